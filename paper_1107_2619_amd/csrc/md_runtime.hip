// Host runtime behind include/md.h: validation, workspace layout, the step
// schedule and the error flags.  Device work is enqueued on the caller's
// stream; nothing here allocates device memory (the caller provides the
// workspace).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "md_internal.h"

using namespace mdk;

struct md_ctx {
    // configuration (copied)
    int32_t R = 0, cap = 0, rebuild_every = 1, precision = MD_FP64, nbr_mode = MD_NBR_FULL, lanes = 1;
    bool compact_ok = false;
    bool compact_on = true;  // MD_OPT_COMPACT
    bool nvt = false;        // Nose-Hoover thermostat per replica
    bool gear = false;       // third-order Gear predictor-corrector instead of Verlet
    bool gear_ready = false; // Gear derivatives started since md_bind
    bool pr = false;         // Parrinello-Rahman barostat per replica
    std::vector<double> pr_P, pr_W;  // GPa, eV fs^2 / A^2
    bool tri = false;        // box matrices (sheared cells; the barostat then moves all nine entries)
    std::vector<double> hmat, pr_S;  // [R][9] box matrices (A), external stress (GPa)
    bool chunked_sums = false;  // some replica spans more than kChunkedSumWaves wavefronts
    std::vector<double> nh_T, nh_Q;
    std::vector<double> nh_gkt;  // host copy of nh_param
    std::vector<int64_t> atom_off;
    std::vector<double> box, origin, vp;
    std::vector<uint8_t> periodic;
    double skin = 0.0, dt_fs = 1.0, rc = 0.0, rlist = 0.0, t0_fs = 0.0;
    double rd = 0.0;  // largest density knot: every density function vanishes beyond it
    // potential
    DevPotential pot{};
    bool single = false;
    PotArgs args{};
    // local-polynomial tables (host copies, uploaded at md_bind)
    bool table_ok = false;
    int32_t table_kind = 0;    // 1 = knots on the bin grid, 2 = knots inside bins (split terms)
    bool explicit_ok = false;  // a compiled knot-sum variant covers the knot counts
    int32_t evaluator = 0;  // 0 = tables, 1 = explicit knot sums (FP64 only)
    std::vector<double> tf64, te64, td64;
    std::vector<float> tf32, te32, td32;
    // derived layout
    int64_t N = 0, Np = 0;
    int32_t C = 0, C_alloc = 0, scan_nb = 0;
    // brick path
    int32_t kernel_path = 1;  // 0 = LDS bricks, 1 = global gathers, 2 = LDS bricks with pairs once
    int32_t nchunk = 4;       // neighbour records in flight per thread (global kernels)
    int32_t brick_dims = 0;   // 0 = automatic, else bd[0] + 10 bd[1] + 100 bd[2]
    int32_t brick_block = 512;
    int32_t lds_limit = 65536;
    int32_t halo_cap = 0;
    int32_t halo_cap_max = 0;
    int64_t halo_overflows = 0;  // bricks evaluated from global memory (last md_energy)
    std::vector<int32_t> brick_rep;
    std::vector<DevReplica> reps;
    std::vector<int32_t> rep_of_wave, cell_shift, cell_rep, chunk_rep, chunk_off;
    size_t ws_bytes = 0;
    std::vector<size_t> off;  // workspace offsets, in Buffers field order
    // binding and run state
    md_state st{};
    void* ws = nullptr;
    bool bound = false, have_slots = false, have_list = false, have_energy = false;
    // md_step may continue from its own state: the internal positions and
    // velocities are those it wrote back, and fhalf holds the forces of the
    // final step (cleared by any call that could change either)
    bool resume_ok = false;
    // per-step energies: every energy_every-th step also reduces PE, KE and the
    // virial and appends them to a device ring of ring_len entries
    int32_t energy_every = 0;
    int64_t ring_len = 0;
    std::vector<int64_t> ring_steps;  // step index of every entry appended (host log)
    int64_t ring_read = 0;            // entries already returned by md_energy_history
    Buffers buf{};
    int p = 0, q = 0;
    int64_t step = 0, built_at = -1, n_builds = 0, max_count = 0;
    // automatic rebuilds (MD_OPT_AUTO_REBUILD): a displacement check before
    // every force evaluation and gated rebuild kernels instead of the fixed
    // period; gate_sel picks the device flag set of the next check, auto_builds
    // counts the triggered builds (as of the last md_energy)
    bool auto_rebuild = false;
    int gate_sel = 0;
    int64_t auto_builds = 0;
    std::vector<int64_t> n_mobile;
    std::string err;
    // optional kernel timing: event pairs per group, resolved lazily
    bool timing = false;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double kt_ms[MD_KT_COUNT] = {0, 0, 0, 0};
    int64_t kt_n[MD_KT_COUNT] = {0, 0, 0, 0};
    // HIP graph replay of md_step (MD_OPT_USE_GRAPH): one executable graph per
    // ping-pong state (p + 2 q) and flag set of the automatic rebuild's checks,
    // each covering two list-rebuild periods (kAutoGraphSteps steps with
    // automatic rebuilds)
    bool use_graph = false;
    hipGraphExec_t graph_exec[8] = {};
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_ev[2] = {nullptr, nullptr};
    int64_t graph_launches = 0;
    double tuned_us = 0.0;  // md_autotune's estimate of one step of the chosen configuration
    void drop_graphs()
    {
        for (auto& g : graph_exec)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    ~md_ctx()
    {
        drop_graphs();
        for (hipEvent_t e : graph_ev)
            if (e) (void)hipEventDestroy(e);
        if (graph_stream) (void)hipStreamDestroy(graph_stream);
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    }
};

namespace {

int fail(md_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

bool hip_ok(md_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return true;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Inverse of a 3x3 matrix (row-major) by cofactors.
void invert3(const double* m, double* o)
{
    const double id =
        1.0 / (m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) + m[2] * (m[3] * m[7] - m[4] * m[6]));
    o[0] = (m[4] * m[8] - m[5] * m[7]) * id;
    o[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    o[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    o[3] = (m[5] * m[6] - m[3] * m[8]) * id;
    o[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    o[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    o[6] = (m[3] * m[7] - m[4] * m[6]) * id;
    o[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    o[8] = (m[0] * m[4] - m[1] * m[3]) * id;
}

// Descriptor fields of a sheared cell with box matrix h (the link-cell counts
// nc already set): inverse, build inverse, strain map, compact-record units,
// and the widths between opposite faces in place of edge lengths.
void set_cell_matrix(DevReplica& D, const double* h)
{
    std::memcpy(D.h, h, sizeof D.h);
    invert3(h, D.hinv);
    std::memcpy(D.hbinv, D.hinv, sizeof D.hbinv);
    for (int e = 0; e < 9; ++e) {
        D.mb[e] = (e % 4 == 0) ? 1.0 : 0.0;
        D.qg[e] = std::ldexp(h[e] / (double)D.nc[e % 3], -kCompactBits);
    }
    for (int a = 0; a < 3; ++a) {
        const double* r = D.hinv + 3 * a;
        const double w = 1.0 / std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        D.box[a] = w;
        D.inv_box[a] = 1.0 / w;
        D.cell[a] = w / (double)D.nc[a];
        D.lbuild[a] = w;
    }
}

KernelShape shape(const md_ctx* c)
{
    KernelShape k;
    k.n_slots = c->Np;
    k.n_cells = c->C;
    k.n_replicas = c->R;
    k.cap = c->cap;
    k.lanes = c->lanes > 0 ? std::min(c->lanes, 4) : 2;  // automatic: two lanes per atom
    k.npk = c->pot.npk;
    k.ndk = c->pot.ndk;
    k.table = (c->table_ok && c->evaluator == 0) ? c->table_kind : 0;
    k.n_chunks = (int32_t)c->chunk_rep.size();
    k.n_bricks = (int32_t)c->brick_rep.size();
    // the barostat moves the bricks' box; the brick kernels take orthorhombic boxes only
    // (the automatic rebuild's gated build covers the global list only)
    k.brick = c->kernel_path != 1 && c->nbr_mode == MD_NBR_FULL && !c->pr && !c->tri && !c->auto_rebuild;
    k.pairs = k.brick && c->kernel_path == 2;
    k.halo_cap = c->halo_cap;
    k.block = c->brick_block;
    k.rowlen = (c->cap + 7) / 8 * 8;
    k.compact = c->precision == MD_MIXED && !k.brick && c->compact_ok && c->compact_on && c->nbr_mode == MD_NBR_FULL;
    if (k.compact && c->tri) k.compact = 2;  // fractional in-cell coordinates
    k.tri = c->tri ? 1 : 0;
    k.chunked = c->chunked_sums ? 1 : 0;
    k.lds_limit = c->lds_limit;
    k.nchunk = c->nchunk;
    k.list_types = c->single ? 0 : 1;
    // FP64 density passes gather 24 bytes per neighbour and gain from skipping
    // the outer entries; the 16-byte compact records of mixed precision do not
    k.split_list = c->precision == MD_FP64 ? 1 : 0;
    return k;
}

// Staging records of all bricks: n_bricks x halo_cap entries.  Every atom lies
// in the halo of at most 27 bricks, and the automatic capacity is 1.25 times
// the expected halo rounded up to 64, so 34 Np + 64 (bricks) entries bound it;
// choose_bricks clamps explicit settings to this size.
size_t stage_entries(const md_ctx* c)
{
    size_t max_bricks = 0;
    for (int r = 0; r < c->R; ++r) max_bricks += (size_t)c->reps[r].nc[0] * c->reps[r].nc[1] * c->reps[r].nc[2];
    return 34 * (size_t)c->Np + 64 * max_bricks;
}

// Brick geometry (LDS path).  One workgroup's LDS holds the halo table, the
// staged atoms (32 bytes each plus a type byte) and the tables of the pass.
// Budget: kLdsBudget per workgroup (two workgroups per CU on 160 KB of LDS) or
// the device limit if lower; a shape set through MD_OPT_BRICK_DIMS may use the
// whole device limit.  Automatic shape: the largest candidate whose
// expected halo, with 25% headroom for density fluctuations, fits the budget;
// the staging area is then sized to that halo, not to the budget, so that as
// many workgroups as possible stay resident.
constexpr int64_t kLdsBudget = 80 * 1024;
constexpr double kHaloHeadroom = 1.25;

void choose_bricks(md_ctx* c, int32_t dims)
{
    const size_t rsz = c->precision == MD_MIXED ? 4 : 8;
    const size_t tables = c->table_ok && c->pot.ns == 1
                              ? (size_t)c->args.nbt * (force_stride(c->table_kind) + value_stride(c->table_kind)) * rsz
                              : 0;
    // an explicit shape may use all the LDS a workgroup can have
    const int64_t budget = dims > 0 ? (int64_t)c->lds_limit : std::min<int64_t>(kLdsBudget, c->lds_limit);
    const int64_t max_cap = std::max<int64_t>(64, std::min<int64_t>(65535, (budget - kHaloTableBytes - (int64_t)tables) / 33));
    static const int cand[][3] = {{4, 4, 4}, {4, 4, 3}, {4, 4, 2}, {4, 3, 2}, {4, 2, 2}, {3, 2, 2},
                                  {2, 2, 2}, {2, 2, 1}, {2, 1, 1}, {1, 1, 1}};
    int64_t cells = 0, bricks = 0;
    double need = 0.0;
    c->brick_rep.clear();
    for (int r = 0; r < c->R; ++r) {
        DevReplica& D = c->reps[r];
        const double vol_cell = (D.box[0] / D.nc[0]) * (D.box[1] / D.nc[1]) * (D.box[2] / D.nc[2]);
        const double vol = D.box[0] * D.box[1] * D.box[2];
        const double apc = D.n_atoms > 0 ? D.n_atoms / vol * vol_cell : 0.0;
        auto halo_of = [&](const int* bd) {
            double h = kHaloHeadroom * apc;
            for (int a = 0; a < 3; ++a) h *= std::min(bd[a], D.nc[a]) + 2;
            return h;
        };
        int bd[3] = {1, 1, 1};
        if (dims > 0) {
            bd[0] = dims % 10;
            bd[1] = (dims / 10) % 10;
            bd[2] = (dims / 100) % 10;
        } else {
            for (const auto& cd : cand)
                if (halo_of(cd) <= max_cap) {
                    for (int a = 0; a < 3; ++a) bd[a] = cd[a];
                    break;
                }
        }
        for (int a = 0; a < 3; ++a) {
            bd[a] = std::max(1, std::min(bd[a], std::min(kBrickMaxDim, D.nc[a])));
            D.bd[a] = bd[a];
            D.nbk[a] = (D.nc[a] + bd[a] - 1) / bd[a];
        }
        need = std::max(need, halo_of(bd));
        D.cpb = bd[0] * bd[1] * bd[2];
        D.cell_off = (int32_t)cells;
        D.brick_off = (int32_t)bricks;
        const int64_t nb = (int64_t)D.nbk[0] * D.nbk[1] * D.nbk[2];
        for (int64_t k = 0; k < nb; ++k) c->brick_rep.push_back(r);
        bricks += nb;
        cells += nb * D.cpb;
    }
    // staging capacity: the largest expected halo (with headroom), whole wavefronts
    int64_t cap = ((int64_t)std::ceil(need) + 63) / 64 * 64;
    const int64_t rec_cap = (int64_t)(stage_entries(c) / std::max<size_t>(c->brick_rep.size(), 1));
    c->halo_cap_max = (int32_t)std::max<int64_t>(64, std::min<int64_t>(max_cap, rec_cap));
    c->halo_cap = (int32_t)std::max<int64_t>(64, std::min<int64_t>(cap, c->halo_cap_max));
    c->C = (int32_t)std::max<int64_t>(cells, 1);
    c->cell_shift.assign(c->C_alloc, 0);
    c->cell_rep.assign(c->C_alloc, -1);
    for (int r = 0; r < c->R; ++r) {
        const DevReplica& D = c->reps[r];
        const int64_t nc = (int64_t)D.nbk[0] * D.nbk[1] * D.nbk[2] * D.cpb;
        for (int64_t k = 0; k < nc; ++k) {
            c->cell_shift[D.cell_off + k] = D.slot_off - D.atom_off;
            c->cell_rep[D.cell_off + k] = r;
        }
    }
    c->brick_dims = dims;
}

// Upload the replica table and the brick/cell maps (after md_bind or a
// change of brick shape); the next call rebuilds the list.
// Link-cell adjacency table on the device (once per geometry; synchronous).
bool build_cell_table(md_ctx* c)
{
    launch_cell_table(c->buf, shape(c), nullptr);
    return hip_ok(c, hipGetLastError(), "cell table") && hip_ok(c, hipStreamSynchronize(nullptr), "cell table");
}

// Edge-dependent fields of a replica descriptor for edges L.
void set_edges(DevReplica& D, const double L[3])
{
    for (int a = 0; a < 3; ++a) {
        D.box[a] = L[a];
        D.inv_box[a] = 1.0 / L[a];
        D.cell[a] = L[a] / (double)D.nc[a];
        D.qs[a] = std::ldexp(D.cell[a], -kCompactBits);
        D.iqs[a] = std::ldexp(1.0 / D.cell[a], kCompactBits);
    }
}

bool upload_geometry(md_ctx* c)
{
    if (!c->bound) return true;
    c->have_list = false;
    if (c->pr) {  // the device holds the barostat's current box: keep it
        std::vector<DevReplica> cur(c->reps.size());
        if (!hip_ok(c, hipMemcpy(cur.data(), c->buf.reps, cur.size() * sizeof(DevReplica), hipMemcpyDeviceToHost), "upload"))
            return false;
        for (size_t r = 0; r < cur.size(); ++r) {
            if (c->tri) {
                DevReplica& D = c->reps[r];
                std::memcpy(D.h, cur[r].h, sizeof D.h);
                std::memcpy(D.hinv, cur[r].hinv, sizeof D.hinv);
                std::memcpy(D.hbinv, cur[r].hbinv, sizeof D.hbinv);
                std::memcpy(D.mb, cur[r].mb, sizeof D.mb);
                std::memcpy(D.qg, cur[r].qg, sizeof D.qg);
                for (int a = 0; a < 3; ++a) {
                    D.box[a] = cur[r].box[a];
                    D.inv_box[a] = cur[r].inv_box[a];
                }
                continue;
            }
            set_edges(c->reps[r], cur[r].box);
            for (int a = 0; a < 3; ++a) c->reps[r].lbuild[a] = cur[r].lbuild[a];
        }
    }
    return hip_ok(c, hipMemcpy(c->buf.reps, c->reps.data(), c->reps.size() * sizeof(DevReplica), hipMemcpyHostToDevice), "upload") &&
           hip_ok(c, hipMemcpy(c->buf.cell_shift, c->cell_shift.data(), c->cell_shift.size() * 4, hipMemcpyHostToDevice), "upload") &&
           hip_ok(c, hipMemcpy(c->buf.cell_rep, c->cell_rep.data(), c->cell_rep.size() * 4, hipMemcpyHostToDevice), "upload") &&
           (c->brick_rep.empty() ||
            hip_ok(c, hipMemcpy(c->buf.brick_rep, c->brick_rep.data(), c->brick_rep.size() * 4, hipMemcpyHostToDevice), "upload")) &&
           build_cell_table(c);
}

// Exact re-expansion of every cubic-knot sum on a grid of bins of width w.
// Inside a bin the set of knots switched on across the whole bin is fixed, so
// their sum f(b w + u) = sum_k a_k (D_k - u)^3, D_k = r_k - b w, is one cubic
// c0 + c1 u + c2 u^2 + c3 u^3.  Kind 1: every knot lies on the bin grid (a
// bin edge), so that cubic is the whole function.  Kind 2 (knots on no common
// grid, as in any coefficient file of "Available potentials"): a bin may hold
// one knot of each function strictly inside; that knot's term a (D - u)^3
// H(D - u) is stored beside the cubic as (D, a) and added in the kernels.
// Returns false only when two knots of one function are closer than the
// finest bin width allowed (4096 bins up to the cutoff).
bool build_tables(md_ctx* c)
{
    const DevPotential& P = c->pot;
    const int n2 = P.ns * P.ns;
    auto on_grid = [](double rk, double w) {
        const double x = rk / w;
        return std::fabs(x - std::nearbyint(x)) <= 1e-9 * std::max(1.0, x);
    };
    // every function's knots: (amplitudes, positions, count)
    struct Fn {
        const double *a, *r;
        int n;
    };
    std::vector<Fn> fns;
    for (int ab = 0; ab < n2; ++ab) {
        fns.push_back({P.pair_a[ab], P.pair_r[ab], P.npk});
        fns.push_back({P.dens_a[ab], P.dens_r[ab], P.ndk});
    }
    auto all_on_grid = [&](double w) {
        for (const Fn& f : fns)
            for (int k = 0; k < f.n; ++k)
                if (f.a[k] != 0.0 && !on_grid(f.r[k], w)) return false;
        return true;
    };
    // kind 2 needs at most one knot of each function strictly inside any bin
    auto one_per_bin = [&](double w) {
        for (const Fn& f : fns) {
            std::vector<int64_t> inside;
            for (int k = 0; k < f.n; ++k)
                if (f.a[k] != 0.0 && !on_grid(f.r[k], w)) inside.push_back((int64_t)std::floor(f.r[k] / w));
            std::sort(inside.begin(), inside.end());
            if (std::adjacent_find(inside.begin(), inside.end()) != inside.end()) return false;
        }
        return true;
    };
    static const double cand[] = {0.02, 0.025, 0.01, 0.05, 0.04, 0.0125, 0.005, 0.002, 0.001};
    double w = 0.0;
    int kind = 1;
    for (double wc : cand)
        if (c->rc / wc <= 4096.0 && all_on_grid(wc)) {
            w = wc;
            break;
        }
    if (w == 0.0) {
        kind = 2;
        for (double wc = 0.02; c->rc / wc <= 4096.0; wc *= 0.5)
            if (one_per_bin(wc)) {
                w = wc;
                break;
            }
    }
    if (w == 0.0) return false;
    const int nb = (int)std::ceil(c->rc / w - 1e-9);
    const int nbt = nb + 2;  // two all-zero bins beyond the cutoff absorb rounding at r -> r_c
    const int FS = force_stride(kind), VS = value_stride(kind);
    c->table_kind = kind;
    c->args.w = w;
    c->args.inv_w = 1.0 / w;
    c->args.nbt = nbt;
    c->tf64.assign((size_t)n2 * nbt * FS, 0.0);
    c->te64.assign((size_t)n2 * nbt * VS, 0.0);
    c->td64.assign((size_t)n2 * nbt * VS, 0.0);
    // out[0..3]: cubic of the knots on across bin b; out[4], out[5]: offset and
    // amplitude of the knot strictly inside bin b (0, 0 if none)
    auto expand = [&](const double* amp, const double* rk, int nk, int b, double out[6]) {
        for (int i = 0; i < 6; ++i) out[i] = 0.0;
        const double base = b * w;
        for (int k = 0; k < nk; ++k) {
            if (amp[k] == 0.0) continue;
            const bool grid = on_grid(rk[k], w);
            // a knot on the grid closes bin llround(rk / w) - 1 and is on across
            // it and every bin below; a knot inside bin kb is on across the bins
            // below kb and becomes a split term of bin kb
            const int64_t kb = grid ? std::llround(rk[k] / w) : (int64_t)std::floor(rk[k] / w);
            const double D = rk[k] - base, a = amp[k];
            if (b < kb) {  // switched on across the whole bin
                out[0] += a * D * D * D;
                out[1] += -3.0 * a * D * D;
                out[2] += 3.0 * a * D;
                out[3] += -a;
            } else if (kb == b && !grid) {
                out[4] = D;
                out[5] = a;
            }
        }
    };
    for (int ab = 0; ab < n2; ++ab)
        for (int b = 0; b < nbt; ++b) {
            double ph[6], rh[6];
            expand(P.pair_a[ab], P.pair_r[ab], P.npk, b, ph);
            expand(P.dens_a[ab], P.dens_r[ab], P.ndk, b, rh);
            double* f = &c->tf64[((size_t)ab * nbt + b) * FS];
            f[0] = ph[1];
            f[1] = 2.0 * ph[2];
            f[2] = 3.0 * ph[3];
            f[3] = rh[1];
            f[4] = 2.0 * rh[2];
            f[5] = 3.0 * rh[3];
            if (kind == 2) {
                f[6] = ph[4];
                f[7] = -3.0 * ph[5];
                f[8] = rh[4];
                f[9] = -3.0 * rh[5];
            }
            for (int i = 0; i < VS; ++i) {
                c->te64[((size_t)ab * nbt + b) * VS + i] = ph[i];
                c->td64[((size_t)ab * nbt + b) * VS + i] = rh[i];
            }
        }
    c->tf32.assign(c->tf64.begin(), c->tf64.end());
    c->te32.assign(c->te64.begin(), c->te64.end());
    c->td32.assign(c->td64.begin(), c->td64.end());
    return true;
}

// Workspace layout: every array 256-byte aligned.  The order here is the
// order of the assignments in bind_buffers.
void plan_workspace(md_ctx* c)
{
    const size_t Np = (size_t)c->Np, C = (size_t)c->C_alloc;
    size_t max_bricks = 0;
    for (int r = 0; r < c->R; ++r)
        max_bricks += (size_t)c->reps[r].nc[0] * c->reps[r].nc[1] * c->reps[r].nc[2];
    // forces kept per slot: the half list's accumulators, the thermostat's,
    // barostat's and Gear's kick, and the forces an md_step call resumes from
    const bool keep_f = true;
    const size_t gear = c->gear ? Np * 8 : 0;
    std::vector<size_t> sizes = {
        Np * 32, Np * 32,                                    // pos[2]
        Np * 8, Np * 8, Np * 8, Np * 8, Np * 8, Np * 8,      // vel[2][3]
        Np * 4, Np * 4,                                      // id[2]
        Np, Np,                                              // type[2]
        Np * 8, Np * 8,                                      // pwork[2]
        Np * 4, Np * 4, Np * 4, Np * 4, Np * 4, Np * 4,      // img[2][3]
        Np * 32,                                             // xbuild
        Np * 8,                                              // femb
        Np * 4 * (size_t)((c->cap + 2 * kChunk - 1) / kChunk * kChunk),  // nbr (nbr_at), a padding group
        Np * 4,                                              // ncount
        Np * 4,                                              // cell_of
        Np * 4,                                              // perm
        C * 4, C * 4, C * 4, C * 4,                          // cell start/count/cursor/shift (C_alloc)
        (size_t)c->scan_nb * 4,                              // scan_blocks
        Np / kWave * 4,                                      // rep_of_wave
        (size_t)c->R * sizeof(DevReplica),                   // reps
        sizeof(DevPotential),                                // pot
        Np * kEnergyTerms * 8,                               // eslot
        (size_t)c->R * kEnergySlots * 8,                     // energies
        c->chunk_rep.size() * 4, c->chunk_off.size() * 4,     // reduction chunks
        c->chunk_rep.size() * kEnergySlots * 8,
        keep_f ? Np * 8 : 0,  // fhalf[3] (also the forces kept by the thermostat and the Gear steps)
        keep_f ? Np * 8 : 0,
        keep_f ? Np * 8 : 0,
        c->nbr_mode == MD_NBR_HALF_ATOMIC ? Np * 8 : 0,     // rhalf
        c->nbr_mode == MD_NBR_HALF_ATOMIC ? Np * 8 : 0,     // ehalf
        (size_t)c->R * 16, (size_t)c->R * 32,                // nh_param, nh_state
        Np / kWave * 8,                                      // nh_partial
        F_COUNT * 4,                                         // flags
        c->tf64.size() * 8, c->te64.size() * 8, c->td64.size() * 8,  // tables FP64
        c->tf32.size() * 4, c->te32.size() * 4, c->td32.size() * 4,  // tables FP32
        (Np * (size_t)((c->cap + 7) / 8 * 8) + 64) * 2,     // nbr16 rows (+ one padding row for prefetches)
        Np * 4,                                              // perm_sorted
        std::max<size_t>(max_bricks, 1) * 4,                 // brick_rep (bricks <= cells)
        std::max<size_t>(max_bricks, 1) * 16,                // brick_info
        stage_entries(c) * 4,                                // stage_src
        Np * 2,                                              // own_li
        Np * 16, Np * 16,                                    // rec[2]
        Np * 16,                                             // cellxyz
        C * 4,                                               // cell_rep (C_alloc)
        C * 27 * 8,                                          // cell_adj
        C * 4,                                               // cell_coord
        (size_t)c->N * 8, (size_t)c->N * 8, (size_t)c->N * 8,  // x0[3]
        (size_t)c->N,                                        // ctype
        std::max<size_t>(c->chunk_rep.size(), 1) * 2 * MD_MAX_SPECIES * 8,  // msd_partial
        (size_t)c->R * 2 * MD_MAX_SPECIES * 8,               // msd_out
        gear, gear, gear, gear, gear, gear,                  // acc[2][3]
        gear, gear, gear, gear, gear, gear,                  // jrk[2][3]
        c->pr ? (size_t)c->R * 16 : 0,                       // pr_param
        c->pr ? (size_t)c->R * (c->tri ? kPrtState : kPrState) * 8 : 0,  // pr_state
        c->pr ? Np / kWave * (c->tri ? 12 : 6) * 8 : 0,      // pr_partial
        (size_t)c->ring_len * c->R * kEnergySlots * 8,       // ering
        16,                                                  // ering_count, ticket
        c->single ? 0 : Np * (size_t)((c->cap + 2 * kChunk - 1) / kChunk * kChunk),  // ntype (several species)
        Np / kWave * kEnergyTerms * 8,                       // wave_terms
        C * 4,                                               // bin_count (C_alloc)
        2 * ((size_t)c->R + 1) * 4,                          // gate
    };
    c->off.clear();
    size_t o = 0;
    for (size_t s : sizes) {
        c->off.push_back(o);
        o = align_up(o + std::max<size_t>(s, 1), 256);
    }
    c->ws_bytes = o;
}

void bind_buffers(md_ctx* c)
{
    char* w = static_cast<char*>(c->ws);
    size_t i = 0;
    auto at = [&](auto*& ptr) { ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(w + c->off[i++]); };
    Buffers& b = c->buf;
    at(b.pos[0]);
    at(b.pos[1]);
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 3; ++a) at(b.vel[k][a]);
    at(b.id[0]);
    at(b.id[1]);
    at(b.type[0]);
    at(b.type[1]);
    at(b.pwork[0]);
    at(b.pwork[1]);
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 3; ++a) at(b.img[k][a]);
    at(b.xbuild);
    at(b.femb);
    at(b.nbr);
    at(b.ncount);
    at(b.cell_of);
    at(b.perm);
    at(b.cell_start);
    at(b.cell_count);
    at(b.cell_cursor);
    at(b.cell_shift);
    at(b.scan_blocks);
    at(b.rep_of_wave);
    at(b.reps);
    at(b.pot);
    at(b.eslot);
    at(b.energies);
    at(b.chunk_rep);
    at(b.chunk_off);
    at(b.chunk_partial);
    for (int a = 0; a < 3; ++a) at(b.fhalf[a]);
    at(b.rhalf);
    at(b.ehalf);
    at(b.nh_param);
    at(b.nh_state);
    at(b.nh_partial);
    at(b.flags);
    at(b.tab_force64);
    at(b.tab_energy64);
    at(b.tab_dens64);
    at(b.tab_force32);
    at(b.tab_energy32);
    at(b.tab_dens32);
    at(b.nbr16);
    at(b.perm_sorted);
    at(b.brick_rep);
    at(b.brick_info);
    at(b.stage_src);
    at(b.own_li);
    at(b.rec[0]);
    at(b.rec[1]);
    at(b.cellxyz);
    at(b.cell_rep);
    at(b.cell_adj);
    at(b.cell_coord);
    for (int a = 0; a < 3; ++a) at(b.x0[a]);
    at(b.ctype);
    at(b.msd_partial);
    at(b.msd_out);
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 3; ++a) at(b.acc[k][a]);
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < 3; ++a) at(b.jrk[k][a]);
    if (!c->gear)  // the sort moves Gear state only where it exists
        for (int k = 0; k < 2; ++k)
            for (int a = 0; a < 3; ++a) b.acc[k][a] = b.jrk[k][a] = nullptr;
    at(b.pr_param);
    at(b.pr_state);
    at(b.pr_partial);
    at(b.ering);
    at(b.ering_count);
    at(b.ntype);
    at(b.wave_terms);
    at(b.bin_count);
    at(b.gate);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int check_launch(md_ctx* c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, MD_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return MD_OK;
}

// Kernel-group timing (MD_OPT_TIMING): an event before and after each group.
hipEvent_t next_event(md_ctx* c)
{
    if (c->event_next == c->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->event_pool.push_back(e);
    }
    return c->event_pool[c->event_next++];
}

struct Timed {
    md_ctx* c;
    int group;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(md_ctx* c_, int g, hipStream_t s_) : c(c_), group(g), s(s_)
    {
        if (!c->timing) return;
        a = next_event(c);
        b = next_event(c);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~Timed()
    {
        if (!c->timing || !a || !b) return;
        (void)hipEventRecord(b, s);
        c->pending.push_back({group, {a, b}});
    }
};

// Resolve recorded event pairs (the stream has been synchronised).
void collect_times(md_ctx* c)
{
    for (auto& pr : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.second.first, pr.second.second) == hipSuccess) {
            c->kt_ms[pr.first] += ms;
            c->kt_n[pr.first] += 1;
        }
    }
    c->pending.clear();
    c->event_next = 0;
}

void ensure_slots(md_ctx* c, hipStream_t s)
{
    if (c->have_slots) return;
    launch_init_slots(c->buf, c->q, c->st, shape(c), s);
    c->have_slots = true;
}

// List build.  Scheduled builds (check_skin) verify that no atom moved more
// than skin/2 since the previous build, i.e. that the list just retired was
// complete; an explicit md_build_neighbours starts afresh.
void rebuild(md_ctx* c, hipStream_t s, bool check_skin)
{
    const KernelShape k = shape(c);
    // under the barostat the skin is shared: 0.4 skin per atom and 0.2 skin for the strain
    const double guard = c->pr ? 0.4 * c->skin : 0.5 * c->skin;
    const double half_skin2 = (c->have_list && check_skin) ? guard * guard : -1.0;
    Timed tm(c, MD_KT_BUILD, s);
    launch_rebuild(c->buf, c->p, c->q, k, half_skin2, c->nbr_mode == MD_NBR_HALF_ATOMIC, nullptr, s);
    c->p ^= 1;
    c->q ^= 1;
    if (k.brick)
        launch_brick_list(c->buf, c->p, c->q, k, c->rlist * c->rlist, k.pairs,
                          k.pairs ? pair_slots(k, c->args, c->precision) : 0, s);
    else {
        // inner entries: within r_d + skin, so a pair left out stays beyond r_d
        // (every density function's last knot) until the next build
        const double rdl = std::min(c->rd + c->skin, c->rlist);
        launch_build_list(c->buf, c->p, c->q, k, c->rlist * c->rlist, rdl * rdl, c->nbr_mode == MD_NBR_HALF_ATOMIC,
                          nullptr, 0, s);
    }
    if (c->pr) launch_pr_mark_build(c->buf, k, s);
    c->have_list = true;
    c->built_at = c->step;
    ++c->n_builds;
}

// Flag set `sel` of the automatic rebuild (two sets alternate: each check
// writes one and clears the other, whose readers have run).
int32_t* gate_set(md_ctx* c, int sel) { return c->buf.gate + (size_t)sel * (c->R + 1); }

// Automatic rebuild ("The Neighbourlist calculation": the list must hold every
// pair that comes within r_c before it is rebuilt): before a force evaluation,
// each replica with an atom more than skin/2 from its position at the last
// build is re-sorted and gets a new list; the others keep theirs.  The rebuild
// kernels run every time and exit at once where nothing is flagged, so a
// captured step needs no host decision.  The sorted state is gathered into the
// other ping-pong buffers and copied back by the list kernel, which leaves the
// buffer indices (fixed in a captured graph) as they were.
void auto_check(md_ctx* c, hipStream_t s)
{
    const KernelShape k = shape(c);
    const int half = c->nbr_mode == MD_NBR_HALF_ATOMIC;
    int32_t* gate = gate_set(c, c->gate_sel);
    const double guard = 0.5 * c->skin;
    const double rdl = std::min(c->rd + c->skin, c->rlist);
    Timed tm(c, MD_KT_BUILD, s);
    launch_skin_check(c->buf, c->p, k, guard * guard, gate, gate_set(c, c->gate_sel ^ 1), s);
    launch_rebuild(c->buf, c->p, c->q, k, -1.0, half, gate, s);
    launch_build_list(c->buf, c->p ^ 1, c->q ^ 1, k, c->rlist * c->rlist, rdl * rdl, half, gate, 1, s);
    c->gate_sel ^= 1;
}

// Caller state -> internal slots at the start of every call.  Compact records
// (mixed mode, global path) follow the positions unless a list build, which
// writes them, comes next.
void load_state(md_ctx* c, hipStream_t s, bool build_next)
{
    const KernelShape k = shape(c);
    ensure_slots(c, s);
    launch_load_state(c->buf, c->p, c->q, c->st, k, s);
    if (k.compact && c->have_list && !build_next) launch_compact_records(c->buf, c->p, k, s);
}

// Automatic rebuilds at the start of a call, after load_state(c, s, true): the
// check on the caller's positions, then the compact records of the replicas
// that kept their list.
void check_loaded(md_ctx* c, hipStream_t s)
{
    auto_check(c, s);
    const KernelShape k = shape(c);
    if (k.compact) launch_compact_records(c->buf, c->p, k, s);
}

// waves: the force pass summed the energy terms per wavefront (energy mode 4)
void reduce_energies(md_ctx* c, const KernelShape& k, hipStream_t s, bool waves = false)
{
    Timed tm(c, MD_KT_REDUCE, s);
    // W = -sum over pairs of g d d / r: the full list sees each pair from both atoms
    const double scale = c->nbr_mode == MD_NBR_HALF_ATOMIC ? -1.0 : -0.5;
    // steps on the per-step energy schedule also append the totals to the ring
    // (the device counter picks the entry, so graph replays append in turn)
    const bool ring = c->ring_len > 0 && c->energy_every > 0 && c->step % c->energy_every == 0;
    if (waves) launch_reduce_waves(c->buf, k, scale, ring ? c->ring_len : 0, s);
    else launch_reduce_energies(c->buf, k, scale, ring ? c->ring_len : 0, s);
    c->have_energy = true;
    if (ring) c->ring_steps.push_back(c->step);
}

// Density and force passes.  reduce = false leaves the energy reduction to
// the caller (the thermostat scales the kinetic terms first).
void forces(md_ctx* c, ForceFlags fl, hipStream_t s, bool reduce = true)
{
    const KernelShape k = shape(c);
    const int half = c->nbr_mode == MD_NBR_HALF_ATOMIC;
    // energy steps of the global kernels whose totals are reduced right away
    // (velocity Verlet, md_eam_forces) sum the energy terms per wavefront in the
    // force pass; the thermostat, barostat and Gear steps rework them per atom
    const bool waves = fl.energy == 1 && reduce && !k.brick && !half && (fl.writeback || (fl.close && fl.open));
    if (waves) fl.energy = 4;
    {
        Timed tm(c, MD_KT_DENSITY, s);
        const int fe = fl.energy == 1 || fl.energy == 4;  // barostat steps (energy 2, 3) need no embedding energies
        if (k.pairs) launch_pair_density(c->buf, c->p, c->q, k, c->args, c->precision, fe, s);
        else if (k.brick) launch_brick_density(c->buf, c->p, c->q, k, c->args, c->precision, fe, s);
        else launch_density(c->buf, c->p, c->q, k, c->args, c->precision, half, fe, s);
    }
    {
        Timed tm(c, MD_KT_FORCE, s);
        if (k.pairs) launch_pair_force(c->buf, c->p, c->q, k, c->args, c->precision, fl, c->dt_fs, c->st, s);
        else if (k.brick) launch_brick_force(c->buf, c->p, c->q, k, c->args, c->precision, fl, c->dt_fs, c->st, s);
        else launch_force(c->buf, c->p, c->q, k, c->args, c->precision, half, fl, c->dt_fs, c->st, s);
    }
    if (fl.open) c->p ^= 1;
    if ((fl.energy == 1 || fl.energy == 4) && reduce) reduce_energies(c, k, s, waves);
}

// Thermostatted step boundary: kinetic energy, `halves` thermostat half steps,
// then the scaled opening kick and drift (which moves the positions to p^1).
void nh_boundary(md_ctx* c, int halves, hipStream_t s)
{
    const KernelShape k = shape(c);
    Timed tm(c, MD_KT_FORCE, s);
    launch_nh_update(c->buf, c->q, k, c->args, halves, c->dt_fs, s);
    launch_nh_open(c->buf, c->p, c->q, k, c->args, c->dt_fs, 1, s);
    c->p ^= 1;
}

// A scheduled list build at this step (none with automatic rebuilds).
bool due(const md_ctx* c) { return !c->auto_rebuild && c->step % c->rebuild_every == 0 && c->built_at != c->step; }

// Before a force evaluation inside md_step: the scheduled build, or the
// automatic rebuild's check.
void before_forces(md_ctx* c, hipStream_t s)
{
    if (due(c)) rebuild(c, s, true);
    else if (c->auto_rebuild) auto_check(c, s);
}

// Steps per captured graph: two rebuild periods (the pattern of scheduled
// builds repeats), or a fixed span with automatic rebuilds.
constexpr int64_t kAutoGraphSteps = 16;
int64_t graph_period(const md_ctx* c) { return c->auto_rebuild ? kAutoGraphSteps : 2 * (int64_t)c->rebuild_every; }

// Barostat step boundary: the stress tensor, the box half kicks (closing,
// opening or both), and with `open` the box drift and the particles' opening
// friction, kick and drift (into pos[p^1]).
void pr_boundary(md_ctx* c, int close, int open, hipStream_t s)
{
    const KernelShape k = shape(c);
    Timed tm(c, MD_KT_FORCE, s);
    if (c->tri) {
        launch_prt_update(c->buf, c->q, k, c->args, close, open, c->dt_fs, c->rlist, 0.2 * c->skin, c->nvt, s);
        if (open) {
            launch_prt_open(c->buf, c->p, c->q, k, c->args, c->dt_fs, s);
            c->p ^= 1;
        }
        return;
    }
    launch_pr_update(c->buf, c->q, k, c->args, close, open, c->dt_fs, c->rlist, 0.2 * c->skin, c->nvt, s);
    if (open) {
        launch_pr_open(c->buf, c->p, c->q, k, c->args, c->dt_fs, s);
        c->p ^= 1;
    }
}

// One Gear step ("Time integration") from predicted positions in pos[p]: the
// list rebuild on schedule (at the predicted positions, where the forces are
// taken), the force pass, then the corrector, which within a call also
// predicts the next step.  The last step of a call also produces the energies
// and writes the caller's state.
void gear_step(md_ctx* c, bool last, hipStream_t s)
{
    ++c->step;
    before_forces(c, s);
    forces(c, last ? ForceFlags{1, 0, 0, 1} : ForceFlags{0, 0, 0, 0}, s, false);
    const KernelShape k = shape(c);
    {
        Timed tm(c, MD_KT_FORCE, s);
        launch_gear_correct(c->buf, c->p, c->q, k, c->args, c->dt_fs, c->st, last ? 1 : 0, s);
    }
    c->p ^= 1;
    if (last) reduce_energies(c, k, s);
}

// The middle steps of md_step (closing kick, list rebuild on schedule, force
// pass, opening kick and drift), `n` of them.
void middle_steps(md_ctx* c, int64_t n, hipStream_t s)
{
    for (int64_t k = 0; k < n; ++k) {
        if (c->gear) {
            gear_step(c, false, s);
            continue;
        }
        ++c->step;
        before_forces(c, s);
        if (c->pr) {
            // closing kick and the virial (the whole tensor for a box matrix), forces kept
            forces(c, ForceFlags{c->tri ? 3 : 2, 1, 0, 0}, s, false);
            pr_boundary(c, 1, 1, s);
        } else if (c->nvt) {
            forces(c, ForceFlags{0, 1, 0, 0}, s);  // closing kick, forces kept
            nh_boundary(c, 2, s);
        } else {
            const int e = c->energy_every > 0 && c->step % c->energy_every == 0 ? 1 : 0;
            forces(c, ForceFlags{e, 1, 1, 0}, s);
        }
    }
}

// Two rebuild periods of middle steps from a step that is a multiple of
// 2 * rebuild_every, replayed from a captured graph.  Over such a span every
// ping-pong index flips an even number of times and the rebuild pattern is
// fixed, so one graph per (p, q) state serves every replay.  With automatic
// rebuilds the span is kAutoGraphSteps steps, each with its check (an even
// number of checks: the flag set in use is the same at both ends).  Capture
// runs the host logic once (advancing the counters as a real run would)
// without executing; a replay advances the counters by the same amounts.
bool replay_period(md_ctx* c, hipStream_t s)
{
    const int64_t P = graph_period(c);
    if (!c->graph_stream) {
        if (!hip_ok(c, hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking), "graph stream") ||
            !hip_ok(c, hipEventCreateWithFlags(&c->graph_ev[0], hipEventDisableTiming), "graph event") ||
            !hip_ok(c, hipEventCreateWithFlags(&c->graph_ev[1], hipEventDisableTiming), "graph event"))
            return false;
    }
    hipStream_t gs = c->graph_stream;
    const int key = c->p + 2 * c->q + 4 * c->gate_sel;
    const int64_t step0 = c->step, builds0 = c->n_builds;
    if (!c->graph_exec[key]) {
        hipGraph_t g = nullptr;
        if (!hip_ok(c, hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed), "graph capture")) return false;
        middle_steps(c, P, gs);
        if (!hip_ok(c, hipStreamEndCapture(gs, &g), "graph capture")) return false;
        const bool ok = hip_ok(c, hipGraphInstantiate(&c->graph_exec[key], g, nullptr, nullptr, 0), "graph instantiate");
        (void)hipGraphDestroy(g);
        if (!ok) {
            c->graph_exec[key] = nullptr;
            return false;
        }
        if (c->p + 2 * c->q + 4 * c->gate_sel != key)
            return fail(c, MD_ERR_STATE, "graph period changed the ping-pong state") == MD_OK;
    } else {
        c->step = step0 + P;
        if (!c->auto_rebuild) {
            c->n_builds = builds0 + 2;
            c->built_at = c->step;
        }
        if (c->ring_len > 0 && c->energy_every > 0 && !c->nvt && !c->pr && !c->gear)
            for (int64_t t = step0 + 1; t <= step0 + P; ++t)
                if (t % c->energy_every == 0) c->ring_steps.push_back(t);
    }
    ++c->graph_launches;
    return hip_ok(c, hipEventRecord(c->graph_ev[0], s), "graph launch") &&
           hip_ok(c, hipStreamWaitEvent(gs, c->graph_ev[0], 0), "graph launch") &&
           hip_ok(c, hipGraphLaunch(c->graph_exec[key], gs), "graph launch") &&
           hip_ok(c, hipEventRecord(c->graph_ev[1], gs), "graph launch") &&
           hip_ok(c, hipStreamWaitEvent(s, c->graph_ev[1], 0), "graph launch");
}

// Per-replica quantities from the reduced totals v[kEnergySlots] of one
// state (nh, pr: the thermostat and barostat states of all replicas, read only
// with those enabled).
void fill_energies(const md_ctx* c, int r, const double* v, const std::vector<double>& nh,
                   const std::vector<double>& pr, int64_t step, md_energies& o)
{
    const int nps = c->tri ? kPrtState : kPrState;
    std::memset(&o, 0, sizeof o);
    const DevReplica& D = c->reps[r];
    const bool has_rigid = c->n_mobile[r] < D.n_atoms;
    const int64_t dof = has_rigid ? 3 * c->n_mobile[r] : 3 * c->n_mobile[r] - 3;
    o.pe = v[E_PE];
    o.ke = v[E_KE];
    o.temperature = dof > 0 ? 2.0 * o.ke / ((double)dof * kBoltzmannEv) : 0.0;
    if (c->tri) {
        // the box matrix, its edge lengths and volume; with the barostat the
        // energy P Omega + W tr(dh/dt^T dh/dt) / 2 + Omega0 tr((S - P) eps),
        // eps = (h0^-T h^T h h0^-1 - 1) / 2 the strain from the bound box h0
        const double* h = c->pr ? &pr[(size_t)nps * r] : &c->hmat[9 * (size_t)r];
        std::memcpy(o.h, h, sizeof o.h);
        for (int a = 0; a < 3; ++a) o.box[a] = std::sqrt(h[a] * h[a] + h[3 + a] * h[3 + a] + h[6 + a] * h[6 + a]);
        o.volume = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) + h[2] * (h[3] * h[7] - h[4] * h[6]);
        if (c->pr) {
            const double* hd = &pr[(size_t)nps * r + 9];
            const double* h0 = &c->hmat[9 * (size_t)r];
            double kb = 0.0;
            for (int e = 0; e < 9; ++e) kb += hd[e] * hd[e];
            double h0i[9], f[9], eps[9];
            invert3(h0, h0i);
            for (int i = 0; i < 3; ++i)  // f = h h0^-1
                for (int j = 0; j < 3; ++j) f[3 * i + j] = h[3 * i] * h0i[j] + h[3 * i + 1] * h0i[3 + j] + h[3 * i + 2] * h0i[6 + j];
            for (int i = 0; i < 3; ++i)  // eps = (f^T f - 1) / 2
                for (int j = 0; j < 3; ++j)
                    eps[3 * i + j] = 0.5 * (f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j] - (i == j ? 1.0 : 0.0));
            const double om0 = h0[0] * (h0[4] * h0[8] - h0[5] * h0[7]) - h0[1] * (h0[3] * h0[8] - h0[5] * h0[6]) +
                               h0[2] * (h0[3] * h0[7] - h0[4] * h0[6]);
            double el = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    el += (c->pr_S[9 * (size_t)r + 3 * i + j] - (i == j ? c->pr_P[r] : 0.0)) * eps[3 * j + i];
            o.pr_energy = (c->pr_P[r] * o.volume + om0 * el) / kEvPerA3InGpa + 0.5 * c->pr_W[r] * kb;
        }
    } else {
        for (int a = 0; a < 3; ++a) o.box[a] = c->pr ? pr[(size_t)kPrState * r + a] : D.box[a];
        for (int a = 0; a < 3; ++a) o.h[4 * a] = o.box[a];
        o.volume = o.box[0] * o.box[1] * o.box[2];
        if (c->pr) {
            const double* ld = &pr[(size_t)kPrState * r + 3];
            o.pr_energy = c->pr_P[r] / kEvPerA3InGpa * o.volume + 0.5 * c->pr_W[r] * (ld[0] * ld[0] + ld[1] * ld[1] + ld[2] * ld[2]);
        }
    }
    for (int k = 0; k < 6; ++k) o.virial[k] = v[E_W0 + k];
    o.pressure_gpa = (2.0 * o.ke + o.virial[0] + o.virial[1] + o.virial[2]) / (3.0 * o.volume) * kEvPerA3InGpa;
    o.piston_work = v[E_PW];
    o.step = step;
    o.n_atoms = D.n_atoms;
    o.n_mobile = c->n_mobile[r];
    if (c->nvt) {
        const double Q = c->nh_gkt[2 * r], gkt = c->nh_gkt[2 * r + 1], pi = nh[4 * r], xi = nh[4 * r + 1];
        o.nh_pi = pi;
        o.nh_energy = 0.5 * Q * pi * pi + gkt * xi;
    }
}

}  // namespace

extern "C" {

int md_create(const md_config* cfg, const md_potential* pot, md_ctx** out)
{
    if (!out) return MD_ERR_ARG;
    *out = nullptr;
    if (!cfg || !pot) return MD_ERR_ARG;
    md_ctx* c = new md_ctx();
    auto reject = [&](int code, const std::string& msg) {
        // keep the context so md_last_error can explain; the caller destroys it
        c->err = msg;
        *out = c;
        return code;
    };
    // ---- configuration
    if (cfg->n_replicas < 1) return reject(MD_ERR_ARG, "n_replicas must be >= 1");
    if (!cfg->atom_offset || !(cfg->box || cfg->box_matrix) || !cfg->periodic)
        return reject(MD_ERR_ARG, "atom_offset, box (or box_matrix) and periodic are required");
    if (cfg->max_neighbours < 1) return reject(MD_ERR_ARG, "max_neighbours must be >= 1");
    if (cfg->rebuild_every < 1) return reject(MD_ERR_ARG, "rebuild_every must be >= 1");
    if (cfg->precision != MD_FP64 && cfg->precision != MD_MIXED) return reject(MD_ERR_ARG, "precision must be MD_FP64 or MD_MIXED");
    if (cfg->nbr_mode != MD_NBR_FULL && cfg->nbr_mode != MD_NBR_HALF_ATOMIC) return reject(MD_ERR_ARG, "nbr_mode must be MD_NBR_FULL or MD_NBR_HALF_ATOMIC");
    if (!(cfg->lanes_per_atom == 0 || cfg->lanes_per_atom == 1 || cfg->lanes_per_atom == 2 || cfg->lanes_per_atom == 4))
        return reject(MD_ERR_ARG, "lanes_per_atom must be 0, 1, 2 or 4");
    if (!(cfg->skin >= 0.0) || !std::isfinite(cfg->skin)) return reject(MD_ERR_ARG, "skin must be finite and >= 0");
    if (!(cfg->dt_fs > 0.0) || !std::isfinite(cfg->dt_fs)) return reject(MD_ERR_ARG, "dt_fs must be finite and > 0");
    c->R = cfg->n_replicas;
    c->cap = cfg->max_neighbours;
    c->rebuild_every = cfg->rebuild_every;
    c->precision = cfg->precision;
    c->nbr_mode = cfg->nbr_mode;
    c->lanes = cfg->lanes_per_atom;  // 0 = automatic
    c->skin = cfg->skin;
    c->dt_fs = cfg->dt_fs;
    if ((cfg->nh_temperature == nullptr) != (cfg->nh_mass == nullptr))
        return reject(MD_ERR_ARG, "nh_temperature and nh_mass go together (both NULL for NVE)");
    c->nvt = cfg->nh_temperature != nullptr;
    if (cfg->integrator != MD_VERLET && cfg->integrator != MD_GEAR3) return reject(MD_ERR_ARG, "integrator must be MD_VERLET or MD_GEAR3");
    c->gear = cfg->integrator == MD_GEAR3;
    if (c->gear && c->nvt) return reject(MD_ERR_ARG, "the Gear integrator runs NVE only (no thermostat)");
    if ((cfg->pr_pressure_gpa == nullptr) != (cfg->pr_mass == nullptr))
        return reject(MD_ERR_ARG, "pr_pressure_gpa and pr_mass go together (both NULL for a fixed box)");
    c->pr = cfg->pr_pressure_gpa != nullptr;
    if (c->pr) {
        if (c->gear) return reject(MD_ERR_ARG, "the barostat runs with velocity Verlet");
        if (cfg->nbr_mode != MD_NBR_FULL) return reject(MD_ERR_ARG, "the barostat needs the full neighbour list");
        c->pr_P.assign(cfg->pr_pressure_gpa, cfg->pr_pressure_gpa + c->R);
        c->pr_W.assign(cfg->pr_mass, cfg->pr_mass + c->R);
        for (int r = 0; r < c->R; ++r) {
            if (!std::isfinite(c->pr_P[r])) return reject(MD_ERR_ARG, "pr_pressure_gpa must be finite");
            if (!(c->pr_W[r] > 0.0) || !std::isfinite(c->pr_W[r])) return reject(MD_ERR_ARG, "pr_mass must be finite and > 0");
        }
    }
    if (c->nvt) {
        c->nh_T.assign(cfg->nh_temperature, cfg->nh_temperature + c->R);
        c->nh_Q.assign(cfg->nh_mass, cfg->nh_mass + c->R);
        for (int r = 0; r < c->R; ++r) {
            if (!(c->nh_T[r] >= 0.0) || !std::isfinite(c->nh_T[r])) return reject(MD_ERR_ARG, "nh_temperature must be finite and >= 0");
            if (!(c->nh_Q[r] > 0.0) || !std::isfinite(c->nh_Q[r])) return reject(MD_ERR_ARG, "nh_mass must be finite and > 0");
        }
    }
    c->atom_off.assign(cfg->atom_offset, cfg->atom_offset + c->R + 1);
    if (c->atom_off[0] != 0) return reject(MD_ERR_ARG, "atom_offset[0] must be 0");
    for (int r = 0; r < c->R; ++r)
        if (c->atom_off[r + 1] < c->atom_off[r]) return reject(MD_ERR_ARG, "atom_offset must be non-decreasing");
    c->N = c->atom_off[c->R];
    c->periodic.assign(cfg->periodic, cfg->periodic + 3 * c->R);
    // box matrices: a sheared cell per replica, or the full-matrix barostat
    // (an external stress) starting from orthorhombic boxes
    if (cfg->pr_stress_gpa && !c->pr) return reject(MD_ERR_ARG, "pr_stress_gpa needs the barostat (pr_pressure_gpa and pr_mass)");
    c->tri = cfg->box_matrix != nullptr || cfg->pr_stress_gpa != nullptr;
    if (c->tri) {
        c->hmat.assign(9 * (size_t)c->R, 0.0);
        c->box.assign(3 * (size_t)c->R, 0.0);
        for (int r = 0; r < c->R; ++r) {
            double* h = &c->hmat[9 * (size_t)r];
            if (cfg->box_matrix) std::memcpy(h, cfg->box_matrix + 9 * (size_t)r, 9 * sizeof(double));
            else
                for (int a = 0; a < 3; ++a) h[4 * a] = cfg->box[3 * (size_t)r + a];
            for (int e = 0; e < 9; ++e)
                if (!std::isfinite(h[e])) return reject(MD_ERR_BOX, "box_matrix entries must be finite");
            const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) + h[2] * (h[3] * h[7] - h[4] * h[6]);
            if (!(det > 0.0)) return reject(MD_ERR_BOX, "box_matrix must have a positive determinant (right-handed edge vectors)");
            for (int a = 0; a < 3; ++a) {
                if (cfg->periodic[3 * (size_t)r + a] != 1) return reject(MD_ERR_ARG, "a box matrix needs every axis periodic");
                // width between the faces spanned by the other two edges: volume / |their cross product|
                const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
                const double cx = h[3 + b1] * h[6 + b2] - h[6 + b1] * h[3 + b2];
                const double cy = h[6 + b1] * h[b2] - h[b1] * h[6 + b2];
                const double cz = h[b1] * h[3 + b2] - h[3 + b1] * h[b2];
                c->box[3 * (size_t)r + a] = det / std::sqrt(cx * cx + cy * cy + cz * cz);
            }
        }
        if (c->pr) {
            c->pr_S.assign(9 * (size_t)c->R, 0.0);
            for (int r = 0; r < c->R; ++r) {
                double* S = &c->pr_S[9 * (size_t)r];
                if (cfg->pr_stress_gpa) std::memcpy(S, cfg->pr_stress_gpa + 9 * (size_t)r, 9 * sizeof(double));
                else
                    for (int a = 0; a < 3; ++a) S[4 * a] = c->pr_P[r];
                double scale = 0.0;
                for (int e = 0; e < 9; ++e) {
                    if (!std::isfinite(S[e])) return reject(MD_ERR_ARG, "pr_stress_gpa entries must be finite");
                    scale = std::max(scale, std::fabs(S[e]));
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = a + 1; b < 3; ++b)
                        if (std::fabs(S[3 * a + b] - S[3 * b + a]) > 1e-12 * scale)
                            return reject(MD_ERR_ARG, "pr_stress_gpa must be symmetric");
            }
        }
    } else {
        c->box.assign(cfg->box, cfg->box + 3 * c->R);
    }
    c->origin.assign(3 * c->R, 0.0);
    if (cfg->origin) c->origin.assign(cfg->origin, cfg->origin + 3 * c->R);
    c->vp.assign(3 * c->R, 0.0);
    if (cfg->rigid_velocity) c->vp.assign(cfg->rigid_velocity, cfg->rigid_velocity + 3 * c->R);
    for (int i = 0; i < 3 * c->R; ++i) {
        if (!(c->box[i] > 0.0) || !std::isfinite(c->box[i])) return reject(MD_ERR_BOX, "box lengths must be finite and > 0");
        if (c->periodic[i] > 1) return reject(MD_ERR_ARG, "periodic flags must be 0 or 1");
        if (!std::isfinite(c->origin[i]) || !std::isfinite(c->vp[i])) return reject(MD_ERR_ARG, "origin and rigid_velocity must be finite");
    }

    // ---- potential (paper: the material module must accept the species, else
    // the run halts before it starts - the analogue of a non-zero ierror)
    const int ns = pot->n_species, npk = pot->n_pair_knots, ndk = pot->n_dens_knots;
    if (ns < 1 || ns > MD_MAX_SPECIES) return reject(MD_ERR_POTENTIAL, "n_species must be 1..4");
    if (npk < 1 || npk > MD_MAX_KNOTS || ndk < 1 || ndk > MD_MAX_KNOTS) return reject(MD_ERR_POTENTIAL, "knot counts must be 1..16");
    if (pot->reserved != 0) return reject(MD_ERR_POTENTIAL, "reserved must be 0");
    if (!pot->pair_a || !pot->pair_r || !pot->dens_A || !pot->dens_R || !pot->emb_c || !pot->mass_amu)
        return reject(MD_ERR_POTENTIAL, "potential arrays are required");
    DevPotential& P = c->pot;
    P.ns = ns;
    P.npk = npk;
    P.ndk = ndk;
    double rc = 0.0;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const int ab = a * ns + b, ba = b * ns + a;
            for (int k = 0; k < npk; ++k) {
                const double A = pot->pair_a[ab * npk + k], Rk = pot->pair_r[ab * npk + k];
                if (!std::isfinite(A) || !std::isfinite(Rk) || Rk < 0.0) return reject(MD_ERR_POTENTIAL, "pair coefficients must be finite, knots >= 0");
                if (A != pot->pair_a[ba * npk + k] || Rk != pot->pair_r[ba * npk + k])
                    return reject(MD_ERR_POTENTIAL, "pair potential must be symmetric in the two species");
                P.pair_a[ab][k] = A;
                P.pair_d[ab][k] = -3.0 * A;
                P.pair_r[ab][k] = Rk;
                rc = std::max(rc, Rk);
            }
            for (int k = 0; k < ndk; ++k) {
                const double A = pot->dens_A[ab * ndk + k], Rk = pot->dens_R[ab * ndk + k];
                if (!(A > 0.0) || !std::isfinite(A) || !std::isfinite(Rk) || !(Rk > 0.0))
                    return reject(MD_ERR_POTENTIAL, "density amplitudes and knots must be finite and > 0 (rho must stay >= 0)");
                P.dens_a[ab][k] = A;
                P.dens_d[ab][k] = -3.0 * A;
                P.dens_r[ab][k] = Rk;
                rc = std::max(rc, Rk);
            }
        }
    c->t0_fs = std::sqrt(kAmuKg * 1.0e-20 / kEvJ) * 1.0e15;
    for (int a = 0; a < ns; ++a) {
        const double m = pot->mass_amu[a], ec = pot->emb_c[a];
        if (!(m > 0.0) || !std::isfinite(m)) return reject(MD_ERR_POTENTIAL, "masses must be finite and > 0");
        if (!(ec >= 0.0) || !std::isfinite(ec)) return reject(MD_ERR_POTENTIAL, "emb_c must be finite and >= 0");
        P.emb_c[a] = ec;
        P.accel[a] = 1.0 / (m * c->t0_fs * c->t0_fs);
        P.half_m[a] = 0.5 * m * c->t0_fs * c->t0_fs;
    }
    if (!(rc > 0.0)) return reject(MD_ERR_POTENTIAL, "cutoff (largest knot) must be > 0");
    c->rc = rc;
    c->rlist = rc + c->skin;
    c->rd = 0.0;
    for (int ab = 0; ab < ns * ns; ++ab)
        for (int k = 0; k < ndk; ++k) c->rd = std::max(c->rd, P.dens_r[ab][k]);
    P.rc = rc;
    P.rc2 = rc * rc;
    P.rlist2 = c->rlist * c->rlist;
    c->single = ns == 1;
    c->args.ns = ns;
    c->args.rc2 = P.rc2;
    c->table_ok = build_tables(c);
    // term-by-term sums: <= 8 + 8 knots, or one species with <= 16 pair and <= 4
    // density knots (a 13 + 2 iron potential of the paper's benchmark fits)
    c->explicit_ok = (npk <= 8 && ndk <= 8) || (ns == 1 && npk <= 16 && ndk <= 4);
    // mixed precision meets its tolerances only through the exact tables: its
    // FP32 knot sums lose the per-atom energies to cancellation between terms
    if (c->precision == MD_MIXED && !c->table_ok)
        return reject(MD_ERR_POTENTIAL, "mixed precision needs the exact tables, and two knots of one function "
                                        "lie closer than the finest table bin (r_c / 4096)");
    if (!c->table_ok && !c->explicit_ok)
        return reject(MD_ERR_POTENTIAL, "more than 8 knots need the tables, and two knots of one function lie "
                                        "closer than the finest table bin (or one species with at most 4 "
                                        "density knots)");
    if (c->single) {
        PotArgs& A = c->args;
        for (int k = 0; k < MD_MAX_KNOTS; ++k) {
            A.pair_a[k] = P.pair_a[0][k];
            A.pair_d[k] = P.pair_d[0][k];
            A.pair_r[k] = P.pair_r[0][k];
            A.dens_a[k] = P.dens_a[0][k];
            A.dens_d[k] = P.dens_d[0][k];
            A.dens_r[k] = P.dens_r[0][k];
            A.pair_af[k] = (float)A.pair_a[k];
            A.pair_df[k] = (float)A.pair_d[k];
            A.dens_af[k] = (float)A.dens_a[k];
            A.dens_df[k] = (float)A.dens_d[k];
        }
        A.emb_c = P.emb_c[0];
        A.accel = P.accel[0];
        A.half_m = P.half_m[0];
    }

    // ---- replicas, wavefront-aligned slot ranges, link-cell grids
    // (paper: link cells at least the potential range plus the padding rpad)
    int64_t slot = 0, cells_alloc = 0;
    double cell_min = 1e300;
    c->reps.resize(c->R);
    for (int r = 0; r < c->R; ++r) {
        DevReplica& D = c->reps[r];
        const int64_t n = c->atom_off[r + 1] - c->atom_off[r];
        D.slot_off = (int32_t)slot;
        D.n_atoms = (int32_t)n;
        D.atom_off = (int32_t)c->atom_off[r];
        D.periodic_mask = 0;
        int64_t worst = 1;
        for (int a = 0; a < 3; ++a) {
            const double L = c->box[3 * r + a];
            const bool per = c->periodic[3 * r + a];
            if (per && !(L > 2.0 * c->rlist)) {
                char msg[160];
                std::snprintf(msg, sizeof msg, "replica %d axis %d: periodic length %.6g must exceed 2*(cutoff+skin) = %.6g", r, a, L,
                              2.0 * c->rlist);
                return reject(MD_ERR_BOX, msg);
            }
            D.box[a] = L;
            D.inv_box[a] = 1.0 / L;
            D.origin[a] = c->origin[3 * r + a];
            D.vp[a] = c->vp[3 * r + a];
            // under the barostat the grid leaves 5% room for compression
            int64_t nc = (int64_t)std::floor(L / (c->pr ? 1.05 * c->rlist : c->rlist));
            nc = std::max<int64_t>(1, std::min<int64_t>(nc, 1023));
            if (c->tri && nc < 3) {  // L is the width between opposite faces here
                char msg[200];
                std::snprintf(msg, sizeof msg,
                              "replica %d: a box matrix needs at least three link cells between each pair of faces "
                              "(width %.6g, list radius %.6g)", r, L, c->rlist);
                return reject(MD_ERR_BOX, msg);
            }
            if (c->pr && (!per || nc < 3)) {
                char msg[160];
                std::snprintf(msg, sizeof msg, "replica %d axis %d: the barostat needs a periodic axis of at least three link cells", r, a);
                return reject(c->pr && !per ? MD_ERR_ARG : MD_ERR_BOX, msg);
            }
            D.nc[a] = (int32_t)nc;
            D.cell[a] = L / (double)nc;
            D.qs[a] = std::ldexp(D.cell[a], -kCompactBits);
            D.iqs[a] = std::ldexp(1.0 / D.cell[a], kCompactBits);
            D.lbuild[a] = L;
            cell_min = std::min(cell_min, D.cell[a]);
            if (per) D.periodic_mask |= 1 << a;
            worst *= nc + kBrickMaxDim - 1;  // cells of the grid padded to whole bricks
        }
        D.tri = c->tri ? 1 : 0;
        if (c->tri) set_cell_matrix(D, &c->hmat[9 * (size_t)r]);
        slot += (n + kWave - 1) / kWave * kWave;
        cells_alloc += worst;
        if (slot > (int64_t)kIndexMask || cells_alloc > (int64_t)INT32_MAX / 2)
            return reject(MD_ERR_ARG, "system too large: at most 2^25 atom slots and 2^30 link cells");
    }
    c->Np = std::max<int64_t>(slot, kWave);
    for (const DevReplica& D : c->reps)
        if ((D.n_atoms + kWave - 1) / kWave > kChunkedSumWaves) c->chunked_sums = true;
    // compact records hold coordinates up to kCompactCells cell edges from
    // their cell; cells under half the list radius (a free axis of a thin
    // slab) could see atoms beyond that between builds
    c->compact_ok = cell_min >= 0.5 * c->rlist;
    c->C_alloc = (int32_t)std::max<int64_t>(cells_alloc, 1);
    c->scan_nb = (c->C_alloc + 1023) / 1024;
    if (c->scan_nb > 1024 * 64) return reject(MD_ERR_ARG, "too many link cells");
    c->rep_of_wave.assign(c->Np / kWave, 0);
    for (int r = 0; r < c->R; ++r) {
        const int64_t w0 = c->reps[r].slot_off / kWave;
        const int64_t w1 = (c->reps[r].slot_off + c->reps[r].n_atoms + kWave - 1) / kWave;
        for (int64_t w = w0; w < w1; ++w) c->rep_of_wave[w] = r;
    }
    // energy-reduction chunks of kReduceChunk slots, per replica
    c->chunk_off.assign(c->R + 1, 0);
    c->chunk_rep.clear();
    for (int r = 0; r < c->R; ++r) {
        const int64_t nch = (c->reps[r].n_atoms + kReduceChunk - 1) / kReduceChunk;
        for (int64_t k = 0; k < nch; ++k) c->chunk_rep.push_back(r);
        c->chunk_off[r + 1] = (int32_t)c->chunk_rep.size();
    }
    // LDS available to one workgroup (a device query when a GPU is visible)
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            c->lds_limit = lds;
        (void)hipGetLastError();
    }
    choose_bricks(c, 0);
    plan_workspace(c);
    *out = c;
    return MD_OK;
}

int md_workspace_bytes(const md_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return MD_ERR_ARG;
    *bytes = c->ws_bytes;
    return MD_OK;
}

int md_bind(md_ctx* c, const md_state* st, void* workspace, size_t bytes)
{
    if (!c || !st || !workspace) return fail(c, MD_ERR_ARG, "md_bind: NULL argument");
    if (!c->err.empty() && c->ws_bytes == 0) return fail(c, MD_ERR_STATE, "md_bind: context was not created successfully");
    if (bytes < c->ws_bytes) return fail(c, MD_ERR_ARG, "md_bind: workspace smaller than md_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(c, MD_ERR_ARG, "md_bind: workspace must be 256-byte aligned");
    if (c->N > 0 && (!st->x || !st->y || !st->z || !st->vx || !st->vy || !st->vz || !st->fx || !st->fy || !st->fz || !st->species))
        return fail(c, MD_ERR_ARG, "md_bind: x, v, f and species are required");
    c->st = *st;
    c->ws = workspace;
    bind_buffers(c);
    if (c->pr)  // the barostat restarts from the configured box
        for (int r = 0; r < c->R; ++r) {
            DevReplica& D = c->reps[r];
            if (c->tri) {
                set_cell_matrix(D, &c->hmat[9 * (size_t)r]);
                continue;
            }
            set_edges(D, &c->box[3 * (size_t)r]);
            for (int a = 0; a < 3; ++a) D.lbuild[a] = c->box[3 * (size_t)r + a];
        }
    if (!hip_ok(c, hipMemcpy(c->buf.reps, c->reps.data(), c->reps.size() * sizeof(DevReplica), hipMemcpyHostToDevice), "md_bind upload") ||
        !hip_ok(c, hipMemcpy(c->buf.pot, &c->pot, sizeof(DevPotential), hipMemcpyHostToDevice), "md_bind upload") ||
        !hip_ok(c, hipMemcpy(c->buf.rep_of_wave, c->rep_of_wave.data(), c->rep_of_wave.size() * 4, hipMemcpyHostToDevice), "md_bind upload") ||
        !hip_ok(c, hipMemcpy(c->buf.cell_shift, c->cell_shift.data(), c->cell_shift.size() * 4, hipMemcpyHostToDevice), "md_bind upload") ||
        !hip_ok(c, hipMemcpy(c->buf.cell_rep, c->cell_rep.data(), c->cell_rep.size() * 4, hipMemcpyHostToDevice), "md_bind upload") ||
        (!c->brick_rep.empty() &&
         !hip_ok(c, hipMemcpy(c->buf.brick_rep, c->brick_rep.data(), c->brick_rep.size() * 4, hipMemcpyHostToDevice), "md_bind upload")) ||
        !hip_ok(c, hipMemcpy(c->buf.chunk_off, c->chunk_off.data(), c->chunk_off.size() * 4, hipMemcpyHostToDevice), "md_bind upload") ||
        (!c->chunk_rep.empty() &&
         !hip_ok(c, hipMemcpy(c->buf.chunk_rep, c->chunk_rep.data(), c->chunk_rep.size() * 4, hipMemcpyHostToDevice), "md_bind upload")) ||
        !hip_ok(c, hipMemset(c->buf.flags, 0, F_COUNT * 4), "md_bind flags") ||
        !hip_ok(c, hipMemset(c->buf.ering_count, 0, 16), "md_bind energy ring") ||
        !hip_ok(c, hipMemset(c->buf.bin_count, 0, (size_t)c->C_alloc * 4), "md_bind cell counters") ||
        !hip_ok(c, hipMemset(c->buf.gate, 0, 2 * ((size_t)c->R + 1) * 4), "md_bind rebuild flags"))
        return MD_ERR_DEVICE;
    if (c->table_ok &&
        (!hip_ok(c, hipMemcpy(c->buf.tab_force64, c->tf64.data(), c->tf64.size() * 8, hipMemcpyHostToDevice), "md_bind tables") ||
         !hip_ok(c, hipMemcpy(c->buf.tab_energy64, c->te64.data(), c->te64.size() * 8, hipMemcpyHostToDevice), "md_bind tables") ||
         !hip_ok(c, hipMemcpy(c->buf.tab_dens64, c->td64.data(), c->td64.size() * 8, hipMemcpyHostToDevice), "md_bind tables") ||
         !hip_ok(c, hipMemcpy(c->buf.tab_force32, c->tf32.data(), c->tf32.size() * 4, hipMemcpyHostToDevice), "md_bind tables") ||
         !hip_ok(c, hipMemcpy(c->buf.tab_energy32, c->te32.data(), c->te32.size() * 4, hipMemcpyHostToDevice), "md_bind tables") ||
         !hip_ok(c, hipMemcpy(c->buf.tab_dens32, c->td32.data(), c->td32.size() * 4, hipMemcpyHostToDevice), "md_bind tables")))
        return MD_ERR_DEVICE;
    // species range and mobile counts per replica, checked once on the host
    std::vector<uint8_t> sp(c->N), rg(c->N, 0);
    if (c->N > 0) {
        if (!hip_ok(c, hipMemcpy(sp.data(), st->species, c->N, hipMemcpyDeviceToHost), "md_bind species")) return MD_ERR_DEVICE;
        if (st->rigid && !hip_ok(c, hipMemcpy(rg.data(), st->rigid, c->N, hipMemcpyDeviceToHost), "md_bind rigid")) return MD_ERR_DEVICE;
    }
    for (int64_t i = 0; i < c->N; ++i)
        if (sp[i] >= c->pot.ns) return fail(c, MD_ERR_POTENTIAL, "md_bind: species index out of range of the potential");
    c->n_mobile.assign(c->R, 0);
    for (int r = 0; r < c->R; ++r)
        for (int64_t i = c->atom_off[r]; i < c->atom_off[r + 1]; ++i) c->n_mobile[r] += rg[i] ? 0 : 1;
    {
        // thermostat: mass Q and g k_B T per replica (g as in the temperature), pi = xi = 0
        std::vector<double> param(2 * (size_t)c->R, 0.0), state(4 * (size_t)c->R, 0.0);
        for (int r = 0; r < c->R; ++r) {
            const bool has_rigid = c->n_mobile[r] < c->reps[r].n_atoms;
            const double dof = std::max<double>(0.0, has_rigid ? 3.0 * c->n_mobile[r] : 3.0 * c->n_mobile[r] - 3.0);
            param[2 * r] = c->nvt ? c->nh_Q[r] : 1.0;
            param[2 * r + 1] = c->nvt ? dof * kBoltzmannEv * c->nh_T[r] : 0.0;
            state[4 * r + 2] = 1.0;
        }
        if (!hip_ok(c, hipMemcpy(c->buf.nh_param, param.data(), param.size() * 8, hipMemcpyHostToDevice), "md_bind thermostat") ||
            !hip_ok(c, hipMemcpy(c->buf.nh_state, state.data(), state.size() * 8, hipMemcpyHostToDevice), "md_bind thermostat"))
            return MD_ERR_DEVICE;
        c->nh_gkt.assign(param.begin(), param.end());
    }
    if (c->pr) {
        // barostat: W and P per replica; the box starts at the configured edges at rest
        for (int r = 0; r < c->R; ++r)
            if (c->n_mobile[r] < c->reps[r].n_atoms) return fail(c, MD_ERR_ARG, "md_bind: the barostat takes no rigid atoms");
        const int ns = c->tri ? kPrtState : kPrState;
        std::vector<double> param(2 * (size_t)c->R), state((size_t)ns * c->R, 0.0);
        for (int r = 0; r < c->R; ++r) {
            param[2 * r] = c->pr_W[r];
            param[2 * r + 1] = c->pr_P[r] / kEvPerA3InGpa;
            if (c->tri) {
                // h, dh/dt = 0, Sigma = Omega0 h0^-1 (S - P) h0^-T (eV), identity maps
                double* st = &state[(size_t)ns * r];
                const double* h0 = &c->hmat[9 * (size_t)r];
                double hi[9], sp[9];
                invert3(h0, hi);
                const double om0 = h0[0] * (h0[4] * h0[8] - h0[5] * h0[7]) - h0[1] * (h0[3] * h0[8] - h0[5] * h0[6]) +
                                   h0[2] * (h0[3] * h0[7] - h0[4] * h0[6]);
                for (int e = 0; e < 9; ++e) sp[e] = (c->pr_S[9 * (size_t)r + e] - (e % 4 == 0 ? c->pr_P[r] : 0.0)) / kEvPerA3InGpa;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double v = 0.0;
                        for (int k = 0; k < 3; ++k)
                            for (int l = 0; l < 3; ++l) v += hi[3 * i + k] * sp[3 * k + l] * hi[3 * j + l];
                        st[18 + 3 * i + j] = om0 * v;
                    }
                std::memcpy(st, h0, 9 * sizeof(double));
                for (int e = 0; e < 9; e += 4) st[27 + e] = st[36 + e] = st[54 + e] = 1.0;
                continue;
            }
            for (int a = 0; a < 3; ++a) {
                state[(size_t)kPrState * r + a] = c->box[3 * r + a];
                state[(size_t)kPrState * r + 6 + a] = 1.0;
                state[(size_t)kPrState * r + 9 + a] = 1.0;
                state[(size_t)kPrState * r + 15 + a] = 1.0;
            }
        }
        if (!hip_ok(c, hipMemcpy(c->buf.pr_param, param.data(), param.size() * 8, hipMemcpyHostToDevice), "md_bind barostat") ||
            !hip_ok(c, hipMemcpy(c->buf.pr_state, state.data(), state.size() * 8, hipMemcpyHostToDevice), "md_bind barostat"))
            return MD_ERR_DEVICE;
    }
    if (c->N > 0) {
        // mean square displacement: species and rigid flag in caller order, and
        // the bound positions as the origin
        std::vector<uint8_t> ct(c->N);
        for (int64_t i = 0; i < c->N; ++i) ct[i] = (uint8_t)(sp[i] | (rg[i] ? kRigidBit : 0));
        const size_t nb = (size_t)c->N * 8;
        if (!hip_ok(c, hipMemcpy(c->buf.ctype, ct.data(), c->N, hipMemcpyHostToDevice), "md_bind msd") ||
            !hip_ok(c, hipMemcpy(c->buf.x0[0], st->x, nb, hipMemcpyDeviceToDevice), "md_bind msd") ||
            !hip_ok(c, hipMemcpy(c->buf.x0[1], st->y, nb, hipMemcpyDeviceToDevice), "md_bind msd") ||
            !hip_ok(c, hipMemcpy(c->buf.x0[2], st->z, nb, hipMemcpyDeviceToDevice), "md_bind msd"))
            return MD_ERR_DEVICE;
    }
    c->bound = true;
    c->gear_ready = false;
    c->resume_ok = false;
    c->ring_steps.clear();
    c->ring_read = 0;
    c->drop_graphs();
    if (!build_cell_table(c)) return MD_ERR_DEVICE;
    c->have_slots = c->have_list = c->have_energy = false;
    c->p = c->q = 0;
    c->step = 0;
    c->built_at = -1;
    c->n_builds = 0;
    c->auto_builds = 0;
    c->gate_sel = 0;
    c->max_count = 0;
    c->err.clear();
    return MD_OK;
}

int md_build_neighbours(md_ctx* c, void* stream)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_build_neighbours: call md_bind first");
    c->resume_ok = false;
    hipStream_t s = as_stream(stream);
    load_state(c, s, true);
    rebuild(c, s, false);
    return check_launch(c);
}

int md_eam_forces(md_ctx* c, int want_energy, void* stream)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_eam_forces: call md_bind first");
    c->resume_ok = false;
    hipStream_t s = as_stream(stream);
    load_state(c, s, !c->have_list || c->auto_rebuild);
    if (!c->have_list) rebuild(c, s, false);
    else if (c->auto_rebuild) check_loaded(c, s);
    forces(c, ForceFlags{want_energy ? 1 : 0, 0, 0, 1}, s);
    return check_launch(c);
}

int md_step(md_ctx* c, int32_t nsteps, void* stream)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_step: call md_bind first");
    if (nsteps < 1) return fail(c, MD_ERR_ARG, "md_step: nsteps must be >= 1");
    hipStream_t s = as_stream(stream);
    // continuing from the last md_step call (no md_state_changed, md_bind or
    // other call in between): the internal state and the kept forces are
    // current, so the step starts with the opening kick and drift alone
    const bool resume = c->resume_ok && !c->gear && !c->pr && c->have_list && !due(c);
    c->resume_ok = false;
    const bool build = !resume && (!c->have_list || due(c));
    if (!resume) load_state(c, s, build || c->auto_rebuild);
    if (build) rebuild(c, s, true);
    else if (!resume && c->auto_rebuild) check_loaded(c, s);
    if (resume) {
        if (c->nvt) {
            nh_boundary(c, 1, s);  // thermostat half step, opening kick, drift
        } else {
            Timed tm(c, MD_KT_FORCE, s);
            launch_nh_open(c->buf, c->p, c->q, shape(c), c->args, c->dt_fs, 0, s);  // opening kick, drift
            c->p ^= 1;
        }
    } else if (c->gear) {
        if (!c->gear_ready) {
            forces(c, ForceFlags{0, 0, 0, 0}, s);  // f(x0): a = f/m, da/dt = 0
            launch_gear_start(c->buf, c->q, shape(c), c->args, s);
            c->gear_ready = true;
        }
        {
            Timed tm(c, MD_KT_FORCE, s);  // first prediction of the call
            launch_gear_predict(c->buf, c->p, c->q, shape(c), c->args, c->dt_fs, s);
        }
        c->p ^= 1;
    } else if (c->pr) {
        forces(c, ForceFlags{c->tri ? 3 : 2, 0, 0, 0}, s, false);  // f(x0) and the virial
        pr_boundary(c, 0, 1, s);                      // box half kick and drift, opening kick and drift
    } else if (c->nvt) {
        forces(c, ForceFlags{0, 0, 0, 0}, s);  // f(x0) kept for the kick
        nh_boundary(c, 1, s);                  // thermostat half step, opening kick, drift
    } else {
        forces(c, ForceFlags{0, 0, 1, 0}, s);  // f(x0), opening half kick, drift
    }
    const int64_t P = graph_period(c);
    int64_t left = nsteps - 1;  // middle steps
    while (left > 0) {
        if (c->use_graph && !c->timing && c->step % P == 0 && left >= P) {
            if (!replay_period(c, s)) return c->err.empty() ? fail(c, MD_ERR_DEVICE, "graph replay") : MD_ERR_DEVICE;
            left -= P;
            continue;
        }
        // eager steps up to the next period boundary (or the end)
        const int64_t n = c->use_graph ? std::min(left, P - c->step % P) : left;
        middle_steps(c, n, s);
        left -= n;
    }
    if (c->gear) {
        gear_step(c, true, s);
        return check_launch(c);
    }
    ++c->step;
    before_forces(c, s);
    if (c->pr) {
        forces(c, ForceFlags{1, 1, 0, 1}, s, false);  // closing kick, energies, write back
        const KernelShape k = shape(c);
        {
            Timed tm(c, MD_KT_FORCE, s);
            if (c->tri) {
                launch_prt_update(c->buf, c->q, k, c->args, 1, 0, c->dt_fs, c->rlist, 0.2 * c->skin, c->nvt, s);
                launch_prt_close_scale(c->buf, c->q, k, c->args, c->st, s);
            } else {
                launch_pr_update(c->buf, c->q, k, c->args, 1, 0, c->dt_fs, c->rlist, 0.2 * c->skin, c->nvt, s);  // closing halves
                launch_pr_close_scale(c->buf, c->q, k, c->args, c->st, s);
            }
        }
        reduce_energies(c, k, s);
    } else if (c->nvt) {
        forces(c, ForceFlags{1, 1, 0, 1}, s, false);  // closing kick, energies, write back
        const KernelShape k = shape(c);
        {
            Timed tm(c, MD_KT_FORCE, s);
            launch_nh_update(c->buf, c->q, k, c->args, 1, c->dt_fs, s);  // closing thermostat half step
            launch_nh_scale(c->buf, c->q, k, c->st, 1, s);
        }
        reduce_energies(c, k, s);
    } else {
        forces(c, ForceFlags{1, 1, 0, 1}, s);  // closing kick, energies, write back
    }
    const int rc = check_launch(c);
    c->resume_ok = rc == MD_OK && !c->gear && !c->pr;
    return rc;
}

int md_energy(md_ctx* c, md_energies* out, void* stream)
{
    if (!c || !out) return fail(c, MD_ERR_ARG, "md_energy: NULL argument");
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_energy: call md_bind first");
    hipStream_t s = as_stream(stream);
    std::vector<double> e((size_t)c->R * kEnergySlots, 0.0);
    int32_t flags[F_COUNT] = {};
    if (!hip_ok(c, hipStreamSynchronize(s), "md_energy sync")) return MD_ERR_DEVICE;
    collect_times(c);
    if (!hip_ok(c, hipMemcpy(flags, c->buf.flags, sizeof flags, hipMemcpyDeviceToHost), "md_energy flags")) return MD_ERR_DEVICE;
    if (c->have_energy && !hip_ok(c, hipMemcpy(e.data(), c->buf.energies, e.size() * 8, hipMemcpyDeviceToHost), "md_energy copy"))
        return MD_ERR_DEVICE;
    c->max_count = flags[F_MAX_COUNT];
    c->auto_builds = flags[F_AUTO_BUILDS];
    std::vector<double> nh((size_t)c->R * 4, 0.0);
    if (c->nvt && !hip_ok(c, hipMemcpy(nh.data(), c->buf.nh_state, nh.size() * 8, hipMemcpyDeviceToHost), "md_energy thermostat"))
        return MD_ERR_DEVICE;
    const int nps = c->tri ? kPrtState : kPrState;
    std::vector<double> pr((size_t)c->R * nps, 0.0);
    if (c->pr && !hip_ok(c, hipMemcpy(pr.data(), c->buf.pr_state, pr.size() * 8, hipMemcpyDeviceToHost), "md_energy barostat"))
        return MD_ERR_DEVICE;
    for (int r = 0; r < c->R; ++r) fill_energies(c, r, e.data() + (size_t)r * kEnergySlots, nh, pr, c->step, out[r]);
    // a non-finite state first: it also trips the displacement checks
    for (int r = 0; r < c->R; ++r) {
        const double* v = e.data() + (size_t)r * kEnergySlots;
        if (v[E_NONFINITE] != 0.0 || !std::isfinite(v[E_PE]) || !std::isfinite(v[E_KE]))
            return fail(c, MD_ERR_NONFINITE, "non-finite energy or force in replica " + std::to_string(r));
    }
    if (flags[F_RANGE] > 0)
        return fail(c, MD_ERR_NONFINITE, "a pair term exceeded the range of the pair kernels' fixed-point accumulators "
                                         "(|share| >= 1024; atoms closer than the potential is meant for?)");
    if (flags[F_MAX_COUNT] > c->cap) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "neighbour list overflow: an atom has %d entries, max_neighbours is %d (set it >= %d)",
                      flags[F_MAX_COUNT], c->cap, flags[F_MAX_COUNT]);
        return fail(c, MD_ERR_NBR_OVERFLOW, msg);
    }
    c->halo_overflows = flags[F_HALO];
    if (flags[F_PR_BOX] > 0)
        return fail(c, MD_ERR_BOX, c->tri ? "barostat: the cell narrowed below its link cells' list radius between a pair of faces "
                                            "(more than the 5% the grid allows), or the box velocity is too large for the step"
                                          : "barostat: a box edge shrank below its link cells' list radius (more than the 5% the grid allows)");
    if (flags[F_SKIN] > 0) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "skin violation: %d atom(s) moved more than %.4g A between list builds%s", flags[F_SKIN],
                      (c->pr ? 0.4 : 0.5) * c->skin, c->pr ? " (or the box strained more than 0.2 skin / list radius)" : "");
        return fail(c, MD_ERR_SKIN, msg);
    }
    if (flags[F_COMPACT] > 0) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "skin violation: %d atom(s) moved %.3g link cells or more from their cell between list builds",
                      flags[F_COMPACT], kCompactCells);
        return fail(c, MD_ERR_SKIN, msg);
    }
    return MD_OK;
}

int md_energy_history(md_ctx* c, md_energies* out, int64_t max_entries, int64_t* n_out, void* stream)
{
    if (!c || !n_out || (max_entries > 0 && !out)) return fail(c, MD_ERR_ARG, "md_energy_history: NULL argument");
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_energy_history: call md_bind first");
    *n_out = 0;
    if (max_entries < 0) return fail(c, MD_ERR_ARG, "md_energy_history: max_entries must be >= 0");
    if (c->ring_len == 0) return MD_OK;
    if (!hip_ok(c, hipStreamSynchronize(as_stream(stream)), "md_energy_history sync")) return MD_ERR_DEVICE;
    const int64_t pushed = (int64_t)c->ring_steps.size();
    // entries older than the ring holds were overwritten: skip them
    c->ring_read = std::max(c->ring_read, pushed - c->ring_len);
    const int64_t n = std::min(pushed - c->ring_read, max_entries);
    const size_t per = (size_t)c->R * kEnergySlots;
    std::vector<double> v(per);
    const std::vector<double> none;
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = c->ring_read + j;
        if (!hip_ok(c, hipMemcpy(v.data(), c->buf.ering + (size_t)(i % c->ring_len) * per, per * 8,
                                 hipMemcpyDeviceToHost), "md_energy_history copy"))
            return MD_ERR_DEVICE;
        for (int r = 0; r < c->R; ++r)
            fill_energies(c, r, v.data() + (size_t)r * kEnergySlots, none, none, c->ring_steps[i], out[j * c->R + r]);
    }
    c->ring_read += n;
    *n_out = n;
    return MD_OK;
}

int md_state_changed(md_ctx* c)
{
    if (!c) return MD_ERR_ARG;
    c->resume_ok = false;
    return MD_OK;
}

int md_copy_neighbours(md_ctx* c, int32_t* counts, int32_t* list, int32_t cap, void* stream)
{
    if (!c || !counts || !list) return fail(c, MD_ERR_ARG, "md_copy_neighbours: NULL argument");
    if (!c->bound || !c->have_list) return fail(c, MD_ERR_STATE, "md_copy_neighbours: no list built");
    if (cap < c->cap) return fail(c, MD_ERR_ARG, "md_copy_neighbours: cap smaller than max_neighbours");
    if (shape(c).brick) launch_brick_list_to_slots(c->buf, shape(c), as_stream(stream));
    if (!hip_ok(c, hipStreamSynchronize(as_stream(stream)), "md_copy_neighbours sync")) return MD_ERR_DEVICE;
    const size_t Np = (size_t)c->Np;
    std::vector<int32_t> cnt(Np), ids(Np), nb(Np * (size_t)((c->cap + kChunk - 1) / kChunk * kChunk));
    if (!hip_ok(c, hipMemcpy(cnt.data(), c->buf.ncount, Np * 4, hipMemcpyDeviceToHost), "copy") ||
        !hip_ok(c, hipMemcpy(ids.data(), c->buf.id[c->q], Np * 4, hipMemcpyDeviceToHost), "copy") ||
        !hip_ok(c, hipMemcpy(nb.data(), c->buf.nbr, nb.size() * 4, hipMemcpyDeviceToHost), "copy"))
        return MD_ERR_DEVICE;
    for (size_t t = 0; t < Np; ++t) {
        const int32_t a = ids[t];
        if (a < 0) continue;
        counts[a] = cnt[t];
        for (int k = 0; k < cnt[t]; ++k) list[(size_t)a * cap + k] = ids[nb[nbr_at(k, (int64_t)t, (int64_t)Np)] & kIndexMask];
    }
    return MD_OK;
}

int md_msd(md_ctx* c, double* msd, int64_t* count, void* stream)
{
    if (!c || !msd) return fail(c, MD_ERR_ARG, "md_msd: NULL argument");
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_msd: call md_bind first");
    hipStream_t s = as_stream(stream);
    launch_msd(c->buf, shape(c), c->st, s);
    const int ns = c->pot.ns;
    std::vector<double> out((size_t)c->R * 2 * MD_MAX_SPECIES);
    if (!hip_ok(c, hipGetLastError(), "md_msd launch") ||
        !hip_ok(c, hipMemcpyAsync(out.data(), c->buf.msd_out, out.size() * 8, hipMemcpyDeviceToHost, s), "md_msd copy") ||
        !hip_ok(c, hipStreamSynchronize(s), "md_msd sync"))
        return MD_ERR_DEVICE;
    for (int r = 0; r < c->R; ++r)
        for (int k = 0; k < ns; ++k) {
            msd[(size_t)r * ns + k] = out[(size_t)r * 2 * MD_MAX_SPECIES + k];
            if (count) count[(size_t)r * ns + k] = (int64_t)out[(size_t)r * 2 * MD_MAX_SPECIES + MD_MAX_SPECIES + k];
        }
    return MD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Device scratch of md_msd_static: a file-scope array in every GPU's memory,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, so its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.
namespace {
constexpr size_t kScratchDoubles = (size_t)1 << 17;  // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device (nullptr and a message on failure).
double* scratch_on_device(md_ctx* c)
{
    int dev = 0;
    if (!hip_ok(c, hipGetDevice(&dev), "md_msd_static device")) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        c->err = "md_msd_static: device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (!hip_ok(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "md_msd_static scratch address")) return nullptr;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int md_msd_static(md_ctx* c, double* msd, int64_t* count, void* stream)
{
    if (!c || !msd || !count) return fail(c, MD_ERR_ARG, "md_msd_static: NULL argument");
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_msd_static: call md_bind first");
    const KernelShape k = shape(c);
    const int ns = c->pot.ns;
    // layout: chunk partials | per-replica sums | msd [R][ns] | count [R][ns]
    const size_t n_part = (size_t)k.n_chunks * 2 * MD_MAX_SPECIES, n_out = (size_t)c->R * 2 * MD_MAX_SPECIES;
    const size_t n_res = (size_t)c->R * ns;
    if (n_part + n_out + 2 * n_res > kScratchDoubles)
        return fail(c, MD_ERR_ARG, "md_msd_static: " + std::to_string(n_part + n_out + 2 * n_res) +
                                       " scratch doubles needed, the static scratch holds " +
                                       std::to_string(kScratchDoubles));
    double* base = scratch_on_device(c);
    if (!base) return MD_ERR_DEVICE;
    hipStream_t s = as_stream(stream);
    Buffers b = c->buf;  // the same kernels, their partials and results in the scratch
    b.msd_partial = base;
    b.msd_out = base + n_part;
    double* d_msd = base + n_part + n_out;
    int64_t* d_cnt = reinterpret_cast<int64_t*>(d_msd + n_res);
    launch_msd(b, k, c->st, s);
    launch_msd_pack(b.msd_out, c->R, ns, d_msd, d_cnt, s);
    if (!hip_ok(c, hipGetLastError(), "md_msd_static launch") ||
        !hip_ok(c, hipMemcpyAsync(msd, d_msd, n_res * 8, hipMemcpyDeviceToHost, s), "md_msd_static copy") ||
        !hip_ok(c, hipMemcpyAsync(count, d_cnt, n_res * 8, hipMemcpyDeviceToHost, s), "md_msd_static copy") ||
        !hip_ok(c, hipStreamSynchronize(s), "md_msd_static sync"))
        return MD_ERR_DEVICE;
    return MD_OK;
}

int md_msd_origin(md_ctx* c, void* stream)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_msd_origin: call md_bind first");
    if (c->N == 0) return MD_OK;
    hipStream_t s = as_stream(stream);
    const size_t nb = (size_t)c->N * 8;
    if (!hip_ok(c, hipMemcpyAsync(c->buf.x0[0], c->st.x, nb, hipMemcpyDeviceToDevice, s), "md_msd_origin") ||
        !hip_ok(c, hipMemcpyAsync(c->buf.x0[1], c->st.y, nb, hipMemcpyDeviceToDevice, s), "md_msd_origin") ||
        !hip_ok(c, hipMemcpyAsync(c->buf.x0[2], c->st.z, nb, hipMemcpyDeviceToDevice, s), "md_msd_origin"))
        return MD_ERR_DEVICE;
    return MD_OK;
}

int md_set_option(md_ctx* c, int32_t option, int64_t value)
{
    if (!c) return MD_ERR_ARG;
    if (option != MD_OPT_TIMING) c->drop_graphs();  // captured launches hold the old settings
    // options that change the list or the evaluation make the next md_step
    // start afresh; timing, graph replay and the energy schedule do not
    if (option != MD_OPT_TIMING && option != MD_OPT_USE_GRAPH && option != MD_OPT_ENERGY_EVERY) c->resume_ok = false;
    switch (option) {
    case MD_OPT_ENERGY_EVERY:
        if (value < 0 || value > (int64_t)1 << 30) return fail(c, MD_ERR_ARG, "energy_every must be 0..2^30");
        if (value > 0 && (c->nvt || c->pr || c->gear))
            return fail(c, MD_ERR_ARG, "per-step energies are for velocity-Verlet NVE runs");
        c->energy_every = (int32_t)value;
        return MD_OK;
    case MD_OPT_ENERGY_RING:
        if (c->bound) return fail(c, MD_ERR_STATE, "set the energy ring length before md_bind");
        if (value < 0 || value > (int64_t)1 << 24) return fail(c, MD_ERR_ARG, "energy ring length must be 0..2^24");
        c->ring_len = value;
        plan_workspace(c);  // the ring lives in the workspace
        return MD_OK;
    case MD_OPT_LANES_PER_ATOM:
        if (value != 0 && value != 1 && value != 2 && value != 4) return fail(c, MD_ERR_ARG, "lanes per atom must be 0 (automatic), 1, 2 or 4");
        c->lanes = (int32_t)value;
        return MD_OK;
    case MD_OPT_USE_GRAPH:
        if (value != 0 && value != 1) return fail(c, MD_ERR_ARG, "use_graph must be 0 or 1");
        c->use_graph = value != 0;
        return MD_OK;
    case MD_OPT_COMPACT:
        if (value != 0 && value != 1) return fail(c, MD_ERR_ARG, "compact must be 0 or 1");
        if ((value != 0) != c->compact_on) {
            c->compact_on = value != 0;
            c->have_list = false;  // the list entries carry a different code
        }
        return MD_OK;
    case MD_OPT_NEIGHBOUR_CHUNK:
        if (value != 2 && value != 4 && value != 8) return fail(c, MD_ERR_ARG, "neighbour chunk must be 2, 4 or 8");
        c->nchunk = (int32_t)value;
        return MD_OK;
    case MD_OPT_AUTO_REBUILD: {
        if (value != 0 && value != 1) return fail(c, MD_ERR_ARG, "auto_rebuild must be 0 or 1");
        if (value != 0 && c->pr)
            return fail(c, MD_ERR_ARG, "automatic rebuilds are not available under the barostat (its build guard "
                                       "also bounds the box strain)");
        const bool brick = shape(c).brick != 0;
        c->auto_rebuild = value != 0;
        if ((shape(c).brick != 0) != brick) c->have_list = false;  // the brick lists have their own format
        return MD_OK;
    }
    case MD_OPT_TIMING:
        if (!value && !c->pending.empty()) return fail(c, MD_ERR_STATE, "read md_kernel_times before turning timing off");
        c->timing = value != 0;
        return MD_OK;
    case MD_OPT_EVALUATOR:
        if (value != 0 && value != 1) return fail(c, MD_ERR_ARG, "evaluator must be 0 (tables) or 1 (knot sums)");
        if (value == 0 && !c->table_ok) return fail(c, MD_ERR_ARG, "two knots of one function share a table bin");
        if (value == 1 && c->precision == MD_MIXED)
            return fail(c, MD_ERR_ARG, "the knot sums are FP64 only: in FP32 they miss the mixed-precision "
                                       "energy tolerance");
        if (value == 1 && !c->explicit_ok) return fail(c, MD_ERR_ARG, "no knot-sum variant for these knot counts");
        c->evaluator = (int32_t)value;
        return MD_OK;
    case MD_OPT_KERNEL:
        if (value != 0 && value != 1 && value != 2)
            return fail(c, MD_ERR_ARG, "kernel path must be 0 (LDS bricks), 1 (global gathers) or 2 (LDS bricks, pairs once)");
        if (value != c->kernel_path) {
            c->kernel_path = (int32_t)value;
            c->have_list = false;  // the two paths keep different list formats
        }
        return MD_OK;
    case MD_OPT_BRICK_DIMS: {
        const int64_t d0 = value % 10, d1 = (value / 10) % 10, d2 = (value / 100) % 10;
        if (value != 0 && (value >= 1000 || d0 < 1 || d1 < 1 || d2 < 1 || d0 > kBrickMaxDim || d1 > kBrickMaxDim || d2 > kBrickMaxDim))
            return fail(c, MD_ERR_ARG, "brick dims: 0 (automatic) or bx + 10 by + 100 bz with each in 1..4");
        choose_bricks(c, (int32_t)value);
        return upload_geometry(c) ? MD_OK : MD_ERR_DEVICE;
    }
    case MD_OPT_HALO_CAP:
        // shrink the staging area (testing the global fallback, tuning occupancy)
        if (value < 64 || value > c->halo_cap_max) return fail(c, MD_ERR_ARG, "halo capacity out of range");
        c->halo_cap = (int32_t)value;
        c->have_list = false;  // staging records are laid out by capacity
        return MD_OK;
    case MD_OPT_BRICK_BLOCK:
        if (value != 64 && value != 128 && value != 256 && value != 512 && value != 1024)
            return fail(c, MD_ERR_ARG, "brick workgroup size must be 64, 128, 256, 512 or 1024");
        c->brick_block = (int32_t)value;
        return MD_OK;
    default:
        return fail(c, MD_ERR_ARG, "unknown or read-only option");
    }
}

int md_autotune(md_ctx* c, int32_t trials, void* stream)
{
    if (!c) return MD_ERR_ARG;
    if (!c->bound) return fail(c, MD_ERR_STATE, "md_autotune: call md_bind first");
    c->resume_ok = false;
    if (trials < 1 || trials > 1000) return fail(c, MD_ERR_ARG, "md_autotune: trials must be 1..1000");
    if (c->timing) return fail(c, MD_ERR_STATE, "md_autotune: turn MD_OPT_TIMING off first");
    hipStream_t s = as_stream(stream);
    struct Cand {
        int32_t kernel, dims, lanes, block, evaluator, nchunk;
    };
    // FP64 may take either evaluator (both meet its tolerance); mixed keeps the
    // current one, since its explicit FP32 knot sums do not
    std::vector<int32_t> evals = {(c->table_ok && c->evaluator == 0) ? 0 : 1};
    if (c->precision == MD_FP64 && c->table_ok && c->explicit_ok) evals = {0, 1};
    std::vector<Cand> cands;
    for (int32_t e : evals) {
        for (int32_t nch : {4, 2, 8}) cands.push_back({1, 0, 0, 512, e, nch});
        // the brick kernels take fixed orthorhombic boxes and scheduled builds
        if (c->nbr_mode == MD_NBR_FULL && !c->pr && !c->tri && !c->auto_rebuild)
            // (the pair kernels, MD_OPT_KERNEL = 2, are left out: their LDS
            // atomics make them several times slower on this device)
            for (int32_t dims : {0, 444, 222})
                for (int32_t lanes : {1, 2})
                    for (int32_t block : {512, 1024}) cands.push_back({0, dims, lanes, block, e, 4});
    }
    hipEvent_t ev[3];
    for (auto& e : ev)
        if (!hip_ok(c, hipEventCreate(&e), "md_autotune events")) return MD_ERR_DEVICE;
    // two rounds over the candidates, each candidate scored by its faster round
    // (one round alone mis-ranks close candidates now and then)
    std::vector<double> cost_of(cands.size(), 1e300);
    int rc = MD_OK;
    for (int round = 0; round < 2 && rc == MD_OK; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Cand& cd = cands[ci];
            if ((rc = md_set_option(c, MD_OPT_KERNEL, cd.kernel)) != MD_OK || (rc = md_set_option(c, MD_OPT_BRICK_DIMS, cd.dims)) != MD_OK ||
                (rc = md_set_option(c, MD_OPT_LANES_PER_ATOM, cd.lanes)) != MD_OK ||
                (rc = md_set_option(c, MD_OPT_BRICK_BLOCK, cd.block)) != MD_OK ||
                (rc = md_set_option(c, MD_OPT_EVALUATOR, cd.evaluator)) != MD_OK ||
                (rc = md_set_option(c, MD_OPT_NEIGHBOUR_CHUNK, cd.nchunk)) != MD_OK)
                break;
            ensure_slots(c, s);
            launch_load_state(c->buf, c->p, c->q, c->st, shape(c), s);
            (void)hipEventRecord(ev[0], s);
            rebuild(c, s, false);
            (void)hipEventRecord(ev[1], s);
            // the plain force pass (forces kept in the slots, no state change)
            for (int32_t t = 0; t < trials; ++t) forces(c, ForceFlags{0, 0, 0, 0}, s);
            (void)hipEventRecord(ev[2], s);
            if ((rc = check_launch(c)) != MD_OK) break;
            float t_build = 0.0f, t_force = 0.0f;
            if (!hip_ok(c, hipEventSynchronize(ev[2]), "md_autotune") || !hip_ok(c, hipEventElapsedTime(&t_build, ev[0], ev[1]), "md_autotune") ||
                !hip_ok(c, hipEventElapsedTime(&t_force, ev[1], ev[2]), "md_autotune")) {
                rc = MD_ERR_DEVICE;
                break;
            }
            // cost of one step: force passes plus the list build spread over its period
            cost_of[ci] = std::min(cost_of[ci], (double)t_force / trials + (double)t_build / c->rebuild_every);
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc != MD_OK) return rc;
    const size_t pick = (size_t)(std::min_element(cost_of.begin(), cost_of.end()) - cost_of.begin());
    const Cand choice = cands[pick];
    const double best = cost_of[pick];
    if ((rc = md_set_option(c, MD_OPT_KERNEL, choice.kernel)) != MD_OK || (rc = md_set_option(c, MD_OPT_BRICK_DIMS, choice.dims)) != MD_OK ||
        (rc = md_set_option(c, MD_OPT_LANES_PER_ATOM, choice.lanes)) != MD_OK ||
        (rc = md_set_option(c, MD_OPT_BRICK_BLOCK, choice.block)) != MD_OK ||
        (rc = md_set_option(c, MD_OPT_EVALUATOR, choice.evaluator)) != MD_OK ||
        (rc = md_set_option(c, MD_OPT_NEIGHBOUR_CHUNK, choice.nchunk)) != MD_OK)
        return rc;
    c->tuned_us = best * 1e3;
    c->have_list = false;  // the next call builds the list of the chosen configuration
    return MD_OK;
}

int md_get_option(const md_ctx* c, int32_t option, int64_t* value)
{
    if (!c || !value) return MD_ERR_ARG;
    switch (option) {
    case MD_OPT_LANES_PER_ATOM: *value = shape(c).lanes; return MD_OK;
    case MD_OPT_USE_GRAPH: *value = c->use_graph ? 1 : 0; return MD_OK;
    case MD_OPT_GRAPH_LAUNCHES: *value = c->graph_launches; return MD_OK;
    case MD_OPT_TUNED_NS: *value = (int64_t)(c->tuned_us * 1e3); return MD_OK;
    case MD_OPT_COMPACT: *value = shape(c).compact ? 1 : 0; return MD_OK;
    case MD_OPT_MAX_COUNT: *value = c->max_count; return MD_OK;
    case MD_OPT_N_BUILDS: *value = c->n_builds + c->auto_builds; return MD_OK;
    case MD_OPT_AUTO_REBUILD: *value = c->auto_rebuild ? 1 : 0; return MD_OK;
    case MD_OPT_TIMING: *value = c->timing ? 1 : 0; return MD_OK;
    case MD_OPT_EVALUATOR: *value = (c->table_ok && c->evaluator == 0) ? 0 : 1; return MD_OK;
    case MD_OPT_KERNEL: *value = shape(c).brick ? (shape(c).pairs ? 2 : 0) : 1; return MD_OK;
    case MD_OPT_BRICK_DIMS: *value = c->reps.empty() ? 0 : c->reps[0].bd[0] + 10 * c->reps[0].bd[1] + 100 * c->reps[0].bd[2]; return MD_OK;
    case MD_OPT_BRICK_BLOCK: *value = c->brick_block; return MD_OK;
    case MD_OPT_HALO_CAP: *value = c->halo_cap; return MD_OK;
    case MD_OPT_HALO_OVERFLOWS: *value = c->halo_overflows; return MD_OK;
    case MD_OPT_ENERGY_EVERY: *value = c->energy_every; return MD_OK;
    case MD_OPT_ENERGY_RING: *value = c->ring_len; return MD_OK;
    case MD_OPT_NEIGHBOUR_CHUNK: *value = c->nchunk; return MD_OK;
    default: return MD_ERR_ARG;
    }
}

int md_kernel_times(md_ctx* c, double* ms, int64_t* launches, int reset, void* stream)
{
    if (!c || !ms || !launches) return fail(c, MD_ERR_ARG, "md_kernel_times: NULL argument");
    if (!hip_ok(c, hipStreamSynchronize(as_stream(stream)), "md_kernel_times sync")) return MD_ERR_DEVICE;
    collect_times(c);
    for (int g = 0; g < MD_KT_COUNT; ++g) {
        ms[g] = c->kt_ms[g];
        launches[g] = c->kt_n[g];
        if (reset) {
            c->kt_ms[g] = 0.0;
            c->kt_n[g] = 0;
        }
    }
    return MD_OK;
}

void md_destroy(md_ctx* c) { delete c; }

const char* md_last_error(const md_ctx* c)
{
    if (!c) return "NULL context";
    return c->err.empty() ? "no error" : c->err.c_str();
}

}  // extern "C"
