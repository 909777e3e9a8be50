// gfx950 kernels of the embedded-atom force loop.
//
// Global-gather kernels and the cell sort.  Data layout (all in the
// caller-provided workspace, see md_runtime.hip):
//   - atoms live in "slots" sorted by link cell (paper, "OpenMP
//     Parallelisation": particles ordered by link-cell index so cell members
//     are contiguous); replica r owns a wavefront-aligned slot range;
//   - positions as double4 {x, y, z, F'}: one 32-byte gather per neighbour
//     brings the position and the embedding derivative the force pass needs;
//   - the Verlet list is one int32 row per atom (slot index + periodic shift
//     code), read 8 entries per two 16-byte loads;
//   - the full (symmetric) list lets each atom gather its own density and
//     force with no atomics; the half list with FP64 atomics is kept as the
//     comparison variant (paper, "OpenMP Parallelisation", on the trade
//     between a symmetric list and synchronised updates).
#include "md_device.h"

namespace mdk {
namespace {
// ---------------------------------------------------------------------------
// Utility kernels.
__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// First placement: slot_off + local index, caller order within a replica.
__global__ void k_init_slots(Buffers b, int q, const uint8_t* __restrict__ species,
                             const uint8_t* __restrict__ rigid, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const int64_t local = t - R.slot_off;
    if (local < R.n_atoms) {
        const int64_t a = R.atom_off + local;
        b.id[q][t] = (int32_t)a;
        uint8_t ty = species[a] & 0x3F;
        if (rigid && rigid[a]) ty |= kRigidBit;
        b.type[q][t] = ty;
    } else {
        b.id[q][t] = -1;
        b.type[q][t] = kEmptySlot;
    }
    b.pwork[q][t] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) b.img[q][a][t] = 0;
}

// Caller state (caller order, unwrapped) -> slots.  Inside the library a
// position is kept as x - n L along periodic axes (x - h n in a sheared cell),
// with the integer image
// count n of the slot fixed at the last list build, so that list entries can
// carry their periodic shift and the force loop needs no minimum image.
__global__ void k_load_state(Buffers b, int p, int q, md_state st, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const int32_t a = b.id[q][t];
    if (a >= 0) {
        double sh[3];
        lattice_shift(R, b.img[q][0][t], b.img[q][1][t], b.img[q][2][t], sh);
        b.pos[p][t] = make_double4(st.x[a] - sh[0], st.y[a] - sh[1], st.z[a] - sh[2], 0.0);
        b.vel[q][0][t] = st.vx[a];
        b.vel[q][1][t] = st.vy[a];
        b.vel[q][2][t] = st.vz[a];
    } else {
        b.pos[p][t] = make_double4(0.0, 0.0, 0.0, 0.0);
        b.vel[q][0][t] = 0.0;
        b.vel[q][1][t] = 0.0;
        b.vel[q][2][t] = 0.0;
    }
}

// counter[key] += 1 for every lane with key >= 0; returns the lane's old value
// plus its rank among the lanes of its run.  Lanes with equal keys usually sit
// side by side (the slots are cell-sorted from the previous build), so each
// run of equal keys issues one atomic instead of one per lane.  Must be called
// by every lane of the wavefront.
__device__ __forceinline__ int wave_run_add(int32_t* counter, int key)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int prev = __shfl_up(key, 1, kWave);
    const uint64_t heads = __ballot(lane == 0 || key != prev);
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1);
    const int head = 63 - __clzll(heads & upto);  // first lane of this run
    const uint64_t later = heads & ~upto;
    const int next = later ? __ffsll((unsigned long long)later) - 1 : kWave;
    int base = 0;
    if (lane == head && key >= 0) base = atomicAdd(&counter[key], next - lane);
    base = __shfl(base, head, kWave);
    return base + (lane - head);
}


// ---------------------------------------------------------------------------
// Rebuild stage 1 of 5: link cell of every atom, cell populations, and the skin
// guard (net displacement since the previous build must stay below skin/2).
// Every rebuild kernel takes `gate`: NULL for a build of all replicas, else
// the automatic rebuild's flags, and then it leaves alone every replica r with
// gate[1 + r] == 0 (slot ranges and link cells are per replica, so a kept
// replica's slots, cells and list stay exactly as they are).  Gated builds run
// at every step and mostly find nothing flagged: they launch a capped grid
// whose threads stride over the elements (whole wavefronts per stride, as
// replicas are wave aligned), so that such a launch ends at once; builds of
// all replicas take one element per thread.
constexpr int64_t kGatedBlocks = 2048;

__device__ __forceinline__ bool replica_kept(const Buffers& b, const int32_t* gate, int64_t t)
{
    return gate && gate[1 + uniform(b.rep_of_wave[t / kWave])] == 0;
}

__device__ __forceinline__ void bin_slot(const Buffers& b, int p, int q, int64_t t, double half_skin2, int check_skin)
{
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const bool valid = b.id[q][t] >= 0;
    const Box bx = load_box(R);
    const double3 x = load_xyz(b.pos[p], t);
    int c[3];
    cell_coords(bx, x.x, x.y, x.z, c);
    const int cell = valid ? cell_index(R, c[0], c[1], c[2]) : -1;
    b.cell_of[t] = cell;
    wave_run_add(b.bin_count, cell);
    if (!valid) return;
    if (check_skin) {
        // displacement since the build, after mapping the build position into
        // the current box (the two boxes differ only under the barostat)
        const double3 x0 = load_xyz(b.xbuild, t);
        double dx, dy, dz;
        if (bx.tri) {  // strained by the homogeneous map mb since the build
            const double u[3] = {x0.x - bx.o[0], x0.y - bx.o[1], x0.z - bx.o[2]};
            dx = (x.x - bx.o[0]) - (R.mb[0] * u[0] + R.mb[1] * u[1] + R.mb[2] * u[2]);
            dy = (x.y - bx.o[1]) - (R.mb[3] * u[0] + R.mb[4] * u[1] + R.mb[5] * u[2]);
            dz = (x.z - bx.o[2]) - (R.mb[6] * u[0] + R.mb[7] * u[1] + R.mb[8] * u[2]);
        } else {
            dx = (x.x - bx.o[0]) - (x0.x - bx.o[0]) * (R.box[0] / R.lbuild[0]);
            dy = (x.y - bx.o[1]) - (x0.y - bx.o[1]) * (R.box[1] / R.lbuild[1]);
            dz = (x.z - bx.o[2]) - (x0.z - bx.o[2]) * (R.box[2] / R.lbuild[2]);
        }
        if (dx * dx + dy * dy + dz * dz > half_skin2) atomicAdd(&b.flags[F_SKIN], 1);
    }
    // atoms beyond the grid extent of a free axis (clamped into edge cells)
    for (int a = 0; a < 3; ++a) {
        if (bx.pmask & (1 << a)) continue;
        const double xa = a == 0 ? x.x : (a == 1 ? x.y : x.z);
        const double f = (xa - bx.o[a]) * bx.iL[a];
        if (f < 0.0 || f >= 1.0) {
            atomicAdd(&b.flags[F_OUTSIDE], 1);
            break;
        }
    }
}

__global__ void k_bin(Buffers b, int p, int q, int64_t n_slots, double half_skin2, int check_skin,
                      const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = global_thread(); t < n_slots; t += stride)
        if (!replica_kept(b, gate, t)) bin_slot(b, p, q, t, half_skin2, check_skin);
}

// Rebuild stage 2: exclusive scan of cell populations in two phases (block scan, then
// each block adds the sum of the block totals before it), shifted into slot numbering
// with the per-cell replica shift.  The populations binned by stage 1 are taken over
// (and their counters cleared for the next build); a kept replica's cells keep theirs.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* sh, int32_t& total)
{
    // Hillis-Steele over the workgroup in LDS (1024 entries).
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        const int32_t add = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    total = sh[kScanBlock - 1];
    return sh[tid] - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_local(Buffers b, int32_t n, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    __shared__ int32_t sh[kScanBlock];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    int32_t v = 0;
    if (i < n) {
        const int r = b.cell_rep[i];
        if (gate && r >= 0 && gate[1 + r] == 0) {
            v = b.cell_count[i];
        } else {
            v = b.bin_count[i];
            b.cell_count[i] = v;
            b.bin_count[i] = 0;
            b.cell_cursor[i] = 0;
        }
    }
    int32_t total;
    const int32_t ex = block_exclusive_scan(v, sh, total);
    if (i < n) b.cell_start[i] = ex;
    if (threadIdx.x == 0) b.scan_blocks[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(Buffers b, int32_t n, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    // the totals of the blocks before this one (integers: any order is exact)
    __shared__ int32_t part[kScanBlock / kWave];
    int32_t run = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kScanBlock) run += b.scan_blocks[k];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) run += __shfl_xor(run, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = run;
    __syncthreads();
    int32_t before = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / kWave; ++w) before += part[w];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) b.cell_start[i] += before + b.cell_shift[i];
    if (gate && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&b.flags[F_AUTO_BUILDS], 1);
}

// Rebuild stage 3: place every atom in its cell's slot range (arbitrary order within
// the cell, fixed by the next kernel).
__global__ void k_scatter(Buffers b, int64_t n_slots, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = global_thread(); t < n_slots; t += stride) {
        if (replica_kept(b, gate, t)) continue;
        const int c = b.cell_of[t];
        const int k = wave_run_add(b.cell_cursor, c);
        if (c >= 0) b.perm[b.cell_start[c] + k] = (int32_t)t;
    }
}

// Rebuild stage 4: order each cell's members by caller index, making the slot order
// (and so every later floating-point sum) independent of atomics' timing.
__global__ void k_sort_cells(Buffers b, int q, int32_t n_cells, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    if (gate) {
        const int r = b.cell_rep[c];
        if (r < 0 || gate[1 + r] == 0) return;
    }
    const int beg = b.cell_start[c], cnt = b.cell_count[c];
    int32_t* m = b.perm + beg;
    const int32_t* id = b.id[q];
    for (int i = 1; i < cnt; ++i) {
        const int32_t v = m[i];
        const int32_t key = id[v];
        int j = i - 1;
        while (j >= 0 && id[m[j]] > key) {
            m[j + 1] = m[j];
            --j;
        }
        m[j + 1] = v;
    }
}

// Rebuild stage 5: gather the whole atom state into the new slot order.
__device__ __forceinline__ void gather_slot(const Buffers& b, int p, int q, int64_t u)
{
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[u / kWave])];
    const int pn = p ^ 1, qn = q ^ 1;
    if (u - R.slot_off < R.n_atoms) {
        const int32_t t = b.perm[u];
        const double3 x = load_xyz(b.pos[p], t);
        double xw[3] = {x.x, x.y, x.z};
        // re-wrap atoms that left the primary box on a periodic axis
        if (R.tri) {  // sheared cell: whole edge vectors, from the fractional coordinates
            double f[3];
            frac_coords(R.hinv, R.origin, xw[0], xw[1], xw[2], f);
            double k[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                k[a] = floor(f[a]);
                b.img[qn][a][u] = b.img[q][a][t] + (int32_t)k[a];
            }
            double sh[3];
            lattice_shift(R, k[0], k[1], k[2], sh);
#pragma unroll
            for (int a = 0; a < 3; ++a) xw[a] -= sh[a];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int32_t n = b.img[q][a][t];
                if (R.periodic_mask & (1 << a)) {
                    const double s = floor((xw[a] - R.origin[a]) * R.inv_box[a]);
                    if (s != 0.0) {
                        xw[a] -= s * R.box[a];
                        n += (int32_t)s;
                    }
                }
                b.img[qn][a][u] = n;
            }
        }
        const double4 x4 = make_double4(xw[0], xw[1], xw[2], 0.0);
        b.pos[pn][u] = x4;
        b.xbuild[u] = x4;
#pragma unroll
        for (int a = 0; a < 3; ++a) b.vel[qn][a][u] = b.vel[q][a][t];
        b.id[qn][u] = b.id[q][t];
        b.type[qn][u] = b.type[q][t];
        b.cell_sorted[u] = b.cell_of[t];
        b.pwork[qn][u] = b.pwork[q][t];
        if (b.acc[q][0]) {  // Gear integrator state travels with its atom
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b.acc[qn][a][u] = b.acc[q][a][t];
                b.jrk[qn][a][u] = b.jrk[q][a][t];
            }
        }
    } else {
        const double4 z = make_double4(0.0, 0.0, 0.0, 0.0);
        b.pos[pn][u] = z;
        b.xbuild[u] = z;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b.vel[qn][a][u] = 0.0;
            b.img[qn][a][u] = 0;
        }
        b.id[qn][u] = -1;
        b.type[qn][u] = kEmptySlot;
        b.pwork[qn][u] = 0.0;
        b.cell_sorted[u] = -1;
        if (b.acc[q][0]) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b.acc[qn][a][u] = 0.0;
                b.jrk[qn][a][u] = 0.0;
            }
        }
    }
}

__global__ void k_gather(Buffers b, int p, int q, int64_t n_slots, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = global_thread(); u < n_slots; u += stride)
        if (!replica_kept(b, gate, u)) gather_slot(b, p, q, u);
}

// Verlet list from the link cells (paper, "The Neighbourlist calculation":
// each cell's atoms are tested against the atoms of the 27 cells around it).  One wavefront per link
// cell.  The up to 27 adjacent cells (fewer on free faces; on a periodic axis
// with under three cells each distinct cell once) become one candidate
// sequence: cell by cell (x fastest), atoms in slot order.  The wavefront
// holds 64 x kCandPasses candidates in registers, shifted by the periodic
// image of their cell, and tests every atom of its own cell against them;
// the in-range lanes of each test are packed with a ballot, so list entries
// come out in candidate order.  Full list: every j != i with r < r_c + skin;
// half list: only j with a larger slot index.
//
// Entries: slot | code << kIndexBits, 2 bits per axis, and kInnerBit for a
// pair closer than r_d + skin.  FP64 mode: the periodic image (0 none, 1 +L,
// 2 -L); compact mixed mode: the unwrapped link-cell offset plus one.  Axes with one or two periodic cells have no
// unique image per cell; there the image is the minimum one of each pair.
// Layout: groups of four entries per slot (nbr_at).  Overflow keeps counting, so the
// required capacity can be reported.
// Adjacency of every link cell, once per geometry: entry k of cell c is the
// cell at offset (k % 3 - 1, k / 3 % 3 - 1, k / 9 - 1), or -1 where a free
// face ends the grid or a periodic axis of under three cells would list a
// cell twice.  .y: periodic image of that cell (2 bits per axis, 1 = +L,
// 2 = -L) and, from bit 8, its unwrapped offset plus one.  On periodic axes
// with under three cells the image is left to the pair (minimum image) and
// the offset is the plain one between the two cells.
__global__ void k_cell_table(Buffers b, int32_t n_cells)
{
    const int64_t t = global_thread();
    if (t >= (int64_t)n_cells * 27) return;
    const int cell = (int)(t / 27), k = (int)(t - (int64_t)cell * 27);
    const int r = b.cell_rep[cell];
    if (r < 0) {
        b.cell_adj[t] = make_int2(-1, 0);
        if (k == 13) b.cell_coord[cell] = 0;
        return;
    }
    const DevReplica& R = b.reps[r];
    const int local = cell - R.cell_off;
    const int brick = local / R.cpb, in = local - brick * R.cpb;
    const int c[3] = {(brick % R.nbk[0]) * R.bd[0] + in % R.bd[0],
                      ((brick / R.nbk[0]) % R.nbk[1]) * R.bd[1] + (in / R.bd[0]) % R.bd[1],
                      (brick / (R.nbk[0] * R.nbk[1])) * R.bd[2] + in / (R.bd[0] * R.bd[1])};
    const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
    bool ok = true;
    int cc[3], wrap = 0, code = 0;
    for (int a = 0; a < 3; ++a) {
        int v = c[a] + o[a], w = 0;
        ok = ok && c[a] < R.nc[a];  // padding cells of the brick grid have no atoms
        if (R.periodic_mask >> a & 1) {
            if (R.nc[a] == 1) ok = ok && o[a] == 0;
            if (R.nc[a] == 2) ok = ok && o[a] >= 0;
            if (v < 0) v += R.nc[a], w = 2;
            if (v >= R.nc[a]) v -= R.nc[a], w = 1;
        } else {
            ok = ok && v >= 0 && v < R.nc[a];
        }
        cc[a] = v;
        const bool few = (R.periodic_mask >> a & 1) && R.nc[a] < 3;
        wrap |= (few ? 0 : w) << (2 * a);
        code |= (few ? v - c[a] + 1 : o[a] + 1) << (2 * a);
    }
    b.cell_adj[t] = make_int2(ok ? cell_index(R, cc[0], cc[1], cc[2]) : -1, wrap | (code << 8));
    if (k == 13) b.cell_coord[cell] = c[0] | (c[1] << 10) | (c[2] << 20);
}

constexpr int kCandPasses = 4;

__device__ __forceinline__ double select_shift(int s, double L) { return s == 1 ? L : (s == 2 ? -L : 0.0); }


// Minimum image of one pair along the axes in `amb` (periodic axes with fewer
// than three cells), with the entry's code field updated: the image shift in
// FP64 mode, the unwrapped link-cell offset plus one in compact mode.
__device__ __forceinline__ void min_image_axis(double& d, double L, double iL, int nc, int a, int compact, int& e)
{
    const double s = rint(d * iL);
    d -= s * L;
    const int sh = kIndexBits + 2 * a;
    const int f = (e >> sh) & 3;
    const int nf = compact ? f - (int)s * nc : (s < 0.0 ? 1 : (s > 0.0 ? 2 : 0));
    e = (e & ~(3 << sh)) | (nf << sh);
}

__device__ __forceinline__ void min_image_pair(const Box& bx, int amb, int compact, double& dx, double& dy, double& dz,
                                               int& e)
{
    if (amb & 1) min_image_axis(dx, bx.L[0], bx.iL[0], bx.nc[0], 0, compact, e);
    if (amb & 2) min_image_axis(dy, bx.L[1], bx.iL[1], bx.nc[1], 1, compact, e);
    if (amb & 4) min_image_axis(dz, bx.L[2], bx.iL[2], bx.nc[2], 2, compact, e);
}

// Where the list build writes.  Lists below 4 GiB are written through raw
// buffer resources: the atom's row start is a scalar byte offset and each lane
// adds its entry's 32-bit offset, so the address costs three vector
// instructions; WIDE lists take 64-bit addresses.  With several species each
// entry also gets its neighbour's type byte, in the same layout (four bytes
// per group of four entries), so the force loop reads them with its entries
// instead of gathering them one by one.
struct ListOut {
    __amdgpu_buffer_rsrc_t rs, ts;  // entries, type bytes
    uint32_t group_bytes;           // n_slots * 16: one group of four entries of every slot
    int32_t* nbr;
    uint8_t* types;
    int64_t n_slots;
    int with_types;
};

typedef int int4v __attribute__((ext_vector_type(4)));

// Tests atoms s0 .. s0 + n - 1 (lane l holds atom s0 + l in xl) against the
// candidates in registers and appends the in-range ones to their rows.
template <int P, bool AMB, bool WIDE, bool SPLIT>
__device__ __forceinline__ void test_candidates(const ListOut& L, int32_t cap, double rlist2, double rdl2,
                                                int half_list, int compact, const Box& bx, int amb, int s0, int n,
                                                const double3& xl,
                                                const double (&cx)[P], const double (&cy)[P], const double (&cz)[P],
                                                const int (&ce)[P], const int (&cj)[P], const int (&ct)[P],
                                                const bool (&live)[P], int& my_count)
{
    const int lane = threadIdx.x & (kWave - 1);
    // j != i (full list) or j > i (half list) as one unsigned compare of j - i - 1
    const uint32_t lim = half_list ? 0x7FFFFFFFu : 0xFFFFFFFFu;
    for (int ii = 0; ii < n; ++ii) {
        const int i = s0 + ii;
        const double xi = bcast_lane(xl.x, ii), yi = bcast_lane(xl.y, ii), zi = bcast_lane(xl.z, ii);
        int base = __builtin_amdgcn_readlane(my_count, ii);
        const uint32_t row = (uint32_t)i * 16u;  // entry k of atom i: row + (k / 4) group_bytes + 4 (k % 4)
#pragma unroll
        for (int u = 0; u < P; ++u) {
            double dx = cx[u] - xi, dy = cy[u] - yi, dz = cz[u] - zi;
            int e = ce[u];
            if (AMB) min_image_pair(bx, amb, compact, dx, dy, dz, e);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool take = live[u] & ((uint32_t)(cj[u] - (i + 1)) < lim) & (r2 < rlist2);
            if (SPLIT && r2 < rdl2) e |= kInnerBit;  // (otherwise every candidate carries it)
            const uint64_t mask = __builtin_amdgcn_ballot_w64(take);
            if (mask == 0) continue;
            const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
            // entry base + rank of atom i (the layout of nbr_at)
            const uint32_t k = (uint32_t)(base + rank);
            if (take && base + rank < cap) {
                if (WIDE) {
                    const int64_t at = nbr_at(base + rank, i, L.n_slots);
                    L.nbr[at] = e;
                    if (L.with_types) L.types[at] = (uint8_t)ct[u];
                } else {
                    const uint32_t off = (k >> 2) * L.group_bytes + ((k & 3u) << 2);
                    __builtin_amdgcn_raw_buffer_store_b32(e, L.rs, off, row, 0);
                    if (L.with_types)  // byte offsets a quarter of the entry's
                        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)ct[u], L.ts, off >> 2, row >> 2, 0);
                }
            }
            base += __popcll(mask);
        }
        if (lane == ii) my_count = base;
    }
}

// TRI: sheared cells (candidate shifts are edge-vector sums), a separate
// instantiation so the orthorhombic build keeps its short candidate loop.
// SPLIT: mark the inner entries (r < r_d + skin); otherwise every entry is
// inner (one precision's density pass gains nothing from the mark).
// WT: several species (each entry's type byte is stored beside it).
// gate: the automatic rebuild's replica flags (NULL: every replica).
// copy_back: also copy each own atom's sorted state from (p, q) into
// (p ^ 1, q ^ 1), the buffers an automatic rebuild keeps using.
template <bool TRI, bool WIDE, bool SPLIT, bool WT>
__device__ __forceinline__ void list_cell(const Buffers& b, int p, int q, int64_t n_slots, int cell, int32_t cap,
                                          double rlist2, double rdl2, int half_list, int compact,
                                          const int32_t* __restrict__ gate, int copy_back)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int r = uniform(b.cell_rep[cell]);
    if (r < 0) return;
    if (gate && gate[1 + r] == 0) return;
    const int n_own = uniform(b.cell_count[cell]);
    if (n_own == 0) return;
    const int s_own = uniform(b.cell_start[cell]);
    const DevReplica& R = b.reps[r];
    const Box bx = load_box(R);
    const int cpk = uniform(b.cell_coord[cell]);
    int c[3] = {cpk & 1023, (cpk >> 10) & 1023, cpk >> 20};
    int amb = 0;  // periodic axes with fewer than three cells
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if ((bx.pmask >> a & 1) && bx.nc[a] < 3) amb |= 1 << a;

    // lane k < 27: adjacent cell k
    int nb_start = 0, nb_count = 0, nb_wrap = 0, nb_code = 0;
    if (lane < 27) {
        const int2 adj = b.cell_adj[(int64_t)cell * 27 + lane];
        nb_wrap = adj.y & 63;
        nb_code = compact ? (adj.y >> 8) & 63 : nb_wrap;
        if (adj.x >= 0) {
            nb_start = b.cell_start[adj.x];
            nb_count = b.cell_count[adj.x];
        }
    }
    // sheared cells: whether any adjacent cell lies across a face (interior
    // cells, most of a large cell, skip the edge-vector shifts)
    const bool any_wrap = TRI && __ballot(nb_wrap != 0) != 0;
    // exclusive prefix of the candidate counts over the 27 lanes
    int incl = nb_count;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int v = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += v;
    }
    const int excl = incl - nb_count;
    const int total = uniform(__shfl(incl, kWave - 1, kWave));

    // candidate table of this wave: slot and codes of candidate m, written by
    // the 27 lanes of the adjacent cells (lane k its own cell's run), read back
    // by candidate index.  A wave's LDS operations complete in order, so the
    // wave-scope fence suffices.  Larger stencils search the prefix instead.
    __shared__ int2 cand_table[kBlock / kWave][kCandTable];
    int2* tab = cand_table[threadIdx.x / kWave];
    const bool tabled = total <= kCandTable;
    if (tabled) {
        const int wc = nb_wrap | (nb_code << 8);
        for (int qq = 0; qq < nb_count; ++qq) tab[excl + qq] = make_int2(nb_start + qq, wc);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    const double4* __restrict__ pos = b.pos[p];
    // (WIDE: the buffer resources are unused; their sizes wrap harmlessly)
    ListOut L;
    L.group_bytes = (uint32_t)n_slots * 16u;
    const uint32_t n_groups = (uint32_t)((cap + 2 * kChunk - 1) / kChunk);
    L.rs = __builtin_amdgcn_make_buffer_rsrc(b.nbr, (short)0, (int)(L.group_bytes * n_groups), (int)kBufferWord3);
    L.ts = __builtin_amdgcn_make_buffer_rsrc(b.ntype, (short)0, (int)(L.group_bytes / 4 * n_groups), (int)kBufferWord3);
    L.nbr = b.nbr;
    L.types = b.ntype;
    L.n_slots = n_slots;
    L.with_types = WT;
    for (int i0 = 0; i0 < n_own; i0 += kWave) {
        const int n_chunk = min(kWave, n_own - i0);
        // lane l holds atom s_own + i0 + l; the test loop broadcasts it
        const double3 xl = load_xyz(pos, s_own + i0 + min(lane, n_chunk - 1));
        int my_count = 0;  // lane l: entries of that atom so far
        for (int g0 = 0; g0 < total; g0 += kWave * kCandPasses) {
            double cx[kCandPasses], cy[kCandPasses], cz[kCandPasses];
            int ce[kCandPasses], cj[kCandPasses], ct[kCandPasses];
            bool live[kCandPasses];
#pragma unroll
            for (int u = 0; u < kCandPasses; ++u) {
                const int m0 = g0 + u * kWave + lane;
                const int m = min(m0, total - 1);
                int j, w, code;
                if (tabled) {
                    const int2 tv = tab[m];
                    j = tv.x;
                    w = tv.y & 63;
                    code = (tv.y >> 8) & 63;
                } else {
                    // the adjacent cell holding candidate m: the last k with excl_k <= m
                    int k = 0;
#pragma unroll
                    for (int step = kWave / 2; step > 0; step >>= 1)
                        if (__shfl(excl, k + step, kWave) <= m) k += step;
                    j = __shfl(nb_start, k, kWave) + (m - __shfl(excl, k, kWave));
                    w = __shfl(nb_wrap, k, kWave);
                    code = __shfl(nb_code, k, kWave);
                }
                const double3 xj = load_xyz(pos, j);
                if (TRI) {  // the image cell's edge-vector shift
                    double dsh[3] = {0.0, 0.0, 0.0};
                    if (any_wrap) apply_shift(bx, w & 63, dsh[0], dsh[1], dsh[2]);
                    cx[u] = xj.x + dsh[0];
                    cy[u] = xj.y + dsh[1];
                    cz[u] = xj.z + dsh[2];
                } else {
                    cx[u] = xj.x + select_shift(w & 3, bx.L[0]);
                    cy[u] = xj.y + select_shift((w >> 2) & 3, bx.L[1]);
                    cz[u] = xj.z + select_shift((w >> 4) & 3, bx.L[2]);
                }
                ce[u] = j | (code << kIndexBits) | (SPLIT ? 0 : kInnerBit);
                cj[u] = j;
                ct[u] = WT ? b.type[q][j] : 0;
                live[u] = m0 < total;
            }
            if (amb)
                test_candidates<kCandPasses, true, WIDE, SPLIT>(L, cap, rlist2, rdl2, half_list, compact, bx, amb,
                                                                s_own + i0, n_chunk, xl, cx, cy, cz, ce, cj, ct, live,
                                                                my_count);
            else
                test_candidates<kCandPasses, false, WIDE, SPLIT>(L, cap, rlist2, rdl2, half_list, compact, bx, amb,
                                                                 s_own + i0, n_chunk, xl, cx, cy, cz, ce, cj, ct, live,
                                                                 my_count);
        }
        // per-atom epilogue: count, overflow flag, compact record
        const int i = s_own + i0 + lane;
        if (lane < n_chunk) {
            b.ncount[i] = min(my_count, cap);
            b.cellxyz[i] = make_int4(c[0], c[1], c[2], 0);
            if (compact) {
                int4 rq;
                if (!compact_coords<TRI ? 2 : 1>(R, c, xl.x, xl.y, xl.z, rq)) atomicAdd(&b.flags[F_COMPACT], 1);
                b.rec[0][i] = rq;
            }
            if (copy_back) {  // (no lane of this kernel reads the buffers written here)
                const int pn = p ^ 1, qn = q ^ 1;
                b.pos[pn][i] = pos[i];
                b.id[qn][i] = b.id[q][i];
                b.type[qn][i] = b.type[q][i];
                b.pwork[qn][i] = b.pwork[q][i];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    b.vel[qn][a][i] = b.vel[q][a][i];
                    b.img[qn][a][i] = b.img[q][a][i];
                }
                if (b.acc[q][0]) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        b.acc[qn][a][i] = b.acc[q][a][i];
                        b.jrk[qn][a][i] = b.jrk[q][a][i];
                    }
                }
            }
        }
        wave_max_flag(lane < n_chunk ? my_count : 0, &b.flags[F_MAX_COUNT]);
    }
}

// One wavefront per link cell.  LOOP (gated builds): a capped grid, each
// wavefront taking every `waves`-th cell (a wavefront's LDS operations
// complete in order, so its candidate table is simply refilled for the next
// cell); a separate instantiation, since the loop keeps more registers live.
template <bool TRI, bool WIDE, bool SPLIT, bool WT, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_cell_list(Buffers b, int p, int q, int64_t n_slots, int32_t n_cells,
                                                      int32_t cap, double rlist2, double rdl2, int half_list,
                                                      int compact, const int32_t* __restrict__ gate, int copy_back)
{
    const int64_t w0 = logical_block() * (kBlock / kWave) + threadIdx.x / kWave;
    if (!LOOP) {
        if (w0 < n_cells)
            list_cell<TRI, WIDE, SPLIT, WT>(b, p, q, n_slots, uniform((int)w0), cap, rlist2, rdl2, half_list,
                                            compact, nullptr, 0);
        return;
    }
    if (gate[0] == 0) return;
    const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t w = w0; w < n_cells; w += waves)
        list_cell<TRI, WIDE, SPLIT, WT>(b, p, q, n_slots, uniform((int)w), cap, rlist2, rdl2, half_list, compact,
                                        gate, copy_back);
}

// Compact records of all slots from the FP64 positions (mixed mode, at the
// start of a call when the list is kept).
__global__ void k_compact_records(Buffers b, int p, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - R.slot_off >= R.n_atoms) return;
    const int4 c4 = b.cellxyz[t];
    const int c[3] = {c4.x, c4.y, c4.z};
    const double3 x = load_xyz(b.pos[p], t);
    int4 rq;
    if (!compact_coords(R, c, x.x, x.y, x.z, rq)) atomicAdd(&b.flags[F_COMPACT], 1);
    b.rec[0][t] = rq;
}

// Pair separation from compact records.  With the cell offset dc in {-1,0,1}
// per axis, d_a = (q_j - q_i + dc 2^28) h_a 2^-28: the integer part is exact
// in 32 bits (|d| < 8 cells), and the scale is one rounding in FP64.  `qi1`
// holds q_i + 2^28, so the field c = dc + 1 of the entry adds c 2^28.
__device__ __forceinline__ double compact_axis(int code_field, int qj, int qi1, double qs)
{
    const uint32_t dq = ((uint32_t)code_field << kCompactBits) + (uint32_t)qj - (uint32_t)qi1;
    return (double)(int32_t)dq * qs;
}

// CMP = 1: orthorhombic cells.  CMP = 2: a sheared cell, whose records hold
// fractional in-cell coordinates: the integer differences along the three edge
// vectors map through qg = h diag(2^-28 / n_a) into the Cartesian separation.
template <int CMP>
__device__ __forceinline__ void compact_delta(const DevReplica& R, const int4& qi1, const int4& qj, int code,
                                              double& dx, double& dy, double& dz)
{
    if (CMP == 2) {
        const double d0 = compact_axis(code & 3, qj.x, qi1.x, 1.0);
        const double d1 = compact_axis((code >> 2) & 3, qj.y, qi1.y, 1.0);
        const double d2 = compact_axis((code >> 4) & 3, qj.z, qi1.z, 1.0);
        dx = fma(R.qg[0], d0, fma(R.qg[1], d1, R.qg[2] * d2));
        dy = fma(R.qg[3], d0, fma(R.qg[4], d1, R.qg[5] * d2));
        dz = fma(R.qg[6], d0, fma(R.qg[7], d1, R.qg[8] * d2));
        return;
    }
    dx = compact_axis(code & 3, qj.x, qi1.x, R.qs[0]);
    dy = compact_axis((code >> 2) & 3, qj.y, qi1.y, R.qs[1]);
    dz = compact_axis((code >> 4) & 3, qj.z, qi1.z, R.qs[2]);
}

__device__ __forceinline__ int4 compact_base(const int4& q)
{
    constexpr int one = 1 << kCompactBits;
    return make_int4(q.x + one, q.y + one, q.z + one, q.w);
}

// One 16-byte gather through a raw buffer resource: a single load
// instruction with a 32-bit offset (out-of-range offsets read zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t record_rsrc(const int4* p, int64_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int4*>(p), (short)0, (int)(n * 16), (int)kBufferWord3);
}
__device__ __forceinline__ int4 record_load(__amdgpu_buffer_rsrc_t rs, int j)
{
    const int4v v = __builtin_amdgcn_raw_buffer_load_b128(rs, j * 16, 0, 0);
    return make_int4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------
// Global-gather kernels: one thread per atom reads its neighbours straight
// from the cache hierarchy through the transposed int32 list.  Neighbours go
// in chunks of kChunk: all index loads, then all gathers, then the
// arithmetic.  Entries past the end point at the atom itself (masked).
//
// The cost of these loops is set by the number of vector-memory accesses per
// neighbour (the L1 resolves about one cache-line access per clock per CU),
// not by bytes or arithmetic: FP64 mode gathers a 32-byte {x, y, z, F'} record
// (two accesses), the compact mixed mode a 16-byte record (one access).
//
// Density pass (Eq. Ucoh, the argument of F): rho_i = sum_j rho_{s_i s_j}(r_ij),
// then F_i and F'_i.  The sum is accumulated in FP64 in both precision modes.
//
// NCH: neighbour records in flight per thread (2, 4 or 8; the autotuner picks
// it): more hide more gather latency, fewer free registers for more waves.
//
// TL: several species with all their tables staged in LDS, in workgroups of
// kTableBlock threads that share one copy (one species always stages its own).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, int CMP, int NCH, bool TL>
__global__ __launch_bounds__(TL ? kTableBlock : kBlock) void k_density(Buffers b, int p, int q, int64_t n_slots,
                                                                        PotArgs P, int energy)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const R* tab = tables<R>(b).dens;
    if (EV != EV_KNOTS && (SINGLE || TL)) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tab, (SINGLE ? 1 : P.ns * P.ns) * P.nbt * value_stride(EV));
        __syncthreads();
        tab = s;
    }
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - Rp.slot_off >= Rp.n_atoms) return;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const int4* __restrict__ rec = b.rec[0];
    const int32_t* __restrict__ nbr = b.nbr;
    const double3 xi = CMP ? make_double3(0.0, 0.0, 0.0) : load_xyz(pos, t);
    const int4 qi = CMP ? rec[t] : make_int4(0, 0, 0, 0);
    const int4 qb = compact_base(qi);
    const __amdgpu_buffer_rsrc_t rs = record_rsrc(b.rec[0], n_slots);
    const int si = b.type[q][t] & 0x3F;
    const int n = b.ncount[t];
    double rho = 0.0;
    constexpr int GR = NCH >= kChunk ? NCH / kChunk : 1;  // list groups per iteration
    constexpr int SUB = NCH >= kChunk ? 1 : kChunk / NCH;  // record batches per group
    static_assert(kChunk == 4 && NCH * SUB == kChunk * GR, "one int4 list load per four entries");
    for (int k0 = 0; k0 < n; k0 += kChunk * GR) {
        int v[kChunk * GR];
#pragma unroll
        for (int g = 0; g < GR; ++g) {  // 16-byte loads of four entries; groups past cap are padding
            const int4 v4 = reinterpret_cast<const int4*>(nbr)[(int64_t)((k0 >> 2) + g) * n_slots + t];
            v[4 * g] = v4.x;
            v[4 * g + 1] = v4.y;
            v[4 * g + 2] = v4.z;
            v[4 * g + 3] = v4.w;
        }
        uint32_t tv[GR];  // neighbour type bytes of the groups (several species)
#pragma unroll
        for (int g = 0; g < GR; ++g)
            tv[g] = SINGLE ? 0u : reinterpret_cast<const uint32_t*>(b.ntype)[(int64_t)((k0 >> 2) + g) * n_slots + t];
#pragma unroll
        for (int sb = 0; sb < SUB; ++sb) {
            const int kb = k0 + sb * NCH;
            if (kb >= n) break;
            int e[NCH];
            double3 xs[NCH];
            int4 qs[NCH];
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                // FP64: only inner entries (the others lie beyond every density
                // cutoff); mixed-precision lists mark every entry inner
                e[u] = kb + u < n ? v[sb * NCH + u] : (int)t;
                if (sizeof(R) == 4 || e[u] < 0) {
                    if (CMP) qs[u] = record_load(rs, e[u] & kIndexMask);
                    else xs[u] = load_xyz(pos, e[u] & kIndexMask);
                }
            }
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                if (kb + u >= n) break;
                if (sizeof(R) == 8 && e[u] >= 0) continue;
                const int code = ((unsigned)e[u] >> kIndexBits) & kCodeMask;
                double dx, dy, dz;
                if (CMP) {
                    compact_delta<CMP>(Rp, qb, qs[u], code, dx, dy, dz);
                } else {
                    dx = xs[u].x - xi.x;
                    dy = xs[u].y - xi.y;
                    dz = xs[u].z - xi.z;
                    if (code) apply_shift(bx, code, dx, dy, dz);
                }
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                if (!(r2 < P.rc2)) continue;
                const double r = r2 * inv_dist<R>(r2);
                const int ku = sb * NCH + u;  // entry within the groups loaded
                const int sj = SINGLE ? 0 : (int)((tv[ku >> 2] >> (8 * (ku & 3))) & 0x3F);
                rho += (double)density_term<R, SINGLE, NDK, EV>(P, G, tab, si, sj, r);
            }
        }
    }
    double F, dF;
    embed(SINGLE ? P.emb_c : G.emb_c[si], rho, F, dF);
    if (CMP) b.rec[1][t] = make_int4(qi.x, qi.y, qi.z, __float_as_int((float)dF));
    else reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
    if (energy) b.femb[t] = F;
}

// Force pass + velocity Verlet (global gathers).
//
// EN = 4: the energies and virial of energy mode 1, summed per wavefront in the
// kernel (the reduction then reads one record per 64 atoms).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, int EN, bool CLOSE, bool OPEN, bool WRITEBACK,
          int CMP, int NCH, bool TL>
__global__ __launch_bounds__(TL ? kTableBlock : kBlock) void k_force(Buffers b, int p, int q, int64_t n_slots,
                                                                      PotArgs P, double dt, md_state st)
{
    constexpr bool WSUM = EN == 4;
    constexpr int ENERGY = WSUM ? 1 : EN;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tabs<R> T = tables<R>(b);
    const R* tf = T.force;
    const R* te = T.energy;
    if (EV != EV_KNOTS && (SINGLE || TL)) {
        const int nf = (SINGLE ? 1 : P.ns * P.ns) * P.nbt * force_stride(EV);
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tf, nf);
        if (ENERGY == 1) lds_fill(s + nf, te, (SINGLE ? 1 : P.ns * P.ns) * P.nbt * value_stride(EV));
        __syncthreads();
        tf = s;
        te = s + nf;
    }
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    // slots past the replica's atoms: none in energy-sum mode, whose wavefront
    // sums need every lane (those lanes add zeros)
    const bool pad = t - Rp.slot_off >= Rp.n_atoms;
    if (pad && !WSUM) return;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const int4* __restrict__ rec = b.rec[1];
    const int32_t* __restrict__ nbr = b.nbr;
    const double4 pi = pos[t];
    const int4 qi = CMP ? rec[t] : make_int4(0, 0, 0, 0);
    const int4 qb = compact_base(qi);
    const __amdgpu_buffer_rsrc_t rs = record_rsrc(b.rec[1], n_slots);
    const uint8_t ti = b.type[q][t];
    const int si = ti & 0x3F;
    const bool rigid_i = ti & kRigidBit;
    const int n = pad ? 0 : b.ncount[t];
    const R fpi = CMP ? (R)__int_as_float(qi.w) : (R)pi.w;
    PairAcc A;
    constexpr int GR = NCH >= kChunk ? NCH / kChunk : 1;  // list groups per iteration
    constexpr int SUB = NCH >= kChunk ? 1 : kChunk / NCH;  // record batches per group
    static_assert(kChunk == 4 && NCH * SUB == kChunk * GR, "one int4 list load per four entries");
    for (int k0 = 0; k0 < n; k0 += kChunk * GR) {
        int v[kChunk * GR];
#pragma unroll
        for (int g = 0; g < GR; ++g) {  // 16-byte loads of four entries; groups past cap are padding
            const int4 v4 = reinterpret_cast<const int4*>(nbr)[(int64_t)((k0 >> 2) + g) * n_slots + t];
            v[4 * g] = v4.x;
            v[4 * g + 1] = v4.y;
            v[4 * g + 2] = v4.z;
            v[4 * g + 3] = v4.w;
        }
        uint32_t tv[GR];  // neighbour type bytes of the groups (several species)
#pragma unroll
        for (int g = 0; g < GR; ++g)
            tv[g] = SINGLE ? 0u : reinterpret_cast<const uint32_t*>(b.ntype)[(int64_t)((k0 >> 2) + g) * n_slots + t];
#pragma unroll
        for (int sb = 0; sb < SUB; ++sb) {
            const int kb = k0 + sb * NCH;
            if (kb >= n) break;
            int e[NCH];
            double4 ps[NCH];
            int4 qs[NCH];
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                e[u] = kb + u < n ? v[sb * NCH + u] : (int)t;
                if (CMP) qs[u] = record_load(rs, e[u] & kIndexMask);
                else ps[u] = pos[e[u] & kIndexMask];
            }
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                if (kb + u >= n) break;
                const int code = ((unsigned)e[u] >> kIndexBits) & kCodeMask;
                double dx, dy, dz;
                R fpj;
                if (CMP) {
                    compact_delta<CMP>(Rp, qb, qs[u], code, dx, dy, dz);
                    fpj = (R)__int_as_float(qs[u].w);
                } else {
                    dx = ps[u].x - pi.x;
                    dy = ps[u].y - pi.y;
                    dz = ps[u].z - pi.z;
                    if (code) apply_shift(bx, code, dx, dy, dz);
                    fpj = (R)ps[u].w;
                }
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                if (!(r2 < P.rc2)) continue;
                const double ri = inv_dist<R>(r2);
                const double r = r2 * ri;
                // one species: j's type byte matters only for the virial of a rigid
                // atom i (pairs of two rigid atoms stay out of it)
                const int ku = sb * NCH + u;  // entry within the groups loaded
                const uint8_t tj = !SINGLE ? (uint8_t)(tv[ku >> 2] >> (8 * (ku & 3)))
                                           : (ENERGY == 1 && rigid_i) ? b.type[q][e[u] & kIndexMask] : 0;
                R g, phi;
                pair_terms<R, SINGLE, NPK, NDK, EV, ENERGY>(P, G, tf, te, si, tj & 0x3F, r, fpi, fpj, g, phi);
                accumulate<ENERGY>(A, (double)g * ri, dx, dy, dz, (double)phi, rigid_i && (tj & kRigidBit));
            }
        }
    }
    double wv[kEnergyTerms] = {};
    if (!pad) atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK, WSUM>(b, p, q, t, n_slots, Rp, P, G, dt, st, pi, ti,
                                                                      A, wv);
    if (WSUM) wave_sum_terms(b, t, wv);
    if (CMP && OPEN && !pad) {
        // the compact record of the drifted position, for the next density pass
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        const double3 xn = load_xyz(b.pos[p ^ 1], t);
        int4 rq;
        if (!compact_coords<CMP>(Rp, c, xn.x, xn.y, xn.z, rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
}

// Per-replica totals of the per-atom energy terms, in two stages with a fixed
// order that depends only on the replica's own size, so a replica gives bitwise
// the same sums alone or inside a batch.  Stage 1: one workgroup per chunk of
// kReduceChunk slots (counted from the replica's first slot); stage 2: one
// workgroup per replica over its chunk sums.
__device__ __forceinline__ void block_sum_terms(double v[kEnergyTerms], double (*sh)[kBlock])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) sh[k][tid] = v[k];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (tid < off)
#pragma unroll
            for (int k = 0; k < kEnergyTerms; ++k) sh[k][tid] += sh[k][tid + off];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_chunks(Buffers b, int64_t n_slots)
{
    __shared__ double sh[kEnergyTerms][kBlock];
    const int c = blockIdx.x;
    const int r = b.chunk_rep[c];
    const DevReplica& R = b.reps[r];
    const int64_t s0 = R.slot_off + (int64_t)(c - b.chunk_off[r]) * kReduceChunk;
    const int64_t s1 = min(s0 + (int64_t)kReduceChunk, (int64_t)R.slot_off + R.n_atoms);
    double v[kEnergyTerms];
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) v[k] = 0.0;
    for (int64_t t = s0 + threadIdx.x; t < s1; t += kBlock)
#pragma unroll
        for (int k = 0; k < kEnergyTerms; ++k) v[k] += b.eslot[(int64_t)k * n_slots + t];
    block_sum_terms(v, sh);
    if (threadIdx.x < kEnergyTerms) b.chunk_partial[(int64_t)c * kEnergySlots + threadIdx.x] = sh[threadIdx.x][0];
}

// Stage 1 from per-wavefront sums: one wavefront per chunk sums its chunk's
// (at most kReduceChunk / 64) wavefront records by an xor butterfly.
__global__ __launch_bounds__(kWave) void k_reduce_wave_chunks(Buffers b)
{
    static_assert(kReduceChunk / kWave <= kWave, "one lane per wavefront record of a chunk");
    const int c = blockIdx.x;
    const int r = b.chunk_rep[c];
    const DevReplica& R = b.reps[r];
    const int64_t s0 = R.slot_off + (int64_t)(c - b.chunk_off[r]) * kReduceChunk;
    const int64_t s1 = min(s0 + (int64_t)kReduceChunk, (int64_t)R.slot_off + R.n_atoms);
    const int64_t w = s0 / kWave + threadIdx.x;
    const bool live = w < (s1 + kWave - 1) / kWave;
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) {
        double v = live ? b.wave_terms[w * kEnergyTerms + k] : 0.0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        if (threadIdx.x == 0) b.chunk_partial[(int64_t)c * kEnergySlots + k] = v;
    }
}

//
// ring_len > 0: the totals also go to entry (count mod ring_len) of the energy
// ring ("Thermodynamic Quantities", sampled every few steps).  Every workgroup
// reads the count before it takes a ticket, and the last one to take a ticket
// advances the count, so a captured step sequence appends to successive
// entries on every replay.
__global__ __launch_bounds__(kBlock) void k_reduce_replicas(Buffers b, double virial_scale, int64_t ring_len)
{
    __shared__ double sh[kEnergyTerms][kBlock];
    const int r = blockIdx.x;
    const int64_t count =
        ring_len > 0 ? __hip_atomic_load(b.ering_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    double v[kEnergyTerms];
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k) v[k] = 0.0;
    for (int c = b.chunk_off[r] + threadIdx.x; c < b.chunk_off[r + 1]; c += kBlock)
#pragma unroll
        for (int k = 0; k < kEnergyTerms; ++k) v[k] += b.chunk_partial[(int64_t)c * kEnergySlots + k];
    block_sum_terms(v, sh);
    if (threadIdx.x < kEnergySlots) {
        const int k = threadIdx.x;
        double out = k < kEnergyTerms ? sh[k][0] : 0.0;
        if (k >= E_W0 && k < E_W0 + 6) out *= virial_scale;
        b.energies[(int64_t)r * kEnergySlots + k] = out;
        if (ring_len > 0) b.ering[((count % ring_len) * gridDim.x + r) * kEnergySlots + k] = out;
    }
    if (ring_len > 0) {
        __syncthreads();  // this replica's entry is written
        if (threadIdx.x == 0) {
            __threadfence();
            const unsigned long long done = atomicAdd(reinterpret_cast<unsigned long long*>(b.ering_count + 1), 1ull);
            if (done == gridDim.x - 1) {
                b.ering_count[1] = 0;
                __hip_atomic_store(b.ering_count, count + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Nose-Hoover thermostat (paper, "Thermostat NVTp").  The flow of a step is
// split symmetrically: thermostat half step, velocity half kick, drift, forces,
// velocity half kick, thermostat half step.  A thermostat half step of length
// h with kinetic energy K updates pi by (h/2)(2K - g k_B T)/Q, scales the
// velocities by exp(-pi h) (K by its square), advances xi by pi h and updates
// pi again with the scaled K.  Between two steps the two half steps meet, so
// one kinetic-energy reduction per step serves both.

// Kinetic energy of the mobile atoms of each wavefront (a wavefront never
// straddles two replicas): one partial per wave, summed by shuffles in a fixed
// order.  The whole slot range runs in parallel.
__global__ __launch_bounds__(kBlock) void k_nh_ke_waves(Buffers b, int q, int64_t n_slots, PotArgs P)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;  // n_slots is a multiple of the wave size: whole waves leave
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const DevPotential& G = *b.pot;
    double ke = 0.0;
    if (t - R.slot_off < R.n_atoms) {
        const uint8_t ty = b.type[q][t];
        if (!(ty & kRigidBit)) {
            const double vx = b.vel[q][0][t], vy = b.vel[q][1][t], vz = b.vel[q][2][t];
            ke = (P.ns == 1 ? P.half_m : G.half_m[ty & 0x3F]) * (vx * vx + vy * vy + vz * vz);
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) ke += __shfl_down(ke, off, kWave);
    if ((t & (kWave - 1)) == 0) b.nh_partial[t / kWave] = ke;
}

// One workgroup per replica: the kinetic energy from the replica's wave
// partials, or from its chunk sums when `chunked` (a fixed tree either way),
// then on one lane `halves` thermostat half steps of
// length dt/2; nh_state = {pi, xi, total velocity scale, kinetic energy after}.
__global__ __launch_bounds__(kBlock) void k_nh_update(Buffers b, int halves, double dt, int chunked)
{
    __shared__ double sh[kBlock];
    const int r = blockIdx.x;
    double part = 0.0;
    if (chunked) {
        for (int c = b.chunk_off[r] + threadIdx.x; c < b.chunk_off[r + 1]; c += kBlock)
            part += b.chunk_partial[(int64_t)c * kEnergySlots];
    } else {
        const DevReplica& R = b.reps[r];
        const int64_t w0 = R.slot_off / kWave, w1 = (R.slot_off + (int64_t)R.n_atoms + kWave - 1) / kWave;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += kBlock) part += b.nh_partial[w];
    }
    sh[threadIdx.x] = part;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double K = sh[0];
    double* st = b.nh_state + 4 * (int64_t)r;
    const double Q = b.nh_param[2 * r], gkt = b.nh_param[2 * r + 1];
    double pi = st[0], xi = st[1], S = 1.0;
    const double h = 0.5 * dt;
    for (int k = 0; k < halves; ++k) {
        pi += 0.5 * h * (2.0 * K - gkt) / Q;
        const double s = exp(-pi * h);
        S *= s;
        K *= s * s;
        xi += pi * h;
        pi += 0.5 * h * (2.0 * K - gkt) / Q;
    }
    st[0] = pi;
    st[1] = xi;
    st[2] = S;
    st[3] = K;
}

// Scaled opening half kick and drift after a thermostatted boundary: for mobile
// atoms v <- S v + (dt/2) f/m and x <- x + dt v; rigid atoms move on their
// line and account the opening half of their power.  Writes pos[p^1] (and the
// compact record of the new position).
__global__ void k_nh_open(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double dt, int compact, int scaled)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const uint8_t ty = b.type[q][t];
    const double3 x = load_xyz(b.pos[p], t);
    double xn[3] = {x.x, x.y, x.z};
    const double f[3] = {b.fhalf[0][t], b.fhalf[1][t], b.fhalf[2][t]};
    if (ty & kRigidBit) {
        b.pwork[q][t] += -(f[0] * R.vp[0] + f[1] * R.vp[1] + f[2] * R.vp[2]) * 0.5 * dt;
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[a] += dt * R.vp[a];
    } else {
        const double S = scaled ? b.nh_state[4 * (int64_t)r + 2] : 1.0;
        const double acc = P.ns == 1 ? P.accel : G.accel[ty & 0x3F];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = fma(0.5 * dt * acc, f[a], S * b.vel[q][a][t]);
            b.vel[q][a][t] = v;
            xn[a] = fma(dt, v, xn[a]);
        }
    }
    double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
    *reinterpret_cast<double2*>(dst) = make_double2(xn[0], xn[1]);
    dst[2] = xn[2];
    if (compact) {
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        int4 rq;
        if (!compact_coords(R, c, xn[0], xn[1], xn[2], rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
}

// Final thermostat half step of an md_step call: scale the mobile velocities
// (internal and the caller's, already written back) and their kinetic-energy
// terms.
__global__ void k_nh_scale(Buffers b, int q, int64_t n_slots, md_state st, int energy)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    if (b.type[q][t] & kRigidBit) return;
    const double S = b.nh_state[4 * (int64_t)r + 2];
    const int32_t a = b.id[q][t];
    for (int d = 0; d < 3; ++d) b.vel[q][d][t] *= S;
    st.vx[a] *= S;
    st.vy[a] *= S;
    st.vz[a] *= S;
    if (energy) b.eslot[(int64_t)E_KE * n_slots + t] *= S * S;
}

// ---------------------------------------------------------------------------
// Parrinello-Rahman barostat on an orthorhombic box (paper, "Barostat NPTp";
// h = diag(L), hydrostatic external stress).  The step composes exact
// sub-flows symmetrically: box half kick W dL/dt += (h/2)(Omega/L)(pi - P),
// friction half step v *= exp(-(h/2) dL/dt / L), velocity half kick, drift of
// positions and box with dL/dt held, forces, and the mirror image.  Between two
// steps the closing and opening halves meet: the force pass closes the kick,
// k_pr_update takes both box half kicks from one stress tensor and drifts the
// box, k_pr_open applies both friction halves, the opening kick and the drift.

// Per wave: sums of m v_a^2 and of the per-atom virial diagonal (eslot).
__global__ __launch_bounds__(kBlock) void k_pr_tensor_waves(Buffers b, int q, int64_t n_slots, PotArgs P)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;  // whole waves
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const DevPotential& G = *b.pot;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (t - R.slot_off < R.n_atoms) {
        const uint8_t ty = b.type[q][t];
        const double m2 = 2.0 * (P.ns == 1 ? P.half_m : G.half_m[ty & 0x3F]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double va = b.vel[q][a][t];
            v[a] = m2 * va * va;
            v[3 + a] = b.eslot[(int64_t)(E_W0 + a) * n_slots + t];
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
        if ((t & (kWave - 1)) == 0) b.pr_partial[(t / kWave) * 6 + k] = x;
    }
}

// Thermostat and barostat sums, first stage: one wavefront per reduction chunk
// (kReduceChunk slots of one replica) adds the chunk's per-wave partials (N
// terms each) in a fixed shuffle tree into chunk_partial[c][k].  The update
// kernels then read a replica's chunk sums instead of all its wave partials.
template <int N>
__global__ __launch_bounds__(kWave) void k_chunk_sums(Buffers b, const double* __restrict__ part)
{
    const int c = blockIdx.x;
    const int r = b.chunk_rep[c];
    const DevReplica& R = b.reps[r];
    const int64_t s0 = R.slot_off + (int64_t)(c - b.chunk_off[r]) * kReduceChunk;
    const int64_t s1 = min(s0 + (int64_t)kReduceChunk, (int64_t)R.slot_off + R.n_atoms);
    const int64_t w = s0 / kWave + threadIdx.x;
    const bool live = w < (s1 + kWave - 1) / kWave;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double x = live ? part[w * N + k] : 0.0;
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
        if (threadIdx.x == 0) b.chunk_partial[(int64_t)c * kEnergySlots + k] = x;
    }
}

// One workgroup per replica: the stress tensor from the wave partials or, when
// `chunked`, the chunk sums (a fixed tree either way), then on one lane the
// closing and/or opening box half kicks and, with
// `open`, the box drift and the factors of the open pass.
__global__ __launch_bounds__(kBlock) void k_pr_update(Buffers b, int close, int open, double h, double rlist,
                                                      double strain_tol, int nvt, int chunked)
{
    __shared__ double sh[6][kBlock];
    const int r = blockIdx.x;
    DevReplica& R = b.reps[r];
    double part[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (chunked) {
        for (int c = b.chunk_off[r] + threadIdx.x; c < b.chunk_off[r + 1]; c += kBlock)
#pragma unroll
            for (int k = 0; k < 6; ++k) part[k] += b.chunk_partial[(int64_t)c * kEnergySlots + k];
    } else {
        const int64_t w0 = R.slot_off / kWave, w1 = (R.slot_off + (int64_t)R.n_atoms + kWave - 1) / kWave;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += kBlock)
#pragma unroll
            for (int k = 0; k < 6; ++k) part[k] += b.pr_partial[w * 6 + k];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = part[k];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
#pragma unroll
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x != 0 || R.n_atoms == 0) return;  // an empty replica's box stays put
    double* st = b.pr_state + (int64_t)kPrState * r;
    const double W = b.pr_param[2 * r], pext = b.pr_param[2 * r + 1];
    double L[3], Ld[3], lam_c[3], mv2[3];
    for (int a = 0; a < 3; ++a) {
        L[a] = st[a];
        Ld[a] = st[3 + a];
        lam_c[a] = close ? Ld[a] / L[a] : 0.0;
        mv2[a] = sh[a][0] * exp(-h * lam_c[a]);  // m v_a^2 after the closing friction half step
    }
    // with the thermostat (NPT): its half steps sit between the box friction
    // and the box kicks, and scale every velocity of the replica alike
    double* nh = b.nh_state + 4 * (int64_t)r;
    double pi_s = 0.0, xi = 0.0, s_close = 1.0, s_open = 1.0;
    const double Q = nvt ? b.nh_param[2 * r] : 1.0, gkt = nvt ? b.nh_param[2 * r + 1] : 0.0;
    auto thermostat_half = [&](double& scale) {
        const double hh = 0.5 * h;
        double K = 0.5 * (mv2[0] + mv2[1] + mv2[2]);
        pi_s += 0.5 * hh * (2.0 * K - gkt) / Q;
        const double sc = exp(-pi_s * hh);
        scale = sc;
        for (int a = 0; a < 3; ++a) mv2[a] *= sc * sc;
        K *= sc * sc;
        xi += pi_s * hh;
        pi_s += 0.5 * hh * (2.0 * K - gkt) / Q;
    };
    if (nvt) {
        pi_s = nh[0];
        xi = nh[1];
        if (close) thermostat_half(s_close);
    }
    const double omega = L[0] * L[1] * L[2];
    for (int a = 0; a < 3; ++a) {
        // the full-list virial sees every pair from both atoms
        const double pi_aa = (mv2[a] - 0.5 * sh[3 + a][0]) / omega;
        Ld[a] += (close + open) * 0.5 * h * (omega / L[a]) * (pi_aa - pext) / W;
        st[15 + a] = exp(-0.5 * h * lam_c[a]) * s_close;
        st[3 + a] = Ld[a];
    }
    if (nvt && open) thermostat_half(s_open);
    if (nvt) {
        nh[0] = pi_s;
        nh[1] = xi;
        nh[2] = s_close * s_open;
        nh[3] = 0.5 * (mv2[0] + mv2[1] + mv2[2]);
    }
    if (!open) return;
    for (int a = 0; a < 3; ++a) {
        const double lam_o = Ld[a] / L[a];
        const double u = h * lam_o;
        const double phi = u == 0.0 ? 1.0 : log1p(u) / u;
        const double Ln = L[a] + h * Ld[a];
        st[6 + a] = exp(-0.5 * h * (lam_c[a] + lam_o)) * s_close * s_open;
        st[9 + a] = Ln / L[a];
        st[12 + a] = h * phi * (Ln / L[a]);
        st[a] = Ln;
        R.box[a] = Ln;
        R.inv_box[a] = 1.0 / Ln;
        R.cell[a] = Ln / (double)R.nc[a];
        R.qs[a] = ldexp(R.cell[a], -kCompactBits);
        R.iqs[a] = ldexp(1.0 / R.cell[a], kCompactBits);
        if (R.cell[a] < rlist) atomicAdd(&b.flags[F_PR_BOX], 1);
        if (fabs(Ln / R.lbuild[a] - 1.0) * rlist > strain_tol) atomicAdd(&b.flags[F_SKIN], 1);
    }
}

// Both friction halves, the opening kick and the drift of positions (scaled
// about the box origin) into pos[p^1], with the compact record in the new box.
__global__ void k_pr_open(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double h, int compact)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const double* st = b.pr_state + (int64_t)kPrState * r;
    const uint8_t ty = b.type[q][t];
    const double acc = P.ns == 1 ? P.accel : G.accel[ty & 0x3F];
    const double3 x = load_xyz(b.pos[p], t);
    const double xo[3] = {x.x - R.origin[0], x.y - R.origin[1], x.z - R.origin[2]};
    double xn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = fma(0.5 * h * acc, b.fhalf[a][t], st[6 + a] * b.vel[q][a][t]);
        b.vel[q][a][t] = v;
        xn[a] = R.origin[a] + fma(st[12 + a], v, xo[a] * st[9 + a]);
    }
    double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
    *reinterpret_cast<double2*>(dst) = make_double2(xn[0], xn[1]);
    dst[2] = xn[2];
    if (compact) {
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        int4 rq;
        if (!compact_coords<1>(R, c, xn[0], xn[1], xn[2], rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
}

// Closing friction half step of the last step of a call: the internal and the
// caller's velocities and the kinetic terms of the energy record.
__global__ void k_pr_close_scale(Buffers b, int q, int64_t n_slots, PotArgs P, md_state st)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const double* ps = b.pr_state + (int64_t)kPrState * r;
    const uint8_t ty = b.type[q][t];
    const int32_t id = b.id[q][t];
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[a] = b.vel[q][a][t] * ps[15 + a];
        b.vel[q][a][t] = v[a];
    }
    st.vx[id] = v[0];
    st.vy[id] = v[1];
    st.vz[id] = v[2];
    b.eslot[(int64_t)E_KE * n_slots + t] = (P.ns == 1 ? P.half_m : G.half_m[ty & 0x3F]) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// After a list build: the build box of every replica is the current one.
__global__ void k_pr_mark_build(Buffers b, int n_replicas)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_replicas) return;
    DevReplica& R = b.reps[r];
#pragma unroll
    for (int a = 0; a < 3; ++a) R.lbuild[a] = R.box[a];
    if (R.tri)
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            R.hbinv[e] = R.hinv[e];
            R.mb[e] = (e % 4 == 0) ? 1.0 : 0.0;
        }
}

// ---------------------------------------------------------------------------
// Third-order Gear predictor-corrector (paper, "Time integration").  Per
// coordinate the state is x, v, the acceleration a and its time derivative b.
// The predictor is the Taylor series to third order; after the force pass at
// the predicted positions the mismatch d = f/m - a_pred corrects the four
// values with Gear's weights for second-order equations.  In unscaled form
// (step h): x += h^2 d / 12, v += 5 h d / 12, a = f/m, b += d / h.  The force
// pass keeps f (fhalf); the corrector runs as its own pass because every atom
// must see its neighbours' predicted positions first.

// a = f/m of the starting positions, b = 0.
__global__ void k_gear_start(Buffers b, int q, int64_t n_slots, PotArgs P)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const uint8_t ty = b.type[q][t];
    const double acc = (ty & kRigidBit) ? 0.0 : (P.ns == 1 ? P.accel : G.accel[ty & 0x3F]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b.acc[q][a][t] = acc * b.fhalf[a][t];
        b.jrk[q][a][t] = 0.0;
    }
}

// Predicted positions pos[p^1] (and their compact records).  Rigid atoms take
// their next position on x0 + vp t and the first half of the step's work
// from the force of the previous evaluation.
__global__ void k_gear_predict(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double h, int compact)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const uint8_t ty = b.type[q][t];
    const double3 x = load_xyz(b.pos[p], t);
    double xn[3] = {x.x, x.y, x.z};
    if (ty & kRigidBit) {
        const double f[3] = {b.fhalf[0][t], b.fhalf[1][t], b.fhalf[2][t]};
        b.pwork[q][t] += -(f[0] * R.vp[0] + f[1] * R.vp[1] + f[2] * R.vp[2]) * 0.5 * h;
#pragma unroll
        for (int a = 0; a < 3; ++a) xn[a] += h * R.vp[a];
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double inc = b.vel[q][a][t] + h * (0.5 * b.acc[q][a][t] + (h / 6.0) * b.jrk[q][a][t]);
            xn[a] = fma(h, inc, xn[a]);
        }
    }
    double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
    *reinterpret_cast<double2*>(dst) = make_double2(xn[0], xn[1]);
    dst[2] = xn[2];
    if (compact) {
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        int4 rq;
        if (!compact_coords(R, c, xn[0], xn[1], xn[2], rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
}

// Corrector from pos[p] (predicted) into pos[p^1].  Within a call the same
// pass predicts the next step from the corrected values (all of them local to
// the atom), so pos[p^1] receives the next predicted position and its compact
// record, and rigid atoms account both halves of the work at this evaluation.
// The last step of a call stores the corrected position instead, takes f from
// the caller's arrays (its force pass wrote them), keeps it for the next call,
// fixes the kinetic and work terms of the energy record and writes the
// caller's x and v.
__global__ void k_gear_correct(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double h, md_state st, int last,
                               int compact)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const uint8_t ty = b.type[q][t];
    const int32_t id = b.id[q][t];
    const double3 xp = load_xyz(b.pos[p], t);
    double xc[3] = {xp.x, xp.y, xp.z};
    double f[3];
    if (last) {
        f[0] = st.fx[id];
        f[1] = st.fy[id];
        f[2] = st.fz[id];
#pragma unroll
        for (int a = 0; a < 3; ++a) b.fhalf[a][t] = f[a];
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] = b.fhalf[a][t];
    }
    double v[3];
    double ke = 0.0;
    if (ty & kRigidBit) {
        b.pwork[q][t] += -(f[0] * R.vp[0] + f[1] * R.vp[1] + f[2] * R.vp[2]) * (last ? 0.5 * h : h);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = R.vp[a];
            if (!last) xc[a] += h * R.vp[a];
        }
    } else {
        const int si = ty & 0x3F;
        const double acc = P.ns == 1 ? P.accel : G.accel[si];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double a0 = b.acc[q][a][t], j0 = b.jrk[q][a][t];
            const double an = acc * f[a];
            const double d = an - fma(h, j0, a0);
            const double jn = j0 + d / h;
            v[a] = b.vel[q][a][t] + h * (a0 + 0.5 * h * j0) + (5.0 / 12.0) * h * d;
            xc[a] += (h * h / 12.0) * d;
            if (!last) xc[a] = fma(h, v[a] + h * (0.5 * an + (h / 6.0) * jn), xc[a]);  // next prediction
            b.vel[q][a][t] = v[a];
            b.acc[q][a][t] = an;
            b.jrk[q][a][t] = jn;
        }
        ke = (P.ns == 1 ? P.half_m : G.half_m[si]) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
    *reinterpret_cast<double2*>(dst) = make_double2(xc[0], xc[1]);
    dst[2] = xc[2];
    if (compact && !last) {
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        int4 rq;
        if (!compact_coords(R, c, xc[0], xc[1], xc[2], rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
    if (last) {
        b.eslot[(int64_t)E_KE * n_slots + t] = ke;
        b.eslot[(int64_t)E_PW * n_slots + t] = (ty & kRigidBit) ? b.pwork[q][t] : 0.0;
        double sh[3];
        lattice_shift(R, b.img[q][0][t], b.img[q][1][t], b.img[q][2][t], sh);
        st.x[id] = xc[0] + sh[0];
        st.y[id] = xc[1] + sh[1];
        st.z[id] = xc[2] + sh[2];
        st.vx[id] = v[0];
        st.vy[id] = v[1];
        st.vz[id] = v[2];
    }
}

// ---------------------------------------------------------------------------
// Half-list variant (MD_NBR_HALF_ATOMIC): the comparison form in which every
// unordered pair is evaluated once, by its lower slot, and the partner's share
// goes to memory with FP64 atomics; the paper's own OpenMP code resolves the
// same write conflict with link-cell locks (section "OpenMP Parallelisation").
// Density: rho_i and rho_j both receive their term; the embedding then runs as
// its own pass.  Forces: f_i += s d, f_j -= s d; pair energies split in halves;
// the virial counts every pair once.  Integration follows as a separate pass.

// Density pass, half list: accumulates into rhalf (zeroed beforehand).
template <typename R, bool SINGLE, int NPK, int NDK, int EV>
__global__ __launch_bounds__(kBlock) void k_density_half(Buffers b, int p, int q, int64_t n_slots, PotArgs P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const R* tab = tables<R>(b).dens;
    if (EV != EV_KNOTS && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tab, P.nbt * value_stride(EV));
        __syncthreads();
        tab = s;
    }
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - Rp.slot_off >= Rp.n_atoms) return;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const int32_t* __restrict__ nbr = b.nbr;
    const double3 xi = load_xyz(pos, t);
    const int si = b.type[q][t] & 0x3F;
    const int n = b.ncount[t];
    double rho = 0.0;
    for (int k = 0; k < n; ++k) {
        const int e = nbr[nbr_at(k, t, n_slots)];
        const int j = e & kIndexMask;
        const double3 xj = load_xyz(pos, j);
        double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
        const int code = ((unsigned)e >> kIndexBits) & kCodeMask;
        if (code) apply_shift(bx, code, dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < P.rc2)) continue;
        const double r = r2 * inv_dist<R>(r2);
        const int sj = SINGLE ? 0 : (b.type[q][j] & 0x3F);
        const R to_i = density_term<R, SINGLE, NDK, EV>(P, G, tab, si, sj, r);
        const R to_j = SINGLE ? to_i : density_term<R, SINGLE, NDK, EV>(P, G, tab, sj, si, r);
        rho += (double)to_i;
        atomicAdd(&b.rhalf[j], (double)to_j);
    }
    atomicAdd(&b.rhalf[t], rho);
}

// Embedding after the half-list density pass: F_i, F'_i from rho_i.
template <bool SINGLE>
__global__ void k_embed_half(Buffers b, int p, int q, int64_t n_slots, PotArgs P, int energy)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - Rp.slot_off >= Rp.n_atoms) return;
    const DevPotential& G = *b.pot;
    const int si = b.type[q][t] & 0x3F;
    double F, dF;
    embed(SINGLE ? P.emb_c : G.emb_c[si], b.rhalf[t], F, dF);
    reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
    if (energy) b.femb[t] = F;
}

// Force pass, half list: forces and pair energies into fhalf / ehalf (zeroed
// beforehand); the virial of the pairs an atom owns into its energy slots.
template <typename R, bool SINGLE, int NPK, int NDK, int EV, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_force_half(Buffers b, int p, int q, int64_t n_slots, PotArgs P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tabs<R> T = tables<R>(b);
    const R* tf = T.force;
    const R* te = T.energy;
    if (EV != EV_KNOTS && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tf, P.nbt * force_stride(EV));
        if (ENERGY == 1) lds_fill(s + P.nbt * force_stride(EV), te, P.nbt * value_stride(EV));
        __syncthreads();
        tf = s;
        te = s + P.nbt * force_stride(EV);
    }
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - Rp.slot_off >= Rp.n_atoms) return;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const int32_t* __restrict__ nbr = b.nbr;
    const double4 pi = pos[t];
    const uint8_t ti = b.type[q][t];
    const int si = ti & 0x3F;
    const bool rigid_i = ti & kRigidBit;
    const int n = b.ncount[t];
    PairAcc A;
    for (int k = 0; k < n; ++k) {
        const int e = nbr[nbr_at(k, t, n_slots)];
        const int j = e & kIndexMask;
        const double4 pj = pos[j];
        double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        const int code = ((unsigned)e >> kIndexBits) & kCodeMask;
        if (code) apply_shift(bx, code, dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < P.rc2)) continue;
        const double ri = inv_dist<R>(r2);
        const double r = r2 * ri;
        const uint8_t tj = (!SINGLE || ENERGY) ? b.type[q][j] : 0;
        R g, phi;
        pair_terms<R, SINGLE, NPK, NDK, EV, ENERGY>(P, G, tf, te, si, tj & 0x3F, r, (R)pi.w, (R)pj.w, g, phi);
        const double s = (double)g * ri;
        accumulate<ENERGY>(A, s, dx, dy, dz, (double)phi, rigid_i && (tj & kRigidBit));
        atomicAdd(&b.fhalf[0][j], -s * dx);
        atomicAdd(&b.fhalf[1][j], -s * dy);
        atomicAdd(&b.fhalf[2][j], -s * dz);
        if (ENERGY) atomicAdd(&b.ehalf[j], 0.5 * (double)phi);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(&b.fhalf[a][t], A.f[a]);
    if (ENERGY) {
        atomicAdd(&b.ehalf[t], 0.5 * A.epair);
#pragma unroll
        for (int k = 0; k < 6; ++k) b.eslot[(int64_t)(E_W0 + k) * n_slots + t] = A.w[k];
    }
}

// Velocity Verlet and energy terms after the half-list force pass.
template <bool SINGLE, bool ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK>
__global__ void k_integrate_half(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double dt, md_state st)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (t - Rp.slot_off >= Rp.n_atoms) return;
    const DevPotential& G = *b.pot;
    PairAcc A;
#pragma unroll
    for (int a = 0; a < 3; ++a) A.f[a] = b.fhalf[a][t];
    if (ENERGY) {
        A.epair = 2.0 * b.ehalf[t];
#pragma unroll
        for (int k = 0; k < 6; ++k) A.w[k] = b.eslot[(int64_t)(E_W0 + k) * n_slots + t];
    }
    atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK>(b, p, q, t, n_slots, Rp, P, G, dt, st, b.pos[p][t],
                                                         b.type[q][t], A);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, v, n);
}

void launch_init_slots(const Buffers& b, int q, const md_state& st, const KernelShape& k, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_slots, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, st.species,
                       st.rigid, k.n_slots);
}

void launch_load_state(const Buffers& b, int p, int q, const md_state& st, const KernelShape& k,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_load_state, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, st,
                       k.n_slots);
}

void launch_rebuild(const Buffers& b, int p, int q, const KernelShape& k, double half_skin2,
                    int half_list, const int32_t* gate, hipStream_t s)
{
    // p, q: current buffers; the sorted state lands in p^1, q^1.  The cell
    // populations are binned into bin_count, which every build leaves zeroed.
    (void)half_list;
    const int64_t slot_blocks = gate ? std::min<int64_t>(blocks_for(k.n_slots), kGatedBlocks) : blocks_for(k.n_slots);
    hipLaunchKernelGGL(k_bin, dim3(slot_blocks), dim3(kBlock), 0, s, b, p, q, k.n_slots,
                       half_skin2, half_skin2 >= 0.0 ? 1 : 0, gate);
    const int nb = (int)((k.n_cells + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, b, k.n_cells, gate);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, s, b, k.n_cells, gate);
    hipLaunchKernelGGL(k_scatter, dim3(slot_blocks), dim3(kBlock), 0, s, b, k.n_slots, gate);
    hipLaunchKernelGGL(k_sort_cells, dim3(blocks_for(k.n_cells)), dim3(kBlock), 0, s, b, q, k.n_cells, gate);
    hipLaunchKernelGGL(k_gather, dim3(slot_blocks), dim3(kBlock), 0, s, b, p, q, k.n_slots, gate);
}

// Displacement check of the automatic rebuild: the same criterion as the skin
// guard of scheduled builds (no atom may move more than skin/2 between builds
// for a list of r_c + skin to hold every pair closer than r_c), tested at every
// step before the list is used, per replica.  Block 0 also clears the flag set
// of the next check (the rebuild kernels of the previous check, its readers,
// ran before this kernel).
__global__ void k_skin_check(Buffers b, int p, int64_t n_slots, int32_t n_rep, double guard2,
                             int32_t* __restrict__ gate, int32_t* __restrict__ next)
{
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i <= n_rep; i += blockDim.x) next[i] = 0;
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const double3 x = load_xyz(b.pos[p], t);
    const double3 x0 = load_xyz(b.xbuild, t);  // (empty slots: both zero)
    const double dx = x.x - x0.x, dy = x.y - x0.y, dz = x.z - x0.z;
    const bool far = fma(dx, dx, fma(dy, dy, dz * dz)) > guard2;
    if (__ballot(far) != 0 && (threadIdx.x & (kWave - 1)) == 0) {
        atomicOr(&gate[1 + b.rep_of_wave[t / kWave]], 1);
        atomicOr(&gate[0], 1);
    }
}

void launch_skin_check(const Buffers& b, int p, const KernelShape& k, double guard2, int32_t* gate,
                       int32_t* next, hipStream_t s)
{
    hipLaunchKernelGGL(k_skin_check, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, k.n_slots,
                       k.n_replicas, guard2, gate, next);
}

void launch_build_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, double rdl2,
                       int half_list, const int32_t* gate, int copy_back, hipStream_t s)
{
    int64_t blocks = ((int64_t)k.n_cells + kBlock / kWave - 1) / (kBlock / kWave);
    if (gate) blocks = std::min<int64_t>(blocks, kGatedBlocks / 2);
    const bool wide = (uint64_t)k.n_slots * 16 * (uint64_t)((k.cap + 2 * kChunk - 1) / kChunk) >= ((uint64_t)1 << 32);
    const bool split = k.split_list && !half_list && rdl2 < rlist2;
    const int which = (k.tri ? 8 : 0) | (wide ? 4 : 0) | (split ? 2 : 0) | (k.list_types ? 1 : 0);
    using Kern = void (*)(Buffers, int, int, int64_t, int32_t, int32_t, double, double, int, int, const int32_t*, int);
    // [gated][TRI WIDE SPLIT WT]
    static const Kern kerns[2][16] = {
#define MDK_LIST_ROW(G)                                                                                             \
    {k_cell_list<false, false, false, false, G>, k_cell_list<false, false, false, true, G>,                        \
     k_cell_list<false, false, true, false, G>,  k_cell_list<false, false, true, true, G>,                         \
     k_cell_list<false, true, false, false, G>,  k_cell_list<false, true, false, true, G>,                         \
     k_cell_list<false, true, true, false, G>,   k_cell_list<false, true, true, true, G>,                          \
     k_cell_list<true, false, false, false, G>,  k_cell_list<true, false, false, true, G>,                         \
     k_cell_list<true, false, true, false, G>,   k_cell_list<true, false, true, true, G>,                          \
     k_cell_list<true, true, false, false, G>,   k_cell_list<true, true, false, true, G>,                          \
     k_cell_list<true, true, true, false, G>,    k_cell_list<true, true, true, true, G>}
        MDK_LIST_ROW(false), MDK_LIST_ROW(true)};
#undef MDK_LIST_ROW
    hipLaunchKernelGGL(kerns[gate ? 1 : 0][which], dim3(blocks), dim3(kBlock), 0, s, b, p, q, k.n_slots, k.n_cells,
                       k.cap, rlist2, half_list ? rlist2 : rdl2, half_list, k.compact, gate, copy_back);
}

void launch_cell_table(const Buffers& b, const KernelShape& k, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_table, dim3(blocks_for((int64_t)k.n_cells * 27)), dim3(kBlock), 0, s, b, k.n_cells);
}

void launch_compact_records(const Buffers& b, int p, const KernelShape& k, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact_records, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, k.n_slots);
}

template <typename R, bool S, int NP, int ND, int EV, int CMP, bool TL>
static void density_chunked(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                            size_t lds, hipStream_t s)
{
    const int block = TL ? kTableBlock : kBlock;
    const dim3 grid((unsigned)((k.n_slots + block - 1) / block));
    if (k.nchunk == 2)
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, CMP, 2, TL>), grid, dim3(block), lds, s, b, p, q, k.n_slots,
                           P, energy);
    else if (k.nchunk == 8)
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, CMP, 8, TL>), grid, dim3(block), lds, s, b, p, q, k.n_slots,
                           P, energy);
    else
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, CMP, 4, TL>), grid, dim3(block), lds, s, b, p, q, k.n_slots,
                           P, energy);
}

template <typename R, bool S, int NP, int ND, int EV, int CMP>
static void density_tables(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                           hipStream_t s)
{
    // tables in LDS: always for one species, for several when they fit
    const size_t bytes = EV != EV_KNOTS ? (size_t)(S ? 1 : P.ns * P.ns) * P.nbt * value_stride(EV) * sizeof(R) : 0;
    if constexpr (!S && EV != EV_KNOTS) {
        if (bytes <= (size_t)k.lds_limit) {
            density_chunked<R, S, NP, ND, EV, CMP, true>(b, p, q, k, P, energy, bytes, s);
            return;
        }
    }
    density_chunked<R, S, NP, ND, EV, CMP, false>(b, p, q, k, P, energy, S ? bytes : 0, s);
}

template <typename R, bool S, int NP, int ND, int EV>
static void density_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                            hipStream_t s)
{
    if (k.compact == 2) density_tables<R, S, NP, ND, EV, 2>(b, p, q, k, P, energy, s);
    else if (k.compact) density_tables<R, S, NP, ND, EV, 1>(b, p, q, k, P, energy, s);
    else density_tables<R, S, NP, ND, EV, 0>(b, p, q, k, P, energy, s);
}

template <typename R, bool S, int NP, int ND, int EV>
static void density_half_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                                 hipStream_t s)
{
    const size_t lds = (EV != EV_KNOTS && S) ? (size_t)P.nbt * value_stride(EV) * sizeof(R) : 0;
    const dim3 grid(blocks_for(k.n_slots));
    hipLaunchKernelGGL(k_fill_f64, grid, dim3(kBlock), 0, s, b.rhalf, 0.0, k.n_slots);
    hipLaunchKernelGGL((k_density_half<R, S, NP, ND, EV>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P);
    hipLaunchKernelGGL((k_embed_half<S>), grid, dim3(kBlock), 0, s, b, p, q, k.n_slots, P, energy);
}

template <typename R, bool S>
static void density_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int half_list,
                             int energy, hipStream_t s)
{
    // the term-by-term knot sums are FP64 only (the runtime refuses them in mixed precision)
    constexpr bool knots = sizeof(R) == 8;
    if (half_list) {
        if (k.table == 2) density_half_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, energy, s);
        else if (k.table || !knots) density_half_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, energy, s);
        else if constexpr (knots) {
            if (k.ndk == 2) density_half_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, energy, s);  // density knots only
            else density_half_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, energy, s);
        }
        return;
    }
    if (k.table == 2) density_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, energy, s);
    else if (k.table || !knots) density_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, energy, s);
    else if constexpr (knots) {
        if (k.ndk == 2) density_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, energy, s);  // density knots only
        else density_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, energy, s);
    }
}

void launch_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                    int half_list, int energy, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) density_dispatch<float, true>(b, p, q, k, P, half_list, energy, s);
        else density_dispatch<float, false>(b, p, q, k, P, half_list, energy, s);
    } else {
        if (one) density_dispatch<double, true>(b, p, q, k, P, half_list, energy, s);
        else density_dispatch<double, false>(b, p, q, k, P, half_list, energy, s);
    }
}

// The neighbour chunk applies to the velocity-Verlet step kernels (with and
// without energies) and to the plain force pass the autotuner times; the other
// variants run once per call or per barostat step.
template <typename R, bool S, int NP, int ND, int EV, int E, bool C, bool O, bool W, int CMP, bool TL>
static void force_chunked(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                          const md_state& st, size_t lds, hipStream_t s)
{
    const int block = TL ? kTableBlock : kBlock;
    const dim3 grid((unsigned)((k.n_slots + block - 1) / block));
    constexpr bool step = ((E == 0 || E == 1 || E == 4) && C && O && !W) || (E == 0 && !C && !O && !W);
    if constexpr (step) {
        if (k.nchunk == 2) {
            hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, CMP, 2, TL>), grid, dim3(block), lds, s, b, p,
                               q, k.n_slots, P, dt_fs, st);
            return;
        }
        if (k.nchunk == 8) {
            hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, CMP, 8, TL>), grid, dim3(block), lds, s, b, p,
                               q, k.n_slots, P, dt_fs, st);
            return;
        }
    }
    hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, CMP, 4, TL>), grid, dim3(block), lds, s, b, p, q,
                       k.n_slots, P, dt_fs, st);
}

template <typename R, bool S, int NP, int ND, int EV, int E, bool C, bool O, bool W, int CMP>
static void force_tables(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         const md_state& st, hipStream_t s)
{
    // tables in LDS: always for one species, for several when they fit
    const size_t bytes = EV != EV_KNOTS ? (size_t)(S ? 1 : P.ns * P.ns) * P.nbt *
                                              (force_stride(EV) + (E == 1 || E == 4 ? value_stride(EV) : 0)) *
                                              sizeof(R)
                                        : 0;
    if constexpr (!S && EV != EV_KNOTS) {
        if (bytes <= (size_t)k.lds_limit) {
            force_chunked<R, S, NP, ND, EV, E, C, O, W, CMP, true>(b, p, q, k, P, dt_fs, st, bytes, s);
            return;
        }
    }
    force_chunked<R, S, NP, ND, EV, E, C, O, W, CMP, false>(b, p, q, k, P, dt_fs, st, S ? bytes : 0, s);
}

template <typename R, bool S, int NP, int ND, int EV, int E, bool C, bool O, bool W>
static void force_launch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         const md_state& st, hipStream_t s)
{
    if (k.compact == 2) force_tables<R, S, NP, ND, EV, E, C, O, W, 2>(b, p, q, k, P, dt_fs, st, s);
    else if (k.compact) force_tables<R, S, NP, ND, EV, E, C, O, W, 1>(b, p, q, k, P, dt_fs, st, s);
    else force_tables<R, S, NP, ND, EV, E, C, O, W, 0>(b, p, q, k, P, dt_fs, st, s);
}

template <typename R, bool S, int NP, int ND, int EV>
static void force_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, ForceFlags fl,
                          double dt_fs, const md_state& st, hipStream_t s)
{
    if (!fl.close && !fl.open) {
        if (!fl.writeback && fl.energy == 3)  // full-matrix barostat: the whole virial tensor, forces kept
            force_launch<R, S, NP, ND, EV, 3, false, false, false>(b, p, q, k, P, dt_fs, st, s);
        else if (!fl.writeback && fl.energy)  // barostat: the stress of the starting state, forces kept
            force_launch<R, S, NP, ND, EV, 2, false, false, false>(b, p, q, k, P, dt_fs, st, s);
        else if (!fl.writeback) force_launch<R, S, NP, ND, EV, false, false, false, false>(b, p, q, k, P, dt_fs, st, s);
        else if (fl.energy == 4) force_launch<R, S, NP, ND, EV, 4, false, false, true>(b, p, q, k, P, dt_fs, st, s);
        else if (fl.energy) force_launch<R, S, NP, ND, EV, true, false, false, true>(b, p, q, k, P, dt_fs, st, s);
        else force_launch<R, S, NP, ND, EV, false, false, false, true>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.close && fl.open) {
        force_launch<R, S, NP, ND, EV, false, false, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (fl.close && fl.open) {
        if (fl.energy == 4)  // per-step energies, summed per wavefront
            force_launch<R, S, NP, ND, EV, 4, true, true, false>(b, p, q, k, P, dt_fs, st, s);
        else if (fl.energy)  // per-step energies
            force_launch<R, S, NP, ND, EV, true, true, true, false>(b, p, q, k, P, dt_fs, st, s);
        else force_launch<R, S, NP, ND, EV, false, true, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.writeback && fl.energy == 3) {  // full-matrix barostat: closing kick, virial tensor
        force_launch<R, S, NP, ND, EV, 3, true, false, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.writeback && fl.energy) {  // barostat: closing kick with the stress, forces kept
        force_launch<R, S, NP, ND, EV, 2, true, false, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.writeback) {
        force_launch<R, S, NP, ND, EV, false, true, false, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (fl.energy == 4) {  // the last step of a velocity-Verlet call
        force_launch<R, S, NP, ND, EV, 4, true, false, true>(b, p, q, k, P, dt_fs, st, s);
    } else {
        force_launch<R, S, NP, ND, EV, true, true, false, true>(b, p, q, k, P, dt_fs, st, s);
    }
}

template <bool S, bool E, bool C, bool O, bool W>
static void integrate_half(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                           const md_state& st, hipStream_t s)
{
    hipLaunchKernelGGL((k_integrate_half<S, E, C, O, W>), dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q,
                       k.n_slots, P, dt_fs, st);
}

template <typename R, bool S, int NP, int ND, int EV>
static void force_half_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, ForceFlags fl,
                               double dt_fs, const md_state& st, hipStream_t s)
{
    const dim3 grid(blocks_for(k.n_slots));
    for (int a = 0; a < 3; ++a) hipLaunchKernelGGL(k_fill_f64, grid, dim3(kBlock), 0, s, b.fhalf[a], 0.0, k.n_slots);
    if (fl.energy) hipLaunchKernelGGL(k_fill_f64, grid, dim3(kBlock), 0, s, b.ehalf, 0.0, k.n_slots);
    const size_t lds =
        (EV != EV_KNOTS && S) ? (size_t)P.nbt * (force_stride(EV) + (fl.energy ? value_stride(EV) : 0)) * sizeof(R) : 0;
    if (fl.energy)
        hipLaunchKernelGGL((k_force_half<R, S, NP, ND, EV, true>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P);
    else
        hipLaunchKernelGGL((k_force_half<R, S, NP, ND, EV, false>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P);
    if (!fl.close && !fl.open) {
        if (!fl.writeback) integrate_half<S, false, false, false, false>(b, p, q, k, P, dt_fs, st, s);
        else if (fl.energy) integrate_half<S, true, false, false, true>(b, p, q, k, P, dt_fs, st, s);
        else integrate_half<S, false, false, false, true>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.close && fl.open) {
        integrate_half<S, false, false, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (fl.close && fl.open) {
        if (fl.energy) integrate_half<S, true, true, true, false>(b, p, q, k, P, dt_fs, st, s);
        else integrate_half<S, false, true, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.writeback) {
        integrate_half<S, false, true, false, false>(b, p, q, k, P, dt_fs, st, s);
    } else {
        integrate_half<S, true, true, false, true>(b, p, q, k, P, dt_fs, st, s);
    }
}

template <typename R, bool S>
static void force_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int half_list,
                           ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    constexpr bool knots = sizeof(R) == 8;  // knot sums: FP64 only
    if (half_list) {
        if (k.table == 2) force_half_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, fl, dt_fs, st, s);
        else if (k.table || !knots) force_half_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, fl, dt_fs, st, s);
        else if constexpr (knots) {
            if (k.npk == 6 && k.ndk == 2) force_half_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
            else if (k.npk <= 8 && k.ndk <= 8) force_half_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
            else if constexpr (S) force_half_variant<R, S, 16, 4, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
        }
        return;
    }
    if (k.table == 2) force_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, fl, dt_fs, st, s);
    else if (k.table || !knots) force_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, fl, dt_fs, st, s);
    else if constexpr (knots) {
        if (k.npk == 6 && k.ndk == 2) force_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
        else if (k.npk <= 8 && k.ndk <= 8) force_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
        else if constexpr (S) force_variant<R, S, 16, 4, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
    }
}

void launch_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                  int half_list, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) force_dispatch<float, true>(b, p, q, k, P, half_list, fl, dt_fs, st, s);
        else force_dispatch<float, false>(b, p, q, k, P, half_list, fl, dt_fs, st, s);
    } else {
        if (one) force_dispatch<double, true>(b, p, q, k, P, half_list, fl, dt_fs, st, s);
        else force_dispatch<double, false>(b, p, q, k, P, half_list, fl, dt_fs, st, s);
    }
}

void launch_nh_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int halves, double dt_fs,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_nh_ke_waves, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P);
    if (k.chunked && k.n_chunks > 0)
        hipLaunchKernelGGL(k_chunk_sums<1>, dim3(k.n_chunks), dim3(kWave), 0, s, b, b.nh_partial);
    if (k.n_replicas > 0)
        hipLaunchKernelGGL(k_nh_update, dim3(k.n_replicas), dim3(kBlock), 0, s, b, halves, dt_fs, k.chunked);
}

void launch_nh_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                    int scaled, hipStream_t s)
{
    hipLaunchKernelGGL(k_nh_open, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots, P, dt_fs,
                       k.compact, scaled);
}

void launch_pr_chunk_sums(const Buffers& b, const KernelShape& k, int n_terms, hipStream_t s)
{
    if (!k.chunked || k.n_chunks == 0) return;
    if (n_terms == 12) hipLaunchKernelGGL(k_chunk_sums<12>, dim3(k.n_chunks), dim3(kWave), 0, s, b, b.pr_partial);
    else hipLaunchKernelGGL(k_chunk_sums<6>, dim3(k.n_chunks), dim3(kWave), 0, s, b, b.pr_partial);
}

void launch_pr_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int close, int open,
                      double dt_fs, double rlist, double strain_tol, int nvt, hipStream_t s)
{
    hipLaunchKernelGGL(k_pr_tensor_waves, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P);
    launch_pr_chunk_sums(b, k, 6, s);
    if (k.n_replicas > 0)
        hipLaunchKernelGGL(k_pr_update, dim3(k.n_replicas), dim3(kBlock), 0, s, b, close, open, dt_fs, rlist,
                           strain_tol, nvt, k.chunked);
}

void launch_pr_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_pr_open, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots, P, dt_fs,
                       k.compact);
}

void launch_pr_close_scale(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, const md_state& st,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_pr_close_scale, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P, st);
}

void launch_pr_mark_build(const Buffers& b, const KernelShape& k, hipStream_t s)
{
    if (k.n_replicas > 0)
        hipLaunchKernelGGL(k_pr_mark_build, dim3((k.n_replicas + kBlock - 1) / kBlock), dim3(kBlock), 0, s, b,
                           k.n_replicas);
}

void launch_gear_start(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_gear_start, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P);
}

void launch_gear_predict(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_gear_predict, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots, P,
                       dt_fs, k.compact);
}

void launch_gear_correct(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         const md_state& st, int last, hipStream_t s)
{
    hipLaunchKernelGGL(k_gear_correct, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots, P,
                       dt_fs, st, last, k.compact);
}

void launch_nh_scale(const Buffers& b, int q, const KernelShape& k, const md_state& st, int energy, hipStream_t s)
{
    hipLaunchKernelGGL(k_nh_scale, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, st, energy);
}


void launch_reduce_energies(const Buffers& b, const KernelShape& k, double virial_scale, int64_t ring_len,
                            hipStream_t s)
{
    if (k.n_chunks > 0) hipLaunchKernelGGL(k_reduce_chunks, dim3(k.n_chunks), dim3(kBlock), 0, s, b, k.n_slots);
    hipLaunchKernelGGL(k_reduce_replicas, dim3(k.n_replicas), dim3(kBlock), 0, s, b, virial_scale, ring_len);
}

void launch_reduce_waves(const Buffers& b, const KernelShape& k, double virial_scale, int64_t ring_len,
                         hipStream_t s)
{
    if (k.n_chunks > 0) hipLaunchKernelGGL(k_reduce_wave_chunks, dim3(k.n_chunks), dim3(kWave), 0, s, b);
    hipLaunchKernelGGL(k_reduce_replicas, dim3(k.n_replicas), dim3(kBlock), 0, s, b, virial_scale, ring_len);
}

}  // namespace mdk
