// gfx950 kernels of the list build (paper, "The Neighbourlist calculation"):
// binning of the atoms into link cells, the scan of the cell populations, the
// counting sort into cell order (atoms within a cell ordered by caller index),
// the gather of the atom state into the new slot order, the cell adjacency
// table and the Verlet list itself; and the automatic rebuild's displacement
// check with the gating every build kernel takes.
#include "md_device.h"

namespace mdk {
namespace {
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
// (and so every later floating-point sum) independent of atomics' timing.  Every
// member counts the members of its cell with a smaller caller index (indices are
// distinct): that count is its place in the cell, and its old slot goes there in
// perm_sorted.
__global__ void k_sort_cells(Buffers b, int q, int64_t n_slots, const int32_t* __restrict__ gate)
{
    if (gate && gate[0] == 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t* __restrict__ id = b.id[q];
    for (int64_t u = global_thread(); u < n_slots; u += stride) {
        const int rep = uniform(b.rep_of_wave[u / kWave]);
        if (gate && gate[1 + rep] == 0) continue;
        const DevReplica& R = b.reps[rep];
        if (u - R.slot_off >= R.n_atoms) continue;  // slots past the replica's atoms
        const int32_t t = b.perm[u];
        const int c = b.cell_of[t];
        const int beg = b.cell_start[c], cnt = b.cell_count[c];
        const int32_t key = id[t];
        int place = 0;
        for (int j = 0; j < cnt; ++j) place += id[b.perm[beg + j]] < key ? 1 : 0;
        b.perm_sorted[beg + place] = t;
    }
}

// Rebuild stage 5: gather the whole atom state into the new slot order.
__device__ __forceinline__ void gather_slot(const Buffers& b, int p, int q, int64_t u)
{
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[u / kWave])];
    const int pn = p ^ 1, qn = q ^ 1;
    if (u - R.slot_off < R.n_atoms) {
        const int32_t t = b.perm_sorted[u];
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

}  // namespace

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
    hipLaunchKernelGGL(k_sort_cells, dim3(slot_blocks), dim3(kBlock), 0, s, b, q, k.n_slots, gate);
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

}  // namespace mdk
