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
// position is kept as x - n L along periodic axes, with the integer image
// count n of the slot fixed at the last list build, so that list entries can
// carry their periodic shift and the force loop needs no minimum image.
__global__ void k_load_state(Buffers b, int p, int q, md_state st, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const int32_t a = b.id[q][t];
    if (a >= 0) {
        b.pos[p][t] = make_double4(st.x[a] - b.img[q][0][t] * R.box[0], st.y[a] - b.img[q][1][t] * R.box[1],
                                   st.z[a] - b.img[q][2][t] * R.box[2], 0.0);
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

// ---------------------------------------------------------------------------
// List build, step 1: link cell of every atom, cell populations, and the skin
// guard (net displacement since the previous build must stay below skin/2).
__global__ void k_bin(Buffers b, int p, int q, int64_t n_slots, double half_skin2, int check_skin)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    if (b.id[q][t] < 0) {
        b.cell_of[t] = -1;
        return;
    }
    const Box bx = load_box(R);
    const double3 x = load_xyz(b.pos[p], t);
    int c[3];
    cell_coords(bx, x.x, x.y, x.z, c);
    const int cell = cell_index(R, c[0], c[1], c[2]);
    b.cell_of[t] = cell;
    atomicAdd(&b.cell_count[cell], 1);
    if (check_skin) {
        const double3 x0 = load_xyz(b.xbuild, t);
        const double dx = x.x - x0.x, dy = x.y - x0.y, dz = x.z - x0.z;
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

// Exclusive scan of cell populations, three phases (block scan, scan of block
// sums, add), then shifted into slot numbering with the per-cell replica shift.
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

__global__ __launch_bounds__(kScanBlock) void k_scan_local(Buffers b, int32_t n)
{
    __shared__ int32_t sh[kScanBlock];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int32_t v = i < n ? b.cell_count[i] : 0;
    int32_t total;
    const int32_t ex = block_exclusive_scan(v, sh, total);
    if (i < n) b.cell_start[i] = ex;
    if (threadIdx.x == 0) b.scan_blocks[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(Buffers b, int32_t nblocks)
{
    // one workgroup; each thread owns a contiguous run of block sums
    __shared__ int32_t sh[kScanBlock];
    const int per = (nblocks + kScanBlock - 1) / kScanBlock;
    const int beg = threadIdx.x * per;
    int32_t run = 0;
    for (int k = 0; k < per; ++k)
        if (beg + k < nblocks) run += b.scan_blocks[beg + k];
    int32_t total;
    int32_t ex = block_exclusive_scan(run, sh, total);
    for (int k = 0; k < per; ++k)
        if (beg + k < nblocks) {
            const int32_t v = b.scan_blocks[beg + k];
            b.scan_blocks[beg + k] = ex;
            ex += v;
        }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(Buffers b, int32_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) b.cell_start[i] += b.scan_blocks[blockIdx.x] + b.cell_shift[i];
}

// Step 3: place every atom in its cell's slot range (arbitrary order within
// the cell, fixed by the next kernel).
__global__ void k_scatter(Buffers b, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int c = b.cell_of[t];
    if (c < 0) return;
    const int k = atomicAdd(&b.cell_cursor[c], 1);
    b.perm[b.cell_start[c] + k] = (int32_t)t;
}

// Step 4: order each cell's members by caller index, making the slot order
// (and so every later floating-point sum) independent of atomics' timing.
__global__ void k_sort_cells(Buffers b, int q, int32_t n_cells)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
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

// Step 5: gather the whole atom state into the new slot order.
__global__ void k_gather(Buffers b, int p, int q, int64_t n_slots)
{
    const int64_t u = global_thread();
    if (u >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[u / kWave])];
    const int pn = p ^ 1, qn = q ^ 1;
    if (u - R.slot_off < R.n_atoms) {
        const int32_t t = b.perm[u];
        const double3 x = load_xyz(b.pos[p], t);
        double xw[3] = {x.x, x.y, x.z};
        // re-wrap atoms that left the primary box on a periodic axis
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
        const double4 x4 = make_double4(xw[0], xw[1], xw[2], 0.0);
        b.pos[pn][u] = x4;
        b.xbuild[u] = x4;
#pragma unroll
        for (int a = 0; a < 3; ++a) b.vel[qn][a][u] = b.vel[q][a][t];
        b.id[qn][u] = b.id[q][t];
        b.type[qn][u] = b.type[q][t];
        b.cell_sorted[u] = b.cell_of[t];
        b.pwork[qn][u] = b.pwork[q][t];
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
    }
}

// Step 6: the Verlet list from the 27 (or fewer, on boxes under three cells
// per axis) adjacent link cells ("a nested loop over link-cells and their
// adjacent cells").  Full list: every j != i with r < r_c + skin.  Half list:
// only j with a larger slot index.  Overflow keeps counting, so the required
// capacity can be reported.
__global__ void k_build_list(Buffers b, int p, int q, int64_t n_slots, int32_t cap, double rlist2,
                             int half_list, int rowlen)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const bool valid = t - R.slot_off < R.n_atoms;
    const Box bx = load_box(R);
    const double3 xi = load_xyz(b.pos[p], t);
    int c[3];
    cell_coords(bx, xi.x, xi.y, xi.z, c);
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (bx.pmask & (1 << a)) {
            // distinct neighbours only: {-1,0,1}, {0,1} or {0} cells
            lo[a] = bx.nc[a] >= 3 ? -1 : 0;
            hi[a] = bx.nc[a] >= 2 ? 1 : 0;
        } else {
            lo[a] = c[a] > 0 ? -1 : 0;
            hi[a] = c[a] < bx.nc[a] - 1 ? 1 : 0;
        }
    }
    int count = 0;
    int4* row = reinterpret_cast<int4*>(b.nbr + t * (int64_t)rowlen);
    int pk[4] = {0, 0, 0, 0};  // entries buffered until a 16-byte store
    if (!valid) lo[2] = 1, hi[2] = 0;  // empty slot: no cells, count stays 0
    for (int dz = lo[2]; dz <= hi[2]; ++dz) {
        int cz = c[2] + dz;
        if (cz < 0) cz += bx.nc[2];
        if (cz >= bx.nc[2]) cz -= bx.nc[2];
        for (int dy = lo[1]; dy <= hi[1]; ++dy) {
            int cy = c[1] + dy;
            if (cy < 0) cy += bx.nc[1];
            if (cy >= bx.nc[1]) cy -= bx.nc[1];
            for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                int cx = c[0] + dx;
                if (cx < 0) cx += bx.nc[0];
                if (cx >= bx.nc[0]) cx -= bx.nc[0];
                const int cell = cell_index(R, cx, cy, cz);
                const int beg = b.cell_start[cell], end = beg + b.cell_count[cell];
#pragma unroll 4
                for (int j = beg; j < end; ++j) {
                    if (j == t || (half_list && j < t)) continue;
                    const double3 xj = load_xyz(b.pos[p], j);
                    double ddx = xj.x - xi.x, ddy = xj.y - xi.y, ddz = xj.z - xi.z;
                    const int code = image_code(bx, ddx, ddy, ddz);
                    if (ddx * ddx + ddy * ddy + ddz * ddz < rlist2) {
                        if (count < cap) {
                            pk[count & 3] = j | (code << kIndexBits);
                            if ((count & 3) == 3) row[count >> 2] = make_int4(pk[0], pk[1], pk[2], pk[3]);
                        }
                        ++count;
                    }
                }
            }
        }
    }
    const int stored = count < cap ? count : cap;
    if (stored & 3) row[stored >> 2] = make_int4(pk[0], pk[1], pk[2], pk[3]);
    b.ncount[t] = stored;
    wave_max_flag(count, &b.flags[F_MAX_COUNT]);
}

// ---------------------------------------------------------------------------
// Global-gather kernels: one thread per atom reads its neighbours straight
// from HBM/L2 through the int32 list (slot index + periodic shift code).  They
// serve the half-list variant and systems whose brick halo would not fit LDS.
//
// Density pass (Eq. Ucoh, the argument of F): rho_i = sum_j rho_{s_i s_j}(r_ij),
// then F_i and F'_i.  The sum is accumulated in FP64 in both precision modes.
// L lanes share an atom: lane l takes the 8-entry blocks l, l + L, ... of the
// atom's list row, loads the 8 indices with two 16-byte loads and then issues
// all 8 position gathers before using any of them, so one wavefront keeps 8
// gathers per lane in flight (memory-level parallelism is what bounds this
// loop: the arithmetic is a small fraction of the wait).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, int L>
__global__ __launch_bounds__(kBlock) void k_density(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                     int energy, int rowlen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const R* tab = tables<R>(b).dens;
    if (EV == EV_TABLE && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tab, P.nbt * 4);
        __syncthreads();
        tab = s;
    }
    const int64_t gid = global_thread();
    const int64_t t = gid / L;
    const int lane = (int)(gid % L);
    if (t >= n_slots) return;  // whole wavefronts
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const bool valid = t - Rp.slot_off < Rp.n_atoms;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const double3 xi = load_xyz(pos, t);
    const int si = b.type[q][t] & 0x3F;
    const int n = valid ? b.ncount[t] : 0;
    const int4* row = reinterpret_cast<const int4*>(b.nbr + t * (int64_t)rowlen);
    double rho = 0.0;
    for (int blk = lane; blk * 8 < n; blk += L) {
        const int4 v0 = row[2 * blk], v1 = row[2 * blk + 1];
        const int e[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        double3 xs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[u] = load_xyz(pos, blk * 8 + u < n ? (e[u] & kIndexMask) : t);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (blk * 8 + u >= n) break;
            double dx = xs[u].x - xi.x, dy = xs[u].y - xi.y, dz = xs[u].z - xi.z;
            const int code = (unsigned)e[u] >> kIndexBits;
            if (code) apply_shift(bx, code, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < P.rc2)) continue;
            const double r = r2 * inv_dist<R>(r2);
            const int sj = SINGLE ? 0 : (b.type[q][e[u] & kIndexMask] & 0x3F);
            rho += (double)density_term<R, SINGLE, NDK, EV>(P, G, tab, si, sj, r);
        }
    }
    rho = lane_sum<L>(rho);
    if (valid && lane == 0) {
        double F, dF;
        embed(SINGLE ? P.emb_c : G.emb_c[si], rho, F, dF);
        reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
        if (energy) b.femb[t] = F;
    }
}

// Force pass + velocity Verlet (global gathers, lanes as in k_density).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, bool ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK, int L>
__global__ __launch_bounds__(kBlock) void k_force(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                   double dt, md_state st, int rowlen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tabs<R> T = tables<R>(b);
    const R* tf = T.force;
    const R* te = T.energy;
    if (EV == EV_TABLE && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tf, P.nbt * kForceStride);
        if (ENERGY) lds_fill(s + P.nbt * kForceStride, te, P.nbt * 4);
        __syncthreads();
        tf = s;
        te = s + P.nbt * kForceStride;
    }
    const int64_t gid = global_thread();
    const int64_t t = gid / L;
    const int lane = (int)(gid % L);
    if (t >= n_slots) return;  // whole wavefronts
    const DevReplica& Rp = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const bool valid = t - Rp.slot_off < Rp.n_atoms;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const double4 pi = pos[t];
    const uint8_t ti = b.type[q][t];
    const int si = ti & 0x3F;
    const bool rigid_i = ti & kRigidBit;
    const int n = valid ? b.ncount[t] : 0;
    const R fpi = (R)pi.w;
    const int4* row = reinterpret_cast<const int4*>(b.nbr + t * (int64_t)rowlen);
    PairAcc A;
    for (int blk = lane; blk * 8 < n; blk += L) {
        const int4 v0 = row[2 * blk], v1 = row[2 * blk + 1];
        const int e[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        double4 ps[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ps[u] = pos[blk * 8 + u < n ? (e[u] & kIndexMask) : t];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (blk * 8 + u >= n) break;
            const double4 pj = ps[u];
            double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            const int code = (unsigned)e[u] >> kIndexBits;
            if (code) apply_shift(bx, code, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < P.rc2)) continue;
            const double ri = inv_dist<R>(r2);
            const double r = r2 * ri;
            const uint8_t tj = (!SINGLE || ENERGY) ? b.type[q][e[u] & kIndexMask] : 0;
            R g, phi;
            pair_terms<R, SINGLE, NPK, NDK, EV, ENERGY>(P, G, tf, te, si, tj & 0x3F, r, fpi, (R)pj.w, g, phi);
            accumulate<ENERGY>(A, (double)g * ri, dx, dy, dz, (double)phi, rigid_i && (tj & kRigidBit));
        }
    }
    if (L > 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) A.f[c] = lane_sum<L>(A.f[c]);
        if (ENERGY) {
            A.epair = lane_sum<L>(A.epair);
#pragma unroll
            for (int c = 0; c < 6; ++c) A.w[c] = lane_sum<L>(A.w[c]);
        }
    }
    if (valid && lane == 0)
        atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK>(b, p, q, t, n_slots, Rp, P, G, dt, st, pi, ti, A);
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

__global__ __launch_bounds__(kBlock) void k_reduce_replicas(Buffers b, double virial_scale)
{
    __shared__ double sh[kEnergyTerms][kBlock];
    const int r = blockIdx.x;
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
    }
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
                    int half_list, hipStream_t s)
{
    // p, q: current buffers; the sorted state lands in p^1, q^1.
    (void)half_list;
    launch_fill_i32(b.cell_count, 0, k.n_cells, s);
    launch_fill_i32(b.cell_cursor, 0, k.n_cells, s);
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots,
                       half_skin2, half_skin2 >= 0.0 ? 1 : 0);
    const int nb = (int)((k.n_cells + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, b, k.n_cells);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, b, nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, s, b, k.n_cells);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, k.n_slots);
    hipLaunchKernelGGL(k_sort_cells, dim3(blocks_for(k.n_cells)), dim3(kBlock), 0, s, b, q, k.n_cells);
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots);
}

void launch_build_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, int half_list,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_build_list, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots,
                       k.cap, rlist2, half_list, k.rowlen);
}

template <typename R, bool S, int NP, int ND, int EV>
static void density_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                            hipStream_t s)
{
    const size_t lds = (EV == EV_TABLE && S) ? (size_t)P.nbt * 4 * sizeof(R) : 0;
    const dim3 grid(blocks_for(k.n_slots * k.lanes));
    if (k.lanes == 4)
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, 4>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P, energy,
                           k.rowlen);
    else if (k.lanes == 2)
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, 2>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P, energy,
                           k.rowlen);
    else
        hipLaunchKernelGGL((k_density<R, S, NP, ND, EV, 1>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P, energy,
                           k.rowlen);
}

// Knot counts are compile-time so the explicit sums unroll: the 6-pair /
// 2-density shape of every table used here, and a padded 8 / 8 fallback (zero
// amplitudes contribute nothing).  The table evaluator does not depend on them.
template <typename R, bool S>
static void density_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                             hipStream_t s)
{
    if (k.table) density_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, energy, s);
    else if (k.npk == 6 && k.ndk == 2) density_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, energy, s);
    else density_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, energy, s);
}

void launch_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                    int half_list, int energy, hipStream_t s)
{
    (void)half_list;
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) density_dispatch<float, true>(b, p, q, k, P, energy, s);
        else density_dispatch<float, false>(b, p, q, k, P, energy, s);
    } else {
        if (one) density_dispatch<double, true>(b, p, q, k, P, energy, s);
        else density_dispatch<double, false>(b, p, q, k, P, energy, s);
    }
}

template <typename R, bool S, int NP, int ND, int EV, bool E, bool C, bool O, bool W>
static void force_launch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         const md_state& st, hipStream_t s)
{
    const size_t lds = (EV == EV_TABLE && S) ? (size_t)P.nbt * (kForceStride + (E ? 4 : 0)) * sizeof(R) : 0;
    const dim3 grid(blocks_for(k.n_slots * k.lanes));
    if (k.lanes == 4)
        hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, 4>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P,
                           dt_fs, st, k.rowlen);
    else if (k.lanes == 2)
        hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, 2>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P,
                           dt_fs, st, k.rowlen);
    else
        hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W, 1>), grid, dim3(kBlock), lds, s, b, p, q, k.n_slots, P,
                           dt_fs, st, k.rowlen);
}

template <typename R, bool S, int NP, int ND, int EV>
static void force_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, ForceFlags fl,
                          double dt_fs, const md_state& st, hipStream_t s)
{
    if (!fl.close && !fl.open) {
        if (fl.energy) force_launch<R, S, NP, ND, EV, true, false, false, true>(b, p, q, k, P, dt_fs, st, s);
        else force_launch<R, S, NP, ND, EV, false, false, false, true>(b, p, q, k, P, dt_fs, st, s);
    } else if (!fl.close && fl.open) {
        force_launch<R, S, NP, ND, EV, false, false, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else if (fl.close && fl.open) {
        force_launch<R, S, NP, ND, EV, false, true, true, false>(b, p, q, k, P, dt_fs, st, s);
    } else {
        force_launch<R, S, NP, ND, EV, true, true, false, true>(b, p, q, k, P, dt_fs, st, s);
    }
}

template <typename R, bool S>
static void force_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, ForceFlags fl,
                           double dt_fs, const md_state& st, hipStream_t s)
{
    if (k.table) force_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, fl, dt_fs, st, s);
    else if (k.npk == 6 && k.ndk == 2) force_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
    else force_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, fl, dt_fs, st, s);
}

void launch_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                  int half_list, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    (void)half_list;
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) force_dispatch<float, true>(b, p, q, k, P, fl, dt_fs, st, s);
        else force_dispatch<float, false>(b, p, q, k, P, fl, dt_fs, st, s);
    } else {
        if (one) force_dispatch<double, true>(b, p, q, k, P, fl, dt_fs, st, s);
        else force_dispatch<double, false>(b, p, q, k, P, fl, dt_fs, st, s);
    }
}

void launch_reduce_energies(const Buffers& b, const KernelShape& k, double virial_scale, hipStream_t s)
{
    if (k.n_chunks > 0) hipLaunchKernelGGL(k_reduce_chunks, dim3(k.n_chunks), dim3(kBlock), 0, s, b, k.n_slots);
    hipLaunchKernelGGL(k_reduce_replicas, dim3(k.n_replicas), dim3(kBlock), 0, s, b, virial_scale);
}

}  // namespace mdk
