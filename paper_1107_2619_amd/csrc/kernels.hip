// gfx950 kernels of the embedded-atom force loop.
//
// Data layout (all in the caller-provided workspace, see md_runtime.hip):
//   - atoms live in "slots" sorted by link cell (paper, "OpenMP
//     Parallelisation": particles ordered by link-cell index so cell members
//     are contiguous); replica r owns a wavefront-aligned slot range;
//   - positions as double4 {x, y, z, F'}: one 32-byte gather per neighbour
//     brings the position and the embedding derivative the force pass needs;
//   - the Verlet list is transposed ELL, nbr[k * Np + slot], so the k-th
//     entries of consecutive atoms are contiguous (coalesced index loads);
//   - the full (symmetric) list lets each atom gather its own density and
//     force with no atomics; the half list with FP64 atomics is kept as the
//     comparison variant (paper, "OpenMP Parallelisation", on the trade
//     between a symmetric list and synchronised updates).
#include "md_internal.h"

namespace mdk {
namespace {

// ---------------------------------------------------------------------------
// Launch geometry.  The hardware hands workgroup b to accelerator die b % 8;
// remap so each die receives one contiguous range of slots: cell-sorted
// neighbours then share that die's L2 instead of being fetched by all eight.
__device__ __forceinline__ int64_t logical_block()
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t full = (nb / kNumXcd) * kNumXcd;
    if (b >= full) return b;
    const int64_t per = nb / kNumXcd;
    return (b % kNumXcd) * per + (b / kNumXcd);
}

__device__ __forceinline__ int64_t global_thread() { return logical_block() * blockDim.x + threadIdx.x; }

inline int64_t blocks_for(int64_t n) { return (n + kBlock - 1) / kBlock; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Geometry helpers (paper, "Boundary conditions": minimum image along periodic
// axes, plain differences along free ones; positions unwrapped).
struct Box {
    double L[3], iL[3], o[3];
    int pmask;
    int nc[3];
    int cell_off;
};

__device__ __forceinline__ Box load_box(const DevReplica& R)
{
    Box b;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        b.L[a] = R.box[a];
        b.iL[a] = R.inv_box[a];
        b.o[a] = R.origin[a];
        b.nc[a] = R.nc[a];
    }
    b.pmask = R.periodic_mask;
    b.cell_off = R.cell_off;
    return b;
}

__device__ __forceinline__ void min_image(const Box& b, double& dx, double& dy, double& dz)
{
    if (b.pmask & 1) dx -= b.L[0] * rint(dx * b.iL[0]);
    if (b.pmask & 2) dy -= b.L[1] * rint(dy * b.iL[1]);
    if (b.pmask & 4) dz -= b.L[2] * rint(dz * b.iL[2]);
}

// Link cell along one axis: periodic axes wrap the fractional coordinate into
// [0, 1); free axes clamp (monotone, so atoms closer than one cell edge still
// land in the same or adjacent cells).
__device__ __forceinline__ int cell_axis(double x, double o, double iL, int nc, bool periodic)
{
    double f = (x - o) * iL;
    if (periodic) f -= floor(f);
    int c = (int)floor(f * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ void cell_coords(const Box& b, double x, double y, double z, int c[3])
{
    c[0] = cell_axis(x, b.o[0], b.iL[0], b.nc[0], b.pmask & 1);
    c[1] = cell_axis(y, b.o[1], b.iL[1], b.nc[1], b.pmask & 2);
    c[2] = cell_axis(z, b.o[2], b.iL[2], b.nc[2], b.pmask & 4);
}

__device__ __forceinline__ double3 load_xyz(const double4* p, int64_t i)
{
    // 16 + 8 byte loads: never touches .w, which the density pass writes.
    const double2 xy = *reinterpret_cast<const double2*>(p + i);
    const double z = reinterpret_cast<const double*>(p + i)[2];
    return make_double3(xy.x, xy.y, z);
}

// ---------------------------------------------------------------------------
// Cubic-knot sums (paper, "Available potentials"): f(r) = sum_k a_k (r_k - r)^3
// H(r_k - r).  `amp_d` holds -3 a_k so the derivative is sum amp_d t^2.
// The distance r and the knot positions are FP64 in both precision modes; the
// offset t = r_k - r is formed in FP64 (no cancellation error) and the cubic
// is evaluated in the working precision R.
template <typename R, int NK>
__device__ __forceinline__ R knot_deriv(const R* amp_d, const double* rk, double r)
{
    R d = R(0);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        R t = (R)(rk[k] - r);
        t = t > R(0) ? t : R(0);
        d = fma(amp_d[k], t * t, d);
    }
    return d;
}

template <typename R, int NK>
__device__ __forceinline__ R knot_value(const R* amp, const double* rk, double r)
{
    R v = R(0);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        R t = (R)(rk[k] - r);
        t = t > R(0) ? t : R(0);
        v = fma(amp[k] * t, t * t, v);
    }
    return v;
}

template <typename R, int NK>
__device__ __forceinline__ void knot_both(const R* amp, const R* amp_d, const double* rk, double r, R& v, R& d)
{
    v = R(0);
    d = R(0);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        R t = (R)(rk[k] - r);
        t = t > R(0) ? t : R(0);
        const R t2 = t * t;
        d = fma(amp_d[k], t2, d);
        v = fma(amp[k] * t, t2, v);
    }
}

// Coefficient views for one species pair: amplitudes in the working
// precision, knot positions in FP64.
template <typename R>
struct Coef {
    const R *pa, *pd;
    const double* pr;
    const R *da, *dd;
    const double* dr;
};

template <typename R>
__device__ __forceinline__ Coef<R> single_coef(const PotArgs& P);

template <>
__device__ __forceinline__ Coef<double> single_coef<double>(const PotArgs& P)
{
    return {P.pair_a, P.pair_d, P.pair_r, P.dens_a, P.dens_d, P.dens_r};
}

template <>
__device__ __forceinline__ Coef<float> single_coef<float>(const PotArgs& P)
{
    return {P.pair_af, P.pair_df, P.pair_r, P.dens_af, P.dens_df, P.dens_r};
}

// Multi-species tables are FP64 in global memory; the mixed path converts the
// amplitudes it needs per pair.
template <typename R, int NK>
struct KnotSet {
    R a[NK], d[NK];
    double r[NK];
};

template <typename R, int NK>
__device__ __forceinline__ void load_knots(const double* a, const double* d, const double* r, KnotSet<R, NK>& s)
{
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        s.a[k] = (R)a[k];
        s.d[k] = (R)d[k];
        s.r[k] = r[k];
    }
}

// 1/r from r^2 (FP64): the hardware FP32 reciprocal square root as a seed,
// then Newton steps y <- y (3 - r^2 y^2) / 2, each squaring the relative
// error (~1e-7 -> ~2e-14 -> rounding level).  FP64 mode takes two steps, the
// mixed mode one (its pair terms are FP32 anyway).
template <typename R>
__device__ __forceinline__ double inv_dist(double r2)
{
    double y = (double)__builtin_amdgcn_rsqf((float)r2);
    const double h = 0.5 * r2;
    y = y * fma(-h * y, y, 1.5);
    if (sizeof(R) == 8) y = y * fma(-h * y, y, 1.5);
    return y;
}

// Embedding F(rho) = -c sqrt(rho), F'(rho) = -c / (2 sqrt(rho)); zero for an
// atom with no density (the limit of the energy; the derivative is singular).
__device__ __forceinline__ void embed(double c, double rho, double& F, double& dF)
{
    if (rho > 0.0) {
        const double s = sqrt(rho);
        F = -c * s;
        dF = -0.5 * c / s;
    } else {
        F = 0.0;
        dF = 0.0;
    }
}

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
}

// Caller state (caller order) -> slots.
__global__ void k_load_state(Buffers b, int p, int q, md_state st, int64_t n_slots)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int32_t a = b.id[q][t];
    if (a >= 0) {
        b.pos[p][t] = make_double4(st.x[a], st.y[a], st.z[a], 0.0);
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
    const int cell = bx.cell_off + (c[2] * bx.nc[1] + c[1]) * bx.nc[0] + c[0];
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
        const double4 x4 = make_double4(x.x, x.y, x.z, 0.0);
        b.pos[pn][u] = x4;
        b.xbuild[u] = x4;
#pragma unroll
        for (int a = 0; a < 3; ++a) b.vel[qn][a][u] = b.vel[q][a][t];
        b.id[qn][u] = b.id[q][t];
        b.type[qn][u] = b.type[q][t];
        b.pwork[qn][u] = b.pwork[q][t];
    } else {
        const double4 z = make_double4(0.0, 0.0, 0.0, 0.0);
        b.pos[pn][u] = z;
        b.xbuild[u] = z;
#pragma unroll
        for (int a = 0; a < 3; ++a) b.vel[qn][a][u] = 0.0;
        b.id[qn][u] = -1;
        b.type[qn][u] = kEmptySlot;
        b.pwork[qn][u] = 0.0;
    }
}

// Step 6: the Verlet list from the 27 (or fewer, on boxes under three cells
// per axis) adjacent link cells ("a nested loop over link-cells and their
// adjacent cells").  Full list: every j != i with r < r_c + skin.  Half list:
// only j with a larger slot index.  Overflow keeps counting, so the required
// capacity can be reported.
// Largest list length over the wavefront, one atomic per wavefront.
__device__ __forceinline__ void wave_max_flag(int v, int32_t* flag)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && v > 0) atomicMax(flag, v);
}

__global__ void k_build_list(Buffers b, int p, int q, int64_t n_slots, int32_t cap, double rlist2,
                             int half_list)
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
                const int cell = bx.cell_off + (cz * bx.nc[1] + cy) * bx.nc[0] + cx;
                const int beg = b.cell_start[cell], end = beg + b.cell_count[cell];
                for (int j = beg; j < end; ++j) {
                    if (j == t || (half_list && j < t)) continue;
                    const double3 xj = load_xyz(b.pos[p], j);
                    double ddx = xj.x - xi.x, ddy = xj.y - xi.y, ddz = xj.z - xi.z;
                    min_image(bx, ddx, ddy, ddz);
                    if (ddx * ddx + ddy * ddy + ddz * ddz < rlist2) {
                        if (count < cap) b.nbr[(int64_t)count * n_slots + t] = j;
                        ++count;
                    }
                }
            }
        }
    }
    b.ncount[t] = count < cap ? count : cap;
    wave_max_flag(count, &b.flags[F_MAX_COUNT]);
}

// ---------------------------------------------------------------------------
// Pair-function evaluation.  EV_TABLE: every cubic-knot sum is re-expanded
// exactly as a cubic in the local coordinate u = r - b w of a bin b of width w
// whose edges include every knot, so no knot falls inside a bin and the
// expansion reproduces the sum up to rounding.  With u < w small, the FP32
// evaluation keeps full FP32 relative accuracy (no cancellation between knot
// terms).  Coefficients live in LDS for one species, in the L1-cached global
// table for several.  EV_KNOTS: the sums term by term (fallback when the knots
// share no grid; also the explicit-evaluation comparison of the paper's
// "Parallel benchmarks").
enum { EV_KNOTS = 0, EV_TABLE = 1 };

template <typename R>
struct Tabs {
    const R *force, *energy, *dens;  // [ns*ns][nbt][8], [..][4], [..][4]
};
template <typename R>
__device__ __forceinline__ Tabs<R> tables(const Buffers& b);
template <>
__device__ __forceinline__ Tabs<double> tables<double>(const Buffers& b)
{
    return {b.tab_force64, b.tab_energy64, b.tab_dens64};
}
template <>
__device__ __forceinline__ Tabs<float> tables<float>(const Buffers& b)
{
    return {b.tab_force32, b.tab_energy32, b.tab_dens32};
}

template <typename R>
__device__ __forceinline__ void lds_fill(R* dst, const R* src, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

template <typename R>
__device__ __forceinline__ R cubic(const R* c, R u)
{
    return fma(fma(fma(c[3], u, c[2]), u, c[1]), u, c[0]);
}

template <typename R>
__device__ __forceinline__ R quadratic(const R* c, R u)
{
    return fma(fma(c[2], u, c[1]), u, c[0]);
}

// ---------------------------------------------------------------------------
// Density pass (Eq. Ucoh, the argument of F): rho_i = sum_j rho_{s_i s_j}(r_ij),
// then F_i and F'_i.  One thread per atom over its full list; the sum is
// accumulated in FP64 in both precision modes.
template <typename R, bool SINGLE, int NPK, int NDK, int EV>
__global__ __launch_bounds__(kBlock) void k_density(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                     int energy)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const R* tab = tables<R>(b).dens;
    if (EV == EV_TABLE && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tab, P.nbt * 4);
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
    const Coef<R> C1 = single_coef<R>(P);
    const double rc2 = P.rc2;
    double rho = 0.0;
    for (int k = 0; k < n; ++k) {
        const int j = nbr[(int64_t)k * n_slots + t];
        const double3 xj = load_xyz(pos, j);
        double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
        min_image(bx, dx, dy, dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 < rc2)) continue;
        const double r = r2 * inv_dist<R>(r2);
        const int sj = SINGLE ? 0 : (b.type[q][j] & 0x3F);
        R term;
        if (EV == EV_TABLE) {
            const int bin = (int)(r * P.inv_w);
            const R u = (R)fma(-(double)bin, P.w, r);
            const int ab = SINGLE ? 0 : si * G.ns + sj;
            term = cubic(tab + ((int64_t)ab * P.nbt + bin) * 4, u);
        } else if (SINGLE) {
            term = knot_value<R, NDK>(C1.da, C1.dr, r);
        } else {
            const int ab = si * G.ns + sj;
            KnotSet<R, NDK> ks;
            load_knots<R, NDK>(G.dens_a[ab], G.dens_d[ab], G.dens_r[ab], ks);
            term = knot_value<R, NDK>(ks.a, ks.r, r);
        }
        rho += (double)term;
    }
    double F, dF;
    embed(SINGLE ? P.emb_c : G.emb_c[si], rho, F, dF);
    reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
    if (energy) b.femb[t] = F;
}

// ---------------------------------------------------------------------------
// Force pass + velocity Verlet.  g_ij = phi'(r) + F'_i rho'_{ij}(r) + F'_j rho'_{ji}(r),
// f_i = sum_j g_ij d_ij / r.  The same thread then integrates its atom
// (paper, "Time integration"): closing half kick v += dt/2 a (completing the
// previous step), opening half kick and drift into the other position buffer.
// Rigid atoms ("Fixed atoms") move at their replica's prescribed velocity and
// accumulate the work -f.v_p dt/2 per half step (trapezoid rule).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, bool ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK>
__global__ __launch_bounds__(kBlock) void k_force(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                   double dt, md_state st)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tabs<R> T = tables<R>(b);
    const R* tf = T.force;
    const R* te = T.energy;
    if (EV == EV_TABLE && SINGLE) {
        R* s = reinterpret_cast<R*>(smem);
        lds_fill(s, tf, P.nbt * 8);
        if (ENERGY) lds_fill(s + P.nbt * 8, te, P.nbt * 4);
        __syncthreads();
        tf = s;
        te = s + P.nbt * 8;
    }
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r_id = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& Rp = b.reps[r_id];
    const bool valid = t - Rp.slot_off < Rp.n_atoms;
    const Box bx = load_box(Rp);
    const DevPotential& G = *b.pot;
    const double4* __restrict__ pos = b.pos[p];
    const int32_t* __restrict__ nbr = b.nbr;

    double fx = 0.0, fy = 0.0, fz = 0.0;
    double epair = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
    double pe = 0.0, ke = 0.0, pw = 0.0;
    int nonfinite = 0;
    if (valid) {
        const double4 pi = pos[t];
        const uint8_t ti = b.type[q][t];
        const int si = ti & 0x3F;
        const bool rigid_i = ti & kRigidBit;
        const int n = b.ncount[t];
        const Coef<R> C1 = single_coef<R>(P);
        const double rc2 = P.rc2;
        const R fpi = (R)pi.w;
        for (int k = 0; k < n; ++k) {
            const int j = nbr[(int64_t)k * n_slots + t];
            const double4 pj = pos[j];
            double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
            min_image(bx, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < rc2)) continue;
            const double ri = inv_dist<R>(r2);
            const double r = r2 * ri;
            R g, phi = R(0);
            uint8_t tj = 0;
            if (!SINGLE || ENERGY) tj = b.type[q][j];
            if (EV == EV_TABLE) {
                const int bin = (int)(r * P.inv_w);
                const R u = (R)fma(-(double)bin, P.w, r);
                if (SINGLE) {
                    const R* c = tf + bin * 8;
                    g = quadratic(c, u) + (fpi + (R)pj.w) * quadratic(c + 3, u);
                    if (ENERGY) phi = cubic(te + bin * 4, u);
                } else {
                    const int sj = tj & 0x3F;
                    const int64_t ab = si * G.ns + sj, ba = sj * G.ns + si;
                    const R* c = tf + (ab * P.nbt + bin) * 8;
                    const R* c2 = tf + (ba * P.nbt + bin) * 8;
                    g = quadratic(c, u) + fpi * quadratic(c + 3, u) + (R)pj.w * quadratic(c2 + 3, u);
                    if (ENERGY) phi = cubic(te + (ab * P.nbt + bin) * 4, u);
                }
            } else if (SINGLE) {
                R dphi;
                if (ENERGY) knot_both<R, NPK>(C1.pa, C1.pd, C1.pr, r, phi, dphi);
                else dphi = knot_deriv<R, NPK>(C1.pd, C1.pr, r);
                const R drho = knot_deriv<R, NDK>(C1.dd, C1.dr, r);
                g = dphi + (fpi + (R)pj.w) * drho;
            } else {
                const int sj = tj & 0x3F;
                const int ab = si * G.ns + sj, ba = sj * G.ns + si;
                KnotSet<R, NPK> kp;
                load_knots<R, NPK>(G.pair_a[ab], G.pair_d[ab], G.pair_r[ab], kp);
                R dphi;
                if (ENERGY) knot_both<R, NPK>(kp.a, kp.d, kp.r, r, phi, dphi);
                else dphi = knot_deriv<R, NPK>(kp.d, kp.r, r);
                KnotSet<R, NDK> kab, kba;
                load_knots<R, NDK>(G.dens_a[ab], G.dens_d[ab], G.dens_r[ab], kab);
                load_knots<R, NDK>(G.dens_a[ba], G.dens_d[ba], G.dens_r[ba], kba);
                g = dphi + fpi * knot_deriv<R, NDK>(kab.d, kab.r, r) +
                    (R)pj.w * knot_deriv<R, NDK>(kba.d, kba.r, r);
            }
            const double s = (double)g * ri;
            fx = fma(s, dx, fx);
            fy = fma(s, dy, fy);
            fz = fma(s, dz, fz);
            if (ENERGY) {
                epair += (double)phi;
                if (!(rigid_i && (tj & kRigidBit))) {
                    w[0] = fma(s * dx, dx, w[0]);
                    w[1] = fma(s * dy, dy, w[1]);
                    w[2] = fma(s * dz, dz, w[2]);
                    w[3] = fma(s * dx, dy, w[3]);
                    w[4] = fma(s * dx, dz, w[4]);
                    w[5] = fma(s * dy, dz, w[5]);
                }
            }
        }

        // ---- integration
        double v[3] = {b.vel[q][0][t], b.vel[q][1][t], b.vel[q][2][t]};
        double xn[3] = {pi.x, pi.y, pi.z};
        const double f[3] = {fx, fy, fz};
        if (rigid_i) {
            const double p_half = -(f[0] * Rp.vp[0] + f[1] * Rp.vp[1] + f[2] * Rp.vp[2]) * 0.5 * dt;
            double acc = b.pwork[q][t];
            if (CLOSE) acc += p_half;
            if (OPEN) acc += p_half;
            if (CLOSE || OPEN) b.pwork[q][t] = acc;
            pw = acc;
            if (OPEN) {
#pragma unroll
                for (int a = 0; a < 3; ++a) xn[a] += dt * Rp.vp[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a] = Rp.vp[a];
        } else {
            const double acc = SINGLE ? P.accel : G.accel[si];
            if (CLOSE) {
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a] = fma(0.5 * dt * acc, f[a], v[a]);
            }
            if (ENERGY) ke = (SINGLE ? P.half_m : G.half_m[si]) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (OPEN) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    v[a] = fma(0.5 * dt * acc, f[a], v[a]);
                    xn[a] = fma(dt, v[a], xn[a]);
                }
            }
            if (CLOSE || OPEN) {
#pragma unroll
                for (int a = 0; a < 3; ++a) b.vel[q][a][t] = v[a];
            }
        }
        if (OPEN) {
            double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
            *reinterpret_cast<double2*>(dst) = make_double2(xn[0], xn[1]);
            dst[2] = xn[2];
        }
        if (ENERGY) {
            pe = 0.5 * epair + b.femb[t];
            if (!isfinite(pe) || !isfinite(ke) || !isfinite(fx + fy + fz)) nonfinite = 1;
        }
        if (WRITEBACK) {
            const int32_t a = b.id[q][t];
            st.fx[a] = fx;
            st.fy[a] = fy;
            st.fz[a] = fz;
            if (CLOSE) {
                st.x[a] = xn[0];
                st.y[a] = xn[1];
                st.z[a] = xn[2];
                st.vx[a] = v[0];
                st.vy[a] = v[1];
                st.vz[a] = v[2];
            }
            if (ENERGY && st.e_atom) st.e_atom[a] = pe;
        }
    }

    if (ENERGY) {
        // one record per wavefront (a wavefront never mixes replicas)
        double vals[kEnergySlots] = {pe, ke, w[0], w[1], w[2], w[3], w[4], w[5], pw, (double)nonfinite, 0, 0};
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
            for (int k = 0; k < 10; ++k) vals[k] += __shfl_xor(vals[k], off, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            double* out = b.partial + (t / kWave) * kEnergySlots;
#pragma unroll
            for (int k = 0; k < kEnergySlots; ++k) out[k] = vals[k];
        }
    }
}

// Per-replica totals from the per-wavefront records, in a fixed order that
// depends only on the replica's own size (so a replica gives the same sums
// alone or inside a batch).
__global__ __launch_bounds__(kBlock) void k_reduce_energies(Buffers b, double virial_scale)
{
    __shared__ double sh[kBlock];
    const DevReplica& R = b.reps[blockIdx.x];
    const int64_t w0 = R.slot_off / kWave, w1 = (R.slot_off + R.n_atoms + kWave - 1) / kWave;
    for (int k = 0; k < kEnergySlots; ++k) {
        double acc = 0.0;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += kBlock) acc += b.partial[w * kEnergySlots + k];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double v = sh[0];
            if (k >= E_W0 && k < E_W0 + 6) v *= virial_scale;
            b.energies[blockIdx.x * kEnergySlots + k] = v;
        }
        __syncthreads();
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
                       k.cap, rlist2, half_list);
}

template <typename R, bool S, int NP, int ND, int EV>
static void density_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int energy,
                            hipStream_t s)
{
    const size_t lds = (EV == EV_TABLE && S) ? (size_t)P.nbt * 4 * sizeof(R) : 0;
    hipLaunchKernelGGL((k_density<R, S, NP, ND, EV>), dim3(blocks_for(k.n_slots)), dim3(kBlock), lds, s, b, p, q,
                       k.n_slots, P, energy);
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
    const size_t lds = (EV == EV_TABLE && S) ? (size_t)P.nbt * (E ? 12 : 8) * sizeof(R) : 0;
    hipLaunchKernelGGL((k_force<R, S, NP, ND, EV, E, C, O, W>), dim3(blocks_for(k.n_slots)), dim3(kBlock), lds, s,
                       b, p, q, k.n_slots, P, dt_fs, st);
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

void launch_reduce_energies(const Buffers& b, const KernelShape& k, hipStream_t s)
{
    // full list: every pair was seen from both atoms
    hipLaunchKernelGGL(k_reduce_energies, dim3(k.n_replicas), dim3(kBlock), 0, s, b, -0.5);
}

}  // namespace mdk
