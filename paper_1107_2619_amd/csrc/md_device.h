// Device helpers shared by the gfx950 kernel families (global-gather and
// LDS-brick): launch geometry, periodic images, cubic-knot and tabulated
// pair functions, the embedding, and the velocity-Verlet epilogue.
#pragma once

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

// Value of lane `l` (wave-uniform) of a double.
__device__ __forceinline__ double bcast_lane(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Geometry helpers (paper, "Boundary conditions": minimum image along periodic
// axes, plain differences along free ones; positions unwrapped).
struct Box {
    double L[3], iL[3], o[3];
    int pmask;
    int nc[3];
    int cell_off;
    int tri;             // sheared cell: images and cells along the edge vectors
    const double* h;     // its box matrix (edge vectors as columns, row-major)
    const double* hinv;
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
    b.tri = R.tri;
    b.h = R.h;
    b.hinv = R.hinv;
    return b;
}

// Lattice translation by the integer image counts n: n_a L_a along each axis of
// an orthorhombic box, h n in a sheared cell.
__device__ __forceinline__ void lattice_shift(const DevReplica& R, double n0, double n1, double n2, double out[3])
{
    if (R.tri) {
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = R.h[3 * a] * n0 + R.h[3 * a + 1] * n1 + R.h[3 * a + 2] * n2;
    } else {
        out[0] = n0 * R.box[0];
        out[1] = n1 * R.box[1];
        out[2] = n2 * R.box[2];
    }
}

// Fractional coordinates s = h^-1 (x - o) of a point in a sheared cell.
__device__ __forceinline__ void frac_coords(const double* hinv, const double o[3], double x, double y, double z,
                                            double s[3])
{
    const double d[3] = {x - o[0], y - o[1], z - o[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = hinv[3 * a] * d[0] + hinv[3 * a + 1] * d[1] + hinv[3 * a + 2] * d[2];
}

// Minimum image of d at list-build time: applies the shortest periodic image
// to d and returns its shift code (2 bits per axis: 0 = none, 1 = +L, 2 = -L),
// stored in the top bits of the list entry so the force loop can reapply it.
__device__ __forceinline__ int image_code(const Box& b, double& dx, double& dy, double& dz)
{
    double* d[3] = {&dx, &dy, &dz};
    int code = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!(b.pmask & (1 << a))) continue;
        const double m = rint(*d[a] * b.iL[a]);
        if (m != 0.0) {
            *d[a] -= m * b.L[a];
            code |= (m < 0.0 ? 1 : 2) << (2 * a);
        }
    }
    return code;
}

// Reapply a stored periodic shift (rare: only pairs across a box face).  In a
// sheared cell the shift is the sum of the edge vectors the code names.
__device__ __forceinline__ void apply_shift(const Box& b, int code, double& dx, double& dy, double& dz)
{
    if (b.tri) {
        const double k0 = (code & 3) ? ((code & 1) ? 1.0 : -1.0) : 0.0;
        const double k1 = (code & 12) ? ((code & 4) ? 1.0 : -1.0) : 0.0;
        const double k2 = (code & 48) ? ((code & 16) ? 1.0 : -1.0) : 0.0;
        dx += b.h[0] * k0 + b.h[1] * k1 + b.h[2] * k2;
        dy += b.h[3] * k0 + b.h[4] * k1 + b.h[5] * k2;
        dz += b.h[6] * k0 + b.h[7] * k1 + b.h[8] * k2;
        return;
    }
    if (code & 3) dx += (code & 1) ? b.L[0] : -b.L[0];
    if (code & 12) dy += (code & 4) ? b.L[1] : -b.L[1];
    if (code & 48) dz += (code & 16) ? b.L[2] : -b.L[2];
}

// Link cell along one axis: periodic axes wrap the fractional coordinate into
// [0, 1); free axes clamp (monotone, so atoms closer than one cell edge still
// land in the same or adjacent cells).
__device__ __forceinline__ int cell_of_frac(double f, int nc, bool periodic)
{
    if (periodic) f -= floor(f);
    int c = (int)floor(f * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ int cell_axis(double x, double o, double iL, int nc, bool periodic)
{
    double f = (x - o) * iL;
    if (periodic) f -= floor(f);
    int c = (int)floor(f * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ void cell_coords(const Box& b, double x, double y, double z, int c[3])
{
    if (b.tri) {  // cells along the edge vectors: fractional coordinates, all axes periodic
        double f[3];
        frac_coords(b.hinv, b.o, x, y, z, f);
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] = cell_of_frac(f[a], b.nc[a], true);
        return;
    }
    c[0] = cell_axis(x, b.o[0], b.iL[0], b.nc[0], b.pmask & 1);
    c[1] = cell_axis(y, b.o[1], b.iL[1], b.nc[1], b.pmask & 2);
    c[2] = cell_axis(z, b.o[2], b.iL[2], b.nc[2], b.pmask & 4);
}

// Compact record of a slot: cell-local coordinates in units of h_a 2^-28 (the
// mixed mode's gather image of the FP64 positions).  In a sheared cell the
// coordinates are fractional, along the edge vectors: (s_a n_a - c_a) 2^28 with
// s = h^-1 (x - o).  Returns false if a coordinate lies too far outside its
// link cell to encode.  KIND: 0 reads the cell type from the descriptor, 1
// orthorhombic, 2 sheared (for kernels specialised on it).
template <int KIND = 0>
__device__ __forceinline__ bool compact_coords(const DevReplica& R, const int c[3], double x, double y, double z,
                                               int4& out)
{
    double u[3];
    if (KIND == 0 ? R.tri != 0 : KIND == 2) {
        double f[3];
        frac_coords(R.hinv, R.origin, x, y, z, f);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = ldexp(fma(f[a], (double)R.nc[a], -(double)c[a]), kCompactBits);
    } else {
        const double xs[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = (xs[a] - (R.origin[a] + c[a] * R.cell[a])) * R.iqs[a];
    }
    int q[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ok = ok && fabs(u[a]) < kCompactCells * (double)(1 << kCompactBits);
        q[a] = ok ? (int)rint(u[a]) : 0;
    }
    out = make_int4(q[0], q[1], q[2], 0);
    return ok;
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

// Largest list length over the wavefront, one atomic per wavefront.
__device__ __forceinline__ void wave_max_flag(int v, int32_t* flag)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    // The flag only grows, so a plain (possibly stale) read filters out the
    // atomics that cannot raise it: a kernel with many wavefronts would
    // otherwise serialise on one address.
    if ((threadIdx.x & (kWave - 1)) == 0 && v > 0 && v > *flag) atomicMax(flag, v);
}

// ---------------------------------------------------------------------------
// Pair-function evaluation.  EV_TABLE: every cubic-knot sum is re-expanded
// exactly as a cubic in the local coordinate u = r - b w of a bin b of width w
// whose edges include every knot, so no knot falls inside a bin and the
// expansion reproduces the sum up to rounding.  With u < w small, the FP32
// evaluation keeps full FP32 relative accuracy (no cancellation between knot
// terms).  EV_SPLIT: the same for knots that share no grid (any coefficient
// file, "Available potentials"): a bin may hold one knot of each function,
// whose term a (D - u)^3 H(D - u) (D the knot's offset from the bin start)
// is added to the cubic of the knots switched on across the whole bin; still
// exact up to rounding, and still free of cancellation since D - u < w.
// Coefficients live in LDS for one species, in the L1-cached global table for
// several.  EV_KNOTS: the sums term by term (the explicit-evaluation
// comparison of the paper's "Parallel benchmarks"; FP64 only).
enum { EV_KNOTS = 0, EV_TABLE = 1, EV_SPLIT = 2 };

template <typename R>
struct Tabs {
    const R *force, *energy, *dens;  // [ns*ns][nbt][force_stride], [..][value_stride] twice
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

// Sum a value over the L lanes that share one atom (consecutive lanes).
template <int L>
__device__ __forceinline__ double lane_sum(double v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One pair's contribution to the density of the site atom (species si) from
// a neighbour of species sj at distance r: rho_{si sj}(r).
// Knot term inside a bin, added to acc: amp (D - u)^2 (P = 2, derivative
// records) or amp (D - u)^3 (P = 3, value records), zero for u >= D.  The
// fused forms are explicit so that every kernel variant rounds alike.
template <typename R, int PW>
__device__ __forceinline__ R split_term(const R* c, R u, R acc)
{
    R t = c[0] - u;
    t = t > R(0) ? t : R(0);
    return PW == 3 ? fma(c[1] * t * t, t, acc) : fma(c[1] * t, t, acc);
}

template <typename R, bool SINGLE, int NDK, int EV>
__device__ __forceinline__ R density_term(const PotArgs& P, const DevPotential& G, const R* tab, int si, int sj,
                                          double r)
{
    if (EV != EV_KNOTS) {
        constexpr int VS = value_stride(EV);
        const int bin = (int)(r * P.inv_w);
        const R u = (R)fma(-(double)bin, P.w, r);
        const int ab = SINGLE ? 0 : si * G.ns + sj;
        const R* c = tab + ((int64_t)ab * P.nbt + bin) * VS;
        if (EV == EV_SPLIT) return split_term<R, 3>(c + 4, u, cubic(c, u));
        return cubic(c, u);
    } else if (SINGLE) {
        const Coef<R> C1 = single_coef<R>(P);
        return knot_value<R, NDK>(C1.da, C1.dr, r);
    } else {
        const int ab = si * G.ns + sj;
        KnotSet<R, NDK> ks;
        load_knots<R, NDK>(G.dens_a[ab], G.dens_d[ab], G.dens_r[ab], ks);
        return knot_value<R, NDK>(ks.a, ks.r, r);
    }
}

// g_ij = phi'_{ij}(r) + F'_i rho'_{ij}(r) + F'_j rho'_{ji}(r) and, on energy
// steps, phi_{ij}(r).  Tables: tf = [ns*ns][nbt][kForceStride] derivative quadratics,
// te = [ns*ns][nbt][4] value cubics.  DENS = false: a pair beyond every density
// cutoff, whose rho' terms vanish (the caller knows it from the list).
template <typename R, bool SINGLE, int NPK, int NDK, int EV, int ENERGY, bool DENS = true>
__device__ __forceinline__ void pair_terms(const PotArgs& P, const DevPotential& G, const R* tf, const R* te,
                                           int si, int sj, double r, R fpi, R fpj, R& g, R& phi)
{
    phi = R(0);
    if (EV != EV_KNOTS) {
        constexpr int FS = force_stride(EV), VS = value_stride(EV);
        const int bin = (int)(r * P.inv_w);
        const R u = (R)fma(-(double)bin, P.w, r);
        if (SINGLE) {
            const R* c = tf + bin * FS;
            R dphi = quadratic(c, u);
            if (EV == EV_SPLIT) dphi = split_term<R, 2>(c + 6, u, dphi);
            g = dphi;
            if (DENS) {  // explicit fused forms: every kernel variant rounds alike
                R drho = quadratic(c + 3, u);
                if (EV == EV_SPLIT) drho = split_term<R, 2>(c + 8, u, drho);
                g = fma(fpi + fpj, drho, dphi);
            }
            if (ENERGY == 1) {
                const R* e = te + bin * VS;
                phi = cubic(e, u);
                if (EV == EV_SPLIT) phi = split_term<R, 3>(e + 4, u, phi);
            }
        } else {
            const int64_t ab = si * G.ns + sj, ba = sj * G.ns + si;
            const R* c = tf + (ab * P.nbt + bin) * FS;
            R dphi = quadratic(c, u);
            if (EV == EV_SPLIT) dphi = split_term<R, 2>(c + 6, u, dphi);
            g = dphi;
            if (DENS) {
                const R* c2 = tf + (ba * P.nbt + bin) * FS;
                R dab = quadratic(c + 3, u), dba = quadratic(c2 + 3, u);
                if (EV == EV_SPLIT) {
                    dab = split_term<R, 2>(c + 8, u, dab);
                    dba = split_term<R, 2>(c2 + 8, u, dba);
                }
                g = fma(fpi, dab, fma(fpj, dba, dphi));
            }
            if (ENERGY == 1) {
                const R* e = te + (ab * P.nbt + bin) * VS;
                phi = cubic(e, u);
                if (EV == EV_SPLIT) phi = split_term<R, 3>(e + 4, u, phi);
            }
        }
    } else if (SINGLE) {
        const Coef<R> C1 = single_coef<R>(P);
        R dphi;
        if (ENERGY == 1) knot_both<R, NPK>(C1.pa, C1.pd, C1.pr, r, phi, dphi);
        else dphi = knot_deriv<R, NPK>(C1.pd, C1.pr, r);
        g = DENS ? fma(fpi + fpj, knot_deriv<R, NDK>(C1.dd, C1.dr, r), dphi) : dphi;
    } else {
        const int ab = si * G.ns + sj, ba = sj * G.ns + si;
        KnotSet<R, NPK> kp;
        load_knots<R, NPK>(G.pair_a[ab], G.pair_d[ab], G.pair_r[ab], kp);
        R dphi;
        if (ENERGY == 1) knot_both<R, NPK>(kp.a, kp.d, kp.r, r, phi, dphi);
        else dphi = knot_deriv<R, NPK>(kp.d, kp.r, r);
        g = dphi;
        if (DENS) {
            KnotSet<R, NDK> kab, kba;
            load_knots<R, NDK>(G.dens_a[ab], G.dens_d[ab], G.dens_r[ab], kab);
            load_knots<R, NDK>(G.dens_a[ba], G.dens_d[ba], G.dens_r[ba], kba);
            g = fma(fpi, knot_deriv<R, NDK>(kab.d, kab.r, r), fma(fpj, knot_deriv<R, NDK>(kba.d, kba.r, r), g));
        }
    }
}

// Pair accumulation into the site atom: force, and on energy steps
// (ENERGY = 1) the pair energy and the virial tensor (pairs of two rigid atoms
// excluded); ENERGY = 2 (barostat steps) keeps only the virial diagonal and
// ENERGY = 3 (steps of the full-matrix barostat) the whole virial tensor.
struct PairAcc {
    double f[3] = {0.0, 0.0, 0.0};
    double epair = 0.0;
    double w[6] = {0, 0, 0, 0, 0, 0};
};

template <int ENERGY>
__device__ __forceinline__ void accumulate(PairAcc& A, double s, double dx, double dy, double dz, double phi,
                                           bool both_rigid)
{
    A.f[0] = fma(s, dx, A.f[0]);
    A.f[1] = fma(s, dy, A.f[1]);
    A.f[2] = fma(s, dz, A.f[2]);
    if (ENERGY == 1) {
        A.epair += phi;
        if (!both_rigid) {
            A.w[0] = fma(s * dx, dx, A.w[0]);
            A.w[1] = fma(s * dy, dy, A.w[1]);
            A.w[2] = fma(s * dz, dz, A.w[2]);
            A.w[3] = fma(s * dx, dy, A.w[3]);
            A.w[4] = fma(s * dx, dz, A.w[4]);
            A.w[5] = fma(s * dy, dz, A.w[5]);
        }
    } else if (ENERGY == 2 || ENERGY == 3) {  // the barostat takes no rigid atoms
        A.w[0] = fma(s * dx, dx, A.w[0]);
        A.w[1] = fma(s * dy, dy, A.w[1]);
        A.w[2] = fma(s * dz, dz, A.w[2]);
        if (ENERGY == 3) {
            A.w[3] = fma(s * dx, dy, A.w[3]);
            A.w[4] = fma(s * dx, dz, A.w[4]);
            A.w[5] = fma(s * dy, dz, A.w[5]);
        }
    }
}

// Velocity Verlet for one atom after its force is known (paper, "Time
// integration"): closing half kick v += dt/2 a (completing the previous step),
// opening half kick and drift x += dt v into the other position buffer.
// Rigid atoms ("Fixed atoms") move at their replica's prescribed velocity and
// accumulate the work -f.v_p dt/2 per half step (trapezoid rule).  On energy
// steps the atom's energy terms go to its slot of `eslot`; with WRITEBACK the
// final state returns to the caller's arrays (caller order, unwrapped).
//
// WSUM: the energy terms go to `wv` for a wavefront sum instead of `eslot`.
template <bool SINGLE, int ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK, bool WSUM = false>
__device__ __forceinline__ void atom_epilogue(const Buffers& b, int p, int q, int64_t t, int64_t n_slots,
                                              const DevReplica& Rp, const PotArgs& P, const DevPotential& G,
                                              double dt, const md_state& st, const double4& pi, uint8_t ti,
                                              const PairAcc& A, double* wv = nullptr)
{
    const int si = ti & 0x3F;
    const bool rigid_i = ti & kRigidBit;
    double v[3] = {b.vel[q][0][t], b.vel[q][1][t], b.vel[q][2][t]};
    double xn[3] = {pi.x, pi.y, pi.z};
    const double* f = A.f;
    double ke = 0.0, pw = 0.0;
    if (rigid_i) {
        const double p_half = -(f[0] * Rp.vp[0] + f[1] * Rp.vp[1] + f[2] * Rp.vp[2]) * 0.5 * dt;
        double acc = b.pwork[q][t];
        if (CLOSE) acc += p_half;
        pw = acc;  // the work up to this state
        if (OPEN) acc += p_half;
        if (CLOSE || OPEN) b.pwork[q][t] = acc;
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
        if (ENERGY == 1) ke = (SINGLE ? P.half_m : G.half_m[si]) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
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
    double pe = 0.0;
    if (ENERGY == 1) {
        pe = 0.5 * A.epair + b.femb[t];
        const int nonfinite = (!isfinite(pe) || !isfinite(ke) || !isfinite(f[0] + f[1] + f[2])) ? 1 : 0;
        const double vals[kEnergyTerms] = {pe, ke, A.w[0], A.w[1], A.w[2], A.w[3], A.w[4], A.w[5], pw, (double)nonfinite};
#pragma unroll
        for (int k = 0; k < kEnergyTerms; ++k) {
            if (WSUM) wv[k] = vals[k];
            else b.eslot[(int64_t)k * n_slots + t] = vals[k];
        }
    } else if (ENERGY == 2 || ENERGY == 3) {  // barostat steps: the virial diagonal, or the whole tensor
#pragma unroll
        for (int k = 0; k < (ENERGY == 3 ? 6 : 3); ++k) b.eslot[(int64_t)(E_W0 + k) * n_slots + t] = A.w[k];
    }
    if (!OPEN) {
        // kept for the opening kick that runs later: after the thermostat's
        // kinetic-energy reduction, or at the start of the next md_step call
#pragma unroll
        for (int a = 0; a < 3; ++a) b.fhalf[a][t] = f[a];
    }
    if (WRITEBACK) {
        const int32_t a = b.id[q][t];
        st.fx[a] = f[0];
        st.fy[a] = f[1];
        st.fz[a] = f[2];
        if (CLOSE) {
            double sh[3];
            lattice_shift(Rp, b.img[q][0][t], b.img[q][1][t], b.img[q][2][t], sh);
            st.x[a] = xn[0] + sh[0];
            st.y[a] = xn[1] + sh[1];
            st.z[a] = xn[2] + sh[2];
            st.vx[a] = v[0];
            st.vy[a] = v[1];
            st.vz[a] = v[2];
        }
        if (ENERGY == 1 && st.e_atom) st.e_atom[a] = pe;
    }
}

// Sum of each energy term over the wavefront (a wavefront never straddles two
// replicas), by an xor butterfly: every lane ends with the same bits.  Lane 0
// stores the sums of wavefront t / 64.  Called by all lanes of the wavefront.
__device__ __forceinline__ void wave_sum_terms(const Buffers& b, int64_t t, double (&v)[kEnergyTerms])
{
#pragma unroll
    for (int k = 0; k < kEnergyTerms; ++k)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int k = 0; k < kEnergyTerms; ++k) b.wave_terms[(t / kWave) * kEnergyTerms + k] = v[k];
}

}  // namespace
}  // namespace mdk
