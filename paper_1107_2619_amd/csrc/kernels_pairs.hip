// LDS-brick pair kernels (MD_OPT_KERNEL = 2): the density and force passes
// over brick lists that keep each pair of two own atoms of a brick once
// (k_brick_list with half = 1).  The lane of the atom with the smaller
// staging index evaluates such a pair and adds the other atom's share
// (rho_{s_j s_i}(r), -g d / r, phi) into LDS accumulators of the brick's own
// atoms; after a workgroup barrier every atom adds its accumulator to what its
// own lane summed.  Pairs with a halo atom are evaluated from both sides, as in
// the full list, since each side belongs to a different workgroup.  For a
// brick of 4 x 4 x 4 link cells about three quarters of the pairs are internal,
// so the passes evaluate about 0.6 of the full list's pairs.
//
// The shared accumulators add 64-bit fixed-point integers (LDS integer atomics
// are exact, so the sums do not depend on the order the lanes arrive in and a
// run is bitwise reproducible): a share x becomes round(x 2^40), |x| < 2^10
// (a larger share sets F_RANGE, reported as an error).  The rounding is at most
// 4.6e-13 per share, against forces and densities of order 0.1 - 100.
// Bricks whose list holds every pair from both atoms (brick_info.w = 0: halo
// larger than the staging area, or more own atoms than one round of lanes)
// run as the full-list brick kernels do.
#include <algorithm>

#include "brick_common.h"

namespace mdk {
namespace {

constexpr double kFixedScale = 0x1p40;       // fixed-point unit of the shared accumulators: 2^-40
constexpr double kFixedInv = 0x1p-40;
constexpr double kFixedRange = 1024.0;       // largest share the accumulators take
constexpr double kFixedMagic = 0x1.8p52;     // 1.5 2^52: adding it puts round(x 2^40) in the low mantissa bits
constexpr long long kFixedMagicBits = 0x4338000000000000LL;

// round(x 2^40) as a two's-complement 64-bit integer (|x| < 2^11): the sum
// 1.5 2^52 + x 2^40 has unit weight in its last mantissa bit, so its bit
// pattern minus that of 1.5 2^52 is the rounded integer.
__device__ __forceinline__ unsigned long long to_fixed(double x)
{
    return (unsigned long long)(__double_as_longlong(fma(x, kFixedScale, kFixedMagic)) - kFixedMagicBits);
}

__device__ __forceinline__ double from_fixed(unsigned long long v) { return (double)(long long)v * kFixedInv; }

__device__ __forceinline__ void share(unsigned long long* acc, double x, int32_t* flags)
{
    if (!(fabs(x) < kFixedRange)) atomicAdd(&flags[F_RANGE], 1);
    atomicAdd(acc, to_fixed(x));
}

// LDS layout: Halo | staged atoms [halo_cap] | accumulators [n_acc][slots] | tables, types.
__host__ __device__ inline size_t pair_acc_offset(int halo_cap)
{
    return halo_bytes() + (size_t)halo_cap * sizeof(double4);
}

// Density pass (Eq. Ucoh, the argument of F), pairs of own atoms once.
template <typename R, bool SINGLE, int NDK, int EV, int L>
__global__ __launch_bounds__(1024) void k_pair_density(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                       int energy, int halo_cap, int rowlen, int slots)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + halo_bytes());
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + pair_acc_offset(halo_cap));
    unsigned char* tail = smem + pair_acc_offset(halo_cap) + (size_t)slots * 8;
    const R* tab = tables<R>(b).dens;
    uint8_t* ltype = reinterpret_cast<uint8_t*>(tail);
    if (EV != EV_KNOTS && SINGLE) {
        R* s = reinterpret_cast<R*>(tail);
        lds_fill(s, tab, P.nbt * value_stride(EV));
        tab = s;
    }
    const int brick = brick_of_block();
    const DevReplica& Rp = b.reps[b.brick_rep[brick]];
    const int4 info = b.brick_info[brick];  // own slot range, halo size, pairs-once flag at the last build
    const bool staged = info.z <= halo_cap;
    const bool pairs = info.w != 0;  // implies staged and one round of lanes
    const int n_own = info.y - info.x;
    if (pairs)
        for (int i = threadIdx.x; i < n_own; i += blockDim.x) acc[i] = 0ull;
    if (staged) {
        stage_recorded(b, Rp, b.stage_src + (int64_t)brick * halo_cap, info.z, p, q, false, lpos,
                       SINGLE ? nullptr : ltype);
    } else {
        stage_brick(b, Rp, brick - Rp.brick_off, p, false, halo_cap, M, lpos);  // halo table for halo_fetch
    }
    const DevPotential& G = *b.pot;
    const int lane = threadIdx.x % L;
    const int per_round = blockDim.x / L;
    double rho_kept = 0.0;
    int si_kept = 0;
    for (int a0 = 0; a0 < n_own; a0 += per_round) {
        const int a = a0 + threadIdx.x / L;
        const bool live = a < n_own;
        const int64_t t = info.x + (live ? a : 0);
        const int li = b.own_li[t];
        const double4 xi = staged ? lpos[li] : halo_fetch(b, Rp, M, p, li);
        const int si = SINGLE ? 0 : ((staged ? ltype[li] : halo_type(b, M, q, li)) & 0x3F);
        const int n = live ? b.ncount[t] : 0;
        double rho = 0.0;
        const uint4* row = reinterpret_cast<const uint4*>(b.nbr16 + t * (int64_t)rowlen);
        const int nblk = (n + 7) >> 3;
        uint4 cur = row[lane];  // rows are padded: loads past the list are harmless
        for (int blk = lane; blk < nblk; blk += L) {
            const uint4 nxt = row[blk + L];
            const uint32_t w4[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                double4 xs[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * hf + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    const bool ok = blk * 8 + hf * 4 + u < n;
                    xs[u] = staged ? lpos[ok ? e : li] : halo_fetch(b, Rp, M, p, ok ? e : li);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * hf + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    if (blk * 8 + hf * 4 + u >= n) break;
                    const double dx = xs[u].x - xi.x, dy = xs[u].y - xi.y, dz = xs[u].z - xi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < P.rc2)) continue;
                    const double r = r2 * inv_dist<R>(r2);
                    const int sj = SINGLE ? 0 : ((staged ? ltype[e] : halo_type(b, M, q, e)) & 0x3F);
                    const R v = density_term<R, SINGLE, NDK, EV>(P, G, tab, si, sj, r);
                    rho += (double)v;
                    if (pairs && e < n_own) {  // the other atom's density from this one
                        const R vj = SINGLE ? v : density_term<R, SINGLE, NDK, EV>(P, G, tab, sj, si, r);
                        share(acc + e, (double)vj, b.flags);
                    }
                }
            }
            cur = nxt;
        }
        rho = lane_sum<L>(rho);
        if (!pairs && live && lane == 0) {
            double F, dF;
            embed(SINGLE ? P.emb_c : G.emb_c[si], rho, F, dF);
            reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
            if (energy) b.femb[t] = F;
        }
        rho_kept = rho;
        si_kept = si;
    }
    if (pairs) {  // one round: every lane still holds its atom's own sum
        __syncthreads();
        const int a = threadIdx.x / L;
        if (a < n_own && lane == 0) {
            const int64_t t = info.x + a;
            double F, dF;
            embed(SINGLE ? P.emb_c : G.emb_c[si_kept], rho_kept + from_fixed(acc[a]), F, dF);
            reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
            if (energy) b.femb[t] = F;
        }
    }
}

// Force pass + velocity Verlet, pairs of own atoms once.  The accumulators
// hold -g d / r (three components) and, on energy steps, phi for the atom with
// the larger staging index of each such pair.  The virial of a pair evaluated
// once is entered twice, so that the reduction's factor 1/2 of the full list
// applies to every pair.
template <typename R, bool SINGLE, int NPK, int NDK, int EV, bool ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK, int L>
__global__ __launch_bounds__(1024) void k_pair_force(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double dt,
                                                     md_state st, int halo_cap, int rowlen, int slots)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + halo_bytes());
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + pair_acc_offset(halo_cap));
    constexpr int n_acc = ENERGY ? 4 : 3;
    unsigned char* tail = smem + pair_acc_offset(halo_cap) + (size_t)slots * 8 * n_acc;
    const Tabs<R> T = tables<R>(b);
    const R* tf = T.force;
    const R* te = T.energy;
    uint8_t* ltype = reinterpret_cast<uint8_t*>(tail);
    if (EV != EV_KNOTS && SINGLE) {
        R* s = reinterpret_cast<R*>(tail);
        lds_fill(s, tf, P.nbt * force_stride(EV));
        if (ENERGY) lds_fill(s + P.nbt * force_stride(EV), te, P.nbt * value_stride(EV));
        tf = s;
        te = s + P.nbt * force_stride(EV);
        ltype = reinterpret_cast<uint8_t*>(
            tail + (size_t)P.nbt * (force_stride(EV) + (ENERGY ? value_stride(EV) : 0)) * sizeof(R));
    }
    const bool need_type = !SINGLE || ENERGY;
    const int brick = brick_of_block();
    const DevReplica& Rp = b.reps[b.brick_rep[brick]];
    const int4 info = b.brick_info[brick];
    const bool staged = info.z <= halo_cap;
    const bool pairs = info.w != 0;
    const int n_own = info.y - info.x;
    if (pairs)
        for (int i = threadIdx.x; i < n_acc * slots; i += blockDim.x) acc[i] = 0ull;
    if (staged) {
        stage_recorded(b, Rp, b.stage_src + (int64_t)brick * halo_cap, info.z, p, q, true, lpos,
                       need_type ? ltype : nullptr);
    } else {
        stage_brick(b, Rp, brick - Rp.brick_off, p, true, halo_cap, M, lpos);
    }
    const DevPotential& G = *b.pot;
    const int lane = threadIdx.x % L;
    const int per_round = blockDim.x / L;
    PairAcc A;
    for (int a0 = 0; a0 < n_own; a0 += per_round) {
        const int a = a0 + threadIdx.x / L;
        const bool live = a < n_own;
        const int64_t t = info.x + (live ? a : 0);
        const int li = b.own_li[t];
        const double4 pi = staged ? lpos[li] : halo_fetch(b, Rp, M, p, li);
        const uint8_t ti = (need_type && staged) ? ltype[li] : b.type[q][t];
        const int si = ti & 0x3F;
        const bool rigid_i = ti & kRigidBit;
        const int n = live ? b.ncount[t] : 0;
        const R fpi = (R)pi.w;
        A = PairAcc();
        const uint4* row = reinterpret_cast<const uint4*>(b.nbr16 + t * (int64_t)rowlen);
        const int nblk = (n + 7) >> 3;
        uint4 cur = row[lane];
        for (int blk = lane; blk < nblk; blk += L) {
            const uint4 nxt = row[blk + L];
            const uint32_t w4[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                double4 ps[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * hf + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    const bool ok = blk * 8 + hf * 4 + u < n;
                    ps[u] = staged ? lpos[ok ? e : li] : halo_fetch(b, Rp, M, p, ok ? e : li);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * hf + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    if (blk * 8 + hf * 4 + u >= n) break;
                    const double4 pj = ps[u];
                    const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < P.rc2)) continue;
                    const double ri = inv_dist<R>(r2);
                    const double r = r2 * ri;
                    const uint8_t tj = need_type ? (staged ? ltype[e] : halo_type(b, M, q, e)) : 0;
                    R g, phi;
                    pair_terms<R, SINGLE, NPK, NDK, EV, ENERGY>(P, G, tf, te, si, tj & 0x3F, r, fpi, (R)pj.w, g, phi);
                    const double s = (double)g * ri;
                    const bool both_rigid = rigid_i && (tj & kRigidBit);
                    accumulate<ENERGY>(A, s, dx, dy, dz, (double)phi, both_rigid);
                    if (pairs && e < n_own) {  // the other atom's share of a pair kept once
                        share(acc + e, -s * dx, b.flags);
                        share(acc + slots + e, -s * dy, b.flags);
                        share(acc + 2 * slots + e, -s * dz, b.flags);
                        if (ENERGY) {
                            share(acc + 3 * slots + e, (double)phi, b.flags);
                            if (!both_rigid) {
                                A.w[0] = fma(s * dx, dx, A.w[0]);
                                A.w[1] = fma(s * dy, dy, A.w[1]);
                                A.w[2] = fma(s * dz, dz, A.w[2]);
                                A.w[3] = fma(s * dx, dy, A.w[3]);
                                A.w[4] = fma(s * dx, dz, A.w[4]);
                                A.w[5] = fma(s * dy, dz, A.w[5]);
                            }
                        }
                    }
                }
            }
            cur = nxt;
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
        if (!pairs && live && lane == 0)
            atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK>(b, p, q, t, n_slots, Rp, P, G, dt, st, pi, ti, A);
    }
    if (pairs) {  // one round: every lane still holds its atom's own sums
        __syncthreads();
        const int a = threadIdx.x / L;
        if (a < n_own && lane == 0) {
            const int64_t t = info.x + a;
            const double4 pi = lpos[a];
            const uint8_t ti = need_type ? ltype[a] : b.type[q][t];
#pragma unroll
            for (int c = 0; c < 3; ++c) A.f[c] += from_fixed(acc[c * slots + a]);
            if (ENERGY) A.epair += from_fixed(acc[3 * slots + a]);
            atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK>(b, p, q, t, n_slots, Rp, P, G, dt, st, pi, ti, A);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
int pair_slots(const KernelShape& k, const PotArgs& P, int precision)
{
    // room for four accumulators per slot (the force pass on energy steps)
    // beside the larger of the passes' staging areas, at most one round of lanes
    const size_t used = std::max(brick_lds_bytes(k, P, precision, 1, 1), brick_lds_bytes(k, P, precision, 2, 1));
    const int64_t room = ((int64_t)k.lds_limit - (int64_t)used) / 32;
    return (int)std::max<int64_t>(0, std::min<int64_t>(k.block / pair_lanes(k), room));
}

static size_t pair_lds_bytes(const KernelShape& k, const PotArgs& P, int precision, int pass, int energy, int slots)
{
    const size_t accb = (size_t)slots * 8 * (pass == 1 ? 1 : (energy ? 4 : 3));
    return brick_lds_bytes(k, P, precision, pass, energy) + accb;
}

template <typename R, bool S, int ND, int EV, int L>
static void pair_density_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                 int precision, int energy, hipStream_t s)
{
    const int slots = pair_slots(k, P, precision);
    hipLaunchKernelGGL((k_pair_density<R, S, ND, EV, L>), dim3(k.n_bricks), dim3(k.block),
                       pair_lds_bytes(k, P, precision, 1, energy, slots), s, b, p, q, k.n_slots, P, energy,
                       k.halo_cap, k.rowlen, slots);
}

template <typename R, bool S, int ND, int EV>
static void pair_density_lanes(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                               int energy, hipStream_t s)
{
    if (pair_lanes(k) == 2) pair_density_variant<R, S, ND, EV, 2>(b, p, q, k, P, precision, energy, s);
    else pair_density_variant<R, S, ND, EV, 1>(b, p, q, k, P, precision, energy, s);
}

template <typename R, bool S>
static void pair_density_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                  int precision, int energy, hipStream_t s)
{
    constexpr bool knots = sizeof(R) == 8;  // knot sums: FP64 only
    if (k.table == 2) pair_density_lanes<R, S, 8, EV_SPLIT>(b, p, q, k, P, precision, energy, s);
    else if (k.table || !knots) pair_density_lanes<R, S, 8, EV_TABLE>(b, p, q, k, P, precision, energy, s);
    else if constexpr (knots) {
        if (k.ndk == 2) pair_density_lanes<R, S, 2, EV_KNOTS>(b, p, q, k, P, precision, energy, s);
        else pair_density_lanes<R, S, 8, EV_KNOTS>(b, p, q, k, P, precision, energy, s);
    }
}

void launch_pair_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                         int energy, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) pair_density_dispatch<float, true>(b, p, q, k, P, precision, energy, s);
        else pair_density_dispatch<float, false>(b, p, q, k, P, precision, energy, s);
    } else {
        if (one) pair_density_dispatch<double, true>(b, p, q, k, P, precision, energy, s);
        else pair_density_dispatch<double, false>(b, p, q, k, P, precision, energy, s);
    }
}

template <typename R, bool S, int NP, int ND, int EV, bool E, bool C, bool O, bool W>
static void pair_force_launch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                              double dt_fs, const md_state& st, hipStream_t s)
{
    const int slots = pair_slots(k, P, precision);
    const size_t lds = pair_lds_bytes(k, P, precision, 2, E, slots);
    if (pair_lanes(k) == 2)
        hipLaunchKernelGGL((k_pair_force<R, S, NP, ND, EV, E, C, O, W, 2>), dim3(k.n_bricks), dim3(k.block), lds, s, b,
                           p, q, k.n_slots, P, dt_fs, st, k.halo_cap, k.rowlen, slots);
    else
        hipLaunchKernelGGL((k_pair_force<R, S, NP, ND, EV, E, C, O, W, 1>), dim3(k.n_bricks), dim3(k.block), lds, s, b,
                           p, q, k.n_slots, P, dt_fs, st, k.halo_cap, k.rowlen, slots);
}

template <typename R, bool S, int NP, int ND, int EV>
static void pair_force_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                               ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    if (!fl.close && !fl.open) {
        if (!fl.writeback)
            pair_force_launch<R, S, NP, ND, EV, false, false, false, false>(b, p, q, k, P, precision, dt_fs, st, s);
        else if (fl.energy)
            pair_force_launch<R, S, NP, ND, EV, true, false, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
        else pair_force_launch<R, S, NP, ND, EV, false, false, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (!fl.close && fl.open) {
        pair_force_launch<R, S, NP, ND, EV, false, false, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (fl.close && fl.open) {
        if (fl.energy)  // per-step energies
            pair_force_launch<R, S, NP, ND, EV, true, true, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
        else pair_force_launch<R, S, NP, ND, EV, false, true, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (!fl.writeback) {
        pair_force_launch<R, S, NP, ND, EV, false, true, false, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else {
        pair_force_launch<R, S, NP, ND, EV, true, true, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
    }
}

template <typename R, bool S>
static void pair_force_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                                ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    constexpr bool knots = sizeof(R) == 8;  // knot sums: FP64 only
    if (k.table == 2) pair_force_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    else if (k.table || !knots) pair_force_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    else if constexpr (knots) {
        if (k.npk == 6 && k.ndk == 2)
            pair_force_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else if (k.npk <= 8 && k.ndk <= 8)
            pair_force_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else if constexpr (S) pair_force_variant<R, S, 16, 4, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    }
}

void launch_pair_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                       ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) pair_force_dispatch<float, true>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else pair_force_dispatch<float, false>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    } else {
        if (one) pair_force_dispatch<double, true>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else pair_force_dispatch<double, false>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    }
}

}  // namespace mdk
