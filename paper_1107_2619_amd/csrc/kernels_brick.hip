// LDS brick kernels (MD_OPT_KERNEL = 0): the list build, the density pass and
// the force pass with neighbour reads from LDS.  The autotuner picks them where
// they win (FP64 on a large single crystal); the global-gather kernels are the
// default.
//
// The link-cell grid of each replica is cut into bricks (a few cells per axis;
// see cell_index in md_internal.h) and one workgroup owns one brick.  It first
// stages into LDS the positions of every atom of the brick and of the one-cell
// halo around it, cell by cell in a fixed order, each halo cell shifted into
// the brick's periodic frame.  The Verlet list of an atom then stores 16-bit
// LDS indices into that staging order, which stays valid until the next cell
// sort because cell contents only change there (staging order: the brick's
// own atoms first, then the halo ring; brick_common.h).  Every neighbour read
// of the three passes is an LDS read: HBM/L2 see each halo atom once per workgroup
// (about 3-5 times the brick's own atoms) instead of one 128-byte line per
// neighbour gather, and no periodic image is computed in the force loop.
#include <algorithm>

#include "brick_common.h"

namespace mdk {
namespace {

// ---------------------------------------------------------------------------
// List build (paper, "The Neighbourlist calculation": every atom of a link
// cell against the atoms of the 27 cells around it, r < r_c + skin).  One
// wavefront per own cell of the brick: its lanes hold up to 64 candidates at a
// time from the 27 cells (staging order), and each atom of the cell is tested
// against them in turn, the in-range lanes packed with a ballot.  Entries are
// staging (LDS) indices, uint16, collected per atom in an LDS row and written
// out once per cell: the cell's atoms are consecutive slots, so their rows are
// one contiguous run of global memory.  half = 1 keeps a pair of two own
// atoms once, in the row of the one with the smaller staging index (the pair
// kernels then add its share to both atoms); pairs with a halo atom are kept
// in full, since the other atom's brick keeps them too.  A brick keeps full
// rows instead (brick_info.w = 0) when its halo did not fit the staging area
// or it holds more than pair_slots own atoms (one pair-kernel round).
constexpr int kListBlock = 1024;  // threads per list-build workgroup
constexpr int kListPasses = 4;    // candidates per lane held in registers
constexpr int kRowAtoms = 16;    // most atoms of one cell whose rows a wavefront collects at a time

__global__ __launch_bounds__(kListBlock) void k_brick_list(Buffers b, int p, int64_t n_slots, int32_t cap,
                                                           double rlist2, int halo_cap, int rowlen, int row_atoms,
                                                           int half, int pair_slots)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + ((sizeof(Halo) + 15) / 16) * 16);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave, n_waves = blockDim.x / kWave;
    uint16_t* rows = reinterpret_cast<uint16_t*>(lpos + halo_cap) + (size_t)wave * row_atoms * rowlen;
    const int brick = brick_of_block();
    const DevReplica& R = b.reps[b.brick_rep[brick]];
    stage_brick(b, R, brick - R.brick_off, p, false, halo_cap, M, lpos, b.stage_src + (int64_t)brick * halo_cap);
    const bool staged = M.total <= halo_cap;
    const int n_own = M.own_end - M.own_begin;
    half = half && staged && n_own <= pair_slots;
    if (threadIdx.x == 0) b.brick_info[brick] = make_int4(M.own_begin, M.own_end, M.total, half);
    for (int a = threadIdx.x; a < n_own; a += blockDim.x) b.own_li[M.own_begin + a] = (uint16_t)a;
    int most = 0;
    const int n_cells = M.m[0] * M.m[1] * M.m[2];
    for (int lc = wave; lc < n_cells; lc += n_waves) {
        const int lx = lc % M.m[0], ly = (lc / M.m[0]) % M.m[1], lz = lc / (M.m[0] * M.m[1]);
        const int h = ((lz + 1) * M.hy + (ly + 1)) * M.hx + (lx + 1);
        const int n_cell = M.cnt[h], s_cell = M.start[h];
        if (n_cell == 0) continue;
        // lane k < 27: neighbour cell k of the stencil, its staging range
        int nb_start = 0, nb_count = 0;
        if (lane < 27) {
            const int hh = h + ((lane / 9 - 1) * M.hy + (lane / 3 % 3 - 1)) * M.hx + (lane % 3 - 1);
            nb_start = M.start[hh];
            nb_count = M.cnt[hh];
        }
        int incl = nb_count;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int v = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += v;
        }
        const int excl = incl - nb_count;
        const int total = uniform(__shfl(incl, kWave - 1, kWave));
        for (int i0 = 0; i0 < n_cell; i0 += row_atoms) {
            const int nn = min(row_atoms, n_cell - i0);
            // lane ii < nn holds atom i0 + ii of the cell; the tests broadcast it
            const int l0 = s_cell + i0 + min(lane, nn - 1);
            const double4 xl = staged ? lpos[l0] : halo_fetch(b, R, M, p, l0);
            int my_count = 0;  // lane ii: entries of atom i0 + ii so far
            for (int g0 = 0; g0 < total; g0 += kWave * kListPasses) {
                // kListPasses candidates per lane: the stencil cell holding candidate
                // m is the last k with excl_k <= m (lanes past the stencil hold
                // excl = total, so k stays below 27)
                double cx[kListPasses], cy[kListPasses], cz[kListPasses];
                int ce[kListPasses];
                bool live[kListPasses];
#pragma unroll
                for (int u = 0; u < kListPasses; ++u) {
                    const int m0 = g0 + u * kWave + lane;
                    const int m = min(m0, total - 1);
                    int k = 0;
#pragma unroll
                    for (int step = kWave / 2; step > 0; step >>= 1)
                        if (__shfl(excl, k + step, kWave) <= m) k += step;
                    const int e = __shfl(nb_start, k, kWave) + (m - __shfl(excl, k, kWave));
                    const double4 xj = staged ? lpos[e] : halo_fetch(b, R, M, p, e);
                    cx[u] = xj.x;
                    cy[u] = xj.y;
                    cz[u] = xj.z;
                    ce[u] = e;
                    live[u] = m0 < total;
                }
                for (int ii = 0; ii < nn; ++ii) {
                    const int li = s_cell + i0 + ii;
                    const double xi = bcast_lane(xl.x, ii), yi = bcast_lane(xl.y, ii), zi = bcast_lane(xl.z, ii);
                    int base = __builtin_amdgcn_readlane(my_count, ii);
#pragma unroll
                    for (int u = 0; u < kListPasses; ++u) {
                        const double dx = cx[u] - xi, dy = cy[u] - yi, dz = cz[u] - zi;
                        bool take = live[u] && ce[u] != li && dx * dx + dy * dy + dz * dz < rlist2;
                        if (half) take = take && (ce[u] >= n_own || ce[u] > li);
                        const uint64_t mask = __ballot(take);
                        if (mask == 0) continue;
                        const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
                        if (take && base + rank < cap) rows[ii * rowlen + base + rank] = (uint16_t)ce[u];
                        base += __popcll(mask);
                    }
                    if (lane == ii) my_count = base;
                }
            }
            // counts, and the rows of these atoms: one contiguous run of nn rows
            const int64_t t0 = (int64_t)M.own_begin + s_cell + i0;
            if (lane < nn) {
                b.ncount[t0 + lane] = min(my_count, cap);
                most = max(most, my_count);
            }
            const uint4* src = reinterpret_cast<const uint4*>(rows);
            uint4* dst = reinterpret_cast<uint4*>(b.nbr16 + t0 * rowlen);
            for (int c = lane; c < nn * rowlen / 8; c += kWave) dst[c] = src[c];
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) most = max(most, __shfl_xor(most, off, kWave));
    if (lane == 0 && most > 0 && most > b.flags[F_MAX_COUNT]) atomicMax(&b.flags[F_MAX_COUNT], most);
}

// ---------------------------------------------------------------------------
// Density pass over the brick (arithmetic as in k_density).  L lanes share an
// atom: lane l takes list entries l, l + L, ...; the partial sums meet in a
// cross-lane reduction.
template <typename R, bool SINGLE, int NDK, int EV, int L>
__global__ __launch_bounds__(1024) void k_brick_density(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                        int energy, int halo_cap, int rowlen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + halo_bytes());
    unsigned char* tail = smem + halo_bytes() + (size_t)halo_cap * sizeof(double4);
    const R* tab = tables<R>(b).dens;
    uint8_t* ltype = reinterpret_cast<uint8_t*>(tail);
    if (EV != EV_KNOTS && SINGLE) {
        R* s = reinterpret_cast<R*>(tail);
        lds_fill(s, tab, P.nbt * value_stride(EV));
        tab = s;
    } else if (EV != EV_KNOTS) {
        ltype = reinterpret_cast<uint8_t*>(tail);
    }
    const int brick = brick_of_block();
    const DevReplica& Rp = b.reps[b.brick_rep[brick]];
    const int4 info = b.brick_info[brick];  // own slot range and halo size at the last build
    const bool staged = info.z <= halo_cap;
    if (staged) {
        stage_recorded(b, Rp, b.stage_src + (int64_t)brick * halo_cap, info.z, p, q, false, lpos,
                       SINGLE ? nullptr : ltype);
    } else {
        stage_brick(b, Rp, brick - Rp.brick_off, p, false, halo_cap, M, lpos);  // halo table for halo_fetch
    }
    const DevPotential& G = *b.pot;
    const int lane = threadIdx.x % L;
    const int n_own = info.y - info.x;
    // every lane group runs the same number of rounds (the cross-lane sums
    // need whole wavefronts); atoms past the end are masked
    const int per_round = blockDim.x / L;
    for (int a0 = 0; a0 < n_own; a0 += per_round) {
        const int a = a0 + threadIdx.x / L;
        const bool live = a < n_own;
        const int64_t t = info.x + (live ? a : 0);
        const int li = b.own_li[t];
        const double4 xi = staged ? lpos[li] : halo_fetch(b, Rp, M, p, li);
        const int si = SINGLE ? 0 : ((staged ? ltype[li] : halo_type(b, M, q, li)) & 0x3F);
        const int n = live ? b.ncount[t] : 0;
        double rho = 0.0;
        // lane l takes the 8-entry blocks l, l + L, ... of the atom's row; the
        // next block's 16-byte load is issued before the current one is used
        const uint4* row = reinterpret_cast<const uint4*>(b.nbr16 + t * (int64_t)rowlen);
        const int nblk = (n + 7) >> 3;
        uint4 cur = row[lane];  // rows are padded: loads past the list are harmless
        for (int blk = lane; blk < nblk; blk += L) {
            const uint4 nxt = row[blk + L];
            const uint32_t w4[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                double4 xs[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * half + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    const bool ok = blk * 8 + half * 4 + u < n;
                    xs[u] = staged ? lpos[ok ? e : li] : halo_fetch(b, Rp, M, p, ok ? e : li);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * half + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    if (blk * 8 + half * 4 + u >= n) break;
                    const double dx = xs[u].x - xi.x, dy = xs[u].y - xi.y, dz = xs[u].z - xi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < P.rc2)) continue;
                    const double r = r2 * inv_dist<R>(r2);
                    const int sj = SINGLE ? 0 : ((staged ? ltype[e] : halo_type(b, M, q, e)) & 0x3F);
                    rho += (double)density_term<R, SINGLE, NDK, EV>(P, G, tab, si, sj, r);
                }
            }
            cur = nxt;
        }
        rho = lane_sum<L>(rho);
        if (live && lane == 0) {
            double F, dF;
            embed(SINGLE ? P.emb_c : G.emb_c[si], rho, F, dF);
            reinterpret_cast<double*>(b.pos[p] + t)[3] = dF;
            if (energy) b.femb[t] = F;
        }
    }
}

// ---------------------------------------------------------------------------
// Force pass + velocity Verlet over the brick (arithmetic as in k_force).
// Staged atoms carry F' in .w.
template <typename R, bool SINGLE, int NPK, int NDK, int EV, bool ENERGY, bool CLOSE, bool OPEN, bool WRITEBACK, int L>
__global__ __launch_bounds__(1024) void k_brick_force(Buffers b, int p, int q, int64_t n_slots, PotArgs P,
                                                      double dt, md_state st, int halo_cap, int rowlen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + halo_bytes());
    unsigned char* tail = smem + halo_bytes() + (size_t)halo_cap * sizeof(double4);
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
    if (staged) {
        stage_recorded(b, Rp, b.stage_src + (int64_t)brick * halo_cap, info.z, p, q, true, lpos,
                       need_type ? ltype : nullptr);
    } else {
        stage_brick(b, Rp, brick - Rp.brick_off, p, true, halo_cap, M, lpos);
    }
    const DevPotential& G = *b.pot;
    const int lane = threadIdx.x % L;
    const int n_own = info.y - info.x;
    const int per_round = blockDim.x / L;
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
        PairAcc A;
        const uint4* row = reinterpret_cast<const uint4*>(b.nbr16 + t * (int64_t)rowlen);
        const int nblk = (n + 7) >> 3;
        uint4 cur = row[lane];  // rows are padded: loads past the list are harmless
        for (int blk = lane; blk < nblk; blk += L) {
            const uint4 nxt = row[blk + L];
            const uint32_t w4[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                double4 ps[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * half + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    const bool ok = blk * 8 + half * 4 + u < n;
                    ps[u] = staged ? lpos[ok ? e : li] : halo_fetch(b, Rp, M, p, ok ? e : li);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = (w4[2 * half + (u >> 1)] >> (16 * (u & 1))) & 0xFFFF;
                    if (blk * 8 + half * 4 + u >= n) break;
                    const double4 pj = ps[u];
                    const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < P.rc2)) continue;
                    const double ri = inv_dist<R>(r2);
                    const double r = r2 * ri;
                    const uint8_t tj = need_type ? (staged ? ltype[e] : halo_type(b, M, q, e)) : 0;
                    R g, phi;
                    pair_terms<R, SINGLE, NPK, NDK, EV, ENERGY>(P, G, tf, te, si, tj & 0x3F, r, fpi, (R)pj.w, g, phi);
                    accumulate<ENERGY>(A, (double)g * ri, dx, dy, dz, (double)phi, rigid_i && (tj & kRigidBit));
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
        // own cells are never shifted, so pi is the atom's own position
        if (live && lane == 0)
            atom_epilogue<SINGLE, ENERGY, CLOSE, OPEN, WRITEBACK>(b, p, q, t, n_slots, Rp, P, G, dt, st, pi, ti, A);
    }
}

// LDS index -> slot for every list entry (md_copy_neighbours, tests): writes
// the global-slot list `nbr` from the brick list `nbr16`.
__global__ __launch_bounds__(1024) void k_brick_list_to_slots(Buffers b, int64_t n_slots, int rowlen)
{
    __shared__ Halo M;
    const int brick = brick_of_block();
    const DevReplica& R = b.reps[b.brick_rep[brick]];
    halo_table(b, R, brick - R.brick_off, M);
    for (int64_t t = M.own_begin + threadIdx.x; t < M.own_end; t += blockDim.x) {
        const int n = b.ncount[t];
        for (int k = 0; k < n; ++k) {
            int code;
            b.nbr[nbr_at(k, t, n_slots)] = halo_slot(M, b.nbr16[t * (int64_t)rowlen + k], code);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
size_t brick_lds_bytes(const KernelShape& k, const PotArgs& P, int precision, int pass, int energy)
{
    // pass 0: list build, 1: density, 2: force; every pass may stage one
    // type byte per atom after the tables
    const size_t rsz = precision == MD_MIXED ? 4 : 8;
    size_t bytes = halo_bytes() + (size_t)k.halo_cap * sizeof(double4);
    if (pass == 1 && k.table && P.ns == 1) bytes += (size_t)P.nbt * value_stride(k.table) * rsz;
    if (pass == 2 && k.table && P.ns == 1)
        bytes += (size_t)P.nbt * (force_stride(k.table) + (energy ? value_stride(k.table) : 0)) * rsz;
    if (pass > 0) bytes += (size_t)k.halo_cap;
    return bytes;
}

// half: pairs once, for bricks with at most pair_slots own atoms (pair_slots())
void launch_brick_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, int half,
                       int pair_slots, hipStream_t s)
{
    (void)q;
    const size_t base = halo_bytes() + (size_t)k.halo_cap * sizeof(double4);
    // rows collected per wavefront: as many atoms of a cell as the LDS left allows, up to kRowAtoms
    const size_t per_atom = (size_t)(kListBlock / kWave) * k.rowlen * sizeof(uint16_t);
    const int row_atoms = (int)std::max<int64_t>(
        1, std::min<int64_t>(kRowAtoms, ((int64_t)k.lds_limit - (int64_t)base) / (int64_t)per_atom));
    const size_t lds = base + (size_t)row_atoms * per_atom;
    hipLaunchKernelGGL(k_brick_list, dim3(k.n_bricks), dim3(kListBlock), lds, s, b, p, k.n_slots, k.cap, rlist2,
                       k.halo_cap, k.rowlen, row_atoms, half, pair_slots);
}

template <typename R, bool S, int ND, int EV, int L>
static void brick_density_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                  int precision, int energy, hipStream_t s)
{
    hipLaunchKernelGGL((k_brick_density<R, S, ND, EV, L>), dim3(k.n_bricks), dim3(k.block),
                       brick_lds_bytes(k, P, precision, 1, energy), s, b, p, q, k.n_slots, P, energy, k.halo_cap,
                       k.rowlen);
}

template <typename R, bool S, int ND, int EV>
static void brick_density_lanes(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                int precision, int energy, hipStream_t s)
{
    if (k.lanes == 4) brick_density_variant<R, S, ND, EV, 4>(b, p, q, k, P, precision, energy, s);
    else if (k.lanes == 2) brick_density_variant<R, S, ND, EV, 2>(b, p, q, k, P, precision, energy, s);
    else brick_density_variant<R, S, ND, EV, 1>(b, p, q, k, P, precision, energy, s);
}

template <typename R, bool S>
static void brick_density_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                   int precision, int energy, hipStream_t s)
{
    constexpr bool knots = sizeof(R) == 8;  // knot sums: FP64 only
    if (k.table == 2) brick_density_lanes<R, S, 8, EV_SPLIT>(b, p, q, k, P, precision, energy, s);
    else if (k.table || !knots) brick_density_lanes<R, S, 8, EV_TABLE>(b, p, q, k, P, precision, energy, s);
    else if constexpr (knots) {
        if (k.ndk == 2) brick_density_lanes<R, S, 2, EV_KNOTS>(b, p, q, k, P, precision, energy, s);
        else brick_density_lanes<R, S, 8, EV_KNOTS>(b, p, q, k, P, precision, energy, s);
    }
}

void launch_brick_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                          int energy, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) brick_density_dispatch<float, true>(b, p, q, k, P, precision, energy, s);
        else brick_density_dispatch<float, false>(b, p, q, k, P, precision, energy, s);
    } else {
        if (one) brick_density_dispatch<double, true>(b, p, q, k, P, precision, energy, s);
        else brick_density_dispatch<double, false>(b, p, q, k, P, precision, energy, s);
    }
}

template <typename R, bool S, int NP, int ND, int EV, bool E, bool C, bool O, bool W>
static void brick_force_launch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                               double dt_fs, const md_state& st, hipStream_t s)
{
    const size_t lds = brick_lds_bytes(k, P, precision, 2, E);
    if (k.lanes == 4)
        hipLaunchKernelGGL((k_brick_force<R, S, NP, ND, EV, E, C, O, W, 4>), dim3(k.n_bricks), dim3(k.block), lds, s, b,
                           p, q, k.n_slots, P, dt_fs, st, k.halo_cap, k.rowlen);
    else if (k.lanes == 2)
        hipLaunchKernelGGL((k_brick_force<R, S, NP, ND, EV, E, C, O, W, 2>), dim3(k.n_bricks), dim3(k.block), lds, s, b,
                           p, q, k.n_slots, P, dt_fs, st, k.halo_cap, k.rowlen);
    else
        hipLaunchKernelGGL((k_brick_force<R, S, NP, ND, EV, E, C, O, W, 1>), dim3(k.n_bricks), dim3(k.block), lds, s, b,
                           p, q, k.n_slots, P, dt_fs, st, k.halo_cap, k.rowlen);
}

template <typename R, bool S, int NP, int ND, int EV>
static void brick_force_variant(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                int precision, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    if (!fl.close && !fl.open) {
        if (!fl.writeback)
            brick_force_launch<R, S, NP, ND, EV, false, false, false, false>(b, p, q, k, P, precision, dt_fs, st, s);
        else if (fl.energy) brick_force_launch<R, S, NP, ND, EV, true, false, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
        else brick_force_launch<R, S, NP, ND, EV, false, false, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (!fl.close && fl.open) {
        brick_force_launch<R, S, NP, ND, EV, false, false, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (fl.close && fl.open) {
        if (fl.energy)  // per-step energies
            brick_force_launch<R, S, NP, ND, EV, true, true, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
        else brick_force_launch<R, S, NP, ND, EV, false, true, true, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else if (!fl.writeback) {
        brick_force_launch<R, S, NP, ND, EV, false, true, false, false>(b, p, q, k, P, precision, dt_fs, st, s);
    } else {
        brick_force_launch<R, S, NP, ND, EV, true, true, false, true>(b, p, q, k, P, precision, dt_fs, st, s);
    }
}

template <typename R, bool S>
static void brick_force_dispatch(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P,
                                 int precision, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    constexpr bool knots = sizeof(R) == 8;  // knot sums: FP64 only
    if (k.table == 2) brick_force_variant<R, S, 8, 8, EV_SPLIT>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    else if (k.table || !knots) brick_force_variant<R, S, 8, 8, EV_TABLE>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    else if constexpr (knots) {
        if (k.npk == 6 && k.ndk == 2)
            brick_force_variant<R, S, 6, 2, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else if (k.npk <= 8 && k.ndk <= 8)
            brick_force_variant<R, S, 8, 8, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else if constexpr (S) brick_force_variant<R, S, 16, 4, EV_KNOTS>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    }
}

void launch_brick_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                        ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s)
{
    const bool one = P.ns == 1;
    if (precision == MD_MIXED) {
        if (one) brick_force_dispatch<float, true>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else brick_force_dispatch<float, false>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    } else {
        if (one) brick_force_dispatch<double, true>(b, p, q, k, P, precision, fl, dt_fs, st, s);
        else brick_force_dispatch<double, false>(b, p, q, k, P, precision, fl, dt_fs, st, s);
    }
}

void launch_brick_list_to_slots(const Buffers& b, const KernelShape& k, hipStream_t s)
{
    hipLaunchKernelGGL(k_brick_list_to_slots, dim3(k.n_bricks), dim3(k.block), 0, s, b, k.n_slots, k.rowlen);
}

}  // namespace mdk
