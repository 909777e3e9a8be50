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
// sort because cell contents only change there.  Every neighbour read of the
// three passes is an LDS read: HBM/L2 see each halo atom once per workgroup
// (about 3-5 times the brick's own atoms) instead of one 128-byte line per
// neighbour gather, and no periodic image is computed in the force loop.
#include "md_device.h"

namespace mdk {
namespace {

// Halo bookkeeping of the staged brick (LDS).
struct Halo {
    int32_t cnt[kHaloMax];        // atoms of halo cell h
    int32_t start[kHaloMax + 1];  // first LDS index of halo cell h
    int32_t cstart[kHaloMax];     // first slot of halo cell h
    int32_t code[kHaloMax];       // periodic shift (2 bits per axis: 1 = +L, 2 = -L)
    int32_t hx, hy, hz, H;        // halo extent per axis and cell count
    int32_t cell0;                // first cell of the brick
    int32_t own_begin, own_end;   // slot range of the brick's own atoms
    int32_t total;                // atoms staged
};

__device__ __forceinline__ int brick_of_block()
{
    // same die-aware remap as the slot kernels: each die gets contiguous bricks
    return (int)logical_block();
}

// Fill the halo table and the staged positions.  `with_w` also stages F'.
// A brick whose halo exceeds `cap` stages nothing and is evaluated from global
// memory through the halo table (halo_fetch); flags[F_HALO] counts such
// bricks, a performance (not a correctness) signal.
__device__ void stage_brick(const Buffers& b, const DevReplica& R, int lb, int p, bool with_w, int cap, Halo& M,
                            double4* lpos, int32_t* record = nullptr)
{
    const int tid = threadIdx.x;
    const int bx = lb % R.nbk[0], by = (lb / R.nbk[0]) % R.nbk[1], bz = lb / (R.nbk[0] * R.nbk[1]);
    const int base[3] = {bx * R.bd[0], by * R.bd[1], bz * R.bd[2]};
    int m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) m[a] = min(R.bd[a], R.nc[a] - base[a]);
    const int hx = m[0] + 2, hy = m[1] + 2, hz = m[2] + 2, H = hx * hy * hz;
    if (tid == 0) {
        M.hx = hx;
        M.hy = hy;
        M.hz = hz;
        M.H = H;
        M.cell0 = cell_index(R, base[0], base[1], base[2]);
    }
    for (int h = tid; h < H; h += blockDim.x) {
        const int o[3] = {h % hx - 1, (h / hx) % hy - 1, h / (hx * hy) - 1};
        int c[3], code = 0;
        bool exists = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c[a] = base[a] + o[a];
            if (R.periodic_mask & (1 << a)) {
                if (c[a] < 0) {
                    c[a] += R.nc[a];
                    code |= 2 << (2 * a);
                } else if (c[a] >= R.nc[a]) {
                    c[a] -= R.nc[a];
                    code |= 1 << (2 * a);
                }
            } else if (c[a] < 0 || c[a] >= R.nc[a]) {
                exists = false;
            }
        }
        if (exists) {
            const int cell = cell_index(R, c[0], c[1], c[2]);
            M.cnt[h] = b.cell_count[cell];
            M.cstart[h] = b.cell_start[cell];
        } else {
            M.cnt[h] = 0;
            M.cstart[h] = 0;
        }
        M.code[h] = code;
    }
    __syncthreads();
    if (tid < kWave) {
        // exclusive scan of the halo counts by the first wavefront
        int run = 0;
        for (int h0 = 0; h0 < H; h0 += kWave) {
            const int h = h0 + tid;
            const int v = h < H ? M.cnt[h] : 0;
            int incl = v;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int y = __shfl_up(incl, off, kWave);
                if (tid >= off) incl += y;
            }
            if (h < H) M.start[h] = run + incl - v;
            run += __shfl(incl, kWave - 1, kWave);
        }
        if (tid == 0) {
            M.start[H] = run;
            M.total = run;
            const int last = M.cell0 + R.cpb - 1;
            M.own_begin = b.cell_start[M.cell0];
            M.own_end = b.cell_start[last] + b.cell_count[last];
            if (run > cap) atomicAdd(&b.flags[F_HALO], 1);
        }
    }
    __syncthreads();
    const int total = M.total <= cap ? M.total : 0;
    const double4* __restrict__ pos = b.pos[p];
    for (int i = tid; i < total; i += blockDim.x) {
        // halo cell of staged atom i: last h with start[h] <= i
        int lo = 0, hi = H - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (M.start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        const int slot = M.cstart[lo] + (i - M.start[lo]);
        double4 v = with_w ? pos[slot] : make_double4(0.0, 0.0, 0.0, 0.0);
        if (!with_w) {
            const double3 x = load_xyz(pos, slot);
            v.x = x.x;
            v.y = x.y;
            v.z = x.z;
        }
        const int code = M.code[lo];
        if (code) {
            if (code & 3) v.x += (code & 1) ? R.box[0] : -R.box[0];
            if (code & 12) v.y += (code & 4) ? R.box[1] : -R.box[1];
            if (code & 48) v.z += (code & 16) ? R.box[2] : -R.box[2];
        }
        lpos[i] = v;
        if (record) record[i] = slot | (code << kIndexBits);
    }
    __syncthreads();
}

// Fast staging from the record the list build left: staging position i holds
// slot (src & kIndexMask) shifted by the periodic code (src >> kIndexBits).
// One coalesced read of the record, one gather per atom, no halo search.
__device__ void stage_recorded(const Buffers& b, const DevReplica& R, const int32_t* __restrict__ src, int total,
                               int p, int q, bool with_w, double4* lpos, uint8_t* ltype)
{
    const double4* __restrict__ pos = b.pos[p];
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int e = src[i];
        const int slot = e & kIndexMask, code = (unsigned)e >> kIndexBits;
        double4 v;
        if (with_w) {
            v = pos[slot];
        } else {
            const double3 x = load_xyz(pos, slot);
            v = make_double4(x.x, x.y, x.z, 0.0);
        }
        if (code) {
            if (code & 3) v.x += (code & 1) ? R.box[0] : -R.box[0];
            if (code & 12) v.y += (code & 4) ? R.box[1] : -R.box[1];
            if (code & 48) v.z += (code & 16) ? R.box[2] : -R.box[2];
        }
        lpos[i] = v;
        if (ltype) ltype[i] = b.type[q][slot];
    }
    __syncthreads();
}

// Halo cell and LDS index of an own atom (slot t) of the staged brick.
__device__ __forceinline__ void own_index(const Buffers& b, const DevReplica& R, const Halo& M, int64_t t, int& h,
                                          int& li)
{
    const int local = b.cell_sorted[t] - M.cell0;
    const int lx = local % R.bd[0], ly = (local / R.bd[0]) % R.bd[1], lz = local / (R.bd[0] * R.bd[1]);
    h = ((lz + 1) * M.hy + (ly + 1)) * M.hx + (lx + 1);
    li = M.start[h] + (int)(t - M.cstart[h]);
}

// Slot and periodic shift code of staging position i (binary search over the
// halo cells' first staging positions).
__device__ __forceinline__ int halo_slot(const Halo& M, int i, int& code)
{
    int lo = 0, hi = M.H - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (M.start[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    code = M.code[lo];
    return M.cstart[lo] + (i - M.start[lo]);
}

// Staged atom i read from global memory: the path of a brick whose halo did
// not fit the staging area (same values, same order, only slower).
__device__ __forceinline__ double4 halo_fetch(const Buffers& b, const DevReplica& R, const Halo& M, int p, int i)
{
    int code;
    const int slot = halo_slot(M, i, code);
    double4 v = b.pos[p][slot];
    if (code) {
        if (code & 3) v.x += (code & 1) ? R.box[0] : -R.box[0];
        if (code & 12) v.y += (code & 4) ? R.box[1] : -R.box[1];
        if (code & 48) v.z += (code & 16) ? R.box[2] : -R.box[2];
    }
    return v;
}

__device__ __forceinline__ uint8_t halo_type(const Buffers& b, const Halo& M, int q, int i)
{
    int code;
    return b.type[q][halo_slot(M, i, code)];
}

// ---------------------------------------------------------------------------
// List build: every staged atom in the 27 halo cells around the atom's cell
// with r < r_c + skin (paper, "The Neighbourlist calculation": the cell's
// atoms against those of the cells around it).  Entries are staging (LDS) indices,
// uint16, one row of `rowlen` (a multiple of 8) per atom, written 8 at a time.
__global__ __launch_bounds__(1024) void k_brick_list(Buffers b, int p, int64_t n_slots, int32_t cap, double rlist2,
                                                     int halo_cap, int rowlen)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Halo& M = *reinterpret_cast<Halo*>(smem);
    double4* lpos = reinterpret_cast<double4*>(smem + ((sizeof(Halo) + 15) / 16) * 16);
    const int brick = brick_of_block();
    const DevReplica& R = b.reps[b.brick_rep[brick]];
    stage_brick(b, R, brick - R.brick_off, p, false, halo_cap, M, lpos, b.stage_src + (int64_t)brick * halo_cap);
    const bool staged = M.total <= halo_cap;
    if (threadIdx.x == 0) b.brick_info[brick] = make_int4(M.own_begin, M.own_end, M.total, 0);
    int most = 0;
    for (int64_t t = M.own_begin + threadIdx.x; t < M.own_end; t += blockDim.x) {
        int h, li;
        own_index(b, R, M, t, h, li);
        b.own_li[t] = (uint16_t)li;
        const double4 xi = staged ? lpos[li] : halo_fetch(b, R, M, p, li);
        int count = 0;
        uint4* row = reinterpret_cast<uint4*>(b.nbr16 + t * (int64_t)rowlen);
        uint32_t pk[4] = {0, 0, 0, 0};  // entries buffered until a 16-byte store
        {
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int hh = h + (dz * M.hy + dy) * M.hx + dx;
                        const int beg = M.start[hh], end = beg + M.cnt[hh];
#pragma unroll 4
                        for (int i = beg; i < end; ++i) {
                            if (i == li) continue;
                            const double4 xj = staged ? lpos[i] : halo_fetch(b, R, M, p, i);
                            const double ddx = xj.x - xi.x, ddy = xj.y - xi.y, ddz = xj.z - xi.z;
                            if (ddx * ddx + ddy * ddy + ddz * ddz < rlist2) {
                                if (count < cap) {
                                    const int u = count & 7;
                                    pk[u >> 1] |= (uint32_t)i << (16 * (u & 1));
                                    if (u == 7) {
                                        row[count >> 3] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
                                        pk[0] = pk[1] = pk[2] = pk[3] = 0;
                                    }
                                }
                                ++count;
                            }
                        }
                    }
        }
        const int stored = count < cap ? count : cap;
        if (stored & 7) row[stored >> 3] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        b.ncount[t] = stored;
        most = max(most, count);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) most = max(most, __shfl_xor(most, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && most > 0 && most > b.flags[F_MAX_COUNT])
        atomicMax(&b.flags[F_MAX_COUNT], most);
}

// LDS layout of the density / force kernels: Halo | staged atoms | tables.
__host__ __device__ inline size_t halo_bytes() { return (sizeof(Halo) + 15) / 16 * 16; }

// Stage the species/rigid byte of every staged atom (several species, or
// rigid pairs on energy steps).
__device__ void stage_types(const Buffers& b, int q, const Halo& M, int cap, uint8_t* ltype)
{
    const int total = M.total <= cap ? M.total : 0;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        int lo = 0, hi = M.H - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (M.start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        ltype[i] = b.type[q][M.cstart[lo] + (i - M.start[lo])];
    }
    __syncthreads();
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
    // halo table only (no positions)
    const int lb = brick - R.brick_off;
    const int bx = lb % R.nbk[0], by = (lb / R.nbk[0]) % R.nbk[1], bz = lb / (R.nbk[0] * R.nbk[1]);
    const int base[3] = {bx * R.bd[0], by * R.bd[1], bz * R.bd[2]};
    int m[3];
    for (int a = 0; a < 3; ++a) m[a] = min(R.bd[a], R.nc[a] - base[a]);
    const int hx = m[0] + 2, hy = m[1] + 2, hz = m[2] + 2, H = hx * hy * hz;
    if (threadIdx.x == 0) {
        M.hx = hx;
        M.hy = hy;
        M.hz = hz;
        M.H = H;
        M.cell0 = cell_index(R, base[0], base[1], base[2]);
        int run = 0;
        for (int h = 0; h < H; ++h) {
            const int o[3] = {h % hx - 1, (h / hx) % hy - 1, h / (hx * hy) - 1};
            int c[3];
            bool exists = true;
            for (int a = 0; a < 3; ++a) {
                c[a] = base[a] + o[a];
                if (R.periodic_mask & (1 << a)) c[a] = (c[a] + R.nc[a]) % R.nc[a];
                else if (c[a] < 0 || c[a] >= R.nc[a]) exists = false;
            }
            const int cell = exists ? cell_index(R, c[0], c[1], c[2]) : -1;
            M.cnt[h] = exists ? b.cell_count[cell] : 0;
            M.cstart[h] = exists ? b.cell_start[cell] : 0;
            M.start[h] = run;
            run += M.cnt[h];
        }
        M.start[H] = run;
        const int last = M.cell0 + R.cpb - 1;
        M.own_begin = b.cell_start[M.cell0];
        M.own_end = b.cell_start[last] + b.cell_count[last];
    }
    __syncthreads();
    for (int64_t t = M.own_begin + threadIdx.x; t < M.own_end; t += blockDim.x) {
        const int n = b.ncount[t];
        for (int k = 0; k < n; ++k) {
            const int i = b.nbr16[t * (int64_t)rowlen + k];
            int lo = 0, hi = H - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (M.start[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            b.nbr[(int64_t)k * n_slots + t] = M.cstart[lo] + (i - M.start[lo]);
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

void launch_brick_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, hipStream_t s)
{
    (void)q;
    const size_t lds = halo_bytes() + (size_t)k.halo_cap * sizeof(double4);
    hipLaunchKernelGGL(k_brick_list, dim3(k.n_bricks), dim3(k.block), lds, s, b, p, k.n_slots, k.cap, rlist2,
                       k.halo_cap, k.rowlen);
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
