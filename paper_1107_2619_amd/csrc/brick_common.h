// Link-cell bricks staged in LDS: the halo table, the staging of a brick's own
// and halo atoms, and the accessors the LDS-brick kernel families share (the
// list build and the full-list passes in kernels_brick.hip, the pair passes in
// kernels_pairs.hip).
#pragma once

#include "md_device.h"

namespace mdk {
namespace {

// Halo bookkeeping of the staged brick (LDS).  Staging order: the brick's
// own atoms first, in slot order (own atom t at staging index t - own_begin),
// then the atoms of the ring of halo cells around the brick, cell by cell in
// halo-grid order (x fastest).
struct Halo {
    int32_t cnt[kHaloMax];             // atoms of halo cell h
    int32_t start[kHaloMax];           // first staging index of halo cell h
    int32_t cstart[kHaloMax];          // first slot of halo cell h
    int32_t code[kHaloMax];            // periodic shift (2 bits per axis: 1 = +L, 2 = -L)
    int32_t ring_start[kHaloMax + 1];  // first staging index of the k-th ring cell; [nring] = total
    int16_t ring_h[kHaloMax];          // halo cell of the k-th ring cell
    int32_t hx, hy, hz, H, nring;      // halo extent per axis, cell count, ring cells
    int32_t m[3];                      // own cells per axis (the last brick of an axis may be partial)
    int32_t cell0;                     // first cell of the brick
    int32_t own_begin, own_end;        // slot range of the brick's own atoms
    int32_t total;                     // atoms staged
};
static_assert(sizeof(Halo) <= kHaloTableBytes, "halo table exceeds its LDS budget");

__device__ __forceinline__ int brick_of_block()
{
    // same die-aware remap as the slot kernels: each die gets contiguous bricks
    return (int)logical_block();
}

__device__ __forceinline__ bool interior(const Halo& M, int h)
{
    const int ox = h % M.hx - 1, oy = (h / M.hx) % M.hy - 1, oz = h / (M.hx * M.hy) - 1;
    return ox >= 0 && ox < M.m[0] && oy >= 0 && oy < M.m[1] && oz >= 0 && oz < M.m[2];
}

// Slot and periodic shift code of staging position i.
__device__ __forceinline__ int halo_slot(const Halo& M, int i, int& code)
{
    const int n_own = M.own_end - M.own_begin;
    if (i < n_own) {
        code = 0;
        return M.own_begin + i;
    }
    int lo = 0, hi = M.nring - 1;  // last ring cell whose first staging index is <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (M.ring_start[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int h = M.ring_h[lo];
    code = M.code[h];
    return M.cstart[h] + (i - M.ring_start[lo]);
}

__device__ __forceinline__ double4 shifted(const DevReplica& R, double4 v, int code)
{
    if (code) {
        if (code & 3) v.x += (code & 1) ? R.box[0] : -R.box[0];
        if (code & 12) v.y += (code & 4) ? R.box[1] : -R.box[1];
        if (code & 48) v.z += (code & 16) ? R.box[2] : -R.box[2];
    }
    return v;
}

// Fill the halo table and the staged positions.  `with_w` also stages F'.
// A brick whose halo exceeds `cap` stages nothing and is evaluated from global
// memory through the halo table (halo_fetch); flags[F_HALO] counts such
// bricks, a performance (not a correctness) signal.
__device__ void halo_table(const Buffers& b, const DevReplica& R, int lb, Halo& M)
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
        for (int a = 0; a < 3; ++a) M.m[a] = m[a];
        M.cell0 = cell_index(R, base[0], base[1], base[2]);
        const int last = M.cell0 + R.cpb - 1;
        M.own_begin = b.cell_start[M.cell0];
        M.own_end = b.cell_start[last] + b.cell_count[last];
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
        // own cells index straight into the slot range; ring cells follow the
        // own atoms in halo order (an exclusive scan by the first wavefront)
        const int n_own = M.own_end - M.own_begin;
        int run = n_own, nring = 0;
        for (int h0 = 0; h0 < H; h0 += kWave) {
            const int h = h0 + tid;
            const bool in = h < H;
            const bool ring = in && !interior(M, h);
            const int v = ring ? M.cnt[h] : 0;
            int incl = v;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int y = __shfl_up(incl, off, kWave);
                if (tid >= off) incl += y;
            }
            const uint64_t rmask = __ballot(ring);
            const int rk = nring + __popcll(rmask & ((1ull << tid) - 1));
            if (ring) {
                M.start[h] = run + incl - v;
                M.ring_start[rk] = run + incl - v;
                M.ring_h[rk] = (int16_t)h;
            } else if (in) {
                M.start[h] = M.cstart[h] - M.own_begin;
            }
            run += __shfl(incl, kWave - 1, kWave);
            nring += __popcll(rmask);
        }
        if (tid == 0) {
            M.nring = nring;
            M.ring_start[nring] = run;
            M.total = run;
        }
    }
    __syncthreads();
}

__device__ void stage_brick(const Buffers& b, const DevReplica& R, int lb, int p, bool with_w, int cap, Halo& M,
                            double4* lpos, int32_t* record = nullptr)
{
    const int tid = threadIdx.x;
    halo_table(b, R, lb, M);
    if (tid == 0 && M.total > cap) atomicAdd(&b.flags[F_HALO], 1);
    const int total = M.total <= cap ? M.total : 0;
    const double4* __restrict__ pos = b.pos[p];
    for (int i = tid; i < total; i += blockDim.x) {
        int code;
        const int slot = halo_slot(M, i, code);
        double4 v = with_w ? pos[slot] : make_double4(0.0, 0.0, 0.0, 0.0);
        if (!with_w) {
            const double3 x = load_xyz(pos, slot);
            v.x = x.x;
            v.y = x.y;
            v.z = x.z;
        }
        lpos[i] = shifted(R, v, code);
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
        lpos[i] = shifted(R, v, code);
        if (ltype) ltype[i] = b.type[q][slot];
    }
    __syncthreads();
}

// Staged atom i read from global memory: the path of a brick whose halo did
// not fit the staging area (same values, same order, only slower).
__device__ __forceinline__ double4 halo_fetch(const Buffers& b, const DevReplica& R, const Halo& M, int p, int i)
{
    int code;
    const int slot = halo_slot(M, i, code);
    return shifted(R, b.pos[p][slot], code);
}

__device__ __forceinline__ uint8_t halo_type(const Buffers& b, const Halo& M, int q, int i)
{
    int code;
    return b.type[q][halo_slot(M, i, code)];
}

// LDS layout of the density / force kernels: Halo | staged atoms | tables.
__host__ __device__ inline size_t halo_bytes() { return (sizeof(Halo) + 15) / 16 * 16; }

// Stage the species/rigid byte of every staged atom (several species, or
// rigid pairs on energy steps).
__device__ void stage_types(const Buffers& b, int q, const Halo& M, int cap, uint8_t* ltype)
{
    const int total = M.total <= cap ? M.total : 0;
    for (int i = threadIdx.x; i < total; i += blockDim.x) ltype[i] = halo_type(b, M, q, i);
    __syncthreads();
}


}  // namespace
}  // namespace mdk
