// gfx950 kernels of the embedded-atom force loop.
//
// Global-gather kernels (the list build is in kernels_build.hip).  Data
// layout (all in the caller-provided workspace, see md_runtime.hip):
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
typedef int int4v __attribute__((ext_vector_type(4)));

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
