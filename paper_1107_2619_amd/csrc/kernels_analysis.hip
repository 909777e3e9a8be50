// Mean square displacement per replica and species (paper, "Self-diffusion in
// iron": the diffusion coefficient is the long-time slope of the displacement
// squared, averaged over atoms, divided by 6).  Positions are stored without
// wraparound ("Boundary conditions"), so a displacement is the plain
// difference between the caller's current positions and the origin positions.
//
// Both arrays are read in caller order, where each replica's atoms are one
// contiguous range: the reads are fully coalesced and need no slot mapping.
// Two fixed-order stages (per chunk of kReduceChunk atoms, then per replica)
// make every replica's result independent of the batch around it.
#include "md_device.h"

namespace mdk {
namespace {

constexpr int kMsdValues = 2 * MD_MAX_SPECIES;  // {sum of d^2, count} per species

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}

// First stage: one workgroup per chunk of one replica's atoms.
__global__ __launch_bounds__(kBlock) void k_msd_chunks(Buffers b, md_state st)
{
    __shared__ double sh[kBlock / kWave][kMsdValues];
    const int c = blockIdx.x;
    const int r = b.chunk_rep[c];
    const DevReplica& R = b.reps[r];
    const int64_t a0 = R.atom_off + (int64_t)(c - b.chunk_off[r]) * kReduceChunk;
    const int64_t a1 = min(a0 + (int64_t)kReduceChunk, (int64_t)R.atom_off + R.n_atoms);
    double v[kMsdValues];
#pragma unroll
    for (int k = 0; k < kMsdValues; ++k) v[k] = 0.0;
    for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) {
        const uint8_t ty = b.ctype[i];
        if (ty & kRigidBit) continue;
        const double dx = st.x[i] - b.x0[0][i];
        const double dy = st.y[i] - b.x0[1][i];
        const double dz = st.z[i] - b.x0[2][i];
        const double d2 = dx * dx + dy * dy + dz * dz;
        const int s = ty & 0x3F;
        // select by comparison: a register array indexed at run time would spill
#pragma unroll
        for (int k = 0; k < MD_MAX_SPECIES; ++k) {
            v[k] += k == s ? d2 : 0.0;
            v[MD_MAX_SPECIES + k] += k == s ? 1.0 : 0.0;
        }
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kMsdValues; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) sh[wave][k] = w;
    }
    __syncthreads();
    if (threadIdx.x < kMsdValues) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][threadIdx.x];
        b.msd_partial[(int64_t)c * kMsdValues + threadIdx.x] = t;
    }
}

// Second stage: one thread per (replica, species) sums that replica's chunks in
// order and divides; msd_out[r] = {msd[MD_MAX_SPECIES], count[MD_MAX_SPECIES]}.
__global__ void k_msd_replicas(Buffers b, int n_replicas)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_replicas * MD_MAX_SPECIES) return;
    const int r = t / MD_MAX_SPECIES, s = t % MD_MAX_SPECIES;
    double sum = 0.0, cnt = 0.0;
    for (int c = b.chunk_off[r]; c < b.chunk_off[r + 1]; ++c) {
        sum += b.msd_partial[(int64_t)c * kMsdValues + s];
        cnt += b.msd_partial[(int64_t)c * kMsdValues + MD_MAX_SPECIES + s];
    }
    b.msd_out[(int64_t)r * kMsdValues + s] = cnt > 0.0 ? sum / cnt : 0.0;
    b.msd_out[(int64_t)r * kMsdValues + MD_MAX_SPECIES + s] = cnt;
}

// Per-replica results in the caller's layout: msd[r * ns + s] and the counts
// as int64 (for copies straight into the caller's host arrays).
__global__ void k_msd_pack(const double* __restrict__ out, int n_replicas, int ns, double* __restrict__ msd,
                           int64_t* __restrict__ count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_replicas * ns) return;
    const int r = t / ns, s = t % ns;
    msd[t] = out[(int64_t)r * kMsdValues + s];
    count[t] = (int64_t)out[(int64_t)r * kMsdValues + MD_MAX_SPECIES + s];
}

}  // namespace

void launch_msd_pack(const double* out, int n_replicas, int ns, double* msd, int64_t* count, hipStream_t s)
{
    const int n = n_replicas * ns;
    hipLaunchKernelGGL(k_msd_pack, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, out, n_replicas, ns, msd,
                       count);
}

void launch_msd(const Buffers& b, const KernelShape& k, const md_state& st, hipStream_t s)
{
    if (k.n_chunks > 0) hipLaunchKernelGGL(k_msd_chunks, dim3(k.n_chunks), dim3(kBlock), 0, s, b, st);
    const int n = k.n_replicas * MD_MAX_SPECIES;
    hipLaunchKernelGGL(k_msd_replicas, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, b, k.n_replicas);
}

}  // namespace mdk
