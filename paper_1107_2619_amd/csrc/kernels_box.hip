// Parrinello-Rahman dynamics of the full box matrix (paper, "Barostat NPTp":
// nine box degrees of freedom, external pressure P and external stress S).
//
// With r = o + h s, v = h ds/dt and the internal stress
// pi = (sum m v v^T + W) / Omega, the equations of motion are
//   W d2h/dt2 = (pi - P) sigma - h Sigma,   sigma = Omega h^-T,
//   dv/dt = f/m - h^-T (dh/dt)^T v,   dr/dt = v + (dh/dt) h^-1 (r - o),
// with Sigma = Omega0 h0^-1 (S - P) h0^-T fixed by the reference box h0 (the
// box at md_bind).  A step composes exact sub-flows symmetrically: box half
// kick, thermostat half step (NPT), friction half step
// v <- exp(-(dt/2) h^-T (dh/dt)^T) v, velocity half kick, drift of positions
// and box with dh/dt held, forces, and the mirror image.  The drift maps
// r - o to h' h^-1 (r - o) + dt h' phi(dt h^-1 dh/dt) h^-1 v, h' = h + dt dh/dt,
// phi(z) = z^-1 log(1 + z): the integral of ds/dt = (h + t dh/dt)^-1 v.
//
// As in the orthorhombic barostat, the force pass ends with the closing kick
// and keeps f; here it also writes the whole per-atom virial.  One wavefront
// pass sums m v v^T and the virial; one workgroup per replica then does the
// 3x3 arithmetic on a single lane and leaves the velocity maps and the drift
// matrices for the streaming passes.
#include "md_device.h"

namespace mdk {
namespace {

// 3x3 matrices, row-major.
struct M3 {
    double e[9];
};

__device__ M3 m3_identity()
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = (k % 4 == 0) ? 1.0 : 0.0;
    return m;
}

__device__ M3 m3_load(const double* p)
{
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = p[k];
    return m;
}

__device__ void m3_store(const M3& m, double* p)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = m.e[k];
}

__device__ M3 m3_mul(const M3& a, const M3& b)
{
    M3 o;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            o.e[3 * r + c] = a.e[3 * r] * b.e[c] + a.e[3 * r + 1] * b.e[3 + c] + a.e[3 * r + 2] * b.e[6 + c];
    return o;
}

__device__ M3 m3_t(const M3& a)
{
    M3 o;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) o.e[3 * r + c] = a.e[3 * c + r];
    return o;
}

__device__ M3 m3_scale(const M3& a, double s)
{
    M3 o;
#pragma unroll
    for (int k = 0; k < 9; ++k) o.e[k] = a.e[k] * s;
    return o;
}

__device__ double m3_det(const M3& a)
{
    const double* m = a.e;
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) + m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// Adjugate over the determinant.
__device__ M3 m3_inv(const M3& a)
{
    const double* m = a.e;
    const double id = 1.0 / m3_det(a);
    M3 o;
    o.e[0] = (m[4] * m[8] - m[5] * m[7]) * id;
    o.e[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    o.e[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    o.e[3] = (m[5] * m[6] - m[3] * m[8]) * id;
    o.e[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    o.e[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    o.e[6] = (m[3] * m[7] - m[4] * m[6]) * id;
    o.e[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    o.e[8] = (m[0] * m[4] - m[1] * m[3]) * id;
    return o;
}

__device__ double m3_norm1(const M3& a)
{
    double m = 0.0;
    for (int c = 0; c < 3; ++c) m = fmax(m, fabs(a.e[c]) + fabs(a.e[3 + c]) + fabs(a.e[6 + c]));
    return m;
}

// exp(a): halve until the norm is at most 1/2, sum the Taylor series until a
// term no longer changes the sum, square back.
__device__ M3 m3_exp(const M3& a)
{
    M3 b = a;
    int squarings = 0;
    while (m3_norm1(b) > 0.5 && squarings < 60) {
        b = m3_scale(b, 0.5);
        ++squarings;
    }
    M3 sum = m3_identity(), term = m3_identity();
    for (int k = 1; k < 40; ++k) {
        term = m3_scale(m3_mul(term, b), 1.0 / k);
#pragma unroll
        for (int e = 0; e < 9; ++e) sum.e[e] += term.e[e];
        if (m3_norm1(term) < 1e-18 * m3_norm1(sum)) break;
    }
    for (int k = 0; k < squarings; ++k) sum = m3_mul(sum, sum);
    return sum;
}

// phi(z) = sum_{k>=0} (-z)^k / (k + 1); the caller keeps |z| below 1/2.
__device__ M3 m3_logphi(const M3& z)
{
    M3 sum = m3_identity(), pw = m3_identity();
    for (int k = 1; k < 80; ++k) {
        pw = m3_scale(m3_mul(pw, z), -1.0);
        const M3 term = m3_scale(pw, 1.0 / (k + 1));
#pragma unroll
        for (int e = 0; e < 9; ++e) sum.e[e] += term.e[e];
        if (m3_norm1(term) < 1e-18) break;
    }
    return sum;
}

// Per wavefront: m v_a v_b (xx, yy, zz, xy, xz, yz) and the six per-atom virial
// terms of the last force pass.
__global__ void k_prt_tensor_waves(Buffers b, int q, int64_t n_slots, PotArgs P)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const DevReplica& R = b.reps[uniform(b.rep_of_wave[t / kWave])];
    const DevPotential& G = *b.pot;
    double v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = 0.0;
    if (t - R.slot_off < R.n_atoms) {
        const uint8_t ty = b.type[q][t];
        const double m = 2.0 * (P.ns == 1 ? P.half_m : G.half_m[ty & 0x3F]);
        const double vx = b.vel[q][0][t], vy = b.vel[q][1][t], vz = b.vel[q][2][t];
        v[0] = m * vx * vx;
        v[1] = m * vy * vy;
        v[2] = m * vz * vz;
        v[3] = m * vx * vy;
        v[4] = m * vx * vz;
        v[5] = m * vy * vz;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[6 + k] = b.eslot[(int64_t)(E_W0 + k) * n_slots + t];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off, kWave);
        if ((t & (kWave - 1)) == 0) b.pr_partial[(t / kWave) * 12 + k] = x;
    }
}

// Symmetric 3x3 from (xx, yy, zz, xy, xz, yz).
__device__ M3 m3_sym(const double* v)
{
    M3 m;
    m.e[0] = v[0];
    m.e[4] = v[1];
    m.e[8] = v[2];
    m.e[1] = m.e[3] = v[3];
    m.e[2] = m.e[6] = v[4];
    m.e[5] = m.e[7] = v[5];
    return m;
}

// One workgroup per replica: the stress tensor from the wave partials or, when
// `chunked`, the chunk sums (a fixed tree either way), then on one lane the
// closing friction and thermostat halves, the box
// half kicks and, with `open`, the opening halves, the box drift, the new
// descriptor and the matrices of the open pass.
__global__ __launch_bounds__(kBlock) void k_prt_update(Buffers b, int close, int open, double h, double rlist,
                                                       double strain_tol, int nvt, int chunked)
{
    __shared__ double sh[12][kBlock];
    const int r = blockIdx.x;
    DevReplica& R = b.reps[r];
    double part[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) part[k] = 0.0;
    if (chunked) {
        for (int c = b.chunk_off[r] + threadIdx.x; c < b.chunk_off[r + 1]; c += kBlock)
#pragma unroll
            for (int k = 0; k < 12; ++k) part[k] += b.chunk_partial[(int64_t)c * kEnergySlots + k];
    } else {
        const int64_t w0 = R.slot_off / kWave, w1 = (R.slot_off + (int64_t)R.n_atoms + kWave - 1) / kWave;
        for (int64_t w = w0 + threadIdx.x; w < w1; w += kBlock)
#pragma unroll
            for (int k = 0; k < 12; ++k) part[k] += b.pr_partial[w * 12 + k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) sh[k][threadIdx.x] = part[k];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
#pragma unroll
            for (int k = 0; k < 12; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x != 0 || R.n_atoms == 0) return;  // an empty replica's box stays put
    double* st = b.pr_state + (int64_t)kPrtState * r;
    const double W = b.pr_param[2 * r], pext = b.pr_param[2 * r + 1];
    const M3 H = m3_load(st), Sig = m3_load(st + 18);
    M3 Hd = m3_load(st + 9);
    double kin[6], vir[6];
    for (int k = 0; k < 6; ++k) {
        kin[k] = sh[k][0];
        vir[k] = -0.5 * sh[6 + k][0];  // the full-list virial sees every pair from both atoms
    }
    M3 K = m3_sym(kin);
    const M3 Wv = m3_sym(vir);
    const M3 Hi = m3_inv(H), HiT = m3_t(Hi);
    const double omega = fabs(m3_det(H));
    // closing friction half step: v <- Ec v, so m v v^T <- Ec K Ec^T
    const M3 Ec = close ? m3_exp(m3_scale(m3_mul(HiT, m3_t(Hd)), -0.5 * h)) : m3_identity();
    if (close) K = m3_mul(m3_mul(Ec, K), m3_t(Ec));
    double* nh = b.nh_state + 4 * (int64_t)r;
    double pi_s = 0.0, xi = 0.0, s_close = 1.0, s_open = 1.0;
    const double Q = nvt ? b.nh_param[2 * r] : 1.0, gkt = nvt ? b.nh_param[2 * r + 1] : 0.0;
    auto thermostat_half = [&](double& scale) {
        const double hh = 0.5 * h;
        double ke = 0.5 * (K.e[0] + K.e[4] + K.e[8]);
        pi_s += 0.5 * hh * (2.0 * ke - gkt) / Q;
        const double sc = exp(-pi_s * hh);
        scale = sc;
        K = m3_scale(K, sc * sc);
        ke *= sc * sc;
        xi += pi_s * hh;
        pi_s += 0.5 * hh * (2.0 * ke - gkt) / Q;
    };
    if (nvt) {
        pi_s = nh[0];
        xi = nh[1];
        if (close) thermostat_half(s_close);
    }
    // box half kicks (closing and opening see the same stress)
    {
        M3 pi;
#pragma unroll
        for (int e = 0; e < 9; ++e) pi.e[e] = (K.e[e] + Wv.e[e]) / omega;
        for (int a = 0; a < 3; ++a) pi.e[4 * a] -= pext;
        const M3 drive = m3_mul(pi, m3_scale(HiT, omega)), elastic = m3_mul(H, Sig);
        const double f = (close + open) * 0.5 * h / W;
#pragma unroll
        for (int e = 0; e < 9; ++e) Hd.e[e] += f * (drive.e[e] - elastic.e[e]);
    }
    m3_store(Hd, st + 9);
    m3_store(m3_scale(Ec, s_close), st + 54);
    if (nvt && open) thermostat_half(s_open);
    if (nvt) {
        nh[0] = pi_s;
        nh[1] = xi;
        nh[2] = s_close * s_open;
        nh[3] = 0.5 * (K.e[0] + K.e[4] + K.e[8]);
    }
    if (!open) return;
    const M3 Eo = m3_exp(m3_scale(m3_mul(HiT, m3_t(Hd)), -0.5 * h));
    m3_store(m3_scale(m3_mul(Eo, Ec), s_close * s_open), st + 27);
    // drift with dh/dt held
    const M3 Bz = m3_scale(m3_mul(Hi, Hd), h);
    M3 Phi = m3_identity();
    if (m3_norm1(Bz) < 0.5) Phi = m3_logphi(Bz);
    else atomicAdd(&b.flags[F_PR_BOX], 1);  // the box would move by half its size in one step
    M3 Hn;
#pragma unroll
    for (int e = 0; e < 9; ++e) Hn.e[e] = H.e[e] + h * Hd.e[e];
    m3_store(m3_mul(Hn, Hi), st + 36);
    m3_store(m3_scale(m3_mul(m3_mul(Hn, Phi), Hi), h), st + 45);
    m3_store(Hn, st);
    // new descriptor: box, inverse, strain since the build, widths against the cells
    const M3 Hni = m3_inv(Hn);
    m3_store(Hn, R.h);
    m3_store(Hni, R.hinv);
    const M3 mb = m3_mul(Hn, m3_load(R.hbinv));
    m3_store(mb, R.mb);
#pragma unroll
    for (int e = 0; e < 9; ++e) R.qg[e] = ldexp(Hn.e[e] / (double)R.nc[e % 3], -kCompactBits);
    double strain2 = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double d = mb.e[e] - ((e % 4 == 0) ? 1.0 : 0.0);
        strain2 += d * d;
    }
    if (sqrt(strain2) * rlist > strain_tol) atomicAdd(&b.flags[F_SKIN], 1);
    if (!(m3_det(Hn) > 0.0)) atomicAdd(&b.flags[F_PR_BOX], 1);
    for (int a = 0; a < 3; ++a) {
        const double w = 1.0 / sqrt(Hni.e[3 * a] * Hni.e[3 * a] + Hni.e[3 * a + 1] * Hni.e[3 * a + 1] +
                                    Hni.e[3 * a + 2] * Hni.e[3 * a + 2]);
        R.box[a] = w;
        R.inv_box[a] = 1.0 / w;
        R.cell[a] = w / (double)R.nc[a];
        if (!(w / (double)R.nc[a] >= rlist)) atomicAdd(&b.flags[F_PR_BOX], 1);
    }
}

// Opening velocity map and kick, then the drift into pos[p^1], with the
// compact record in the new cell (mixed mode).
__global__ void k_prt_open(Buffers b, int p, int q, int64_t n_slots, PotArgs P, double h, int compact)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const double* st = b.pr_state + (int64_t)kPrtState * r;
    const double* C = st + 27;
    const double* M = st + 36;
    const double* D = st + 45;
    const uint8_t ty = b.type[q][t];
    const double acc = P.ns == 1 ? P.accel : G.accel[ty & 0x3F];
    const double3 x = load_xyz(b.pos[p], t);
    const double xo[3] = {x.x - R.origin[0], x.y - R.origin[1], x.z - R.origin[2]};
    const double v0[3] = {b.vel[q][0][t], b.vel[q][1][t], b.vel[q][2][t]};
    double v[3], xn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[a] = fma(0.5 * h * acc, b.fhalf[a][t], C[3 * a] * v0[0] + C[3 * a + 1] * v0[1] + C[3 * a + 2] * v0[2]);
        b.vel[q][a][t] = v[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        xn[a] = R.origin[a] + (M[3 * a] * xo[0] + M[3 * a + 1] * xo[1] + M[3 * a + 2] * xo[2]) +
                (D[3 * a] * v[0] + D[3 * a + 1] * v[1] + D[3 * a + 2] * v[2]);
    double* dst = reinterpret_cast<double*>(b.pos[p ^ 1] + t);
    *reinterpret_cast<double2*>(dst) = make_double2(xn[0], xn[1]);
    dst[2] = xn[2];
    if (compact) {
        const int4 c4 = b.cellxyz[t];
        const int c[3] = {c4.x, c4.y, c4.z};
        int4 rq;
        if (!compact_coords<2>(R, c, xn[0], xn[1], xn[2], rq)) atomicAdd(&b.flags[F_COMPACT], 1);
        b.rec[0][t] = rq;
    }
}

// Closing velocity map of the last step of a call: the internal and the
// caller's velocities and the kinetic terms of the energy record.
__global__ void k_prt_close_scale(Buffers b, int q, int64_t n_slots, PotArgs P, md_state st)
{
    const int64_t t = global_thread();
    if (t >= n_slots) return;
    const int r = uniform(b.rep_of_wave[t / kWave]);
    const DevReplica& R = b.reps[r];
    if (t - R.slot_off >= R.n_atoms) return;
    const DevPotential& G = *b.pot;
    const double* C = b.pr_state + (int64_t)kPrtState * r + 54;
    const uint8_t ty = b.type[q][t];
    const int32_t id = b.id[q][t];
    const double v0[3] = {b.vel[q][0][t], b.vel[q][1][t], b.vel[q][2][t]};
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[a] = C[3 * a] * v0[0] + C[3 * a + 1] * v0[1] + C[3 * a + 2] * v0[2];
        b.vel[q][a][t] = v[a];
    }
    st.vx[id] = v[0];
    st.vy[id] = v[1];
    st.vz[id] = v[2];
    b.eslot[(int64_t)E_KE * n_slots + t] =
        (P.ns == 1 ? P.half_m : G.half_m[ty & 0x3F]) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

}  // namespace

void launch_prt_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int close, int open,
                       double dt_fs, double rlist, double strain_tol, int nvt, hipStream_t s)
{
    hipLaunchKernelGGL(k_prt_tensor_waves, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P);
    launch_pr_chunk_sums(b, k, 12, s);
    if (k.n_replicas > 0)
        hipLaunchKernelGGL(k_prt_update, dim3(k.n_replicas), dim3(kBlock), 0, s, b, close, open, dt_fs, rlist,
                           strain_tol, nvt, k.chunked);
}

void launch_prt_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_prt_open, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, p, q, k.n_slots, P, dt_fs,
                       k.compact);
}

void launch_prt_close_scale(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, const md_state& st,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_prt_close_scale, dim3(blocks_for(k.n_slots)), dim3(kBlock), 0, s, b, q, k.n_slots, P, st);
}

}  // namespace mdk
