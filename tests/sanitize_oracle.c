/*
 * Host sanitizer driver for the oracle (test infrastructure): compiled with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with the oracle's
 * source, it runs every entry point on small periodic systems (a bcc crystal
 * of two species, also in a sheared cell) and prints one checksum line.  Any
 * out-of-bounds access, use after free, leak or undefined operation aborts the
 * program with a report.
 */
#include "../oracle/eam_oracle.c"

#include <stdio.h>

#define NC 4
#define N (2 * NC * NC * NC)

static double sum(const double *v, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    return s;
}

int main(void)
{
    /* two species, six pair knots, two density knots */
    double pair_a[4 * 6], pair_r[4 * 6], dens_A[4 * 2], dens_R[4 * 2];
    const double emb_c[2] = {1.0, 0.9}, mass[2] = {55.845, 12.011};
    for (int ab = 0; ab < 4; ++ab) {
        for (int k = 0; k < 6; ++k) {
            pair_r[6 * ab + k] = 2.2 + 0.38 * k;
            pair_a[6 * ab + k] = (k % 2 ? -0.3 : 0.5) / (1.0 + k + ab);
        }
        dens_R[2 * ab] = 3.0;
        dens_R[2 * ab + 1] = 3.6;
        dens_A[2 * ab] = 0.8 + 0.1 * ab;
        dens_A[2 * ab + 1] = 0.4;
    }
    const int s01 = 1, s10 = 2; /* symmetric pair functions */
    for (int k = 0; k < 6; ++k) pair_a[6 * s10 + k] = pair_a[6 * s01 + k];
    const or_potential pot = {2, 6, 2, 0, pair_a, pair_r, dens_A, dens_R, emb_c, mass};

    const double a0 = 2.87, L = NC * a0;
    double x[N], y[N], z[N], vx[N], vy[N], vz[N], f[3 * N], e[N], rho[N], vir[6], pe;
    uint8_t sp[N], rigid[N];
    int64_t i = 0;
    for (int cx = 0; cx < NC; ++cx)
        for (int cy = 0; cy < NC; ++cy)
            for (int cz = 0; cz < NC; ++cz)
                for (int b = 0; b < 2; ++b, ++i) {
                    const double j = 0.013 * (double)((i * 7919) % 17) - 0.1;
                    x[i] = (cx + 0.5 * b) * a0 + j;
                    y[i] = (cy + 0.5 * b) * a0 - 0.5 * j;
                    z[i] = (cz + 0.5 * b) * a0 + 0.3 * j;
                    vx[i] = 1e-3 * (double)((i * 31) % 7 - 3);
                    vy[i] = 1e-3 * (double)((i * 17) % 5 - 2);
                    vz[i] = -1e-3 * (double)((i * 13) % 3 - 1);
                    sp[i] = (uint8_t)(i % 9 == 0);
                    rigid[i] = (uint8_t)(i < 4);
                }
    const double box[3] = {L, L, L}, origin[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.01};
    const uint8_t per[3] = {1, 1, 1}, slab[3] = {1, 1, 0};
    double acc = 0.0;
    int rc = 0;

    rc |= or_forces(N, x, y, z, sp, rigid, box, per, &pot, f, e, rho, vir, &pe);
    acc += pe + sum(f, 3 * N) + sum(vir, 6);
    acc += or_energy(N, x, y, z, sp, box, slab, &pot);
    {
        const int64_t sample[3] = {0, 17, N - 1};
        double fs[9], es[3], rs[3];
        rc |= or_forces_sampled(N, x, y, z, sp, box, per, &pot, 3, sample, fs, es, rs);
        acc += sum(fs, 9);
    }
    double pe_out[6], ke_out[6], w_out[6], nh_out[12], box_out[18], ld_out[18], baro[6], press[6];
    double h_out[54], hd_out[54], st_out[36];
    double X[N], Y[N], Z[N], VX[N], VY[N], VZ[N];
#define RESET()                                  \
    do {                                         \
        memcpy(X, x, sizeof X);                  \
        memcpy(Y, y, sizeof Y);                  \
        memcpy(Z, z, sizeof Z);                  \
        memcpy(VX, vx, sizeof VX);               \
        memcpy(VY, vy, sizeof VY);               \
        memcpy(VZ, vz, sizeof VZ);               \
    } while (0)
    RESET();
    rc |= or_run_verlet(N, X, Y, Z, VX, VY, VZ, sp, rigid, box, per, &pot, 1.0, vp, 5, f, pe_out, ke_out, w_out);
    acc += sum(pe_out, 6) + sum(w_out, 6);
    RESET();
    rc |= or_run_nh(N, X, Y, Z, VX, VY, VZ, sp, NULL, box, per, &pot, 1.0, NULL, 5, 500.0, 50.0, 0.0, f, pe_out,
                    ke_out, NULL, nh_out);
    acc += sum(nh_out, 12);
    RESET();
    rc |= or_run_gear(N, X, Y, Z, VX, VY, VZ, sp, rigid, box, per, &pot, 1.0, vp, 5, f, pe_out, ke_out, w_out);
    acc += sum(ke_out, 6);
    RESET();
    double Lb[3] = {L, L, L};
    rc |= or_run_pr(N, X, Y, Z, VX, VY, VZ, sp, Lb, origin, NULL, &pot, 1.0, 5, 1.0, 1e4, f, pe_out, ke_out,
                    box_out, ld_out, baro, press);
    acc += sum(box_out, 18) + sum(press, 6);
    RESET();
    double Lc[3] = {L, L, L};
    rc |= or_run_npt(N, X, Y, Z, VX, VY, VZ, sp, Lc, origin, &pot, 1.0, 5, 1.0, 1e4, 500.0, 50.0, f, pe_out, ke_out,
                     box_out, baro, press, nh_out);
    acc += sum(baro, 6);

    /* the same crystal in a sheared cell of five cells per edge: [a, b, c + a] */
    {
        const int nc = 5, n = 2 * nc * nc * nc;
        const double Ls = nc * a0;
        double *xs = calloc((size_t)n * 6, sizeof(double)), *fs = calloc((size_t)n * 3, sizeof(double));
        uint8_t *ss = calloc((size_t)n, 1);
        int64_t k = 0;
        for (int cx = 0; cx < nc; ++cx)
            for (int cy = 0; cy < nc; ++cy)
                for (int cz = 0; cz < nc; ++cz)
                    for (int b = 0; b < 2; ++b, ++k) {
                        xs[k] = (cx + 0.5 * b) * a0 + 0.01 * (double)(k % 5);
                        xs[n + k] = (cy + 0.5 * b) * a0;
                        xs[2 * n + k] = (cz + 0.5 * b) * a0 - 0.01 * (double)(k % 3);
                        xs[3 * n + k] = 1e-3 * (double)(k % 3 - 1);
                        ss[k] = (uint8_t)(k % 11 == 0);
                    }
        double h[9] = {Ls, 0.0, Ls, 0.0, Ls, 0.0, 0.0, 0.0, Ls};
        const double stress[9] = {1.0, 0.5, 0.0, 0.5, 1.0, -0.3, 0.0, -0.3, 1.0};
        rc |= or_forces_tri(n, xs, xs + n, xs + 2 * n, ss, NULL, h, &pot, fs, NULL, NULL, vir, &pe);
        acc += pe + sum(vir, 6);
        rc |= or_run_prt(n, xs, xs + n, xs + 2 * n, xs + 3 * n, xs + 4 * n, xs + 5 * n, ss, h, origin, NULL, stress,
                         NULL, &pot, 1.0, 5, 1.0, 1e4, 500.0, 50.0, fs, pe_out, ke_out, h_out, hd_out, baro, st_out,
                         nh_out);
        acc += sum(h_out, 54) + sum(st_out, 36) + sum(hd_out, 54);
        free(xs);
        free(fs);
        free(ss);
    }
    /* error paths: a cell too thin for the cutoff */
    {
        double thin[9] = {5.0, 0.0, 0.0, 0.0, 5.0, 0.0, 0.0, 0.0, 5.0};
        if (or_forces_tri(N, x, y, z, sp, NULL, thin, &pot, f, NULL, NULL, NULL, NULL) != -1) rc |= 4;
        const double small[3] = {5.0, 5.0, 5.0};
        if (or_forces(N, x, y, z, sp, NULL, small, per, &pot, f, NULL, NULL, NULL, NULL) != -1) rc |= 8;
    }
    printf("rc %d checksum %.12e\n", rc, acc);
    return rc != 0 || !isfinite(acc);
}
