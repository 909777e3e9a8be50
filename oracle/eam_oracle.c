/*
 * Plain FP64 CPU oracle for the embedded-atom (EAM / Finnis-Sinclair) force
 * loop and velocity-Verlet integration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header or constant with the GPU path.
 *
 * Everything is brute force O(N^2): no cell list, no neighbour list, no
 * reordering.  Each function states the passage of the paper it follows.
 *
 * Notation (paper, "Theoretical background", Eq. Ucoh):
 *   U = sum_i ( 1/2 sum_{j!=i} phi_{s_i s_j}(r_ij) + F_{s_i}(rho_i) ),
 *   rho_i = sum_{j!=i} rho_{s_i s_j}(r_ij).
 * The paper writes the pair term V and the density term phi; here phi is the
 * pair potential and rho the density function.  The pair double sum is read
 * as counting each unordered pair once (the factor 1/2), which is the only
 * reading under which the force carries phi' once per pair.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Units (paper, section "Units") -------------------------------------
 * Length in Angstrom, mass in amu (1 u = 1.66053886e-27 kg, as printed), energy
 * in eV.  The time unit is sqrt(M L^2 / E), about 1.018e-14 s.  The eV in
 * joules and Boltzmann's constant are not printed; the CODATA-2002 values that
 * go with the printed amu are used. */
#define OR_AMU_KG 1.66053886e-27
#define OR_EV_J 1.60217653e-19
#define OR_KB_EV_PER_K 8.617343e-5
#define OR_EV_PER_A3_IN_GPA 160.217653

double or_time_unit_fs(void) { return sqrt(OR_AMU_KG * 1.0e-20 / OR_EV_J) * 1.0e15; }
double or_boltzmann_ev(void) { return OR_KB_EV_PER_K; }
double or_pressure_unit_gpa(void) { return OR_EV_PER_A3_IN_GPA; }

/* ---- Potential description ------------------------------------------------
 * Cubic-knot form (paper, "Available potentials", coefficient-file example):
 *   f(r) = sum_k a_k (r_k - r)^3 H(r_k - r).
 * pair_a/pair_r: [ns][ns][npk]  phi between species a and b (symmetric).
 * dens_A/dens_R: [ns][ns][ndk]  density at an a-site from a b-neighbour.
 *   (EAM: depends on b only; Finnis-Sinclair: symmetric - "Theoretical
 *   background", the paragraph on the two interpretations.)
 * emb_c: [ns]  F_a(rho) = -emb_c[a] * sqrt(rho) (the FS square root).
 * mass:  [ns]  amu.  */
typedef struct {
    int32_t ns, npk, ndk, pad_;
    const double *pair_a, *pair_r, *dens_A, *dens_R, *emb_c, *mass;
} or_potential;

/* One cubic-knot sum and its derivative with respect to r.  Terms with
 * r_k - r <= 0 are switched off by the Heaviside step (the value, slope and
 * curvature of each term vanish at r = r_k, so the side taken at equality
 * does not matter). */
double or_knot_sum(const double *a, const double *rk, int n, double r, double *deriv)
{
    double v = 0.0, d = 0.0;
    for (int k = 0; k < n; ++k) {
        double t = rk[k] - r;
        if (t > 0.0) {
            v += a[k] * t * t * t;
            d += -3.0 * a[k] * t * t;
        }
    }
    if (deriv) *deriv = d;
    return v;
}

double or_pair(const or_potential *p, int a, int b, double r, double *dphi)
{
    const int off = (a * p->ns + b) * p->npk;
    return or_knot_sum(p->pair_a + off, p->pair_r + off, p->npk, r, dphi);
}

double or_density(const or_potential *p, int a, int b, double r, double *drho)
{
    const int off = (a * p->ns + b) * p->ndk;
    return or_knot_sum(p->dens_A + off, p->dens_R + off, p->ndk, r, drho);
}

/* F(rho) = -c sqrt(rho), F'(rho) = -c / (2 sqrt(rho)).  An atom with no
 * density (isolated) has F = F' = 0: the square root is singular there and
 * the paper is silent; zero is the limit of the energy. */
double or_embed(const or_potential *p, int a, double rho, double *dF)
{
    if (rho <= 0.0) {
        if (dF) *dF = 0.0;
        return 0.0;
    }
    double s = sqrt(rho);
    if (dF) *dF = -p->emb_c[a] / (2.0 * s);
    return -p->emb_c[a] * s;
}

/* Largest knot over every function: beyond it every term is exactly zero. */
double or_cutoff(const or_potential *p)
{
    double rc = 0.0;
    int n2 = p->ns * p->ns;
    for (int i = 0; i < n2 * p->npk; ++i)
        if (p->pair_r[i] > rc) rc = p->pair_r[i];
    for (int i = 0; i < n2 * p->ndk; ++i)
        if (p->dens_R[i] > rc) rc = p->dens_R[i];
    return rc;
}

/* ---- Geometry (paper, "Boundary conditions") -----------------------------
 * Positions are stored unwrapped.  The separation used in Eq. Ucoh is the
 * shortest vector between i and j or any periodic image of j, taken only
 * along periodic axes; free axes use the plain difference. */
static void image_vector(const double *xi, const double *xj, const double *box,
                         const uint8_t *periodic, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = xj[a] - xi[a];
        if (periodic[a]) v -= box[a] * rint(v / box[a]);
        d[a] = v;
    }
}

/* A periodic box given by its matrix h = [a, b, c] (paper, "Barostat NPTp":
 * r = h x, the edge vectors as columns; matrices row-major, m[3 r + c]), or an
 * orthorhombic box with per-axis periodic flags (box != NULL). */
typedef struct {
    const double *box;
    const uint8_t *periodic;
    double h[9], hi[9];
} or_geom;

/* Shortest image with a box matrix: k = rint(h^-1 d) lattice vectors are
 * taken off d.  When every width of the cell (the distance between opposite
 * faces, 1 / |row a of h^-1|) exceeds twice the cutoff, a separation shorter
 * than the cutoff has fractional components below 1/2, so this finds it, and
 * it is the only image in range. */
static void geom_image(const or_geom *g, const double *xi, const double *xj, double d[3])
{
    if (g->box) {
        image_vector(xi, xj, g->box, g->periodic, d);
        return;
    }
    double v[3], k[3];
    for (int a = 0; a < 3; ++a) v[a] = xj[a] - xi[a];
    for (int a = 0; a < 3; ++a) k[a] = rint(g->hi[3 * a] * v[0] + g->hi[3 * a + 1] * v[1] + g->hi[3 * a + 2] * v[2]);
    for (int a = 0; a < 3; ++a) d[a] = v[a] - (g->h[3 * a] * k[0] + g->h[3 * a + 1] * k[1] + g->h[3 * a + 2] * k[2]);
}

static void load_pos(const double *x, const double *y, const double *z, int64_t i, double out[3])
{
    out[0] = x[i];
    out[1] = y[i];
    out[2] = z[i];
}

/* Returns 0 when every periodic length exceeds twice the cutoff (so one image
 * at most lies in range), -1 otherwise. */
static int check_box(const double *box, const uint8_t *periodic, double rc)
{
    for (int a = 0; a < 3; ++a)
        if (periodic[a] && !(box[a] > 2.0 * rc)) return -1;
    return 0;
}

/* Host density rho_i of one atom by brute force over all atoms. */
static double density_of(int64_t i, int64_t n, const double *x, const double *y,
                         const double *z, const uint8_t *species, const or_geom *g,
                         const or_potential *p, double rc)
{
    double xi[3], xj[3], d[3];
    load_pos(x, y, z, i, xi);
    double rho = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        load_pos(x, y, z, j, xj);
        geom_image(g, xi, xj, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r >= rc) continue;
        rho += or_density(p, species[i], species[j], r, NULL);
    }
    return rho;
}

/*
 * Full evaluation (Eq. Ucoh and its gradient).
 *   rho_i   = sum_{j!=i} rho_{s_i s_j}(r_ij)
 *   F_i     = F_{s_i}(rho_i),  F'_i its derivative
 *   g_ij    = phi'_{s_i s_j}(r) + F'_i rho'_{s_i s_j}(r) + F'_j rho'_{s_j s_i}(r)
 *   f_i     = sum_{j!=i} g_ij d_ij / r_ij,   d_ij = r_j - r_i (image vector)
 *   e_i     = 1/2 sum_{j!=i} phi_{s_i s_j}(r_ij) + F_i   (the per-atom split of
 *             "Theoretical background", last paragraph: halves of each pair)
 *   W_ab    = - sum_{i<j} g_ij d_a d_b / r, skipping pairs of two fixed atoms
 *             ("Fixed atoms": the stress ignores forces between fixed atoms)
 * Outputs (any may be NULL except f): f[3n] interleaved (fx,fy,fz per atom),
 * e_atom[n], rho[n], virial[6] (xx,yy,zz,xy,xz,yz), pe (sum of e_atom).
 * rigid may be NULL (no fixed atoms).  Returns 0, or -1 if a periodic length
 * is not larger than twice the cutoff.
 */
static void forces_geom(int64_t n, const double *x, const double *y, const double *z,
                        const uint8_t *species, const uint8_t *rigid, const or_geom *g,
                        const or_potential *p, double rc, double *f, double *e_atom,
                        double *rho_out, double *virial, double *pe)
{

    double *rho = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *dF = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *Fe = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *eat = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *wrow = (double *)calloc((size_t)(n > 0 ? n : 1) * 6, sizeof(double));

    /* Pass 1: densities and embedding. */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        rho[i] = density_of(i, n, x, y, z, species, g, p, rc);
        Fe[i] = or_embed(p, species[i], rho[i], &dF[i]);
    }

    /* Pass 2: forces, per-atom energies, virial rows (j > i only). */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double xi[3], xj[3], d[3];
        load_pos(x, y, z, i, xi);
        double fi[3] = {0.0, 0.0, 0.0};
        double epair = 0.0;
        const int si = species[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load_pos(x, y, z, j, xj);
            geom_image(g, xi, xj, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= rc) continue;
            const int sj = species[j];
            double dphi, drho_ij, drho_ji;
            double phi = or_pair(p, si, sj, r, &dphi);
            or_density(p, si, sj, r, &drho_ij);
            or_density(p, sj, si, r, &drho_ji);
            double g = dphi + dF[i] * drho_ij + dF[j] * drho_ji;
            for (int a = 0; a < 3; ++a) fi[a] += g * d[a] / r;
            epair += phi;
            if (j > i && !(rigid && rigid[i] && rigid[j])) {
                double *w = wrow + 6 * i;
                w[0] -= g * d[0] * d[0] / r;
                w[1] -= g * d[1] * d[1] / r;
                w[2] -= g * d[2] * d[2] / r;
                w[3] -= g * d[0] * d[1] / r;
                w[4] -= g * d[0] * d[2] / r;
                w[5] -= g * d[1] * d[2] / r;
            }
        }
        f[3 * i + 0] = fi[0];
        f[3 * i + 1] = fi[1];
        f[3 * i + 2] = fi[2];
        eat[i] = 0.5 * epair + Fe[i];
        if (e_atom) e_atom[i] = eat[i];
        if (rho_out) rho_out[i] = rho[i];
    }

    if (pe) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += eat[i];
        *pe = s;
    }
    if (virial) {
        for (int c = 0; c < 6; ++c) virial[c] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < 6; ++c) virial[c] += wrow[6 * i + c];
    }
    free(rho);
    free(dF);
    free(Fe);
    free(eat);
    free(wrow);
}

int or_forces(int64_t n, const double *x, const double *y, const double *z,
              const uint8_t *species, const uint8_t *rigid, const double *box,
              const uint8_t *periodic, const or_potential *p, double *f,
              double *e_atom, double *rho_out, double *virial, double *pe)
{
    const double rc = or_cutoff(p);
    if (check_box(box, periodic, rc)) return -1;
    const or_geom g = {box, periodic, {0}, {0}};
    forces_geom(n, x, y, z, species, rigid, &g, p, rc, f, e_atom, rho_out, virial, pe);
    return 0;
}

/* Total energy only (Eq. Ucoh), computed without any derivative: used by the
 * finite-difference pins.  Returns NAN on a bad box. */
double or_energy(int64_t n, const double *x, const double *y, const double *z,
                 const uint8_t *species, const double *box, const uint8_t *periodic,
                 const or_potential *p)
{
    const double rc = or_cutoff(p);
    if (check_box(box, periodic, rc)) return NAN;
    double total = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t i = 0; i < n; ++i) {
        double xi[3], xj[3], d[3];
        load_pos(x, y, z, i, xi);
        double rho = 0.0, epair = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load_pos(x, y, z, j, xj);
            image_vector(xi, xj, box, periodic, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= rc) continue;
            rho += or_density(p, species[i], species[j], r, NULL);
            epair += or_pair(p, species[i], species[j], r, NULL);
        }
        total += 0.5 * epair + or_embed(p, species[i], rho, NULL);
    }
    return total;
}

/*
 * Sampled evaluation for large systems: forces, per-atom energies and host
 * densities of the atoms listed in sample[0..m), each from a brute-force scan
 * over all n atoms.  F'_j of every neighbour j is itself found by a
 * brute-force density scan, so the cost is about (1 + neighbours) * n distance
 * tests per sampled atom.  Same definitions as or_forces.
 * Outputs: f[3m], e_atom[m], rho_out[m] (any of the last two may be NULL).
 */
static int sampled_geom(int64_t n, const double *x, const double *y, const double *z,
                        const uint8_t *species, const or_geom *gp, const or_potential *p, double rc,
                        int64_t m, const int64_t *sample, double *f, double *e_atom, double *rho_out)
{
    const or_geom g = *gp;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t s = 0; s < m; ++s) {
        const int64_t i = sample[s];
        if (i < 0 || i >= n) {
            bad |= 1;
            continue;
        }
        double xi[3], xj[3], d[3];
        load_pos(x, y, z, i, xi);
        const int si = species[i];
        /* neighbours of i within the cutoff */
        int64_t cap = 256, cnt = 0;
        int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * cap);
        double rho_i = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            load_pos(x, y, z, j, xj);
            geom_image(&g, xi, xj, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r >= rc) continue;
            rho_i += or_density(p, si, species[j], r, NULL);
            if (cnt == cap) {
                cap *= 2;
                nb = (int64_t *)realloc(nb, sizeof(int64_t) * cap);
            }
            nb[cnt++] = j;
        }
        double dFi;
        double Fi = or_embed(p, si, rho_i, &dFi);
        double fi[3] = {0.0, 0.0, 0.0}, epair = 0.0;
        for (int64_t q = 0; q < cnt; ++q) {
            const int64_t j = nb[q];
            const int sj = species[j];
            double rho_j = density_of(j, n, x, y, z, species, &g, p, rc);
            double dFj;
            or_embed(p, sj, rho_j, &dFj);
            load_pos(x, y, z, j, xj);
            geom_image(&g, xi, xj, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double dphi, drho_ij, drho_ji;
            double phi = or_pair(p, si, sj, r, &dphi);
            or_density(p, si, sj, r, &drho_ij);
            or_density(p, sj, si, r, &drho_ji);
            double g = dphi + dFi * drho_ij + dFj * drho_ji;
            for (int a = 0; a < 3; ++a) fi[a] += g * d[a] / r;
            epair += phi;
        }
        free(nb);
        f[3 * s + 0] = fi[0];
        f[3 * s + 1] = fi[1];
        f[3 * s + 2] = fi[2];
        if (e_atom) e_atom[s] = 0.5 * epair + Fi;
        if (rho_out) rho_out[s] = rho_i;
    }
    return bad ? -2 : 0;
}

int or_forces_sampled(int64_t n, const double *x, const double *y, const double *z,
                      const uint8_t *species, const double *box, const uint8_t *periodic,
                      const or_potential *p, int64_t m, const int64_t *sample, double *f,
                      double *e_atom, double *rho_out)
{
    const double rc = or_cutoff(p);
    if (check_box(box, periodic, rc)) return -1;
    const or_geom g = {box, periodic, {0}, {0}};
    return sampled_geom(n, x, y, z, species, &g, p, rc, m, sample, f, e_atom, rho_out);
}

/* Sum of the forces on the rigid atoms dotted with their prescribed velocity
 * (Angstrom per time unit): the rate at which the system does work on the
 * moving rigid block, whose negative is the power the block delivers. */
static double rigid_power(int64_t n, const double *f, const uint8_t *rigid, const double *vp)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (rigid && rigid[i]) s += f[3 * i] * vp[0] + f[3 * i + 1] * vp[1] + f[3 * i + 2] * vp[2];
    return s;
}

/*
 * Velocity-Verlet molecular dynamics (paper, "Time integration"; "Fixed
 * atoms"; NVEp ensemble), in the internal unit of time:
 *   v <- v + (dt/2) f/m;   x <- x + dt v;   f <- forces(x);   v <- v + (dt/2) f/m.
 * Fixed atoms (rigid[i] = 1) follow a prescribed straight line
 * x(t) = x(0) + vp t with the velocity vp (Angstrom/fs) instead.
 * Velocities in and out are Angstrom/fs, dt in fs.
 * Per step s = 0..nsteps the function records, if the pointers are non-NULL:
 *   pe[s], ke[s], work[s] = energy delivered by the moving rigid block up to
 *   step s (trapezoid rule over -sum_{rigid} f_i . vp).
 * On return x,y,z,vx,vy,vz hold the final state and f[3n] the final forces.
 */
int or_run_verlet(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                  double *vz, const uint8_t *species, const uint8_t *rigid, const double *box,
                  const uint8_t *periodic, const or_potential *p, double dt_fs,
                  const double *vp_fs, int64_t nsteps, double *f, double *pe_out,
                  double *ke_out, double *work_out)
{
    const double t0 = or_time_unit_fs();
    const double dt = dt_fs / t0;
    double vp[3] = {0.0, 0.0, 0.0};
    if (vp_fs)
        for (int a = 0; a < 3; ++a) vp[a] = vp_fs[a] * t0;
    double *v[3] = {vx, vy, vz};
    double *r[3] = {x, y, z};
    /* internal velocities in Angstrom per time unit */
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] *= t0;
    double *rigid0 = NULL;
    if (rigid) {
        rigid0 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) rigid0[3 * i + a] = r[a][i];
    }
    double pe;
    int rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
    if (rc) goto done;
    double work = 0.0;
    double power_prev = -rigid_power(n, f, rigid, vp);
    for (int64_t s = 0;; ++s) {
        if (pe_out) pe_out[s] = pe;
        if (ke_out) {
            double ke = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (rigid && rigid[i]) continue;
                ke += 0.5 * p->mass[species[i]] *
                      (v[0][i] * v[0][i] + v[1][i] * v[1][i] + v[2][i] * v[2][i]);
            }
            ke_out[s] = ke;
        }
        if (work_out) work_out[s] = work;
        if (s == nsteps) break;
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) {
                double t = (double)(s + 1) * dt;
                for (int a = 0; a < 3; ++a) r[a][i] = rigid0[3 * i + a] + vp[a] * t;
                continue;
            }
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) {
                v[a][i] += 0.5 * dt * f[3 * i + a] / m;
                r[a][i] += dt * v[a][i];
            }
        }
        rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
        if (rc) goto done;
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) continue;
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * dt * f[3 * i + a] / m;
        }
        double power = -rigid_power(n, f, rigid, vp);
        work += 0.5 * dt * (power_prev + power);
        power_prev = power;
    }
done:
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
        if (rigid && rigid[i])
            for (int a = 0; a < 3; ++a) v[a][i] = vp_fs ? vp_fs[a] : 0.0;
    }
    free(rigid0);
    return rc;
}

/*
 * Nose-Hoover NVT molecular dynamics (paper, "Thermostat NVTp"): the particle
 * momenta feel the friction -pi_s p_i and the thermostat momentum obeys
 * Q_s dpi_s/dt = sum_i p_i^2/m_i - g k_B T, with g the degrees of freedom of
 * the temperature definition (3N - 3; 3N_mobile with rigid atoms).  The
 * printed right-hand side halves the kinetic term, which would hold the
 * kinetic energy at twice the one the temperature definition gives; the
 * reading here keeps the fixed point at that definition.
 *
 * The flow is split symmetrically (thermostat half step, velocity half kick,
 * drift, forces, velocity half kick, thermostat half step).  A thermostat
 * half step of length h with kinetic energy K:
 *   pi += (h/2) (2K - g k_B T)/Q;  v *= exp(-pi h);  K *= exp(-2 pi h);
 *   xi += pi h;  pi += (h/2) (2K - g k_B T)/Q.
 * The extended energy PE + KE + Q pi^2/2 + g k_B T xi is conserved.
 * Units: dt in fs, velocities Angstrom/fs, Q in eV fs^2, pi in 1/fs (pi starts
 * at pi0, xi at 0).
 * Per step s = 0..nsteps, nh_out[2 s] = pi and nh_out[2 s + 1] =
 * Q pi^2/2 + g k_B T xi (eV), besides the outputs of or_run_verlet.
 */
static double mobile_ke(int64_t n, double *const v[3], const uint8_t *species, const uint8_t *rigid,
                        const or_potential *p)
{
    double ke = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (rigid && rigid[i]) continue;
        ke += 0.5 * p->mass[species[i]] * (v[0][i] * v[0][i] + v[1][i] * v[1][i] + v[2][i] * v[2][i]);
    }
    return ke;
}

static void nh_half_step(int64_t n, double *const v[3], const uint8_t *species, const uint8_t *rigid,
                         const or_potential *p, double h, double q, double gkt, double *pi, double *xi)
{
    double ke = mobile_ke(n, v, species, rigid, p);
    *pi += 0.5 * h * (2.0 * ke - gkt) / q;
    const double s = exp(-*pi * h);
    for (int64_t i = 0; i < n; ++i) {
        if (rigid && rigid[i]) continue;
        for (int a = 0; a < 3; ++a) v[a][i] *= s;
    }
    ke *= s * s;
    *xi += *pi * h;
    *pi += 0.5 * h * (2.0 * ke - gkt) / q;
}

int or_run_nh(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, const uint8_t *rigid, const double *box, const uint8_t *periodic,
              const or_potential *p, double dt_fs, const double *vp_fs, int64_t nsteps, double t_target,
              double q_ev_fs2, double pi0_per_fs, double *f, double *pe_out, double *ke_out, double *work_out,
              double *nh_out)
{
    const double t0 = or_time_unit_fs();
    const double dt = dt_fs / t0;
    const double q = q_ev_fs2 / (t0 * t0);
    double vp[3] = {0.0, 0.0, 0.0};
    if (vp_fs)
        for (int a = 0; a < 3; ++a) vp[a] = vp_fs[a] * t0;
    double *v[3] = {vx, vy, vz};
    double *r[3] = {x, y, z};
    int64_t n_mobile = 0;
    int has_rigid = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (rigid && rigid[i]) has_rigid = 1;
        else ++n_mobile;
    }
    const double dof = has_rigid ? 3.0 * (double)n_mobile : 3.0 * (double)n_mobile - 3.0;
    const double gkt = dof * OR_KB_EV_PER_K * t_target;
    double pi = pi0_per_fs * t0, xi = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] *= t0;
    double *rigid0 = NULL;
    if (rigid) {
        rigid0 = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) rigid0[3 * i + a] = r[a][i];
    }
    double pe;
    int rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
    if (rc) goto done;
    double work = 0.0;
    double power_prev = -rigid_power(n, f, rigid, vp);
    for (int64_t s = 0;; ++s) {
        if (pe_out) pe_out[s] = pe;
        if (ke_out) ke_out[s] = mobile_ke(n, v, species, rigid, p);
        if (work_out) work_out[s] = work;
        if (nh_out) {
            nh_out[2 * s] = pi / t0;
            nh_out[2 * s + 1] = 0.5 * q * pi * pi + gkt * xi;
        }
        if (s == nsteps) break;
        nh_half_step(n, v, species, rigid, p, 0.5 * dt, q, gkt, &pi, &xi);
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) {
                double t = (double)(s + 1) * dt;
                for (int a = 0; a < 3; ++a) r[a][i] = rigid0[3 * i + a] + vp[a] * t;
                continue;
            }
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) {
                v[a][i] += 0.5 * dt * f[3 * i + a] / m;
                r[a][i] += dt * v[a][i];
            }
        }
        rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
        if (rc) goto done;
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) continue;
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * dt * f[3 * i + a] / m;
        }
        nh_half_step(n, v, species, rigid, p, 0.5 * dt, q, gkt, &pi, &xi);
        double power = -rigid_power(n, f, rigid, vp);
        work += 0.5 * dt * (power_prev + power);
        power_prev = power;
    }
done:
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
        if (rigid && rigid[i])
            for (int a = 0; a < 3; ++a) v[a][i] = vp_fs ? vp_fs[a] : 0.0;
    }
    free(rigid0);
    return rc;
}

/*
 * Third-order Gear predictor-corrector (paper, "Time integration": the
 * alternative to velocity Verlet).  Gear's method for a second-order equation
 * carries four values per coordinate, the position r0 and the scaled time
 * derivatives r1 = h v, r2 = h^2 a / 2, r3 = h^3 b / 6.  Each step:
 *   predict  the Taylor series: r0 += r1 + r2 + r3, r1 += 2 r2 + 3 r3,
 *            r2 += 3 r3 (binomial coefficients);
 *   evaluate the forces at the predicted positions;
 *   correct  with e = h^2 f / (2 m) - r2: r_k += c_k e, c = {1/6, 5/6, 1, 1/3}.
 * Start: a = f(x0) / m, b = 0.  pe_out[s] is the potential energy of the force
 * evaluation of step s (at the predicted positions; s = 0: at x0), ke_out[s]
 * the kinetic energy of the corrected velocities.  Rigid atoms move on
 * x0 + vp t; work_out[s] integrates their power -f . vp over the evaluations
 * of steps 0..s by the trapezoid rule.
 */
int or_run_gear(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
                const uint8_t *species, const uint8_t *rigid, const double *box, const uint8_t *periodic,
                const or_potential *p, double dt_fs, const double *vp_fs, int64_t nsteps, double *f,
                double *pe_out, double *ke_out, double *work_out)
{
    static const double c[4] = {1.0 / 6.0, 5.0 / 6.0, 1.0, 1.0 / 3.0};
    const double t0 = or_time_unit_fs();
    const double h = dt_fs / t0;
    double vp[3] = {0.0, 0.0, 0.0};
    if (vp_fs)
        for (int a = 0; a < 3; ++a) vp[a] = vp_fs[a] * t0;
    double *v[3] = {vx, vy, vz};
    double *r0[3] = {x, y, z};
    const size_t m3 = 3 * (size_t)(n > 0 ? n : 1);
    double *r1 = (double *)malloc(sizeof(double) * m3);
    double *r2 = (double *)malloc(sizeof(double) * m3);
    double *r3 = (double *)malloc(sizeof(double) * m3);
    double *rigid0 = (double *)malloc(sizeof(double) * m3);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            v[a][i] *= t0;
            rigid0[3 * i + a] = r0[a][i];
        }
    double pe, work = 0.0, power_prev = 0.0;
    int rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
    if (rc) goto done;
    power_prev = -rigid_power(n, f, rigid, vp);
    for (int64_t i = 0; i < n; ++i) {
        const double m = p->mass[species[i]];
        for (int a = 0; a < 3; ++a) {
            r1[3 * i + a] = h * v[a][i];
            r2[3 * i + a] = 0.5 * h * h * f[3 * i + a] / m;
            r3[3 * i + a] = 0.0;
        }
    }
    for (int64_t s = 0;; ++s) {
        if (pe_out) pe_out[s] = pe;
        if (ke_out) ke_out[s] = mobile_ke(n, v, species, rigid, p);
        if (work_out) work_out[s] = work;
        if (s == nsteps) break;
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) {
                const double t = (double)(s + 1) * h;
                for (int a = 0; a < 3; ++a) r0[a][i] = rigid0[3 * i + a] + vp[a] * t;
                continue;
            }
            for (int a = 0; a < 3; ++a) {
                const size_t k = 3 * (size_t)i + a;
                r0[a][i] += r1[k] + r2[k] + r3[k];
                r1[k] += 2.0 * r2[k] + 3.0 * r3[k];
                r2[k] += 3.0 * r3[k];
            }
        }
        rc = or_forces(n, x, y, z, species, rigid, box, periodic, p, f, NULL, NULL, NULL, &pe);
        if (rc) goto done;
        for (int64_t i = 0; i < n; ++i) {
            if (rigid && rigid[i]) continue;
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) {
                const size_t k = 3 * (size_t)i + a;
                const double e = 0.5 * h * h * f[k] / m - r2[k];
                r0[a][i] += c[0] * e;
                r1[k] += c[1] * e;
                r2[k] += c[2] * e;
                r3[k] += c[3] * e;
                v[a][i] = r1[k] / h;
            }
        }
        const double power = -rigid_power(n, f, rigid, vp);
        work += 0.5 * h * (power_prev + power);
        power_prev = power;
    }
done:
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
        if (rigid && rigid[i])
            for (int a = 0; a < 3; ++a) v[a][i] = vp_fs ? vp_fs[a] : 0.0;
    }
    free(r1);
    free(r2);
    free(r3);
    free(rigid0);
    return rc;
}

/*
 * Parrinello-Rahman barostat (paper, "Barostat NPTp"), restricted to an
 * orthorhombic box: the box matrix h = diag(L) and a hydrostatic external
 * stress S = P.  The particle equations in the velocities v = h ds/dt read
 * dv/dt = f/m - (dL/dt / L) v per axis and dx/dt = (dL/dt / L)(x - o) + v;
 * the box obeys W d2L_a/dt2 = sigma_aa (pi_aa - P), sigma = Omega h^-T (the
 * reciprocal box, Omega / L_a on the diagonal) and pi = (sum_i m v v + W_vir)
 * / Omega the internal stress.  PE + KE + P Omega + W |dL/dt|^2 / 2 is
 * conserved.  A step composes exact sub-flows symmetrically: box half kick,
 * friction half step v *= exp(-(h/2) dL/dt / L), velocity half kick, drift of
 * positions and box with dL/dt held (s = (x - o)/L moves by v h log1p(u)/(u L),
 * u = h dL/dt / L), forces, then the mirror image.  All axes must be
 * periodic.  Outputs per step s: pe, ke, box[3], ldot[3] (A/fs), the
 * barostat energy P Omega + W |dL/dt|^2 / 2 and the pressure (2 KE + tr W) /
 * (3 Omega) in GPa.  W in eV fs^2 / A^2, P in GPa; ldot0 (A/fs) may be NULL.
 */
static void pr_box_kick(int64_t n, double *const v[3], const uint8_t *species, const or_potential *p,
                        const double vir[6], const double L[3], double tau, double w, double pext,
                        double ldot[3])
{
    double k2[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double m = p->mass[species[i]];
        for (int a = 0; a < 3; ++a) k2[a] += m * v[a][i] * v[a][i];
    }
    const double omega = L[0] * L[1] * L[2];
    for (int a = 0; a < 3; ++a) {
        const double pi_aa = (k2[a] + vir[a]) / omega;
        const double sigma_aa = omega / L[a];
        ldot[a] += tau * sigma_aa * (pi_aa - pext) / w;
    }
}

static void pr_friction(int64_t n, double *const v[3], const double L[3], const double ldot[3], double tau)
{
    for (int a = 0; a < 3; ++a) {
        const double s = exp(-tau * ldot[a] / L[a]);
        for (int64_t i = 0; i < n; ++i) v[a][i] *= s;
    }
}

int or_run_pr(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              const uint8_t *species, double *box, const double *origin, const double *ldot0_fs,
              const or_potential *p, double dt_fs, int64_t nsteps, double p_gpa, double w_ev_fs2_a2, double *f,
              double *pe_out, double *ke_out, double *box_out, double *ldot_out, double *baro_out,
              double *press_out)
{
    const uint8_t periodic[3] = {1, 1, 1};
    const double t0 = or_time_unit_fs();
    const double h = dt_fs / t0;
    const double w = w_ev_fs2_a2 / (t0 * t0);
    const double pext = p_gpa / or_pressure_unit_gpa();
    double *v[3] = {vx, vy, vz};
    double *r[3] = {x, y, z};
    double L[3] = {box[0], box[1], box[2]}, ldot[3] = {0.0, 0.0, 0.0}, vir[6], pe;
    if (ldot0_fs)
        for (int a = 0; a < 3; ++a) ldot[a] = ldot0_fs[a] * t0;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] *= t0;
    int rc = or_forces(n, x, y, z, species, NULL, L, periodic, p, f, NULL, NULL, vir, &pe);
    if (rc) goto done;
    for (int64_t s = 0;; ++s) {
        if (pe_out) pe_out[s] = pe;
        if (ke_out) ke_out[s] = mobile_ke(n, v, species, NULL, p);
        const double omega = L[0] * L[1] * L[2];
        if (box_out)
            for (int a = 0; a < 3; ++a) box_out[3 * s + a] = L[a];
        if (ldot_out)
            for (int a = 0; a < 3; ++a) ldot_out[3 * s + a] = ldot[a] / t0;
        if (baro_out)
            baro_out[s] = pext * omega + 0.5 * w * (ldot[0] * ldot[0] + ldot[1] * ldot[1] + ldot[2] * ldot[2]);
        if (press_out)
            press_out[s] = (2.0 * mobile_ke(n, v, species, NULL, p) + vir[0] + vir[1] + vir[2]) / (3.0 * omega) *
                           or_pressure_unit_gpa();
        if (s == nsteps) break;
        pr_box_kick(n, v, species, p, vir, L, 0.5 * h, w, pext, ldot);
        pr_friction(n, v, L, ldot, 0.5 * h);
        for (int64_t i = 0; i < n; ++i) {
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * h * f[3 * i + a] / m;
        }
        for (int a = 0; a < 3; ++a) {
            const double u = h * ldot[a] / L[a];
            const double phi = u == 0.0 ? 1.0 : log1p(u) / u;
            const double Ln = L[a] + h * ldot[a];
            for (int64_t i = 0; i < n; ++i)
                r[a][i] = origin[a] + (r[a][i] - origin[a] + v[a][i] * h * phi) * (Ln / L[a]);
            L[a] = Ln;
        }
        rc = or_forces(n, x, y, z, species, NULL, L, periodic, p, f, NULL, NULL, vir, &pe);
        if (rc) goto done;
        for (int64_t i = 0; i < n; ++i) {
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * h * f[3 * i + a] / m;
        }
        pr_friction(n, v, L, ldot, 0.5 * h);
        pr_box_kick(n, v, species, p, vir, L, 0.5 * h, w, pext, ldot);
    }
done:
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
    for (int a = 0; a < 3; ++a) box[a] = L[a];
    return rc;
}

/*
 * Parrinello-Rahman barostat with the Nose-Hoover thermostat (paper, "Barostat
 * NPTp": "NPEp (or with Nose, NPTp)"), orthorhombic box.  The particle
 * velocities feel both frictions, -(dL/dt / L) v and -pi_s v; the box and the
 * thermostat follow their own equations as in or_run_pr and or_run_nh.  A step
 * composes the exact sub-flows symmetrically: box half kick, thermostat half
 * step, box friction half step, velocity half kick, drift, forces, and the
 * mirror image.  PE + KE + P Omega + W |dL/dt|^2 / 2 + Q pi_s^2 / 2 + g k_B T xi
 * is conserved.  Outputs as or_run_pr, plus nh_out[2s] = pi_s (1/fs) and
 * nh_out[2s+1] = Q pi_s^2 / 2 + g k_B T xi.
 */
int or_run_npt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
               const uint8_t *species, double *box, const double *origin, const or_potential *p, double dt_fs,
               int64_t nsteps, double p_gpa, double w_ev_fs2_a2, double t_target, double q_ev_fs2, double *f,
               double *pe_out, double *ke_out, double *box_out, double *baro_out, double *press_out, double *nh_out)
{
    const uint8_t periodic[3] = {1, 1, 1};
    const double t0 = or_time_unit_fs();
    const double h = dt_fs / t0;
    const double w = w_ev_fs2_a2 / (t0 * t0);
    const double q = q_ev_fs2 / (t0 * t0);
    const double pext = p_gpa / or_pressure_unit_gpa();
    const double gkt = (3.0 * (double)n - 3.0) * OR_KB_EV_PER_K * t_target;
    double *v[3] = {vx, vy, vz};
    double *r[3] = {x, y, z};
    double L[3] = {box[0], box[1], box[2]}, ldot[3] = {0.0, 0.0, 0.0}, vir[6], pe, pi = 0.0, xi = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] *= t0;
    int rc = or_forces(n, x, y, z, species, NULL, L, periodic, p, f, NULL, NULL, vir, &pe);
    if (rc) goto done;
    for (int64_t s = 0;; ++s) {
        const double omega = L[0] * L[1] * L[2];
        const double ke = mobile_ke(n, v, species, NULL, p);
        if (pe_out) pe_out[s] = pe;
        if (ke_out) ke_out[s] = ke;
        if (box_out)
            for (int a = 0; a < 3; ++a) box_out[3 * s + a] = L[a];
        if (baro_out)
            baro_out[s] = pext * omega + 0.5 * w * (ldot[0] * ldot[0] + ldot[1] * ldot[1] + ldot[2] * ldot[2]);
        if (press_out) press_out[s] = (2.0 * ke + vir[0] + vir[1] + vir[2]) / (3.0 * omega) * or_pressure_unit_gpa();
        if (nh_out) {
            nh_out[2 * s] = pi / t0;
            nh_out[2 * s + 1] = 0.5 * q * pi * pi + gkt * xi;
        }
        if (s == nsteps) break;
        pr_box_kick(n, v, species, p, vir, L, 0.5 * h, w, pext, ldot);
        nh_half_step(n, v, species, NULL, p, 0.5 * h, q, gkt, &pi, &xi);
        pr_friction(n, v, L, ldot, 0.5 * h);
        for (int64_t i = 0; i < n; ++i) {
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * h * f[3 * i + a] / m;
        }
        for (int a = 0; a < 3; ++a) {
            const double u = h * ldot[a] / L[a];
            const double phi = u == 0.0 ? 1.0 : log1p(u) / u;
            const double Ln = L[a] + h * ldot[a];
            for (int64_t i = 0; i < n; ++i)
                r[a][i] = origin[a] + (r[a][i] - origin[a] + v[a][i] * h * phi) * (Ln / L[a]);
            L[a] = Ln;
        }
        rc = or_forces(n, x, y, z, species, NULL, L, periodic, p, f, NULL, NULL, vir, &pe);
        if (rc) goto done;
        for (int64_t i = 0; i < n; ++i) {
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * h * f[3 * i + a] / m;
        }
        pr_friction(n, v, L, ldot, 0.5 * h);
        nh_half_step(n, v, species, NULL, p, 0.5 * h, q, gkt, &pi, &xi);
        pr_box_kick(n, v, species, p, vir, L, 0.5 * h, w, pext, ldot);
    }
done:
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
    for (int a = 0; a < 3; ++a) box[a] = L[a];
    return rc;
}

/* ---- Box matrices (paper, "Barostat NPTp") --------------------------------
 * h = [a, b, c] with the edge vectors as columns, r = h x; row-major storage. */
static void m3_mul(const double *a, const double *b, double *o)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) t[3 * r + c] = a[3 * r] * b[c] + a[3 * r + 1] * b[3 + c] + a[3 * r + 2] * b[6 + c];
    memcpy(o, t, sizeof t);
}

static void m3_transpose(const double *a, double *o)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) t[3 * r + c] = a[3 * c + r];
    memcpy(o, t, sizeof t);
}

static double m3_det(const double *a)
{
    return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

/* Inverse by cofactors over the determinant. */
static void m3_inverse(const double *a, double *o)
{
    const double id = 1.0 / m3_det(a);
    double t[9];
    t[0] = (a[4] * a[8] - a[5] * a[7]) * id;
    t[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    t[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    t[3] = (a[5] * a[6] - a[3] * a[8]) * id;
    t[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    t[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    t[6] = (a[3] * a[7] - a[4] * a[6]) * id;
    t[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    t[8] = (a[0] * a[4] - a[1] * a[3]) * id;
    memcpy(o, t, sizeof t);
}

static void m3_apply(const double *m, const double *v, double *o)
{
    double t[3];
    for (int r = 0; r < 3; ++r) t[r] = m[3 * r] * v[0] + m[3 * r + 1] * v[1] + m[3 * r + 2] * v[2];
    memcpy(o, t, sizeof t);
}

static double m3_norm1(const double *a)
{
    double m = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double s = fabs(a[c]) + fabs(a[3 + c]) + fabs(a[6 + c]);
        if (s > m) m = s;
    }
    return m;
}

/* exp(a): the Taylor series, summed until its terms stop changing the sum,
 * after halving a until its norm is below 1/2 and squaring back. */
static void m3_exp(const double *a, double *o)
{
    int sq = 0;
    double b[9];
    memcpy(b, a, sizeof b);
    while (m3_norm1(b) > 0.5) {
        for (int k = 0; k < 9; ++k) b[k] *= 0.5;
        ++sq;
    }
    double sum[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, term[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int k = 1; k < 40; ++k) {
        m3_mul(term, b, term);
        for (int e = 0; e < 9; ++e) term[e] /= (double)k;
        for (int e = 0; e < 9; ++e) sum[e] += term[e];
        if (m3_norm1(term) < 1e-18 * m3_norm1(sum)) break;
    }
    for (int k = 0; k < sq; ++k) m3_mul(sum, sum, sum);
    memcpy(o, sum, sizeof sum);
}

/* phi(z) = sum_{k>=0} (-z)^k / (k + 1) = z^-1 log(1 + z) for |z| < 1: the
 * integral over t in [0, 1] of (1 + t z)^-1.  Returns -1 if |z| >= 1/2. */
static int m3_logphi(const double *z, double *o)
{
    if (m3_norm1(z) >= 0.5) return -1;
    double sum[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, pw[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int k = 1; k < 80; ++k) {
        m3_mul(pw, z, pw);
        for (int e = 0; e < 9; ++e) pw[e] = -pw[e];
        double term[9];
        for (int e = 0; e < 9; ++e) term[e] = pw[e] / (double)(k + 1);
        for (int e = 0; e < 9; ++e) sum[e] += term[e];
        if (m3_norm1(term) < 1e-18) break;
    }
    memcpy(o, sum, sizeof sum);
    return 0;
}

/* Returns 0 when every width of the cell h exceeds twice the cutoff. */
static int tri_geom(const double *h, double rc, or_geom *g)
{
    g->box = NULL;
    g->periodic = NULL;
    memcpy(g->h, h, sizeof g->h);
    if (!(fabs(m3_det(h)) > 0.0)) return -1;
    m3_inverse(h, g->hi);
    for (int a = 0; a < 3; ++a) {
        const double w = 1.0 / sqrt(g->hi[3 * a] * g->hi[3 * a] + g->hi[3 * a + 1] * g->hi[3 * a + 1] +
                                    g->hi[3 * a + 2] * g->hi[3 * a + 2]);
        if (!(w > 2.0 * rc)) return -1;
    }
    return 0;
}

/* or_forces in a periodic cell with box matrix h[9] (paper, "Barostat NPTp"
 * for h, "Boundary conditions" for the shortest image).  Same outputs.
 * Returns -1 if a width of the cell is not larger than twice the cutoff. */
int or_forces_tri(int64_t n, const double *x, const double *y, const double *z,
                  const uint8_t *species, const uint8_t *rigid, const double *h,
                  const or_potential *p, double *f, double *e_atom, double *rho_out,
                  double *virial, double *pe)
{
    const double rc = or_cutoff(p);
    or_geom g;
    if (tri_geom(h, rc, &g)) return -1;
    forces_geom(n, x, y, z, species, rigid, &g, p, rc, f, e_atom, rho_out, virial, pe);
    return 0;
}

/* or_forces_sampled in a periodic cell with box matrix h[9]. */
int or_forces_sampled_tri(int64_t n, const double *x, const double *y, const double *z,
                          const uint8_t *species, const double *h, const or_potential *p, int64_t m,
                          const int64_t *sample, double *f, double *e_atom, double *rho_out)
{
    const double rc = or_cutoff(p);
    or_geom g;
    if (tri_geom(h, rc, &g)) return -1;
    return sampled_geom(n, x, y, z, species, &g, p, rc, m, sample, f, e_atom, rho_out);
}

/*
 * Parrinello-Rahman dynamics of the full box matrix (paper, "Barostat NPTp":
 * the Lagrangian with nine box degrees of freedom, the external pressure P and
 * the external stress S, and the box equation of motion
 *   W h'' = (pi - P) sigma - h Sigma,
 * sigma = Omega h^-T (columns b x c, c x a, a x b), pi = (sum m v v^T + Wvir) / Omega
 * the internal stress, Sigma = Omega0 h0^-1 (S - P) h0^-T with h0 the starting
 * box (the reading that makes the Lagrangian's elastic term the strain energy
 * Omega0 tr((S - P) eps) of the printed strain eps = (h0^-T h^T h h0^-1 - 1) / 2).
 * With v = h ds/dt the particles obey dv/dt = f/m - h^-T h'^T v and
 * dr/dt = v + h' h^-1 (r - o).  The conserved quantity is
 * PE + KE + P Omega + W tr(h'^T h') / 2 + Omega0 tr((S - P) eps).
 * With a thermostat (q > 0) the velocities also feel -pi_s v and pi_s follows
 * the Nose-Hoover equation of or_run_nh (NPTp); its energy adds Q pi_s^2 / 2 +
 * g k_B T xi.
 *
 * A step composes exact sub-flows symmetrically: box half kick, thermostat half
 * step, friction half step v <- exp(-(h/2) h^-T h'^T) v, velocity half kick,
 * drift with h' held (r <- o + h_new h^-1 (r - o) + dt h_new phi(dt h^-1 h') h^-1 v,
 * h_new = h + dt h', phi(z) = z^-1 log(1 + z)), forces, and the mirror image.
 * w = 0 keeps the box fixed (plain velocity Verlet in a sheared cell).
 *
 * Inputs: h[9] (A, overwritten by the final box), origin[3], hdot0[9] (A/fs,
 * may be NULL), stress[9] (GPa, symmetric; NULL means S = P), href[9] (the
 * reference box h0 of the strain; NULL: the starting box), P in GPa, W in
 * eV fs^2 / A^2, the thermostat target (K) and Q (eV fs^2; q <= 0: none).
 * Outputs per step s = 0..nsteps (each may be NULL): pe, ke, h_out[9 s],
 * hdot_out[9 s] (A/fs), baro_out[s] = P Omega + W tr(h'^T h')/2 + the strain
 * energy, stress_out[6 s] = pi (xx, yy, zz, xy, xz, yz) in GPa, nh_out[2 s] =
 * (pi_s in 1/fs, its energy).  Returns 0, -1 for a cell too thin for the
 * cutoff, -2 if the box moves more than half its size in one step.
 */
int or_run_prt(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
               const uint8_t *species, double *hbox, const double *origin, const double *hdot0_fs,
               const double *stress_gpa, const double *href, const or_potential *p, double dt_fs, int64_t nsteps,
               double p_gpa,
               double w_ev_fs2_a2, double t_target, double q_ev_fs2, double *f, double *pe_out, double *ke_out,
               double *h_out, double *hdot_out, double *baro_out, double *stress_out, double *nh_out)
{
    const double t0 = or_time_unit_fs();
    const double dt = dt_fs / t0;
    const double w = w_ev_fs2_a2 / (t0 * t0);
    const double pext = p_gpa / or_pressure_unit_gpa();
    const int nvt = q_ev_fs2 > 0.0;
    const double q = nvt ? q_ev_fs2 / (t0 * t0) : 1.0;
    const double gkt = (3.0 * (double)n - 3.0) * OR_KB_EV_PER_K * t_target;
    const double rc = or_cutoff(p);
    double *v[3] = {vx, vy, vz};
    double *r[3] = {x, y, z};
    double H[9], Hd[9] = {0}, h0i[9], Sig[9], sp[9], vir[6], pe, pi_s = 0.0, xi = 0.0;
    memcpy(H, hbox, sizeof H);
    if (hdot0_fs)
        for (int k = 0; k < 9; ++k) Hd[k] = hdot0_fs[k] * t0;
    const double *h0 = href ? href : hbox;
    const double omega0 = fabs(m3_det(h0));
    for (int k = 0; k < 9; ++k) sp[k] = (stress_gpa ? stress_gpa[k] / or_pressure_unit_gpa() : 0.0);
    if (!stress_gpa)
        for (int a = 0; a < 3; ++a) sp[4 * a] = pext;
    for (int a = 0; a < 3; ++a) sp[4 * a] -= pext; /* S - P */
    m3_inverse(h0, h0i);
    {
        double t[9], h0it[9];
        m3_transpose(h0i, h0it);
        m3_mul(h0i, sp, t);
        m3_mul(t, h0it, Sig);
        for (int k = 0; k < 9; ++k) Sig[k] *= omega0;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] *= t0;
    or_geom g;
    int rc_ = tri_geom(H, rc, &g);
    if (rc_) goto done;
    forces_geom(n, x, y, z, species, NULL, &g, p, rc, f, NULL, NULL, vir, &pe);

    for (int64_t s = 0;; ++s) {
        const double omega = fabs(m3_det(H));
        double K[9] = {0};
        for (int64_t i = 0; i < n; ++i) {
            const double m = p->mass[species[i]];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) K[3 * a + b] += m * v[a][i] * v[b][i];
        }
        const double ke = 0.5 * (K[0] + K[4] + K[8]);
        if (pe_out) pe_out[s] = pe;
        if (ke_out) ke_out[s] = ke;
        if (h_out) memcpy(h_out + 9 * s, H, sizeof H);
        if (hdot_out)
            for (int k = 0; k < 9; ++k) hdot_out[9 * s + k] = Hd[k] / t0;
        if (baro_out) {
            double kb = 0.0, eps[9], G[9], ht[9], t[9], h0it[9], el = 0.0;
            for (int k = 0; k < 9; ++k) kb += Hd[k] * Hd[k];
            m3_transpose(H, ht);
            m3_mul(ht, H, G);
            m3_transpose(h0i, h0it);
            m3_mul(h0it, G, t);
            m3_mul(t, h0i, eps);
            for (int a = 0; a < 3; ++a) eps[4 * a] -= 1.0;
            for (int k = 0; k < 9; ++k) eps[k] *= 0.5;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) el += sp[3 * a + b] * eps[3 * b + a];
            baro_out[s] = pext * omega + 0.5 * w * kb + omega0 * el;
        }
        if (stress_out) {
            const int ia[6] = {0, 4, 8, 1, 2, 5}, iv[6] = {0, 1, 2, 3, 4, 5};
            for (int c = 0; c < 6; ++c)
                stress_out[6 * s + c] = (K[ia[c]] + vir[iv[c]]) / omega * or_pressure_unit_gpa();
        }
        if (nh_out) {
            nh_out[2 * s] = pi_s / t0;
            nh_out[2 * s + 1] = 0.5 * q * pi_s * pi_s + gkt * xi;
        }
        if (s == nsteps) break;
        for (int half = 0; half < 2; ++half) {
            /* half == 0: box kick, thermostat, friction, kick (then drift);
             * half == 1: kick, friction, thermostat, box kick (after forces) */
            if (half == 1) {
                for (int64_t i = 0; i < n; ++i) {
                    const double m = p->mass[species[i]];
                    for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * dt * f[3 * i + a] / m;
                }
            }
            for (int stage = 0; stage < 3; ++stage) {
                const int op = half == 0 ? stage : 2 - stage; /* 0 box kick, 1 thermostat, 2 friction */
                if (op == 0 && w > 0.0) {
                    double Kt[9] = {0}, pi_t[9], sig[9], hi[9], t[9], hs[9];
                    for (int64_t i = 0; i < n; ++i) {
                        const double m = p->mass[species[i]];
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) Kt[3 * a + b] += m * v[a][i] * v[b][i];
                    }
                    const double om = fabs(m3_det(H));
                    const double wv[9] = {vir[0], vir[3], vir[4], vir[3], vir[1], vir[5], vir[4], vir[5], vir[2]};
                    for (int k = 0; k < 9; ++k) pi_t[k] = (Kt[k] + wv[k]) / om;
                    for (int a = 0; a < 3; ++a) pi_t[4 * a] -= pext;
                    m3_inverse(H, hi);
                    m3_transpose(hi, sig);
                    for (int k = 0; k < 9; ++k) sig[k] *= om;
                    m3_mul(pi_t, sig, t);
                    m3_mul(H, Sig, hs);
                    for (int k = 0; k < 9; ++k) Hd[k] += 0.5 * dt * (t[k] - hs[k]) / w;
                } else if (op == 1 && nvt) {
                    nh_half_step(n, v, species, NULL, p, 0.5 * dt, q, gkt, &pi_s, &xi);
                } else if (op == 2 && w > 0.0) {
                    double hi[9], hit[9], hdt[9], A[9], E[9];
                    m3_inverse(H, hi);
                    m3_transpose(hi, hit);
                    m3_transpose(Hd, hdt);
                    m3_mul(hit, hdt, A);
                    for (int k = 0; k < 9; ++k) A[k] *= -0.5 * dt;
                    m3_exp(A, E);
                    for (int64_t i = 0; i < n; ++i) {
                        double vi[3] = {v[0][i], v[1][i], v[2][i]};
                        m3_apply(E, vi, vi);
                        for (int a = 0; a < 3; ++a) v[a][i] = vi[a];
                    }
                }
            }
            if (half == 1) break;
            for (int64_t i = 0; i < n; ++i) {
                const double m = p->mass[species[i]];
                for (int a = 0; a < 3; ++a) v[a][i] += 0.5 * dt * f[3 * i + a] / m;
            }
            /* drift with h' held */
            double hi[9], B[9], Phi[9], Hn[9], M[9], D[9], t[9];
            m3_inverse(H, hi);
            m3_mul(hi, Hd, B);
            for (int k = 0; k < 9; ++k) B[k] *= dt;
            if (m3_logphi(B, Phi)) {
                rc_ = -2;
                goto done;
            }
            for (int k = 0; k < 9; ++k) Hn[k] = H[k] + dt * Hd[k];
            m3_mul(Hn, hi, M);
            m3_mul(Hn, Phi, t);
            m3_mul(t, hi, D);
            for (int k = 0; k < 9; ++k) D[k] *= dt;
            for (int64_t i = 0; i < n; ++i) {
                double xo[3], vi[3] = {v[0][i], v[1][i], v[2][i]}, a1[3], a2[3];
                for (int a = 0; a < 3; ++a) xo[a] = r[a][i] - origin[a];
                m3_apply(M, xo, a1);
                m3_apply(D, vi, a2);
                for (int a = 0; a < 3; ++a) r[a][i] = origin[a] + a1[a] + a2[a];
            }
            memcpy(H, Hn, sizeof H);
            rc_ = tri_geom(H, rc, &g);
            if (rc_) goto done;
            forces_geom(n, x, y, z, species, NULL, &g, p, rc, f, NULL, NULL, vir, &pe);
        }
    }
done:
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) v[a][i] /= t0;
    memcpy(hbox, H, sizeof H);
    return rc_;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel loops (timing at one thread and at all). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
