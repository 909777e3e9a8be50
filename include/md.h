/*
 * md.h - C ABI of the MI355X embedded-atom molecular-dynamics hot path.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the per-timestep
 * force loop of a short-range embedded-atom / Finnis-Sinclair model as
 * described in the MOLDY paper (Ackland et al., arXiv 1107.2619):
 *
 *   - link-cell binning and the Verlet neighbour list built from adjacent
 *     link cells ("The Neighbourlist calculation");
 *   - the density pass rho_i = sum_j rho_{s_i s_j}(r_ij) and the embedding
 *     F(rho_i) = -c sqrt(rho_i) with its derivative (Eq. Ucoh and the
 *     Finnis-Sinclair square root, "Theoretical background");
 *   - the force pass f_i = sum_j [phi'(r) + F'_i rho'_{ij}(r) + F'_j rho'_{ji}(r)] d_ij / r
 *     (the gradient of Eq. Ucoh);
 *   - velocity-Verlet integration ("Time integration"), rigid atoms moving on
 *     a prescribed line ("Fixed atoms"), and the energy, kinetic-energy and
 *     virial reductions ("Thermodynamic Quantities").
 *
 * Units at the boundary (paper, "Units"): Angstrom, amu, eV, fs; velocities in
 * Angstrom/fs, forces in eV/Angstrom, pressure in GPa.
 *
 * Conventions for every entry point:
 *   - Every function returns an int status: MD_OK (0) or a negative MD_ERR_*.
 *     On failure md_last_error(ctx) returns a message.
 *   - "host" pointers are read during the call only; "device" pointers are
 *     HIP device memory owned by the caller and must stay valid while bound.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued asynchronously on it; only md_energy synchronises.
 *   - Errors raised on the device (neighbour overflow, skin violation,
 *     non-finite energies) are sticky and reported by the next md_energy.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef MDEAM_MD_H
#define MDEAM_MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx; /* opaque; created by md_create, freed by md_destroy */

enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,          /* NULL pointer, bad size or bad enum value            */
    MD_ERR_BOX = -2,          /* periodic length <= 2 (cutoff + skin), or bad box    */
    MD_ERR_POTENTIAL = -3,    /* unsupported species count, knots, or coefficients   */
    MD_ERR_NBR_OVERFLOW = -4, /* an atom has more list entries than max_neighbours   */
    MD_ERR_SKIN = -5,         /* an atom moved more than skin/2 between list builds  */
    MD_ERR_NONFINITE = -6,    /* NaN or Inf in the energies                          */
    MD_ERR_DEVICE = -7,       /* a HIP runtime call failed                           */
    MD_ERR_STATE = -8         /* call out of order (e.g. md_step before md_bind)     */
};

enum { MD_FP64 = 0, MD_MIXED = 1 };              /* md_config.precision */
enum { MD_NBR_FULL = 0, MD_NBR_HALF_ATOMIC = 1 }; /* md_config.nbr_mode  */
enum { MD_VERLET = 0, MD_GEAR3 = 1 };             /* md_config.integrator */

#define MD_MAX_SPECIES 4
#define MD_MAX_KNOTS 16

/*
 * Cubic-knot potential (paper, "Available potentials": the generic ATVF form
 * f(r) = sum_k a_k (r_k - r)^3 H(r_k - r)), one function per species pair.
 *   pair_a, pair_r  [ns][ns][n_pair_knots]  pair potential phi_ab; must be
 *                   symmetric in (a, b).
 *   dens_A, dens_R  [ns][ns][n_dens_knots]  [a][b] = density at an a-site
 *                   from a b-neighbour (EAM: depends on b only; FS:
 *                   symmetric).  Every amplitude must be > 0 so that rho >= 0.
 *   emb_c           [ns]  F_a(rho) = -emb_c[a] sqrt(rho); F = F' = 0 at rho = 0.
 *   mass_amu        [ns]  > 0.
 * All host pointers; md_create copies them.  The cutoff r_c is the largest knot.
 * Evaluation (paper, "Parallel benchmarks": lookup table against direct
 * evaluation, with a 15-spline iron potential): by default the functions are
 * tabulated exactly on uniform bins, one cubic per bin in the bin-local
 * coordinate, plus, where a knot falls strictly inside a bin, that knot's own
 * term (any knot placement; two knots of one function may not share a bin of
 * the finest width r_c / 4096).  In FP64 the knot sums can also be evaluated
 * term by term (MD_OPT_EVALUATOR = 1), for up to 8 pair and 8 density knots,
 * or, for one species, up to 16 pair and 4 density knots.  MD_ERR_POTENTIAL
 * for a potential that fits no evaluator of the chosen precision (mixed
 * precision always evaluates through the tables).
 */
typedef struct {
    int32_t n_species;    /* 1..MD_MAX_SPECIES */
    int32_t n_pair_knots; /* 1..MD_MAX_KNOTS */
    int32_t n_dens_knots; /* 1..MD_MAX_KNOTS */
    int32_t reserved;     /* must be 0 */
    const double *pair_a, *pair_r;
    const double *dens_A, *dens_R;
    const double *emb_c;
    const double *mass_amu;
} md_potential;

/*
 * Run configuration: R >= 1 independent replicas (the paper's Introduction
 * averages results over many equivalent runs), each an orthorhombic box
 * with per-axis periodic or free boundaries ("Boundary conditions"), or a
 * periodic cell given by its box matrix.  Replica
 * r owns atoms [atom_offset[r], atom_offset[r+1]) of the state arrays.
 * All pointers are host pointers, copied by md_create.
 */
typedef struct {
    int32_t n_replicas;     /* R >= 1 */
    int32_t max_neighbours; /* per-atom list capacity (the paper's nnbrs), >= 1 */
    int32_t rebuild_every;  /* list rebuild period in steps (nbrupdate), >= 1 */
    int32_t precision;      /* MD_FP64 or MD_MIXED */
    int32_t nbr_mode;       /* MD_NBR_FULL or MD_NBR_HALF_ATOMIC */
    int32_t lanes_per_atom; /* LDS-brick kernels: lanes sharing one atom's neighbours,
                               0 = automatic, 1, 2 or 4 (the global kernels use one) */
    const int64_t *atom_offset;   /* [R+1], atom_offset[0] = 0, non-decreasing */
    const double *box;            /* [R][3] edge lengths, Angstrom, > 0 */
    const double *origin;         /* [R][3] lower corner (matters on free axes); NULL = 0 */
    const uint8_t *periodic;      /* [R][3] 1 = periodic (minimum image), 0 = free */
    const double *rigid_velocity; /* [R][3] Angstrom/fs of rigid atoms; NULL = 0 */
    double skin;                  /* list padding beyond r_c (the paper's rpad), >= 0 */
    double dt_fs;                 /* time step, fs, > 0 */
    /* Nose-Hoover thermostat per replica ("Thermostat NVTp"): md_step then
     * integrates the NVT equations of motion, the thermostat momentum pi_s
     * obeying Q dpi_s/dt = 2 KE - g k_B T (g = 3N - 3, or 3N_mobile with rigid
     * atoms), split symmetrically around the velocity-Verlet step.  Both NULL =
     * NVE; both set = every replica thermostatted. */
    const double *nh_temperature; /* [R] target temperature, K, >= 0 */
    const double *nh_mass;        /* [R] thermostat mass Q, eV fs^2, > 0 */
    /* Time integration ("Time integration"): MD_VERLET (velocity Verlet) or
     * MD_GEAR3, the third-order Gear predictor-corrector, which carries the
     * acceleration and its time derivative beside x and v.  Those two live in
     * the workspace: the first md_step after md_bind starts them (a = f/m,
     * da/dt = 0) and later calls continue from them, so x and v should change
     * between md_step calls only through md_step (or md_bind again).  Forces
     * and potential energy are those at the predicted positions of the last
     * step; rigid atoms' work uses the trapezoid rule over the evaluations.
     * MD_GEAR3 runs NVE only (no thermostat). */
    int32_t integrator;
    /* Parrinello-Rahman barostat per replica ("Barostat NPTp").  On an
     * orthorhombic box (no box_matrix, no pr_stress_gpa below): h = diag(L)
     * and a hydrostatic external stress.  The
     * box edges obey W d2L_a/dt2 = (Omega / L_a)(pi_aa - P), pi the internal
     * stress tensor, and the particles feel the matching friction
     * -(dL_a/dt / L_a) v_a (NPH; PE + KE + P Omega + W |dL/dt|^2 / 2 is
     * conserved).  Both NULL = fixed box; both set = every replica under its
     * own pressure.  With the thermostat set too, the particles feel both
     * frictions (NPT; pe + ke + pr_energy + nh_energy is conserved).  Needs
     * periodic axes, MD_VERLET, the full list and no rigid atoms; the
     * link-cell grid leaves 5% room for compression (more gives MD_ERR_BOX).
     * The LDS-brick kernels are not used. */
    const double *pr_pressure_gpa; /* [R] external pressure, GPa, finite */
    const double *pr_mass;         /* [R] box mass W, eV fs^2 / Angstrom^2, > 0 */
    /* Box matrices ("Barostat NPTp": r = o + h s with h = [a, b, c], the edge
     * vectors as columns, s the fractional coordinates).  box_matrix [R][9]
     * row-major (h[3 i + j] = component i of edge j), determinant > 0; NULL =
     * the orthorhombic boxes of `box` (which may then be NULL).  A box matrix
     * needs every axis periodic and at least three link cells between each
     * pair of opposite faces (width >= 3 (r_c + skin), 3.15 (r_c + skin) under
     * the barostat); the separation of a pair is its shortest image.  The
     * LDS-brick kernels and the compact mixed-mode records are not used.
     * With the barostat set, a box matrix (or pr_stress_gpa) makes all nine
     * entries of h dynamic: W d2h/dt2 = (pi - P) sigma - h Sigma with
     * sigma = Omega h^-T, Sigma = Omega0 h0^-1 (S - P) h0^-T and h0 the box at
     * md_bind, and the particles feel -h^-T (dh/dt)^T v (the conserved
     * quantity is pe + ke + pr_energy, + nh_energy with the thermostat). */
    const double *box_matrix;      /* [R][9] Angstrom, or NULL */
    const double *pr_stress_gpa;   /* [R][9] external stress S, GPa, symmetric; NULL = P on
                                      the diagonal.  Needs the barostat. */
} md_config;

/*
 * Per-atom state: device pointers, caller-owned, in the caller's atom order
 * (which the library never changes; it keeps its own cell-sorted copy).
 * Positions are unwrapped ("Boundary conditions": no wraparound).
 *   x,y,z     [N] Angstrom (read at each call, written by md_step)
 *   vx,vy,vz  [N] Angstrom/fs (read at each call, written by md_step)
 *   fx,fy,fz  [N] eV/Angstrom (written)
 *   species   [N] uint8 < n_species (read at md_bind)
 *   rigid     [N] uint8, 1 = moves at rigid_velocity of its replica; NULL = none
 *   e_atom    [N] eV per-atom energy 1/2 sum_j phi + F_i (written when
 *             energies are computed), or NULL
 */
typedef struct {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *fx, *fy, *fz;
    const uint8_t *species;
    const uint8_t *rigid;
    double *e_atom;
} md_state;

/* Per-replica thermodynamic quantities of the last evaluated state. */
typedef struct {
    double pe;           /* potential energy, eV (Eq. Ucoh, pairs counted once) */
    double ke;           /* kinetic energy of the mobile atoms, eV */
    double temperature;  /* K; 3N-3 degrees of freedom, 3N_mobile with rigid atoms */
    double pressure_gpa; /* (2 KE + tr W) / (3 V) */
    double volume;       /* box volume, Angstrom^3 */
    double piston_work;  /* energy delivered by rigid atoms since md_bind, eV */
    double virial[6];    /* W_ab = -sum_{i<j} g_ij d_a d_b / r, eV (xx,yy,zz,xy,xz,yz);
                            pairs of two rigid atoms are skipped ("Fixed atoms") */
    int64_t step;        /* time step index of this state */
    int64_t n_atoms, n_mobile;
    double nh_pi;        /* thermostat momentum pi_s, 1/fs (0 without thermostat) */
    double nh_energy;    /* thermostat energy Q pi_s^2 / 2 + g k_B T xi, eV, with
                            xi the time integral of pi_s: pe + ke + nh_energy is
                            conserved by the NVT dynamics */
    double box[3];       /* edge lengths of this state, Angstrom (they move under
                            the barostat) */
    double pr_energy;    /* barostat energy P Omega + W |dL/dt|^2 / 2, eV (0 without
                            barostat): pe + ke + pr_energy is conserved.  With a
                            box matrix: P Omega + W tr(dh/dt^T dh/dt) / 2 +
                            Omega0 tr((S - P) eps), eps = (h0^-T h^T h h0^-1 - 1) / 2 */
    double h[9];         /* box matrix of this state, row-major, edge vectors as
                            columns (diag(box) for an orthorhombic box); box[]
                            then holds the edge lengths */
} md_energies;

/* Validates the configuration and potential on the host (no device work)
 * and returns a new context in *out.  Box lengths on periodic axes must
 * exceed 2 (r_c + skin).  At most 2^25 atom slots (each replica's atoms
 * rounded up to 64; MD_ERR_ARG beyond). */
int md_create(const md_config *cfg, const md_potential *pot, md_ctx **out);

/* Bytes of device workspace md_bind needs for this context. */
int md_workspace_bytes(const md_ctx *ctx, size_t *bytes);

/* Attaches caller state and a caller-allocated device workspace of at least
 * md_workspace_bytes (256-byte aligned).  Neither is owned by the library.
 * Resets the step counter, the piston work and the neighbour list. */
int md_bind(md_ctx *ctx, const md_state *state, void *workspace, size_t bytes);

/* Reads the positions, sorts the atoms by link cell and builds the Verlet
 * list of all pairs closer than r_c + skin (paper, "The Neighbourlist
 * calculation"; full list, or the half list in MD_NBR_HALF_ATOMIC mode). */
int md_build_neighbours(md_ctx *ctx, void *stream);

/* Evaluates rho, F, F' and the forces at the caller's current positions
 * (building the list first if none exists) and writes fx,fy,fz.  With
 * want_energy != 0 also the energies (read with md_energy) and e_atom. */
int md_eam_forces(md_ctx *ctx, int want_energy, void *stream);

/* Advances nsteps >= 1 velocity-Verlet steps from the caller's x, v.  Rebuilds
 * the list whenever the step index is a multiple of rebuild_every.  On
 * completion x, v, f (and e_atom) hold the final state and the energies of
 * that state are ready.  A call that directly follows another md_step call
 * continues from the state and forces that call left (no reload of x, v and
 * no force pass at entry); after the caller writes x or v it must call
 * md_state_changed, and any other call on the context (md_bind, md_set_option,
 * md_eam_forces, md_build_neighbours, md_autotune) also makes the next md_step
 * read x, v afresh and recompute the forces at the starting positions.  The
 * Gear integrator and the barostat always start afresh.  With
 * MD_OPT_ENERGY_EVERY = k > 0 every step whose index is a multiple of k also
 * reduces PE, KE and the virial (paper, "Thermodynamic Quantities") into the
 * ring read by md_energy_history. */
int md_step(md_ctx *ctx, int32_t nsteps, void *stream);

/* Declares that the caller has written the bound x, v (or other state arrays)
 * since the last md_step: the next md_step reloads them and recomputes the
 * forces before its first kick.  Host only; no device work. */
int md_state_changed(md_ctx *ctx);

/* Synchronises the stream, checks the device error flags and copies the
 * per-replica energies of the last evaluated state to out[0..R). */
int md_energy(md_ctx *ctx, md_energies *out, void *stream);

/* Per-step energies (paper, "Thermodynamic Quantities": the quantities are
 * sampled along the run and averaged): the entries md_step appended to the
 * device ring (MD_OPT_ENERGY_RING entries, MD_OPT_ENERGY_EVERY) since the last
 * md_energy_history call or md_bind, oldest first.  out: host array of
 * max_entries * R records, entry j of replica r at out[j * R + r], each with
 * its step index in .step (entries older than the ring holds are skipped);
 * *n_out receives the number of entries written.  Synchronises the stream. */
int md_energy_history(md_ctx *ctx, md_energies *out, int64_t max_entries, int64_t *n_out, void *stream);

/* Mean square displacement per replica and species (paper, "Self-diffusion
 * in iron": D = lim MSD / 6t, the MSD averaged over atoms), from the unwrapped
 * positions ("Boundary conditions": no wraparound).  msd[r * S + s] (Angstrom^2,
 * S = n_species) is the mean of |x_i - x0_i|^2 over the mobile atoms i of
 * replica r with species s, x the positions in the bound state arrays now and
 * x0 the origin: the positions at md_bind or at the last md_msd_origin.
 * count[r * S + s] receives the number of such atoms (msd is 0 where it is 0);
 * count may be NULL.  Rigid atoms are left out.  msd and count are host arrays
 * of R * S entries, written once the work already on the stream has finished
 * (the call synchronises the stream). */
int md_msd(md_ctx *ctx, double *msd, int64_t *count, void *stream);

/* md_msd for callers that cannot allocate device memory or must not call the
 * allocator (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the same kernels, with their per-chunk partial sums and
 * per-replica results in a static device array of the library (1 MiB per GPU,
 * held until the process ends) instead of the workspace; no hipMalloc or
 * hipFree.  msd and count (not NULL here) as for md_msd.  MD_ERR_ARG when the
 * bound system needs more than the array holds (about 8 doubles per
 * 2048-atom chunk of every replica plus 8 + 2 S per replica, 2^17 in all).
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (other streams or threads) race and must be serialised by the caller.
 * Synchronises the stream. */
int md_msd_static(md_ctx *ctx, double *msd, int64_t *count, void *stream);

/* Takes the positions in the bound state arrays as the new origin x0 of md_msd
 * (device copies enqueued on the stream; md_bind sets the origin as well). */
int md_msd_origin(md_ctx *ctx, void *stream);

/* Test and tuning helpers.
 * md_copy_neighbours: synchronises and copies the current list to host memory
 *   in the caller's atom numbering: counts[N] and list[N][cap] (row-major,
 *   entries beyond counts[i] unspecified).  cap must be >= max_neighbours.
 * md_set_option / md_get_option: integer knobs (see MD_OPT_*). */
int md_copy_neighbours(md_ctx *ctx, int32_t *counts, int32_t *list, int32_t cap, void *stream);

enum {
    MD_OPT_LANES_PER_ATOM = 1, /* 0 (automatic), 1, 2 or 4 lanes share one atom      */
    MD_OPT_USE_GRAPH = 2,      /* 1 = md_step replays its middle steps, two list
                                  rebuild periods at a time, from captured HIP
                                  graphs (launched on a library stream ordered after
                                  and before the caller's stream by events; not with
                                  MD_OPT_TIMING).  Any md_set_option or md_bind
                                  drops the captured graphs.                         */
    MD_OPT_MAX_COUNT = 3,      /* read only: largest list length seen (at md_energy)  */
    MD_OPT_N_BUILDS = 4,       /* read only: list builds since md_bind (automatic
                                  ones as of the last md_energy)                     */
    MD_OPT_TIMING = 5,         /* 1 = bracket every kernel group with HIP events      */
    MD_OPT_EVALUATOR = 6,      /* 0 = exact local-polynomial tables (default), 1 =
                                  term-by-term knot sums (the paper's explicit
                                  evaluation; FP64 only: MD_ERR_ARG in mixed
                                  precision, whose FP32 knot sums miss its energy
                                  tolerance, and for knot counts beyond those
                                  md_potential lists) */
    MD_OPT_KERNEL = 7,         /* 0 = LDS link-cell bricks (full list only),
                                  1 = one thread per atom with global gathers
                                      (default),
                                  2 = LDS bricks whose lists keep each pair of two
                                      atoms of one brick once, both atoms' shares
                                      summed in LDS in 64-bit fixed point (2^-40;
                                      a share of 1024 or more is reported as
                                      MD_ERR_NONFINITE); md_copy_neighbours then
                                      returns those pairs once                     */
    MD_OPT_BRICK_DIMS = 8,     /* 0 = automatic, else bx + 10 by + 100 bz cells (1..4) */
    MD_OPT_BRICK_BLOCK = 9,    /* threads per brick workgroup: 64..1024             */
    MD_OPT_HALO_CAP = 10,      /* atoms one brick's LDS staging area holds (set
                                  smaller to shrink LDS use; larger halos fall back) */
    MD_OPT_HALO_OVERFLOWS = 11, /* read only: brick passes whose halo exceeded the
                                  staging area and read global memory instead
                                  (counted since md_bind, read at md_energy)         */
    MD_OPT_GRAPH_LAUNCHES = 12, /* read only: graph replays since md_create          */
    MD_OPT_TUNED_NS = 13,      /* read only: md_autotune's estimate of one step of
                                  the chosen configuration, ns                       */
    MD_OPT_COMPACT = 14,       /* mixed precision, global kernels, full list: 1 =
                                  gather 16-byte cell-relative fixed-point records
                                  (default), 0 = the FP64 position records; reads
                                  back whether compact records are in use            */
    MD_OPT_ENERGY_EVERY = 15,  /* k > 0: every step whose index is a multiple of k
                                  reduces PE, KE and the virial and appends them to
                                  the energy ring (velocity-Verlet NVE only); 0 =
                                  energies on the last step of each md_step only   */
    MD_OPT_ENERGY_RING = 16,   /* entries of the device energy ring (workspace
                                  grows by entries * R * 96 bytes); set before
                                  md_workspace_bytes and md_bind (MD_ERR_STATE
                                  after md_bind).  Default 0: no ring                */
    MD_OPT_NEIGHBOUR_CHUNK = 17, /* global kernels: neighbour records each thread
                                  gathers before it evaluates them, 2, 4 (default)
                                  or 8; md_autotune picks it.  Results do not
                                  depend on it (same terms, same order)              */
    MD_OPT_AUTO_REBUILD = 18   /* 1 = rebuild on displacement instead of every
                                  rebuild_every steps ("The Neighbourlist
                                  calculation": the list of r_c + skin stays
                                  complete while no atom moves more than skin/2
                                  from where it was at the build).  Before every
                                  force evaluation of md_step and md_eam_forces
                                  each replica with an atom past skin/2 is
                                  re-sorted and gets a new list; the others keep
                                  theirs, so a replica runs the same in a batch as
                                  alone, and MD_ERR_SKIN does not occur.
                                  rebuild_every is then unused.  Global kernels
                                  only (MD_OPT_KERNEL reads 1); not with the
                                  barostat (MD_ERR_ARG).  Default 0              */
};
int md_set_option(md_ctx *ctx, int32_t option, int64_t value);
int md_get_option(const md_ctx *ctx, int32_t option, int64_t *value);

/* Autotuner for the kernel configuration of the bound system (the paper finds
 * the best settings machine dependent; section "Parallel benchmarks").  Times,
 * on the current positions, the global-gather kernels and (full list only)
 * LDS-brick shapes {automatic, 4x4x4, 2x2x2} x lanes per atom {1, 2} x
 * workgroup sizes {512, 1024}, in FP64 each with either evaluator (tables or
 * knot sums, MD_OPT_EVALUATOR): one list build plus `trials` density + force
 * passes each (forces are written to the caller's arrays; positions and
 * velocities are untouched), and keeps the configuration with the lowest
 * force-pass time plus build time / rebuild_every, readable through
 * md_get_option.  Synchronises the stream.  trials: 1..1000. */
int md_autotune(md_ctx *ctx, int32_t trials, void *stream);

/* Kernel groups timed when MD_OPT_TIMING is on. */
enum { MD_KT_BUILD = 0, MD_KT_DENSITY = 1, MD_KT_FORCE = 2, MD_KT_REDUCE = 3, MD_KT_COUNT = 4 };

/* Synchronises the stream and returns, per kernel group, the summed elapsed
 * milliseconds (HIP events recorded on the launch stream around each launch
 * group) and the number of launches since timing was last reset; reset != 0
 * clears the totals afterwards.  ms[MD_KT_COUNT], launches[MD_KT_COUNT]. */
int md_kernel_times(md_ctx *ctx, double *ms, int64_t *launches, int reset, void *stream);

/* Frees the context (not the caller's state or workspace).  NULL is a no-op. */
void md_destroy(md_ctx *ctx);

/* Message describing the last failure on ctx (never NULL). */
const char *md_last_error(const md_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MDEAM_MD_H */
