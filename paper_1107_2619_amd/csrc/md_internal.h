// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/md.h"

namespace mdk {

// Physical constants (paper, "Units": amu as printed; eV and k_B from the
// CODATA-2002 set that matches it).  The internal time unit is
// t0 = sqrt(amu A^2 / eV) ~ 10.18 fs; the library works in fs and converts.
constexpr double kAmuKg = 1.66053886e-27;
constexpr double kEvJ = 1.60217653e-19;
constexpr double kBoltzmannEv = 8.617343e-5;
constexpr double kEvPerA3InGpa = 160.217653;

constexpr int kWave = 64;       // CDNA wavefront
constexpr int kBlock = 256;     // threads per workgroup (4 waves)
constexpr int kCandTable = 512; // list build: candidates one wave's LDS table holds
constexpr int kTableBlock = 1024;  // global kernels with several species' tables in LDS
constexpr int kEnergySlots = 12;  // per-wave partial record, see EnergyIndex
constexpr int kNumXcd = 8;      // MI355X: 8 accelerator dies, one L2 each

enum EnergyIndex { E_PE = 0, E_KE = 1, E_W0 = 2, E_PW = 8, E_NONFINITE = 9 };
constexpr int kEnergyTerms = 10;       // per-atom terms written on energy steps
constexpr int kReduceChunk = 2048;
constexpr int kChunkedSumWaves = 512;  // replicas above this many waves sum per chunk first     // slots per first-stage reduction chunk (one workgroup each)
constexpr int kHaloMax = 216;          // halo cells of a brick: (4 + 2)^3 at most
constexpr int kHaloTableBytes = 5120;  // LDS of a brick's halo table (bound checked where it is defined)
constexpr int kBrickMaxDim = 4;

// Neighbour-list entry: slot index in the low kIndexBits bits, the periodic
// image shift (2 bits per axis) in the six above, and in the global list the
// sign bit set for an inner entry: a pair closer than r_d + skin at the build,
// r_d the largest density knot.  The others stay beyond every density cutoff
// until the next build, so the density pass gathers only inner entries.
constexpr int kIndexBits = 25;
constexpr int kIndexMask = (1 << kIndexBits) - 1;
constexpr int kCodeMask = 63;
constexpr int32_t kInnerBit = INT32_MIN;
constexpr int kChunk = 4;  // neighbours whose loads are issued together (one 16-byte list load)

// Neighbour-list layout (global kernels): entry k of slot t at
// nbr[((k / 4) Np + t) 4 + k % 4].  A slot's entries come in groups of four,
// one 16-byte load per lane, and the groups of a wavefront's 64 slots are one
// contiguous kilobyte.
__host__ __device__ inline int64_t nbr_at(int k, int64_t t, int64_t n_slots)
{
    return ((int64_t)(k >> 2) * n_slots + t) * 4 + (k & 3);
}
constexpr int kForceStride = 6;  // coefficients per bin of the force table (phi', rho' quadratics)
// Tables whose bins may hold one knot of each function inside (knots on no
// common grid): every function's record also carries that knot's offset D
// from the bin start and its amplitude, for the term amp (D - u)^p H(D - u).
// Force record: phi' quadratic, rho' quadratic, D_phi, -3 a_phi, D_rho, -3 a_rho;
// value records (phi, rho): cubic, D, a.
constexpr int kForceStrideSplit = 10;
constexpr int kValueStride = 4;
constexpr int kValueStrideSplit = 6;
// table kind: 0 = term-by-term knot sums, 1 = knots on the bin grid, 2 = knots inside bins
constexpr int force_stride(int kind) { return kind == 2 ? kForceStrideSplit : kForceStride; }
constexpr int value_stride(int kind) { return kind == 2 ? kValueStrideSplit : kValueStride; }
// Compact gather record of the mixed mode: cell-local coordinates as 32-bit
// fixed point in units of h_a 2^-kCompactBits (h_a the link-cell edge of axis
// a) and F' as FP32, 16 bytes.  A coordinate may lie up to kCompactCells cell
// edges from its cell's origin.
constexpr int kCompactBits = 28;
constexpr double kCompactCells = 7.5;
constexpr uint32_t kBufferWord3 = 0x00020000;  // raw buffer resource, gfx9 family

// Slot type byte: species in bits 0..5, rigid flag in bit 6; 0xFF = empty slot.
constexpr uint8_t kRigidBit = 0x40;
constexpr uint8_t kEmptySlot = 0xFF;

// Per replica, in device memory.  Slots of replica r are
// [slot_off, slot_off + n_atoms); slot_off is a multiple of the wavefront, so
// a wavefront never mixes replicas and the replica of a slot is a per-wave
// (scalar) value.  Cells of replica r are [cell_off, cell_off + nc.x*nc.y*nc.z).
//
// Link cells are numbered brick-major: the nc[0] x nc[1] x nc[2] grid is cut
// into bricks of bd[0] x bd[1] x bd[2] cells (nbk[a] bricks per axis, the last
// one possibly partial), cell (cx,cy,cz) has index
//   cell_off + brick * cpb + local,  brick = (bz*nbk[1] + by)*nbk[0] + bx,
//   local = (lz*bd[1] + ly)*bd[0] + lx,  c = b*bd + l,  cpb = bd[0]*bd[1]*bd[2],
// so after the cell sort the atoms of a brick occupy one contiguous slot range.
struct DevReplica {
    int32_t slot_off, n_atoms, cell_off, periodic_mask;  // bit a = axis a periodic
    int32_t nc[3], atom_off;                              // atom_off: caller index base
    int32_t bd[3], cpb;                                   // brick shape, cells per brick
    int32_t nbk[3], brick_off;                            // bricks per axis, first global brick
    double box[3], inv_box[3], origin[3];
    double vp[3];    // rigid velocity, A/fs
    double cell[3];  // link-cell edge per axis, box / nc
    double qs[3];    // compact coordinate unit per axis, cell * 2^-kCompactBits
    double iqs[3];   // its inverse
    double lbuild[3];  // edges at the last list build (differ from box only under the barostat)
    // Sheared cell (tri = 1): the box matrix h with the edge vectors as
    // columns (row-major), r = o + h s with s the fractional coordinates; every
    // axis periodic, link cells and image counts along the edge vectors.  box
    // then holds the widths of the cell (distances between opposite faces).
    int32_t tri, pad_tri;
    double h[9], hinv[9];
    double hbinv[9];  // inverse of h at the last list build
    double mb[9];     // h times hbinv: the homogeneous strain since that build
    double qg[9];     // h diag(2^-kCompactBits / nc): compact-record units to Cartesian
};

__host__ __device__ inline int32_t cell_index(const DevReplica& R, int cx, int cy, int cz)
{
    const int bx = cx / R.bd[0], by = cy / R.bd[1], bz = cz / R.bd[2];
    const int lx = cx - bx * R.bd[0], ly = cy - by * R.bd[1], lz = cz - bz * R.bd[2];
    return R.cell_off + ((bz * R.nbk[1] + by) * R.nbk[0] + bx) * R.cpb + (lz * R.bd[1] + ly) * R.bd[0] + lx;
}

// Potential evaluated in the kernels.  Amplitudes are stored premultiplied
// for the derivative (-3 a) beside the value amplitudes.
struct DevPotential {
    int32_t ns, npk, ndk, pad;
    double rc, rc2, rlist2;
    double pair_a[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];
    double pair_d[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];  // -3 a
    double pair_r[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];
    double dens_a[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];
    double dens_d[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];
    double dens_r[MD_MAX_SPECIES * MD_MAX_SPECIES][MD_MAX_KNOTS];
    double emb_c[MD_MAX_SPECIES];
    double accel[MD_MAX_SPECIES];    // (eV/A) -> A/fs^2 : 1 / (m t0^2)
    double half_m[MD_MAX_SPECIES];   // (A/fs)^2 -> eV   : m t0^2 / 2
};

// Potential arguments passed by value (kernel arguments land in scalar
// registers, so every lane reads the same coefficient without a load).  The
// knot coefficients are those of the single species when ns == 1.
struct PotArgs {
    double pair_a[MD_MAX_KNOTS], pair_d[MD_MAX_KNOTS], pair_r[MD_MAX_KNOTS];
    double dens_a[MD_MAX_KNOTS], dens_d[MD_MAX_KNOTS], dens_r[MD_MAX_KNOTS];
    double emb_c, accel, half_m, rc2;
    double w, inv_w;  // bin width of the local-polynomial tables
    int32_t nbt, ns;  // bins per table (incl. two zero bins past r_c), species
    float pair_af[MD_MAX_KNOTS], pair_df[MD_MAX_KNOTS];
    float dens_af[MD_MAX_KNOTS], dens_df[MD_MAX_KNOTS];
};

// Device-side error flags (int32 each).
// F_MAX_COUNT: largest list length found by any build (overflow when > cap);
// F_SKIN: atoms whose net displacement between builds exceeded skin/2;
// F_OUTSIDE: atoms beyond the grid extent of a free axis (clamped; legal).
// F_PR_BOX: the barostat shrank a link-cell edge below the list radius;
// F_HALO: brick passes whose halo did not fit the LDS staging area (those
// read their neighbours from global memory instead).  F_COMPACT: atoms too far
// outside their link cell for the compact mixed-mode record.
// F_RANGE: a pair term beyond the fixed-point range of the pair kernels' shared accumulators.
// F_AUTO_BUILDS: builds the displacement check triggered (automatic rebuilds).
enum FlagIndex {
    F_MAX_COUNT = 0, F_SKIN = 1, F_OUTSIDE = 2, F_HALO = 3, F_COMPACT = 4, F_PR_BOX = 5, F_RANGE = 6,
    F_AUTO_BUILDS = 7, F_COUNT = 8
};

// Pointers into the workspace.
struct Buffers {
    double4* pos[2];      // [Np] x, y, z, F' (w written by the density pass)
    double* vel[2][3];    // [Np] each
    int32_t* id[2];       // [Np] caller index of the slot, -1 = empty
    uint8_t* type[2];     // [Np]
    double* pwork[2];     // [Np] piston work accumulated per rigid atom, eV
    int32_t* img[2][3];   // [Np] periodic image count per axis (caller x = x + img L)
    double4* xbuild;      // [Np] positions at the last list build
    int4* rec[2];         // [Np] compact records (mixed): [0] coordinates, [1] coordinates + F'
    int4* cellxyz;        // [Np] link cell (cx, cy, cz) of each slot at the last build
    double* femb;         // [Np] F_i (energy steps)
    int32_t* nbr;         // [cap][Np] transposed list (global slots + shift code)
    uint8_t* ntype;       // type byte of every list entry, same layout (several species)
    double* wave_terms;   // [Np / 64][kEnergyTerms] per-wavefront energy sums (velocity-Verlet energy steps)
    uint16_t* nbr16;      // [Np][rowlen] rows of staging (LDS) indices (brick path)
    int32_t* perm_sorted; // [Np] old slot of each new slot, cell members in caller-index order
    int32_t* brick_rep;   // [n_bricks] replica of each brick
    int4* brick_info;     // [n_bricks] own slot range [x, y) and halo atoms z at the last build
    int32_t* stage_src;   // [n_bricks][halo_cap] slot | shift code of each staging position
    uint16_t* own_li;     // [Np] staging position of each atom within its own brick
    int32_t* ncount;      // [Np]
    int32_t* cell_of;     // [Np]
    int32_t* perm;        // [Np] new slot -> old slot
    int32_t* cell_start;  // [C]
    int32_t* cell_count;  // [C]
    int32_t* bin_count;   // [C] atoms binned by the build in progress (zero between builds)
    int32_t* cell_cursor; // [C]
    int32_t* cell_shift;  // [C] slot_off - atom_off of the cell's replica
    int32_t* cell_rep;    // [C] replica of each link cell (-1: unused)
    int2* cell_adj;       // [C][27] adjacent cell (-1: none), image and offset codes
    int32_t* cell_coord;  // [C] cell coordinates, 10 bits per axis
    int32_t* scan_blocks; // [scan blocks]
    int32_t* rep_of_wave; // [Np / 64]
    DevReplica* reps;     // [R]
    DevPotential* pot;    // 1
    double* eslot;        // [kEnergyTerms][Np] per-atom energy terms (energy steps)
    double* energies;     // [R][kEnergySlots]
    int32_t* chunk_rep;   // [n_chunks] replica of each reduction chunk
    int32_t* chunk_off;   // [R+1] first chunk of each replica
    double* chunk_partial;  // [n_chunks][kEnergySlots]
    double* fhalf[3];     // [Np] half-list force accumulators (MD_NBR_HALF_ATOMIC)
    double* rhalf;        // [Np] half-list density accumulator
    double* nh_param;     // [R][2] thermostat mass Q (eV fs^2), g k_B T (eV)
    double* nh_state;     // [R][4] pi (1/fs), xi, velocity scale of the last update, KE after it (eV)
    double* nh_partial;   // [Np / 64] kinetic energy per wavefront
    double* ehalf;        // [Np] half-list pair-energy accumulator (half of sum phi)
    double* acc[2][3];    // [Np] Gear integrator: acceleration, A/fs^2 (null with Verlet)
    double* jrk[2][3];    // [Np] Gear integrator: its time derivative, A/fs^3
    double* pr_param;     // [R][2] barostat mass W (eV fs^2/A^2), external pressure (eV/A^3)
    double* pr_state;     // [R][kPrState] box, box velocity and the factors of the open pass
    double* pr_partial;   // [Np / 64][6] per-wave sums of m v_a^2 and of the virial diagonal
                          // ([Np / 64][12]: m v_a v_b and the six virial terms, full box matrix)
    double* x0[3];        // [N] origin positions of the mean square displacement, caller order
    uint8_t* ctype;       // [N] species | rigid bit, caller order
    double* msd_partial;  // [n_chunks][2 * MD_MAX_SPECIES] sums of d^2 and atom counts
    double* msd_out;      // [R][2 * MD_MAX_SPECIES] msd per species, then counts
    // local-polynomial tables, [ns*ns][nbt][force_stride] (phi' and rho' quadratics),
    // [ns*ns][nbt][value_stride] (phi cubic), [ns*ns][nbt][value_stride] (rho cubic)
    double *tab_force64, *tab_energy64, *tab_dens64;
    float *tab_force32, *tab_energy32, *tab_dens32;
    int32_t* flags;       // [F_COUNT]
    double* ering;        // [ring_len][R][kEnergySlots] per-replica totals of the per-step energy steps
    int64_t* ering_count; // [2] entries appended since md_bind (entry i lives at i % ring_len),
                          // then the reduction's workgroup ticket
    int32_t* gate;        // [2][R + 1] automatic rebuilds, two alternating sets: [0] some
                          // replica moved past the guard, [1 + r] replica r did
};

struct KernelShape {
    int64_t n_slots;  // Np
    int32_t n_cells;
    int32_t n_replicas;
    int32_t cap;
    int32_t npk, ndk; // knots per pair / density function
    int32_t table;    // 0 = explicit knot sums, 1 = local-polynomial tables (knots on the
                      // bin grid), 2 = tables whose bins may hold a knot (split terms)
    int32_t n_chunks; // energy-reduction chunks over all replicas
    int32_t n_bricks; // bricks over all replicas
    int32_t brick;    // 1 = LDS brick kernels, 0 = global-gather kernels
    int32_t halo_cap; // atoms the LDS staging area holds
    int32_t block;    // threads per brick workgroup
    int32_t lanes;    // lanes sharing one atom's neighbour list (brick path)
    int32_t rowlen;   // entries per brick-list row: cap rounded up to 8
    int32_t compact;  // mixed mode with compact records (global path): 1 orthorhombic, 2 sheared cells
    int32_t tri;      // 1 = box matrices (sheared cells)
    int32_t lds_limit; // LDS bytes one workgroup may use
    int32_t pairs;     // LDS bricks with each pair of two own atoms once (MD_OPT_KERNEL = 2)
    int32_t nchunk;    // neighbour records in flight per thread in the global kernels: 2, 4 or 8
    int32_t list_types; // the global list also stores its entries' type bytes (several species)
    int32_t split_list; // the global list marks its inner entries (FP64: the density pass then
                        // gathers only those)
    int32_t chunked;  // 1 = per-replica sums of the thermostat and barostat start with
                      // per-chunk sums (some replica spans more than kChunkedSumWaves waves)
};

// Launchers (kernels.hip).  All enqueue on `s`.
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void launch_init_slots(const Buffers& b, int q, const md_state& st, const KernelShape& k, hipStream_t s);
void launch_load_state(const Buffers& b, int p, int q, const md_state& st, const KernelShape& k,
                       hipStream_t s);
// gate: NULL rebuilds every replica; otherwise only the replicas whose entry
// gate[1 + r] is set (automatic rebuilds; every kernel exits at once for the
// others).
void launch_rebuild(const Buffers& b, int p, int q, const KernelShape& k, double half_skin2,
                    int half_list, const int32_t* gate, hipStream_t s);
// rdl2 = (r_d + skin)^2 marks the inner entries (rlist2: every entry).
// copy_back: the list is built from the sorted state in (p, q) and each own
// atom's state is copied into (p ^ 1, q ^ 1) (automatic rebuilds, which keep
// the ping-pong indices).
void launch_build_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, double rdl2,
                       int half_list, const int32_t* gate, int copy_back, hipStream_t s);
// Displacement check of automatic rebuilds: sets gate[0] and gate[1 + r] when
// an atom of replica r moved more than sqrt(guard2) since the last build, and
// clears the other set `next` for the following check.
void launch_skin_check(const Buffers& b, int p, const KernelShape& k, double guard2, int32_t* gate,
                       int32_t* next, hipStream_t s);
void launch_compact_records(const Buffers& b, int p, const KernelShape& k, hipStream_t s);
void launch_cell_table(const Buffers& b, const KernelShape& k, hipStream_t s);
void launch_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                    int half_list, int energy, hipStream_t s);
// energy: 0 none, 1 energies and virial, 2 the virial diagonal only (barostat),
// 3 the whole virial tensor only (full-matrix barostat), 4 energies and virial
// summed per wavefront (velocity-Verlet energy steps of the global kernels)
struct ForceFlags {
    int energy, close, open, writeback;
};
void launch_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                  int half_list, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s);
// ring_len > 0: the totals also go to the next entry of the energy ring.
void launch_reduce_energies(const Buffers& b, const KernelShape& k, double virial_scale, int64_t ring_len,
                            hipStream_t s);
// The same totals from the per-wavefront sums of an energy step of the global kernels.
void launch_reduce_waves(const Buffers& b, const KernelShape& k, double virial_scale, int64_t ring_len,
                         hipStream_t s);
// Nose-Hoover thermostat: kinetic energy per replica and `halves` thermostat
// half steps of length dt/2 (launch_nh_update); then either the scaled opening
// kick and drift (launch_nh_open) or the final scaling (launch_nh_scale).
void launch_nh_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int halves, double dt_fs,
                      hipStream_t s);
// scaled = 1: the thermostat's velocity scale first (NVT); 0: the plain
// opening kick and drift from the kept forces (an md_step call continuing
// from the last one).
void launch_nh_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                    int scaled, hipStream_t s);
void launch_nh_scale(const Buffers& b, int q, const KernelShape& k, const md_state& st, int energy, hipStream_t s);
// Brick path (kernels_brick.hip).
void launch_gear_start(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, hipStream_t s);
void launch_gear_predict(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         hipStream_t s);
void launch_gear_correct(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                         const md_state& st, int last, hipStream_t s);

// Barostat (orthorhombic Parrinello-Rahman).  pr_state per replica:
// [0,3) L, [3,6) dL/dt, [6,9) velocity scale of the open pass, [9,12) L'/L of
// its drift, [12,15) h phi(u) L'/L of its drift, [15,18) closing velocity scale.
constexpr int kPrState = 20;
void launch_pr_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int close, int open,
                      double dt_fs, double rlist, double strain_tol, int nvt, hipStream_t s);
void launch_pr_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                    hipStream_t s);
void launch_pr_close_scale(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, const md_state& st,
                           hipStream_t s);
void launch_pr_mark_build(const Buffers& b, const KernelShape& k, hipStream_t s);
// First stage of the barostat sums: per-wave partials (n_terms = 6 or 12) into
// chunk_partial, one wavefront per reduction chunk.
void launch_pr_chunk_sums(const Buffers& b, const KernelShape& k, int n_terms, hipStream_t s);

// Barostat on the full box matrix.  pr_state per replica (matrices row-major):
// [0,9) h, [9,18) dh/dt (A per time unit), [18,27) Sigma = Omega0 h0^-1 (S - P) h0^-T
// (eV), [27,36) velocity map of the open pass, [36,45) h'h^-1 of its drift,
// [45,54) the velocity term of its drift, [54,63) closing velocity map.
constexpr int kPrtState = 64;
void launch_prt_update(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, int close, int open,
                       double dt_fs, double rlist, double strain_tol, int nvt, hipStream_t s);
void launch_prt_open(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, double dt_fs,
                     hipStream_t s);
void launch_prt_close_scale(const Buffers& b, int q, const KernelShape& k, const PotArgs& P, const md_state& st,
                            hipStream_t s);

// Launchers (kernels_analysis.hip).
void launch_msd(const Buffers& b, const KernelShape& k, const md_state& st, hipStream_t s);
// msd_out [R][2 MD_MAX_SPECIES] -> msd [R][ns], count [R][ns] (int64), on the device.
void launch_msd_pack(const double* out, int n_replicas, int ns, double* msd, int64_t* count, hipStream_t s);

// Lanes per atom of the pair kernels: 1 or 2 (the brick setting, 4 taken as 2).
inline int pair_lanes(const KernelShape& k) { return k.lanes >= 2 ? 2 : 1; }
// half = 1: pairs of two own atoms of a brick once (the pair kernels); 0: every pair from both atoms
void launch_brick_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, int half,
                       int pair_slots, hipStream_t s);
void launch_brick_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                          int energy, hipStream_t s);
void launch_brick_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                        ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s);
void launch_brick_list_to_slots(const Buffers& b, const KernelShape& k, hipStream_t s);
size_t brick_lds_bytes(const KernelShape& k, const PotArgs& P, int precision, int pass, int energy);
// Pair kernels (kernels_pairs.hip): the LDS-brick passes over lists that hold
// each pair of two own atoms once, both atoms' shares accumulated in LDS.
// Own atoms a pair-kernel brick can hold (LDS accumulators, one round of lanes);
// bricks with more keep full lists.
int pair_slots(const KernelShape& k, const PotArgs& P, int precision);
void launch_pair_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                         int energy, hipStream_t s);
void launch_pair_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                       ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s);

}  // namespace mdk
