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
constexpr int kEnergySlots = 12;  // per-wave partial record, see EnergyIndex
constexpr int kNumXcd = 8;      // MI355X: 8 accelerator dies, one L2 each

enum EnergyIndex { E_PE = 0, E_KE = 1, E_W0 = 2, E_PW = 8, E_NONFINITE = 9 };

// Slot type byte: species in bits 0..5, rigid flag in bit 6; 0xFF = empty slot.
constexpr uint8_t kRigidBit = 0x40;
constexpr uint8_t kEmptySlot = 0xFF;

// Per replica, in device memory.  Slots of replica r are
// [slot_off, slot_off + n_atoms); slot_off is a multiple of the wavefront, so
// a wavefront never mixes replicas and the replica of a slot is a per-wave
// (scalar) value.  Cells of replica r are [cell_off, cell_off + nc.x*nc.y*nc.z).
struct DevReplica {
    int32_t slot_off, n_atoms, cell_off, periodic_mask;  // bit a = axis a periodic
    int32_t nc[3], atom_off;                              // atom_off: caller index base
    double box[3], inv_box[3], origin[3];
    double vp[3];  // rigid velocity, A/fs
};

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
enum FlagIndex { F_MAX_COUNT = 0, F_SKIN = 1, F_OUTSIDE = 2, F_COUNT = 4 };

// Pointers into the workspace.
struct Buffers {
    double4* pos[2];      // [Np] x, y, z, F' (w written by the density pass)
    double* vel[2][3];    // [Np] each
    int32_t* id[2];       // [Np] caller index of the slot, -1 = empty
    uint8_t* type[2];     // [Np]
    double* pwork[2];     // [Np] piston work accumulated per rigid atom, eV
    double4* xbuild;      // [Np] positions at the last list build
    double* femb;         // [Np] F_i (energy steps)
    int32_t* nbr;         // [cap][Np] transposed list
    int32_t* ncount;      // [Np]
    int32_t* cell_of;     // [Np]
    int32_t* perm;        // [Np] new slot -> old slot
    int32_t* cell_start;  // [C]
    int32_t* cell_count;  // [C]
    int32_t* cell_cursor; // [C]
    int32_t* cell_shift;  // [C] slot_off - atom_off of the cell's replica
    int32_t* scan_blocks; // [scan blocks]
    int32_t* rep_of_wave; // [Np / 64]
    DevReplica* reps;     // [R]
    DevPotential* pot;    // 1
    double* partial;      // [Np / 64][kEnergySlots]
    double* energies;     // [R][kEnergySlots]
    double* fhalf[3];     // [Np] half-list force accumulators (MD_NBR_HALF_ATOMIC)
    // local-polynomial tables, [ns*ns][nbt][8] (phi' and rho' quadratics),
    // [ns*ns][nbt][4] (phi cubic), [ns*ns][nbt][4] (rho cubic)
    double *tab_force64, *tab_energy64, *tab_dens64;
    float *tab_force32, *tab_energy32, *tab_dens32;
    int32_t* flags;       // [F_COUNT]
};

struct KernelShape {
    int64_t n_slots;  // Np
    int32_t n_cells;
    int32_t n_replicas;
    int32_t cap;
    int32_t lanes;    // lanes per atom
    int32_t npk, ndk; // knots per pair / density function
    int32_t table;    // 1 = local-polynomial tables, 0 = explicit knot sums
};

// Launchers (kernels.hip).  All enqueue on `s`.
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void launch_init_slots(const Buffers& b, int q, const md_state& st, const KernelShape& k, hipStream_t s);
void launch_load_state(const Buffers& b, int p, int q, const md_state& st, const KernelShape& k,
                       hipStream_t s);
void launch_rebuild(const Buffers& b, int p, int q, const KernelShape& k, double half_skin2,
                    int half_list, hipStream_t s);
void launch_build_list(const Buffers& b, int p, int q, const KernelShape& k, double rlist2, int half_list,
                       hipStream_t s);
void launch_density(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                    int half_list, int energy, hipStream_t s);
struct ForceFlags {
    int energy, close, open, writeback;
};
void launch_force(const Buffers& b, int p, int q, const KernelShape& k, const PotArgs& P, int precision,
                  int half_list, ForceFlags fl, double dt_fs, const md_state& st, hipStream_t s);
void launch_reduce_energies(const Buffers& b, const KernelShape& k, hipStream_t s);

}  // namespace mdk
