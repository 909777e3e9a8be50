"""Plain FP64 CPU oracle for the embedded-atom force loop (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does: the two
share no code, header, table or constant.

The arithmetic lives in ``eam_oracle.c`` (brute force O(N^2), FP64); this module
compiles it with gcc and marshals numpy arrays through ctypes.  Every function
follows the paper (MOLDY, "Theoretical background" Eq. Ucoh for the energy,
"Boundary conditions" for the image vector, "Time integration" and "Fixed
atoms" for the integrator, "Thermostat NVTp" for the Nose-Hoover run, "Units"
for the time unit).  The mean square displacement and the diffusion estimate
("Self-diffusion in iron") are plain numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eam_oracle.c")
_LIB = os.path.join(_HERE, "_eam_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over atoms) and return the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Pot(ctypes.Structure):
    _fields_ = [
        ("ns", ctypes.c_int32),
        ("npk", ctypes.c_int32),
        ("ndk", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("pair_a", ctypes.c_void_p),
        ("pair_r", ctypes.c_void_p),
        ("dens_A", ctypes.c_void_p),
        ("dens_R", ctypes.c_void_p),
        ("emb_c", ctypes.c_void_p),
        ("mass", ctypes.c_void_p),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, i64, d, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER(_Pot)
    lib.or_time_unit_fs.restype = d
    lib.or_boltzmann_ev.restype = d
    lib.or_pressure_unit_gpa.restype = d
    lib.or_num_threads.restype = i32
    lib.or_set_num_threads.restype = None
    lib.or_set_num_threads.argtypes = [i32]
    lib.or_knot_sum.restype = d
    lib.or_knot_sum.argtypes = [vp, vp, i32, d, vp]
    lib.or_pair.restype = d
    lib.or_pair.argtypes = [P, i32, i32, d, vp]
    lib.or_density.restype = d
    lib.or_density.argtypes = [P, i32, i32, d, vp]
    lib.or_embed.restype = d
    lib.or_embed.argtypes = [P, i32, d, vp]
    lib.or_cutoff.restype = d
    lib.or_cutoff.argtypes = [P]
    lib.or_forces.restype = i32
    lib.or_forces.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, P, vp, vp, vp, vp, vp]
    lib.or_energy.restype = d
    lib.or_energy.argtypes = [i64, vp, vp, vp, vp, vp, vp, P]
    lib.or_forces_sampled.restype = i32
    lib.or_forces_sampled.argtypes = [i64, vp, vp, vp, vp, vp, vp, P, i64, vp, vp, vp, vp]
    lib.or_run_verlet.restype = i32
    lib.or_run_verlet.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, vp, i64, vp, vp, vp, vp]
    lib.or_run_pr.restype = i32
    lib.or_run_pr.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, i64, d, d, vp, vp, vp, vp, vp, vp,
                              vp]
    lib.or_run_npt.restype = i32
    lib.or_run_npt.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, i64, d, d, d, d, vp, vp, vp, vp, vp,
                               vp, vp]
    lib.or_forces_tri.restype = i32
    lib.or_forces_tri.argtypes = [i64, vp, vp, vp, vp, vp, vp, P, vp, vp, vp, vp, vp]
    lib.or_forces_sampled_tri.restype = i32
    lib.or_forces_sampled_tri.argtypes = [i64, vp, vp, vp, vp, vp, P, i64, vp, vp, vp, vp]
    lib.or_run_prt.restype = i32
    lib.or_run_prt.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, i64, d, d, d, d, vp, vp,
                               vp, vp, vp, vp, vp, vp]
    lib.or_run_gear.restype = i32
    lib.or_run_gear.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, vp, i64, vp, vp, vp, vp]
    lib.or_run_nh.restype = i32
    lib.or_run_nh.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P, d, vp, i64, d, d, d, vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(a):
    return None if a is None else a.ctypes.data


class Potential:
    """Cubic-knot EAM/FS potential in the layout the oracle reads.

    ``pot`` is a mapping with numpy arrays ``pair_a, pair_r`` [ns,ns,npk],
    ``dens_A, dens_R`` [ns,ns,ndk] (density at an a-site from a b-neighbour),
    ``emb_c`` [ns] and ``mass`` [ns] (amu).
    """

    def __init__(self, pot):
        self.pair_a = _f64(pot["pair_a"])
        self.pair_r = _f64(pot["pair_r"])
        self.dens_A = _f64(pot["dens_A"])
        self.dens_R = _f64(pot["dens_R"])
        self.emb_c = _f64(pot["emb_c"])
        self.mass = _f64(pot["mass"])
        ns = self.emb_c.shape[0]
        assert self.pair_a.shape[:2] == (ns, ns) and self.dens_A.shape[:2] == (ns, ns)
        self.s = _Pot(
            ns,
            self.pair_a.shape[2],
            self.dens_A.shape[2],
            0,
            self.pair_a.ctypes.data,
            self.pair_r.ctypes.data,
            self.dens_A.ctypes.data,
            self.dens_R.ctypes.data,
            self.emb_c.ctypes.data,
            self.mass.ctypes.data,
        )

    @property
    def ref(self):
        return ctypes.byref(self.s)


def time_unit_fs() -> float:
    """Internal time unit sqrt(amu A^2 / eV) in fs (paper, "Units")."""
    return _load().or_time_unit_fs()


def boltzmann_ev() -> float:
    return _load().or_boltzmann_ev()


def pressure_unit_gpa() -> float:
    return _load().or_pressure_unit_gpa()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's later parallel loops."""
    _load().or_set_num_threads(int(n))


def num_threads() -> int:
    return _load().or_num_threads()


def knot_sum(a, rk, r):
    """Cubic-knot sum sum_k a_k (r_k - r)^3 H(r_k - r) and its derivative."""
    a, rk = _f64(a), _f64(rk)
    out = ctypes.c_double()
    v = _load().or_knot_sum(a.ctypes.data, rk.ctypes.data, a.shape[0], float(r), ctypes.addressof(out))
    return v, out.value


def pair(pot: Potential, a: int, b: int, r: float):
    out = ctypes.c_double()
    v = _load().or_pair(pot.ref, a, b, float(r), ctypes.addressof(out))
    return v, out.value


def density(pot: Potential, a: int, b: int, r: float):
    out = ctypes.c_double()
    v = _load().or_density(pot.ref, a, b, float(r), ctypes.addressof(out))
    return v, out.value


def embed(pot: Potential, a: int, rho: float):
    out = ctypes.c_double()
    v = _load().or_embed(pot.ref, a, float(rho), ctypes.addressof(out))
    return v, out.value


def cutoff(pot: Potential) -> float:
    return _load().or_cutoff(pot.ref)


@dataclass
class ForceResult:
    f: np.ndarray  # [n,3] eV/A
    e_atom: np.ndarray  # [n] eV
    rho: np.ndarray  # [n]
    virial: np.ndarray  # [6] eV (xx,yy,zz,xy,xz,yz)
    pe: float  # eV


def _split(pos):
    pos = _f64(pos)
    return _f64(pos[:, 0]), _f64(pos[:, 1]), _f64(pos[:, 2])


def forces(pos, species, box, periodic, pot: Potential, rigid=None) -> ForceResult:
    """Brute-force forces, per-atom energies, densities and virial of one system."""
    x, y, z = _split(pos)
    n = x.shape[0]
    sp = _u8(species)
    rg = None if rigid is None else _u8(rigid)
    box = _f64(box)
    per = _u8(periodic)
    f = np.zeros((n, 3))
    e = np.zeros(n)
    rho = np.zeros(n)
    w = np.zeros(6)
    pe = ctypes.c_double()
    rc = _load().or_forces(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, sp.ctypes.data, _ptr(rg), box.ctypes.data,
        per.ctypes.data, pot.ref, f.ctypes.data, e.ctypes.data, rho.ctypes.data, w.ctypes.data,
        ctypes.addressof(pe),
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return ForceResult(f, e, rho, w, pe.value)


def energy(pos, species, box, periodic, pot: Potential) -> float:
    """Total energy of Eq. Ucoh alone (no derivatives)."""
    x, y, z = _split(pos)
    sp = _u8(species)
    box = _f64(box)
    per = _u8(periodic)
    e = _load().or_energy(x.shape[0], x.ctypes.data, y.ctypes.data, z.ctypes.data, sp.ctypes.data,
                          box.ctypes.data, per.ctypes.data, pot.ref)
    if np.isnan(e):
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return e


def forces_sampled(pos, species, box, periodic, pot: Potential, sample):
    """Forces, per-atom energies and densities of the atoms in ``sample`` only."""
    x, y, z = _split(pos)
    sp = _u8(species)
    box = _f64(box)
    per = _u8(periodic)
    idx = np.ascontiguousarray(sample, dtype=np.int64)
    m = idx.shape[0]
    f = np.zeros((m, 3))
    e = np.zeros(m)
    rho = np.zeros(m)
    rc = _load().or_forces_sampled(
        x.shape[0], x.ctypes.data, y.ctypes.data, z.ctypes.data, sp.ctypes.data, box.ctypes.data,
        per.ctypes.data, pot.ref, m, idx.ctypes.data, f.ctypes.data, e.ctypes.data, rho.ctypes.data,
    )
    if rc:
        raise ValueError(f"oracle: sampled evaluation failed ({rc})")
    return ForceResult(f, e, rho, np.full(6, np.nan), float("nan"))


@dataclass
class RunResult:
    pos: np.ndarray
    vel: np.ndarray
    f: np.ndarray
    pe: np.ndarray  # [nsteps+1]
    ke: np.ndarray  # [nsteps+1]
    work: np.ndarray  # [nsteps+1]


def run_verlet(pos, vel, species, box, periodic, pot: Potential, dt_fs, nsteps,
               rigid=None, rigid_velocity=None) -> RunResult:
    """Velocity-Verlet NVE run with brute-force forces at every step."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    rg = None if rigid is None else _u8(rigid)
    vp = None if rigid_velocity is None else _f64(rigid_velocity)
    box = _f64(box)
    per = _u8(periodic)
    f = np.zeros((n, 3))
    pe = np.zeros(nsteps + 1)
    ke = np.zeros(nsteps + 1)
    wk = np.zeros(nsteps + 1)
    rc = _load().or_run_verlet(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data,
        vz.ctypes.data, sp.ctypes.data, _ptr(rg), box.ctypes.data, per.ctypes.data, pot.ref,
        float(dt_fs), _ptr(vp), int(nsteps), f.ctypes.data, pe.ctypes.data, ke.ctypes.data,
        wk.ctypes.data,
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return RunResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, wk)


def run_gear(pos, vel, species, box, periodic, pot: Potential, dt_fs, nsteps, rigid=None,
             rigid_velocity=None) -> RunResult:
    """Third-order Gear predictor-corrector (paper, "Time integration") with
    brute-force forces; pe[s] at the predicted positions of step s, ke[s] of
    the corrected velocities, work[s] by the trapezoid rule over the
    evaluations."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    rg = None if rigid is None else _u8(rigid)
    vp = None if rigid_velocity is None else _f64(rigid_velocity)
    box = _f64(box)
    per = _u8(periodic)
    f = np.zeros((n, 3))
    pe, ke, wk = np.zeros(nsteps + 1), np.zeros(nsteps + 1), np.zeros(nsteps + 1)
    rc = _load().or_run_gear(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data,
        vz.ctypes.data, sp.ctypes.data, _ptr(rg), box.ctypes.data, per.ctypes.data, pot.ref,
        float(dt_fs), _ptr(vp), int(nsteps), f.ctypes.data, pe.ctypes.data, ke.ctypes.data,
        wk.ctypes.data,
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return RunResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, wk)


@dataclass
class PRResult:
    pos: np.ndarray
    vel: np.ndarray
    f: np.ndarray
    pe: np.ndarray
    ke: np.ndarray
    box: np.ndarray    # [nsteps+1, 3] A
    ldot: np.ndarray   # [nsteps+1, 3] A/fs
    baro: np.ndarray   # [nsteps+1] P Omega + W |dL/dt|^2 / 2, eV
    pressure: np.ndarray  # [nsteps+1] (2 KE + tr W) / (3 Omega), GPa


def run_pr(pos, vel, species, box, pot: Potential, dt_fs, nsteps, p_gpa, w_ev_fs2_a2, origin=None,
           ldot0=None) -> PRResult:
    """Parrinello-Rahman NPH run (paper, "Barostat NPTp") with an orthorhombic
    box and hydrostatic external pressure, brute-force forces; every axis
    periodic.  W in eV fs^2 / A^2, P in GPa."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    L = _f64(box).copy()
    o = np.zeros(3) if origin is None else _f64(origin)
    l0 = None if ldot0 is None else _f64(ldot0)
    f = np.zeros((n, 3))
    pe, ke, bx, ld, ba, pr = (np.zeros(nsteps + 1), np.zeros(nsteps + 1), np.zeros(3 * (nsteps + 1)),
                              np.zeros(3 * (nsteps + 1)), np.zeros(nsteps + 1), np.zeros(nsteps + 1))
    rc = _load().or_run_pr(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data, vz.ctypes.data,
        sp.ctypes.data, L.ctypes.data, o.ctypes.data, _ptr(l0), pot.ref, float(dt_fs), int(nsteps), float(p_gpa),
        float(w_ev_fs2_a2), f.ctypes.data, pe.ctypes.data, ke.ctypes.data, bx.ctypes.data, ld.ctypes.data,
        ba.ctypes.data, pr.ctypes.data,
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return PRResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, bx.reshape(-1, 3),
                    ld.reshape(-1, 3), ba, pr)


@dataclass
class NPTResult:
    pos: np.ndarray
    vel: np.ndarray
    f: np.ndarray
    pe: np.ndarray
    ke: np.ndarray
    box: np.ndarray       # [nsteps+1, 3] A
    baro: np.ndarray      # P Omega + W |dL/dt|^2 / 2, eV
    pressure: np.ndarray  # GPa
    pi: np.ndarray        # thermostat momentum, 1/fs
    nh_energy: np.ndarray  # Q pi^2 / 2 + g k_B T xi, eV


def run_npt(pos, vel, species, box, pot: Potential, dt_fs, nsteps, p_gpa, w_ev_fs2_a2, t_target, q_ev_fs2,
            origin=None) -> NPTResult:
    """Parrinello-Rahman barostat with the Nose-Hoover thermostat (paper,
    "Barostat NPTp"), orthorhombic box, hydrostatic pressure; every axis
    periodic, no rigid atoms."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    L = _f64(box).copy()
    o = np.zeros(3) if origin is None else _f64(origin)
    f = np.zeros((n, 3))
    m1 = nsteps + 1
    pe, ke, bx, ba, pr, nh = (np.zeros(m1), np.zeros(m1), np.zeros(3 * m1), np.zeros(m1), np.zeros(m1),
                              np.zeros(2 * m1))
    rc = _load().or_run_npt(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data, vz.ctypes.data,
        sp.ctypes.data, L.ctypes.data, o.ctypes.data, pot.ref, float(dt_fs), int(nsteps), float(p_gpa),
        float(w_ev_fs2_a2), float(t_target), float(q_ev_fs2), f.ctypes.data, pe.ctypes.data, ke.ctypes.data,
        bx.ctypes.data, ba.ctypes.data, pr.ctypes.data, nh.ctypes.data,
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return NPTResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, bx.reshape(-1, 3), ba, pr,
                     nh[0::2].copy(), nh[1::2].copy())


def forces_tri(pos, species, h, pot: Potential, rigid=None) -> ForceResult:
    """Brute-force forces, energies, densities and virial in a periodic cell
    with box matrix ``h`` [3,3] (edge vectors as columns, r = h s)."""
    x, y, z = _split(pos)
    n = x.shape[0]
    sp = _u8(species)
    rg = None if rigid is None else _u8(rigid)
    hm = _f64(np.asarray(h).reshape(9))
    f = np.zeros((n, 3))
    e = np.zeros(n)
    rho = np.zeros(n)
    w = np.zeros(6)
    pe = ctypes.c_double()
    rc = _load().or_forces_tri(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, sp.ctypes.data, _ptr(rg), hm.ctypes.data, pot.ref,
        f.ctypes.data, e.ctypes.data, rho.ctypes.data, w.ctypes.data, ctypes.addressof(pe),
    )
    if rc:
        raise ValueError("oracle: every width of the cell must exceed twice the cutoff")
    return ForceResult(f, e, rho, w, pe.value)


def forces_sampled_tri(pos, species, h, pot: Potential, sample):
    """Forces, per-atom energies and densities of the atoms in ``sample`` only,
    in a periodic cell with box matrix ``h`` [3,3]."""
    x, y, z = _split(pos)
    sp = _u8(species)
    hm = _f64(np.asarray(h).reshape(9))
    idx = np.ascontiguousarray(sample, dtype=np.int64)
    m = idx.shape[0]
    f = np.zeros((m, 3))
    e = np.zeros(m)
    rho = np.zeros(m)
    rc = _load().or_forces_sampled_tri(
        x.shape[0], x.ctypes.data, y.ctypes.data, z.ctypes.data, sp.ctypes.data, hm.ctypes.data, pot.ref, m,
        idx.ctypes.data, f.ctypes.data, e.ctypes.data, rho.ctypes.data,
    )
    if rc == -1:
        raise ValueError("oracle: every width of the cell must exceed twice the cutoff")
    if rc:
        raise ValueError(f"oracle: sampled evaluation failed ({rc})")
    return ForceResult(f, e, rho, np.full(6, np.nan), float("nan"))


@dataclass
class PRTResult:
    pos: np.ndarray
    vel: np.ndarray
    f: np.ndarray
    pe: np.ndarray
    ke: np.ndarray
    h: np.ndarray       # [nsteps+1, 3, 3] box matrix, A (edge vectors as columns)
    hdot: np.ndarray    # [nsteps+1, 3, 3] A/fs
    baro: np.ndarray    # P Omega + W tr(h'^T h') / 2 + Omega0 tr((S - P) eps), eV
    stress: np.ndarray  # [nsteps+1, 6] internal stress (xx,yy,zz,xy,xz,yz), GPa
    pi: np.ndarray      # thermostat momentum, 1/fs (zero without one)
    nh_energy: np.ndarray  # Q pi^2 / 2 + g k_B T xi, eV


def run_prt(pos, vel, species, h, pot: Potential, dt_fs, nsteps, p_gpa=0.0, w_ev_fs2_a2=0.0, stress_gpa=None,
            origin=None, hdot0=None, t_target=0.0, q_ev_fs2=0.0, h_ref=None) -> PRTResult:
    """Parrinello-Rahman dynamics of the full box matrix under pressure P and
    external stress S (paper, "Barostat NPTp"), brute-force forces, every axis
    periodic; with ``q_ev_fs2`` > 0 the Nose-Hoover thermostat too.  W = 0
    keeps the sheared cell fixed (plain velocity Verlet).  ``h_ref`` is the
    reference cell h0 of the strain (default: the starting cell)."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    hm = _f64(np.asarray(h).reshape(9)).copy()
    o = np.zeros(3) if origin is None else _f64(origin)
    hd = None if hdot0 is None else _f64(np.asarray(hdot0).reshape(9))
    sg = None if stress_gpa is None else _f64(np.asarray(stress_gpa).reshape(9))
    hr = None if h_ref is None else _f64(np.asarray(h_ref).reshape(9))
    f = np.zeros((n, 3))
    m1 = nsteps + 1
    pe, ke, ho, hdo, ba, so, nh = (np.zeros(m1), np.zeros(m1), np.zeros(9 * m1), np.zeros(9 * m1), np.zeros(m1),
                                   np.zeros(6 * m1), np.zeros(2 * m1))
    rc = _load().or_run_prt(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data, vz.ctypes.data,
        sp.ctypes.data, hm.ctypes.data, o.ctypes.data, _ptr(hd), _ptr(sg), _ptr(hr), pot.ref, float(dt_fs), int(nsteps),
        float(p_gpa), float(w_ev_fs2_a2), float(t_target), float(q_ev_fs2), f.ctypes.data, pe.ctypes.data,
        ke.ctypes.data, ho.ctypes.data, hdo.ctypes.data, ba.ctypes.data, so.ctypes.data, nh.ctypes.data,
    )
    if rc == -1:
        raise ValueError("oracle: every width of the cell must exceed twice the cutoff")
    if rc:
        raise ValueError("oracle: the box moved more than half its size in one step")
    return PRTResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, ho.reshape(-1, 3, 3),
                     hdo.reshape(-1, 3, 3), ba, so.reshape(-1, 6), nh[0::2].copy(), nh[1::2].copy())


@dataclass
class NHResult:
    pos: np.ndarray
    vel: np.ndarray
    f: np.ndarray
    pe: np.ndarray  # [nsteps+1]
    ke: np.ndarray
    work: np.ndarray
    pi: np.ndarray  # [nsteps+1] thermostat momentum, 1/fs
    nh_energy: np.ndarray  # [nsteps+1] Q pi^2/2 + g k_B T xi, eV


def run_nh(pos, vel, species, box, periodic, pot: Potential, dt_fs, nsteps, t_target, q_ev_fs2,
           rigid=None, rigid_velocity=None, pi0=0.0) -> NHResult:
    """Nose-Hoover NVT run (paper, "Thermostat NVTp") with brute-force forces;
    Q in eV fs^2, thermostat momentum starting at pi0 (1/fs)."""
    x, y, z = (a.copy() for a in _split(pos))
    vx, vy, vz = (a.copy() for a in _split(vel))
    n = x.shape[0]
    sp = _u8(species)
    rg = None if rigid is None else _u8(rigid)
    vp = None if rigid_velocity is None else _f64(rigid_velocity)
    box = _f64(box)
    per = _u8(periodic)
    f = np.zeros((n, 3))
    pe, ke, wk = np.zeros(nsteps + 1), np.zeros(nsteps + 1), np.zeros(nsteps + 1)
    nh = np.zeros(2 * (nsteps + 1))
    rc = _load().or_run_nh(
        n, x.ctypes.data, y.ctypes.data, z.ctypes.data, vx.ctypes.data, vy.ctypes.data, vz.ctypes.data,
        sp.ctypes.data, _ptr(rg), box.ctypes.data, per.ctypes.data, pot.ref, float(dt_fs), _ptr(vp),
        int(nsteps), float(t_target), float(q_ev_fs2), float(pi0), f.ctypes.data, pe.ctypes.data, ke.ctypes.data,
        wk.ctypes.data, nh.ctypes.data,
    )
    if rc:
        raise ValueError("oracle: periodic box length must exceed twice the cutoff")
    return NHResult(np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), f, pe, ke, wk, nh[0::2].copy(),
                    nh[1::2].copy())


def temperature(ke: float, n_mobile: int, has_rigid: bool) -> float:
    """T from the kinetic energy: 3N-3 degrees of freedom once total momentum is
    fixed ("Thermostat NVTp"); 3N when a moving rigid block breaks momentum
    conservation."""
    dof = 3 * n_mobile if has_rigid else 3 * n_mobile - 3
    return 0.0 if dof <= 0 else 2.0 * ke / (dof * boltzmann_ev())


def msd(pos, pos0, species, atom_offset, n_species, rigid=None):
    """Mean square displacement per replica and species ("Self-diffusion in
    iron": the displacement squared, averaged over atoms), from unwrapped
    positions ("Boundary conditions": trajectories are stored without
    wraparound, so a displacement is a plain difference).  Rigid atoms are not
    averaged.  Returns (msd [R, n_species] in A^2, count [R, n_species]); a
    species with no atom in a replica has msd 0."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    pos0 = np.asarray(pos0, np.float64).reshape(-1, 3)
    species = np.asarray(species).astype(np.int64)
    mobile = np.ones(len(pos), bool) if rigid is None else np.asarray(rigid) == 0
    off = np.asarray(atom_offset, np.int64)
    n_rep = len(off) - 1
    out = np.zeros((n_rep, n_species))
    count = np.zeros((n_rep, n_species), np.int64)
    for r in range(n_rep):
        for s in range(n_species):
            total = 0.0
            for i in range(off[r], off[r + 1]):
                if species[i] != s or not mobile[i]:
                    continue
                d = pos[i] - pos0[i]
                total += d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
                count[r, s] += 1
            out[r, s] = total / count[r, s] if count[r, s] else 0.0
    return out, count


def diffusion_coefficient(t_fs, msd_a2):
    """D = lim MSD / (6 t) ("Self-diffusion in iron"), estimated as one sixth of
    the least-squares slope of MSD against t; A^2/fs (x 0.1 gives cm^2/s)."""
    t = np.asarray(t_fs, np.float64)
    m = np.asarray(msd_a2, np.float64)
    tm, mm = t.mean(), m.mean()
    return float(np.sum((t - tm) * (m - mm)) / np.sum((t - tm) ** 2)) / 6.0
