"""Thin ctypes binding of ``include/md.h`` (argument marshalling only).

Every step of the force loop runs in the gfx950 kernels of ``libmdeam.so``;
this module only allocates device tensors with PyTorch, passes their
pointers and the current HIP stream, and converts results.  There is no CPU
fallback: if the library is missing, importing it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdeam.so")

MD_OK = 0
MD_ERR_ARG = -1
MD_ERR_BOX = -2
MD_ERR_POTENTIAL = -3
MD_ERR_NBR_OVERFLOW = -4
MD_ERR_SKIN = -5
MD_ERR_NONFINITE = -6
MD_ERR_DEVICE = -7
MD_ERR_STATE = -8
ERROR_NAMES = {
    MD_ERR_ARG: "MD_ERR_ARG", MD_ERR_BOX: "MD_ERR_BOX", MD_ERR_POTENTIAL: "MD_ERR_POTENTIAL",
    MD_ERR_NBR_OVERFLOW: "MD_ERR_NBR_OVERFLOW", MD_ERR_SKIN: "MD_ERR_SKIN",
    MD_ERR_NONFINITE: "MD_ERR_NONFINITE", MD_ERR_DEVICE: "MD_ERR_DEVICE", MD_ERR_STATE: "MD_ERR_STATE",
}
MD_FP64, MD_MIXED = 0, 1
MD_NBR_FULL, MD_NBR_HALF_ATOMIC = 0, 1
MD_VERLET, MD_GEAR3 = 0, 1
MD_OPT_LANES_PER_ATOM, MD_OPT_USE_GRAPH, MD_OPT_MAX_COUNT, MD_OPT_N_BUILDS, MD_OPT_TIMING = 1, 2, 3, 4, 5
MD_OPT_EVALUATOR = 6
MD_OPT_KERNEL, MD_OPT_BRICK_DIMS, MD_OPT_BRICK_BLOCK, MD_OPT_HALO_CAP, MD_OPT_HALO_OVERFLOWS = 7, 8, 9, 10, 11
MD_OPT_GRAPH_LAUNCHES, MD_OPT_TUNED_NS, MD_OPT_COMPACT = 12, 13, 14
MD_OPT_ENERGY_EVERY, MD_OPT_ENERGY_RING, MD_OPT_NEIGHBOUR_CHUNK, MD_OPT_AUTO_REBUILD = 15, 16, 17, 18
KERNEL_GROUPS = ("build", "density", "force", "reduce")

EXPORTED = [
    "md_create", "md_workspace_bytes", "md_bind", "md_build_neighbours", "md_eam_forces", "md_step",
    "md_energy", "md_copy_neighbours", "md_set_option", "md_get_option", "md_kernel_times", "md_autotune",
    "md_msd", "md_msd_origin", "md_msd_static", "md_energy_history", "md_state_changed", "md_destroy",
    "md_last_error",
]


class MDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Potential(ctypes.Structure):
    _fields_ = [
        ("n_species", ctypes.c_int32), ("n_pair_knots", ctypes.c_int32),
        ("n_dens_knots", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("pair_a", ctypes.c_void_p), ("pair_r", ctypes.c_void_p),
        ("dens_A", ctypes.c_void_p), ("dens_R", ctypes.c_void_p),
        ("emb_c", ctypes.c_void_p), ("mass_amu", ctypes.c_void_p),
    ]


class _Config(ctypes.Structure):
    _fields_ = [
        ("n_replicas", ctypes.c_int32), ("max_neighbours", ctypes.c_int32),
        ("rebuild_every", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nbr_mode", ctypes.c_int32), ("lanes_per_atom", ctypes.c_int32),
        ("atom_offset", ctypes.c_void_p), ("box", ctypes.c_void_p), ("origin", ctypes.c_void_p),
        ("periodic", ctypes.c_void_p), ("rigid_velocity", ctypes.c_void_p),
        ("skin", ctypes.c_double), ("dt_fs", ctypes.c_double),
        ("nh_temperature", ctypes.c_void_p), ("nh_mass", ctypes.c_void_p), ("integrator", ctypes.c_int32),
        ("pr_pressure_gpa", ctypes.c_void_p), ("pr_mass", ctypes.c_void_p),
        ("box_matrix", ctypes.c_void_p), ("pr_stress_gpa", ctypes.c_void_p),
    ]


class _State(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "species", "rigid", "e_atom")]


class _Energies(ctypes.Structure):
    _fields_ = [
        ("pe", ctypes.c_double), ("ke", ctypes.c_double), ("temperature", ctypes.c_double),
        ("pressure_gpa", ctypes.c_double), ("volume", ctypes.c_double),
        ("piston_work", ctypes.c_double), ("virial", ctypes.c_double * 6),
        ("step", ctypes.c_int64), ("n_atoms", ctypes.c_int64), ("n_mobile", ctypes.c_int64),
        ("nh_pi", ctypes.c_double), ("nh_energy", ctypes.c_double), ("box", ctypes.c_double * 3),
        ("pr_energy", ctypes.c_double), ("h", ctypes.c_double * 9),
    ]


_lib = None


def library():
    """Load libmdeam.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1107_2619_amd.build`")
    # PyTorch ships its own copy of the HIP runtime under the same soname.  It
    # has to be loaded (and, with a GPU present, initialised) before this
    # library, which then binds to it; in the other order PyTorch finds no GPU.
    try:
        import torch

        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.md_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(_Potential), ctypes.POINTER(vp)]
    lib.md_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.md_bind.argtypes = [vp, ctypes.POINTER(_State), vp, ctypes.c_size_t]
    lib.md_build_neighbours.argtypes = [vp, vp]
    lib.md_eam_forces.argtypes = [vp, ctypes.c_int, vp]
    lib.md_step.argtypes = [vp, i32, vp]
    lib.md_energy.argtypes = [vp, ctypes.POINTER(_Energies), vp]
    lib.md_copy_neighbours.argtypes = [vp, vp, vp, i32, vp]
    lib.md_set_option.argtypes = [vp, i32, i64]
    lib.md_get_option.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.md_kernel_times.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.md_autotune.argtypes = [vp, i32, vp]
    lib.md_msd.argtypes = [vp, vp, vp, vp]
    lib.md_msd_origin.argtypes = [vp, vp]
    lib.md_msd_static.argtypes = [vp, vp, vp, vp]
    lib.md_energy_history.argtypes = [vp, ctypes.POINTER(_Energies), i64, ctypes.POINTER(i64), vp]
    lib.md_state_changed.argtypes = [vp]
    lib.md_destroy.argtypes = [vp]
    lib.md_destroy.restype = None
    lib.md_last_error.argtypes = [vp]
    lib.md_last_error.restype = ctypes.c_char_p
    for name in EXPORTED[:-2]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Context:
    """Owns one ``md_ctx`` (host side only until ``bind``).

    Per-replica options map onto ``md_config`` (include/md.h): the thermostat
    (``nh_temperature``, ``nh_mass``), the integrator (``"verlet"`` or
    ``"gear3"``), the barostat (``pr_pressure_gpa``, ``pr_mass``), sheared cells
    (``box_matrix`` [R, 3, 3], edge vectors as columns; ``box`` is then ignored)
    and the external stress of the full-matrix barostat (``pr_stress_gpa``
    [R, 3, 3], GPa).  Scalars broadcast over the replicas."""

    def __init__(self, potential: dict, atom_offset, box, periodic, *, origin=None, rigid_velocity=None,
                 skin=0.3, dt_fs=1.0, rebuild_every=10, max_neighbours=64, precision="fp64",
                 nbr_mode="full", lanes_per_atom=0, nh_temperature=None, nh_mass=None, integrator="verlet",
                 pr_pressure_gpa=None, pr_mass=None, box_matrix=None, pr_stress_gpa=None):
        self.lib = library()
        pa = _c(potential["pair_a"], np.float64)
        ns = pa.shape[0]
        self._keep = {
            "pair_a": pa, "pair_r": _c(potential["pair_r"], np.float64),
            "dens_A": _c(potential["dens_A"], np.float64), "dens_R": _c(potential["dens_R"], np.float64),
            "emb_c": _c(potential["emb_c"], np.float64), "mass": _c(potential["mass"], np.float64),
            "off": _c(atom_offset, np.int64), "box": _c(box, np.float64).reshape(-1, 3),
            "periodic": _c(periodic, np.uint8).reshape(-1, 3),
        }
        k = self._keep
        k["origin"] = None if origin is None else _c(origin, np.float64).reshape(-1, 3)
        k["vp"] = None if rigid_velocity is None else _c(rigid_velocity, np.float64).reshape(-1, 3)
        n_rep = len(k["off"]) - 1
        k["nh_t"] = None if nh_temperature is None else np.broadcast_to(
            np.asarray(nh_temperature, np.float64), (n_rep,)).copy()
        k["nh_q"] = None if nh_mass is None else np.broadcast_to(np.asarray(nh_mass, np.float64), (n_rep,)).copy()
        k["pr_p"] = None if pr_pressure_gpa is None else np.broadcast_to(
            np.asarray(pr_pressure_gpa, np.float64), (n_rep,)).copy()
        k["pr_w"] = None if pr_mass is None else np.broadcast_to(np.asarray(pr_mass, np.float64), (n_rep,)).copy()
        # box matrices [R, 3, 3] (edge vectors as columns) and external stresses [R, 3, 3]
        k["hmat"] = None if box_matrix is None else np.broadcast_to(
            np.asarray(box_matrix, np.float64), (n_rep, 3, 3)).copy()
        k["pr_s"] = None if pr_stress_gpa is None else np.broadcast_to(
            np.asarray(pr_stress_gpa, np.float64), (n_rep, 3, 3)).copy()
        pot = _Potential(ns, pa.shape[2], k["dens_A"].shape[2], 0, pa.ctypes.data, k["pair_r"].ctypes.data,
                         k["dens_A"].ctypes.data, k["dens_R"].ctypes.data, k["emb_c"].ctypes.data,
                         k["mass"].ctypes.data)
        prec = {"fp64": MD_FP64, "mixed": MD_MIXED}[precision] if isinstance(precision, str) else precision
        mode = {"full": MD_NBR_FULL, "half": MD_NBR_HALF_ATOMIC}[nbr_mode] if isinstance(nbr_mode, str) else nbr_mode
        cfg = _Config(
            len(k["off"]) - 1, int(max_neighbours), int(rebuild_every), prec, mode, int(lanes_per_atom),
            k["off"].ctypes.data, k["box"].ctypes.data,
            None if k["origin"] is None else k["origin"].ctypes.data, k["periodic"].ctypes.data,
            None if k["vp"] is None else k["vp"].ctypes.data, float(skin), float(dt_fs),
            None if k["nh_t"] is None else k["nh_t"].ctypes.data, None if k["nh_q"] is None else k["nh_q"].ctypes.data,
            {"verlet": MD_VERLET, "gear3": MD_GEAR3}[integrator] if isinstance(integrator, str) else int(integrator),
            None if k["pr_p"] is None else k["pr_p"].ctypes.data, None if k["pr_w"] is None else k["pr_w"].ctypes.data,
            None if k["hmat"] is None else k["hmat"].ctypes.data, None if k["pr_s"] is None else k["pr_s"].ctypes.data,
        )
        h = ctypes.c_void_p()
        rc = self.lib.md_create(ctypes.byref(cfg), ctypes.byref(pot), ctypes.byref(h))
        self.handle = h.value
        if rc != MD_OK:
            msg = self.lib.md_last_error(self.handle).decode() if self.handle else "md_create failed"
            if self.handle:
                self.lib.md_destroy(self.handle)
                self.handle = None
            raise MDError(rc, msg)
        self.n_replicas = len(k["off"]) - 1
        self.n_atoms = int(k["off"][-1])
        self.n_species = ns

    def _check(self, rc):
        if rc != MD_OK:
            raise MDError(rc, self.lib.md_last_error(self.handle).decode())

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.md_workspace_bytes(self.handle, ctypes.byref(n)))
        return n.value

    def set_option(self, opt, value):
        self._check(self.lib.md_set_option(self.handle, int(opt), int(value)))

    def get_option(self, opt) -> int:
        v = ctypes.c_int64()
        self._check(self.lib.md_get_option(self.handle, int(opt), ctypes.byref(v)))
        return v.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self.lib.md_destroy(h)
            self.handle = None


@dataclass
class Energies:
    pe: np.ndarray
    ke: np.ndarray
    temperature: np.ndarray
    pressure_gpa: np.ndarray
    volume: np.ndarray
    piston_work: np.ndarray
    virial: np.ndarray  # [R, 6]
    step: int
    n_atoms: np.ndarray
    n_mobile: np.ndarray
    nh_pi: np.ndarray      # thermostat momentum per replica, 1/fs (0 without a thermostat)
    nh_energy: np.ndarray  # thermostat energy 0.5 Q pi^2 + g k T xi, eV
    box: np.ndarray        # [R, 3] edge lengths, A
    pr_energy: np.ndarray  # barostat energy P Omega + W |dL/dt|^2 / 2 (+ the strain energy), eV
    h: np.ndarray          # [R, 3, 3] box matrices (edge vectors as columns), A


class Simulation:
    """Device state (torch tensors) bound to a Context built from ``system``
    (an ``inputs.System``); the keyword options are those of ``Context``."""

    def __init__(self, system, *, precision="fp64", nbr_mode="full", max_neighbours=None, lanes_per_atom=0,
                 device="cuda:0", want_e_atom=True, rebuild_every=None, skin=None, nh_temperature=None,
                 nh_mass=None, integrator="verlet", pr_pressure_gpa=None, pr_mass=None, box_matrix=None,
                 pr_stress_gpa=None, energy_ring=0):
        import torch

        self.torch = torch
        self.system = system
        self.device = torch.device(device)
        self.cap = int(system.max_neighbours if max_neighbours is None else max_neighbours)
        self.ctx = Context(
            system.potential, system.atom_offset, system.box, system.periodic, origin=system.origin,
            rigid_velocity=system.rigid_velocity, skin=system.skin if skin is None else skin,
            dt_fs=system.dt_fs, rebuild_every=system.rebuild_every if rebuild_every is None else rebuild_every,
            max_neighbours=self.cap,
            precision=precision, nbr_mode=nbr_mode, lanes_per_atom=lanes_per_atom,
            nh_temperature=nh_temperature, nh_mass=nh_mass, integrator=integrator,
            pr_pressure_gpa=pr_pressure_gpa, pr_mass=pr_mass, box_matrix=box_matrix, pr_stress_gpa=pr_stress_gpa,
        )
        if energy_ring:  # sizes the workspace, so before it is allocated
            self.ctx.set_option(MD_OPT_ENERGY_RING, int(energy_ring))
        d = self.device
        f64 = dict(dtype=torch.float64, device=d)
        n = system.n_atoms
        self.x = torch.tensor(system.pos[:, 0], **f64)
        self.y = torch.tensor(system.pos[:, 1], **f64)
        self.z = torch.tensor(system.pos[:, 2], **f64)
        self.vx = torch.tensor(system.vel[:, 0], **f64)
        self.vy = torch.tensor(system.vel[:, 1], **f64)
        self.vz = torch.tensor(system.vel[:, 2], **f64)
        self.fx = torch.zeros(n, **f64)
        self.fy = torch.zeros(n, **f64)
        self.fz = torch.zeros(n, **f64)
        self.species = torch.tensor(system.species, dtype=torch.uint8, device=d)
        self.rigid = torch.tensor(system.rigid, dtype=torch.uint8, device=d) if system.rigid.any() else None
        self.e_atom = torch.zeros(n, **f64) if want_e_atom else None
        nbytes = self.ctx.workspace_bytes()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=d)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._bind()

    def _ptr(self, t):
        return None if t is None else t.data_ptr()

    def _bind(self):
        st = _State(*(self._ptr(t) for t in (self.x, self.y, self.z, self.vx, self.vy, self.vz, self.fx, self.fy,
                                             self.fz, self.species, self.rigid, self.e_atom)))
        self.ctx._check(self.ctx.lib.md_bind(self.ctx.handle, ctypes.byref(st), self._ws_ptr,
                                             self.ctx.workspace_bytes()))

    def set_state(self, pos=None, vel=None):
        """Overwrite positions/velocities (caller order) on the device."""
        t = self.torch
        if pos is not None:
            p = t.as_tensor(np.asarray(pos, np.float64), device=self.device)
            self.x.copy_(p[:, 0]), self.y.copy_(p[:, 1]), self.z.copy_(p[:, 2])
        if vel is not None:
            v = t.as_tensor(np.asarray(vel, np.float64), device=self.device)
            self.vx.copy_(v[:, 0]), self.vy.copy_(v[:, 1]), self.vz.copy_(v[:, 2])
        self.state_changed()

    def state_changed(self):
        """Tell the library the bound arrays were written (md_state_changed)."""
        self.ctx._check(self.ctx.lib.md_state_changed(self.ctx.handle))

    def rebind(self):
        """Re-attach the same buffers (resets step counter, list and piston work)."""
        self._bind()

    @property
    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def build_neighbours(self):
        self.ctx._check(self.ctx.lib.md_build_neighbours(self.ctx.handle, self.stream))

    def eam_forces(self, want_energy=True):
        self.ctx._check(self.ctx.lib.md_eam_forces(self.ctx.handle, int(bool(want_energy)), self.stream))

    def step(self, nsteps: int):
        self.ctx._check(self.ctx.lib.md_step(self.ctx.handle, int(nsteps), self.stream))

    def energy(self) -> Energies:
        R = self.ctx.n_replicas
        out = (_Energies * R)()
        self.ctx._check(self.ctx.lib.md_energy(self.ctx.handle, out, self.stream))
        g = lambda name: np.array([getattr(o, name) for o in out])  # noqa: E731
        return Energies(g("pe"), g("ke"), g("temperature"), g("pressure_gpa"), g("volume"), g("piston_work"),
                        np.array([list(o.virial) for o in out]), int(out[0].step), g("n_atoms"), g("n_mobile"),
                        g("nh_pi"), g("nh_energy"), np.array([list(o.box) for o in out]), g("pr_energy"),
                        np.array([list(o.h) for o in out]).reshape(R, 3, 3))

    def energy_history(self, max_entries=10000) -> list:
        """Per-step energies appended since the last call (md_energy_history):
        a list of Energies, one per sampled step, oldest first."""
        R = self.ctx.n_replicas
        out = (_Energies * (R * max_entries))()
        n = ctypes.c_int64(0)
        self.ctx._check(self.ctx.lib.md_energy_history(self.ctx.handle, out, int(max_entries), ctypes.byref(n),
                                                       self.stream))
        res = []
        for j in range(n.value):
            rec = out[j * R:(j + 1) * R]
            g = lambda name: np.array([getattr(o, name) for o in rec])  # noqa: E731
            res.append(Energies(g("pe"), g("ke"), g("temperature"), g("pressure_gpa"), g("volume"),
                                g("piston_work"), np.array([list(o.virial) for o in rec]), int(rec[0].step),
                                g("n_atoms"), g("n_mobile"), g("nh_pi"), g("nh_energy"),
                                np.array([list(o.box) for o in rec]), g("pr_energy"),
                                np.array([list(o.h) for o in rec]).reshape(R, 3, 3)))
        return res

    def msd(self):
        """(msd [R, n_species] A^2, count [R, n_species]): mean square displacement
        of the mobile atoms from the origin positions (md_msd)."""
        shape = (self.ctx.n_replicas, self.ctx.n_species)
        out = np.zeros(shape)
        cnt = np.zeros(shape, np.int64)
        self.ctx._check(self.ctx.lib.md_msd(self.ctx.handle, out.ctypes.data, cnt.ctypes.data, self.stream))
        return out, cnt

    def msd_static(self):
        """msd() through md_msd_static (no device allocation: static scratch)."""
        shape = (self.ctx.n_replicas, self.ctx.n_species)
        out = np.zeros(shape)
        cnt = np.zeros(shape, np.int64)
        self.ctx._check(self.ctx.lib.md_msd_static(self.ctx.handle, out.ctypes.data, cnt.ctypes.data, self.stream))
        return out, cnt

    def msd_origin(self):
        """Take the current positions as the origin of msd() (md_msd_origin)."""
        self.ctx._check(self.ctx.lib.md_msd_origin(self.ctx.handle, self.stream))

    def neighbours(self):
        """(counts[N], list[N, cap]) in caller numbering."""
        cap = self.cap
        n = self.ctx.n_atoms
        counts = np.zeros(n, np.int32)
        lst = np.full((n, cap), -1, np.int32)
        self.ctx._check(self.ctx.lib.md_copy_neighbours(self.ctx.handle, counts.ctypes.data, lst.ctypes.data,
                                                        cap, self.stream))
        return counts, lst

    def set_option(self, opt, value):
        self.ctx.set_option(opt, value)

    def get_option(self, opt) -> int:
        return self.ctx.get_option(opt)

    def kernel_times(self, reset=True):
        """{group: (total ms, launches)} recorded with MD_OPT_TIMING on."""
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        self.ctx._check(self.ctx.lib.md_kernel_times(self.ctx.handle, ms.ctypes.data, n.ctypes.data, int(reset),
                                                     self.stream))
        return {g: (float(ms[i]), int(n[i])) for i, g in enumerate(KERNEL_GROUPS)}

    def autotune(self, trials=5):
        """Pick the fastest kernel configuration for this system (md_autotune);
        returns the chosen settings and the estimated step time in us."""
        self.ctx._check(self.ctx.lib.md_autotune(self.ctx.handle, int(trials), self.stream))
        opts = {name: self.get_option(opt) for name, opt in (
            ("kernel", MD_OPT_KERNEL), ("brick_dims", MD_OPT_BRICK_DIMS), ("lanes", MD_OPT_LANES_PER_ATOM),
            ("block", MD_OPT_BRICK_BLOCK), ("evaluator", MD_OPT_EVALUATOR), ("nchunk", MD_OPT_NEIGHBOUR_CHUNK))}
        opts["step_us"] = self.get_option(MD_OPT_TUNED_NS) / 1e3
        return opts

    def positions(self) -> np.ndarray:
        return self.torch.stack([self.x, self.y, self.z], 1).cpu().numpy()

    def velocities(self) -> np.ndarray:
        return self.torch.stack([self.vx, self.vy, self.vz], 1).cpu().numpy()

    def forces(self) -> np.ndarray:
        return self.torch.stack([self.fx, self.fy, self.fz], 1).cpu().numpy()

    def atom_energies(self) -> np.ndarray:
        return self.e_atom.cpu().numpy()
