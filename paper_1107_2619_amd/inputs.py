"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the force-loop arithmetic: it builds lattices, removes
vacancies, places interstitials, packs random liquids, draws Maxwell-Boltzmann
velocities and reads/perturbs the cubic-knot potential tables.  Both the CPU
oracle and the GPU library receive exactly what it produces.

Workloads (all synthetic; the paper's own benchmark is itself a synthetic bcc Fe
cube, "Parallel benchmarks"):

* ``bcc_fe``   - bcc Fe, n^3 cells, a = 2.87 A, periodic, optional vacancies.
* ``fcc_piston`` - fcc Cu-like slab periodic in x,y and free in z with a rigid
  bottom layer driven at a fixed velocity (shock-like compression).
* ``fec_replicas`` - many bcc Fe-C replicas of uneven sizes with carbon at
  random octahedral sites.
* ``liquid_replicas`` - many random-packed Fe liquids at 7.0 g/cm^3.

Units at the boundary: Angstrom, amu, eV, fs (velocities in Angstrom/fs).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

# Physical constants (paper, "Units": amu as printed; eV and k_B from the same
# CODATA-2002 set).  Used only to draw thermal velocities.
AMU_KG = 1.66053886e-27
EV_J = 1.60217653e-19
KB_EV = 8.617343e-5
TIME_UNIT_FS = math.sqrt(AMU_KG * 1.0e-20 / EV_J) * 1.0e15

_POT_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "potentials")


# --------------------------------------------------------------------------- potentials
def load_table(name: str) -> dict:
    """Read a base cubic-knot table ``potentials/<name>.json``."""
    with open(os.path.join(_POT_DIR, name + ".json")) as fh:
        return json.load(fh)


def table_to_arrays(tab: dict) -> dict:
    """Convert a JSON table into the dense arrays both sides read.

    pair_a/pair_r [ns,ns,npk] (symmetric), dens_A/dens_R [ns,ns,ndk] with
    [a,b] = density at an a-site from a b-neighbour, emb_c [ns], mass [ns].
    """
    sp = tab["species"]
    ns = len(sp)
    npk = len(next(iter(tab["pair"].values()))["r"])
    ndk = len(next(iter(tab["density"].values()))["R"])
    pa = np.zeros((ns, ns, npk))
    pr = np.zeros((ns, ns, npk))
    da = np.zeros((ns, ns, ndk))
    dr = np.zeros((ns, ns, ndk))
    seen = np.zeros((ns, ns), bool)
    for key, v in tab["pair"].items():
        a, b = (sp.index(s) for s in key.split("-"))
        for (p, q) in ((a, b), (b, a)):
            pa[p, q] = v["a"]
            pr[p, q] = v["r"]
            seen[p, q] = True
    if not seen.all():
        raise ValueError("pair table incomplete")
    seen[:] = False
    for key, v in tab["density"].items():
        a, b = (sp.index(s) for s in key.split("<-"))
        da[a, b] = v["A"]
        dr[a, b] = v["R"]
        seen[a, b] = True
    if not seen.all():
        raise ValueError("density table incomplete")
    return {
        "species": list(sp),
        "pair_a": pa,
        "pair_r": pr,
        "dens_A": da,
        "dens_R": dr,
        "emb_c": np.asarray(tab["emb_c"], float),
        "mass": np.asarray(tab["mass"], float),
    }


def perturbed_potential(name: str, seed: int | None, frac: float = 0.05) -> dict:
    """Base table with every coefficient scaled by (1 + frac*(2U-1)).

    U comes from ``numpy.random.default_rng(seed)``, drawn in file order: for
    each pair function (upper triangle, a <= b) its a_1..a_npk, then for each
    density function its A_1..A_ndk.  Knot positions are not perturbed.
    ``seed=None`` returns the base table unchanged.
    """
    arr = table_to_arrays(load_table(name))
    if seed is None:
        return arr
    rng = np.random.default_rng(seed)
    ns = arr["emb_c"].shape[0]
    for a in range(ns):
        for b in range(a, ns):
            s = 1.0 + frac * (2.0 * rng.random(arr["pair_a"].shape[2]) - 1.0)
            arr["pair_a"][a, b] *= s
            if b != a:
                arr["pair_a"][b, a] = arr["pair_a"][a, b]
    for a in range(ns):
        for b in range(ns):
            s = 1.0 + frac * (2.0 * rng.random(arr["dens_A"].shape[2]) - 1.0)
            arr["dens_A"][a, b] *= s
    return arr


# --------------------------------------------------------------------------- structures
def bcc(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """bcc lattice, 2 atoms per cubic cell (the paper's benchmark cell)."""
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return _lattice(nx, ny, nz, a, basis)


def fcc(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    return _lattice(nx, ny, nz, a, basis)


def _lattice(nx, ny, nz, a, basis):
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    g = g.reshape(-1, 1, 3).astype(float)
    return ((g + basis[None]) * a).reshape(-1, 3)


def bcc_octahedral_sites(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """The 6 octahedral interstitial sites per bcc cubic cell: the three edge
    midpoints (1/2,0,0)-type and the three face centres (1/2,1/2,0)-type."""
    basis = np.array(
        [[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], float
    )
    return _lattice(nx, ny, nz, a, basis)


def random_liquid(n: int, box: float, dmin: float, rng: np.random.Generator, spread: float = 1.15,
                  max_iter: int = 1000) -> np.ndarray:
    """n random points in a periodic cube with every pair at least dmin apart:
    uniform random positions, then overlap relaxation (every pair closer than
    spread * dmin is pushed apart symmetrically along its separation, all pairs
    at once) until no pair is closer than dmin.  The push target above dmin
    gives nearest-neighbour distances spread over [dmin, spread * dmin] instead
    of piling up at dmin."""
    from scipy.spatial import cKDTree

    pts = rng.random((n, 3)) * box
    target = dmin * spread
    for _ in range(max_iter):
        tree = cKDTree(pts, boxsize=box)
        if not len(tree.query_pairs(dmin, output_type="ndarray")):
            return pts
        pairs = tree.query_pairs(target, output_type="ndarray")
        i, j = pairs[:, 0], pairs[:, 1]
        d = pts[j] - pts[i]
        d -= box * np.rint(d / box)
        r = np.linalg.norm(d, axis=1)
        zero = r < 1e-12
        if zero.any():
            d[zero] = rng.normal(size=(int(zero.sum()), 3))
            r[zero] = np.linalg.norm(d[zero], axis=1)
        push = (0.5 * (target - r) / r)[:, None] * d
        disp = np.stack([np.bincount(j, push[:, a], n) - np.bincount(i, push[:, a], n) for a in range(3)], 1)
        pts = (pts + disp) % box
    raise RuntimeError("random packing did not converge")


def maxwell_boltzmann(masses: np.ndarray, temperature: float, rng: np.random.Generator,
                      mobile: np.ndarray | None = None) -> np.ndarray:
    """Gaussian velocity components of variance k_B T / m (A/fs), with the
    mass-weighted centre-of-mass velocity of the mobile atoms removed.  No
    rescaling to the exact target temperature is applied."""
    n = masses.shape[0]
    sig = np.sqrt(KB_EV * temperature / masses) / TIME_UNIT_FS
    v = rng.standard_normal((n, 3)) * sig[:, None]
    mob = np.ones(n, bool) if mobile is None else mobile.astype(bool)
    if mob.sum() > 1:
        m = masses[mob]
        vcm = (m[:, None] * v[mob]).sum(0) / m.sum()
        v[mob] -= vcm
    v[~mob] = 0.0
    return v


# --------------------------------------------------------------------------- systems
@dataclass
class System:
    """A batch of R >= 1 independent replicas, atoms of replica r in
    [atom_offset[r], atom_offset[r+1])."""

    name: str
    pos: np.ndarray  # [N,3] A, unwrapped
    vel: np.ndarray  # [N,3] A/fs
    species: np.ndarray  # [N] uint8
    rigid: np.ndarray  # [N] uint8 (1 = prescribed trajectory)
    atom_offset: np.ndarray  # [R+1] int64
    box: np.ndarray  # [R,3] A
    origin: np.ndarray  # [R,3] A (lower corner; used on free axes)
    periodic: np.ndarray  # [R,3] uint8
    rigid_velocity: np.ndarray  # [R,3] A/fs
    potential: dict
    dt_fs: float
    skin: float
    rebuild_every: int
    steps: int
    temperature: np.ndarray  # [R] K
    max_neighbours: int = 64
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.atom_offset[-1])

    @property
    def n_replicas(self) -> int:
        return int(self.atom_offset.shape[0] - 1)

    def replica(self, r: int) -> "System":
        """Replica r as a stand-alone one-replica system."""
        a, b = int(self.atom_offset[r]), int(self.atom_offset[r + 1])
        return System(
            name=f"{self.name}[{r}]", pos=self.pos[a:b].copy(), vel=self.vel[a:b].copy(),
            species=self.species[a:b].copy(), rigid=self.rigid[a:b].copy(),
            atom_offset=np.array([0, b - a], np.int64), box=self.box[r:r + 1].copy(),
            origin=self.origin[r:r + 1].copy(), periodic=self.periodic[r:r + 1].copy(),
            rigid_velocity=self.rigid_velocity[r:r + 1].copy(), potential=self.potential,
            dt_fs=self.dt_fs, skin=self.skin, rebuild_every=self.rebuild_every, steps=self.steps,
            temperature=self.temperature[r:r + 1].copy(), max_neighbours=self.max_neighbours,
            meta=dict(self.meta),
        )


def _single(name, pos, vel, species, rigid, box, origin, periodic, vp, pot, dt, skin, every, steps,
            temp, cap, meta=None):
    n = pos.shape[0]
    return System(
        name=name, pos=np.ascontiguousarray(pos, float), vel=np.ascontiguousarray(vel, float),
        species=np.ascontiguousarray(species, np.uint8), rigid=np.ascontiguousarray(rigid, np.uint8),
        atom_offset=np.array([0, n], np.int64), box=np.asarray([box], float),
        origin=np.asarray([origin], float), periodic=np.asarray([periodic], np.uint8),
        rigid_velocity=np.asarray([vp], float), potential=pot, dt_fs=float(dt), skin=float(skin),
        rebuild_every=int(every), steps=int(steps), temperature=np.asarray([temp], float),
        max_neighbours=int(cap), meta=meta or {},
    )


def bcc_fe(n: int = 10, a: float = 2.87, temperature: float = 300.0, vacancy_frac: float = 0.0,
           seed: int = 1, pot_seed: int | None = None, dt_fs: float = 1.0, skin: float = 0.3,
           rebuild_every: int = 10, steps: int = 100, displace: float = 0.0,
           name: str = "bcc_fe", potential: str = "fe_fs") -> System:
    """bcc Fe cube of n^3 cells with optional random vacancies, Maxwell-Boltzmann
    velocities and an optional uniform random displacement of every atom
    (the ``dsp`` input of the paper's parameter table).  ``potential`` names the
    base table (``fe_fs``: 6 + 2 knots, ``fe15_fs``: 13 + 2 knots)."""
    rng = np.random.default_rng(seed)
    pot = perturbed_potential(potential, seed if pot_seed is None else pot_seed)
    pos = bcc(n, n, n, a)
    if vacancy_frac > 0:
        nv = int(round(vacancy_frac * pos.shape[0]))
        drop = rng.choice(pos.shape[0], nv, replace=False)
        pos = np.delete(pos, drop, 0)
    if displace > 0:
        pos = pos + displace * (2.0 * rng.random(pos.shape) - 1.0)
    sp = np.zeros(pos.shape[0], np.uint8)
    vel = maxwell_boltzmann(pot["mass"][sp], temperature, rng)
    L = n * a
    return _single(name, pos, vel, sp, np.zeros(pos.shape[0], np.uint8), [L, L, L], [0, 0, 0],
                   [1, 1, 1], [0, 0, 0], pot, dt_fs, skin, rebuild_every, steps, temperature, 48,
                   {"a": a, "cells": n})


def fcc_piston(nx: int = 60, ny: int = 60, nz: int = 200, a: float = 3.615,
               temperature: float = 300.0, piston_cells: int = 3, piston_speed_a_per_fs: float = 0.01,
               seed: int = 3, dt_fs: float = 0.5, skin: float = 0.3, rebuild_every: int = 10,
               steps: int = 2000, z_margin: float = 25.0, name: str = "fcc_piston") -> System:
    """fcc slab periodic in x,y and free in z; atoms below ``piston_cells``
    cubic cells form a rigid piston moving at +piston_speed along z (1 km/s =
    0.01 A/fs)."""
    rng = np.random.default_rng(seed)
    pot = perturbed_potential("cu_fs", seed)
    pos = fcc(nx, ny, nz, a)
    rigid = (pos[:, 2] < piston_cells * a - 1e-9).astype(np.uint8)
    sp = np.zeros(pos.shape[0], np.uint8)
    vel = maxwell_boltzmann(pot["mass"][sp], temperature, rng, mobile=rigid == 0)
    vp = np.array([0.0, 0.0, piston_speed_a_per_fs])
    vel[rigid == 1] = vp
    box = [nx * a, ny * a, nz * a + 2 * z_margin]
    origin = [0.0, 0.0, -z_margin]
    return _single(name, pos, vel, sp, rigid, box, origin, [1, 1, 0], vp, pot, dt_fs, skin,
                   rebuild_every, steps, temperature, 96, {"a": a})


def _near_cubic_cells(n_target: int, nmin: int = 5):
    """(nx,ny,nz) >= nmin with 2*nx*ny*nz closest to n_target, then most cubic."""
    c = max(nmin, int(round((n_target / 2.0) ** (1.0 / 3.0))))
    best = None
    for nx in range(max(nmin, c - 2), c + 3):
        for ny in range(max(nmin, c - 2), c + 3):
            nz = max(nmin, int(round(n_target / (2.0 * nx * ny))))
            key = (abs(2 * nx * ny * nz - n_target), max(nx, ny, nz) - min(nx, ny, nz))
            if best is None or key < best[0]:
                best = (key, (nx, ny, nz))
    return best[1]


def _concat(name, parts, pot, dt, skin, every, steps, cap, meta):
    off = np.zeros(len(parts) + 1, np.int64)
    off[1:] = np.cumsum([p["pos"].shape[0] for p in parts])
    cat = lambda k: np.concatenate([p[k] for p in parts], 0)  # noqa: E731
    return System(
        name=name, pos=cat("pos"), vel=cat("vel"), species=cat("species").astype(np.uint8),
        rigid=cat("rigid").astype(np.uint8), atom_offset=off,
        box=np.array([p["box"] for p in parts], float),
        origin=np.zeros((len(parts), 3)), periodic=np.ones((len(parts), 3), np.uint8),
        rigid_velocity=np.zeros((len(parts), 3)), potential=pot, dt_fs=dt, skin=skin,
        rebuild_every=every, steps=steps, temperature=np.array([p["T"] for p in parts], float),
        max_neighbours=cap, meta=meta,
    )


def _spread_sites(sites: np.ndarray, n: int, box: np.ndarray, min_sep: float,
                  rng: np.random.Generator) -> np.ndarray:
    """n distinct sites in random order, skipping any closer than min_sep
    (periodic) to one already taken."""
    chosen: list[np.ndarray] = []
    for idx in rng.permutation(sites.shape[0]):
        if len(chosen) == n:
            break
        s = sites[idx]
        if chosen:
            d = np.asarray(chosen) - s
            d -= box * np.rint(d / box)
            if np.min(np.sum(d * d, 1)) < min_sep * min_sep:
                continue
        chosen.append(s)
    if len(chosen) < n:
        raise ValueError("too many carbon atoms for the requested separation")
    return np.asarray(chosen).reshape(-1, 3)


def fec_replicas(n_replicas: int = 256, nmin: int = 250, nmax: int = 16000, a: float = 2.87,
                 c_frac: float = 0.005, tmin: float = 300.0, tmax: float = 1200.0,
                 seed0: int = 4000, pot_seed: int = 4, steps: int = 500, dt_fs: float = 1.0,
                 skin: float = 0.8, rebuild_every: int = 5, c_min_sep: float = 1.0,
                 name: str = "fec_replicas") -> System:
    """Independent bcc Fe-C replicas: size ~ U{nmin..nmax}, near-cubic cells,
    round(c_frac * N_Fe) carbon atoms on distinct random octahedral sites,
    temperature ~ U[tmin, tmax], no two carbons closer than c_min_sep lattice
    constants (neighbouring octahedral sites are only a/2 apart, and such
    pairs fly apart at several km/s).  Replica r uses seed seed0 + r.  Carbon at
    1200 K moves up to ~0.26 A in 5 fs in a 2000-atom replica (further in the
    tail of a million-atom batch), so the list uses a 0.8 A skin (guard at
    0.4 A) rebuilt every 5 steps."""
    pot = perturbed_potential("fec_eam", pot_seed)
    parts = []
    for r in range(n_replicas):
        rng = np.random.default_rng(seed0 + r)
        n_r = int(rng.integers(nmin, nmax + 1))
        nx, ny, nz = _near_cubic_cells(n_r)
        fe = bcc(nx, ny, nz, a)
        nc = int(round(c_frac * fe.shape[0]))
        sites = bcc_octahedral_sites(nx, ny, nz, a)
        cpos = _spread_sites(sites, nc, np.array([nx, ny, nz]) * a, c_min_sep * a, rng)
        pos = np.concatenate([fe, cpos], 0)
        sp = np.concatenate([np.zeros(fe.shape[0], np.uint8), np.ones(nc, np.uint8)])
        T = float(rng.uniform(tmin, tmax))
        vel = maxwell_boltzmann(pot["mass"][sp], T, rng)
        parts.append({"pos": pos, "vel": vel, "species": sp, "rigid": np.zeros(pos.shape[0]),
                      "box": [nx * a, ny * a, nz * a], "T": T})
    return _concat(name, parts, pot, dt_fs, skin, rebuild_every, steps, 64, {"a": a})


def vacancy_replicas(temperatures=tuple(range(900, 2001, 100)), per_temperature: int = 16, cells: int = 10,
                     a: float = 2.87, seed0: int = 6000, pot_seed: int = 6, steps: int = 2000,
                     dt_fs: float = 1.0, skin: float = 0.5, rebuild_every: int = 5,
                     name: str = "vacancy_replicas") -> System:
    """The self-diffusion set-up of the paper ("Self-diffusion in iron"): bcc Fe
    of cells^3 unit cells (2000 sites at 10) with one vacancy at a random
    site, at each temperature of ``temperatures`` (900-2000 K in 100 K steps),
    ``per_temperature`` independent replicas each.  Maxwell-Boltzmann
    velocities at the replica's temperature, which is also its thermostat
    target.  At 2000 K the per-axis velocity spread is ~0.0055 A/fs: a 0.5 A
    skin (guard 0.25 A) rebuilt every 5 steps leaves > 8 sigma.  Replica r uses
    seed seed0 + r."""
    pot = perturbed_potential("fe_fs", pot_seed)
    lattice = bcc(cells, cells, cells, a)
    L = cells * a
    parts = []
    r = 0
    for T in temperatures:
        for _ in range(per_temperature):
            rng = np.random.default_rng(seed0 + r)
            pos = np.delete(lattice, int(rng.integers(lattice.shape[0])), 0)
            sp = np.zeros(pos.shape[0], np.uint8)
            vel = maxwell_boltzmann(pot["mass"][sp], float(T), rng)
            parts.append({"pos": pos, "vel": vel, "species": sp, "rigid": np.zeros(pos.shape[0]),
                          "box": [L, L, L], "T": float(T)})
            r += 1
    return _concat(name, parts, pot, dt_fs, skin, rebuild_every, steps, 64, {"a": a, "cells": cells})


LIQUID_VOLUME_PER_ATOM = 13.2475  # A^3 per Fe atom at 7.0 g/cm^3


def _liquid_part(args):
    r, seed0, nmin, nmax, dmin, temperature, mass = args
    rng = np.random.default_rng(seed0 + r)
    n_r = int(rng.integers(nmin, nmax + 1))
    L = (n_r * LIQUID_VOLUME_PER_ATOM) ** (1.0 / 3.0)
    pos = random_liquid(n_r, L, dmin, rng)
    sp = np.zeros(n_r, np.uint8)
    vel = maxwell_boltzmann(np.full(n_r, mass), temperature, rng)
    return {"pos": pos, "vel": vel, "species": sp, "rigid": np.zeros(n_r), "box": [L, L, L], "T": temperature}


def _gpu_initialised() -> bool:
    import sys

    torch = sys.modules.get("torch")
    return bool(torch is not None and torch.cuda.is_initialized())


def liquid_replicas(n_replicas: int = 4096, nmin: int = 128, nmax: int = 2000,
                    temperature: float = 2500.0, dmin: float = 2.0, seed0: int = 5000,
                    pot_seed: int = 5, steps: int = 1000, dt_fs: float = 1.0, skin: float = 0.6,
                    rebuild_every: int = 5, name: str = "liquid_replicas", workers: int = 1) -> System:
    """Independent liquid-like Fe replicas: size ~ U{nmin..nmax}, random
    positions with minimum separation dmin (``random_liquid``) in a periodic
    cube at 7.0 g/cm^3, Maxwell-Boltzmann velocities at ``temperature``.  At
    2500-2800 K an atom moves up to ~0.15 A in 5 fs in a 1000-atom replica and
    ~0.21 A in the tail of a 4-million-atom batch: 0.6 A skin (guard 0.3 A).
    Replica r depends only on seed0 + r, so ``workers`` > 1 (a process pool,
    used only while no GPU context exists in this process) gives the same
    result."""
    pot = perturbed_potential("fe_fs", pot_seed)
    jobs = [(r, seed0, nmin, nmax, dmin, temperature, float(pot["mass"][0])) for r in range(n_replicas)]
    if workers > 1 and n_replicas > 1 and not _gpu_initialised():
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_liquid_part, jobs, chunksize=max(1, n_replicas // (8 * workers)))
    else:
        parts = [_liquid_part(j) for j in jobs]
    return _concat(name, parts, pot, dt_fs, skin, rebuild_every, steps, 96, {})


def workload(name: str, **kw) -> System:
    """Named workloads with the sizes the benchmark and the parity tests use."""
    if name == "bcc2000":  # 2000-atom bcc Fe, 300 K, 100 steps
        return bcc_fe(10, temperature=300.0, seed=1, steps=100, name=name, **kw)
    if name == "bcc31250_fe15":  # 25^3 cells, 31,250 atoms, the 15-spline iron potential, 300 K
        # this softer potential spreads a 10 fs displacement wider (sigma 0.023 A
        # per axis at 300 K against ~0.015 A for fe_fs): a 0.4 A skin keeps the
        # guard at 8.7 sigma
        kw.setdefault("skin", 0.4)
        return bcc_fe(25, temperature=300.0, seed=3, steps=100, name=name, potential="fe15_fs", **kw)
    if name == "bcc1m":  # 80^3 cells, 1% vacancies -> 1,013,760 atoms, 600 K
        # Over 10 fs at 600 K the per-axis displacement has sigma ~0.03 A; with
        # 10^6 atoms a 0.3 A skin (guard at 0.15 A = 5 sigma) is crossed by a
        # handful of atoms per interval, 0.4 A (6.7 sigma) is not.
        kw.setdefault("skin", 0.4)
        return bcc_fe(80, temperature=600.0, vacancy_frac=0.01, seed=2, steps=1000, name=name, **kw)
    if name == "bcc4m":  # 128^3 cells, 1% vacancies -> 4,152,361 atoms, 600 K (beyond the 256 MB cache)
        kw.setdefault("skin", 0.4)
        return bcc_fe(128, temperature=600.0, vacancy_frac=0.01, seed=7, steps=200, name=name, **kw)
    if name == "fcc_piston":
        return fcc_piston(**kw)
    if name == "fec256":
        return fec_replicas(**kw)
    if name == "liquid4096":
        return liquid_replicas(**kw)
    if name == "vacancy192":  # 12 temperatures (900-2000 K) x 16 replicas of 1999 atoms
        return vacancy_replicas(**kw)
    raise KeyError(name)
