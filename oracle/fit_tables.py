"""Write the base cubic-knot potential tables (test infrastructure, run by hand).

The paper's own Fe and Cu coefficient files are not reproduced in it (only the
form, "Available potentials", and a Ni/Al example file), so the workloads use
synthetic tables of the same form.  This script fixes the knot positions and the
density amplitudes and solves for the pair amplitudes a_k by linear least
squares so that the ideal crystal has a chosen cohesive energy, zero pressure,
bulk modulus, and the two cubic shear moduli as soft targets, plus a curvature penalty
that keeps the amplitudes of order one.  Every observable is an energy computed by the oracle on a small
periodic supercell under homogeneous strain, and each is affine in the pair
amplitudes, so the problem is exactly linear.

Usage:  python -m oracle.fit_tables   (writes paper_1107_2619_amd/potentials/*.json)

The tables are inputs, not expected values: parity between the GPU path and the
oracle does not depend on them.
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle as orc

GPA = 160.217653  # eV/A^3 -> GPa
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "paper_1107_2619_amd", "potentials")


def _cubic_supercell(kind, a, reps):
    if kind == "bcc":
        basis = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])
    else:
        basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.stack(np.meshgrid(*(np.arange(reps),) * 3, indexing="ij"), -1).reshape(-1, 1, 3)
    pos = ((g + basis[None]) * a).reshape(-1, 3)
    return pos, np.array([reps * a] * 3)


def _rotated_supercell(kind, a, reps_xy, reps_z):
    """Cell with axes [110], [-110], [001] (orthorhombic, period a*sqrt2, a*sqrt2, a)."""
    big, _ = _cubic_supercell(kind, a, 4 * max(reps_xy, reps_z))
    big = big - big.mean(0)
    s = 1.0 / np.sqrt(2.0)
    rot = np.array([[s, s, 0], [-s, s, 0], [0, 0, 1]])
    p = big @ rot.T
    L = np.array([reps_xy * a * np.sqrt(2), reps_xy * a * np.sqrt(2), reps_z * a])
    frac = p / L
    keep = np.all((frac >= -1e-9) & (frac < 1 - 1e-9), axis=1)
    return p[keep], L


def _energy(pot, pos, L, strain):
    ps = pos * strain[None, :]
    return orc.energy(ps, np.zeros(len(ps), np.uint8), L * strain, [1, 1, 1], pot)


def observables(tab_arrays, kind, a, delta=0.004):
    """E per atom, P (GPa), B, C', C44 (GPa) of the ideal crystal."""
    pot = orc.Potential(tab_arrays)
    pos, L = _cubic_supercell(kind, a, 5 if kind == "bcc" else 4)
    n = len(pos)
    vol = np.prod(L)
    e0 = _energy(pot, pos, L, np.ones(3))
    ep = _energy(pot, pos, L, np.full(3, 1 + delta))
    em = _energy(pot, pos, L, np.full(3, 1 - delta))
    pressure = -(ep - em) / (2 * delta) / (3 * vol) * GPA
    bulk = (ep + em - 2 * e0) / (9 * vol * delta**2) * GPA
    tp = _energy(pot, pos, L, np.array([1 + delta, 1 + delta, 1 - 2 * delta]))
    tm = _energy(pot, pos, L, np.array([1 - delta, 1 - delta, 1 + 2 * delta]))
    cprime = (tp + tm - 2 * e0) / (12 * vol * delta**2) * GPA
    rp, rL = _rotated_supercell(kind, a, 3, 4)
    r0 = _energy(pot, rp, rL, np.ones(3))
    sp_ = _energy(pot, rp, rL, np.array([1 + delta, 1 - delta, 1]))
    sm_ = _energy(pot, rp, rL, np.array([1 - delta, 1 + delta, 1]))
    c44 = (sp_ + sm_ - 2 * r0) / (4 * np.prod(rL) * delta**2) * GPA
    return np.array([e0 / n, pressure, bulk, cprime, c44])


def fit_single(kind, a, knots, dens_A, dens_R, mass, targets, soft_weight, smooth, r_lo,
               core_r, core_val, ridge=0.0):
    """Pair amplitudes of a one-species table.

    Cohesive energy, zero pressure, the bulk modulus and a short-range
    repulsion phi(core_r) = core_val are imposed exactly; the two shear moduli
    are soft targets (weight ``soft_weight``) and the curvature of phi on
    [r_lo, r_max] is penalised (weight ``smooth``), which keeps the amplitudes
    of order one; ``ridge`` adds a penalty on the squared amplitudes, for knot
    sets dense enough that the curvature penalty alone leaves large terms of
    opposite sign.  An equality-constrained least-squares problem, solved
    through its KKT system.  The repulsive core matters for hot runs: without
    it the embedding term makes two atoms pushed closer than ~1.9 A attract.
    """
    npk = len(knots)

    def arrays(amp):
        return {
            "pair_a": np.asarray(amp, float).reshape(1, 1, npk),
            "pair_r": np.asarray(knots, float).reshape(1, 1, npk),
            "dens_A": np.asarray(dens_A, float).reshape(1, 1, -1),
            "dens_R": np.asarray(dens_R, float).reshape(1, 1, -1),
            "emb_c": np.array([1.0]),
            "mass": np.array([mass]),
        }

    base = observables(arrays(np.zeros(npk)), kind, a)
    M = np.array([observables(arrays(np.eye(npk)[k]), kind, a) - base for k in range(npk)]).T
    rhs = np.asarray(targets) - base
    grid = np.linspace(r_lo, knots[-1], 80)
    curv = np.array([[6.0 * max(rk - r, 0.0) for rk in knots] for r in grid]) * np.sqrt(smooth)
    Q = np.vstack([curv, M[3:] * soft_weight, np.eye(npk) * np.sqrt(ridge)])
    q = np.concatenate([np.zeros(len(grid)), rhs[3:] * soft_weight, np.zeros(npk)])
    core = np.array([[max(rk - core_r, 0.0) ** 3 for rk in knots]])
    E, e = np.vstack([M[:3], core]), np.concatenate([rhs[:3], [core_val]])
    kkt = np.block([[Q.T @ Q, E.T], [E, np.zeros((4, 4))]])
    amp = np.linalg.solve(kkt, np.concatenate([Q.T @ q, e]))[:npk]
    return amp, observables(arrays(amp), kind, a)


def _morse_fit(knots, D, r0, alpha, rlo):
    r = np.linspace(rlo, knots[-1], 200)
    tgt = D * ((1 - np.exp(-alpha * (r - r0))) ** 2 - 1)
    A = np.array([[max(rk - x, 0.0) ** 3 for rk in knots] for x in r])
    amp, *_ = np.linalg.lstsq(A, tgt, rcond=None)
    return amp


def main():
    os.makedirs(OUT, exist_ok=True)

    # ---- Fe, bcc, Finnis-Sinclair form: 6 pair knots on [2.2, 4.1], density
    # knots {3.0, 3.6}, F = -sqrt(rho).
    fe_knots = [round(float(v), 10) for v in np.linspace(2.2, 4.1, 6)]
    fe_A, fe_R = [1.0, 2.2], [3.0, 3.6]
    fe_amp, fe_obs = fit_single(
        "bcc", 2.87, fe_knots, fe_A, fe_R, 55.845,
        targets=[-4.28, 0.0, 170.0, 49.0, 116.0], soft_weight=0.05, smooth=0.2, r_lo=2.2,
        core_r=1.8, core_val=5.0,
    )
    fe = {
        "name": "fe_fs",
        "note": "synthetic bcc Fe Finnis-Sinclair table (cubic-knot form); fitted by oracle/fit_tables.py",
        "fit": dict(zip(["E_atom_eV", "P_GPa", "B_GPa", "Cprime_GPa", "C44_GPa"], map(float, fe_obs))),
        "species": ["Fe"],
        "mass": [55.845],
        "emb_c": [1.0],
        "pair": {"Fe-Fe": {"r": fe_knots, "a": list(map(float, fe_amp))}},
        "density": {"Fe<-Fe": {"R": fe_R, "A": fe_A}},
    }

    # ---- Fe with 15 splines in all (the intermediate-complexity iron potential
    # of the lookup-table benchmark, "Parallel benchmarks"): 13 pair knots on
    # [2.3, 4.1] every 0.15 A and the two density knots above; the same targets.
    # Thirteen knots 0.15 A apart admit large terms of opposite sign (amplitudes
    # up to 45 with the curvature penalty alone, and a first-shell pair force
    # 1/100 of its pair-potential part); the amplitude penalty keeps them below
    # 7 at the same elastic constants.
    fe15_knots = [round(float(v), 10) for v in np.linspace(2.3, 4.1, 13)]
    fe15_amp, fe15_obs = fit_single(
        "bcc", 2.87, fe15_knots, fe_A, fe_R, 55.845,
        targets=[-4.28, 0.0, 170.0, 49.0, 116.0], soft_weight=0.05, smooth=0.2, r_lo=2.2,
        core_r=1.8, core_val=5.0, ridge=1.0,
    )
    fe15 = {
        "name": "fe15_fs",
        "note": "synthetic bcc Fe Finnis-Sinclair table with 13 pair and 2 density knots (15 cubic "
                "splines); fitted by oracle/fit_tables.py",
        "fit": dict(zip(["E_atom_eV", "P_GPa", "B_GPa", "Cprime_GPa", "C44_GPa"], map(float, fe15_obs))),
        "species": ["Fe"],
        "mass": [55.845],
        "emb_c": [1.0],
        "pair": {"Fe-Fe": {"r": fe15_knots, "a": list(map(float, fe15_amp))}},
        "density": {"Fe<-Fe": {"R": fe_R, "A": fe_A}},
    }

    # ---- Cu, fcc: 6 pair knots on [2.0, 5.0], density knots {3.5, 4.3}.
    cu_knots = [round(float(v), 10) for v in np.linspace(2.0, 5.0, 6)]
    cu_A, cu_R = [0.3, 0.25], [3.5, 4.3]
    cu_amp, cu_obs = fit_single(
        "fcc", 3.615, cu_knots, cu_A, cu_R, 63.546,
        targets=[-3.54, 0.0, 138.0, 23.5, 75.4], soft_weight=0.3, smooth=0.2, r_lo=2.2,
        core_r=1.7, core_val=5.0,
    )
    cu = {
        "name": "cu_fs",
        "note": "synthetic fcc Cu-like Finnis-Sinclair table (cubic-knot form); fitted by oracle/fit_tables.py",
        "fit": dict(zip(["E_atom_eV", "P_GPa", "B_GPa", "Cprime_GPa", "C44_GPa"], map(float, cu_obs))),
        "species": ["Cu"],
        "mass": [63.546],
        "emb_c": [1.0],
        "pair": {"Cu-Cu": {"r": cu_knots, "a": list(map(float, cu_amp))}},
        "density": {"Cu<-Cu": {"R": cu_R, "A": cu_A}},
    }

    # ---- Fe-C, EAM semantics (density depends on the neighbour's species).
    # Fe-Fe pair and Fe density as above; Fe-C and C-C pairs are least-squares
    # fits of Morse curves in cubic-knot form on [1.6, 4.1]; the carbon density
    # has knots {2.5, 3.3}.
    fc_knots = [round(float(v), 10) for v in np.linspace(1.6, 4.1, 6)]
    fec_amp = _morse_fit(fc_knots, D=0.6, r0=1.85, alpha=2.2, rlo=1.2)
    cc_amp = _morse_fit(fc_knots, D=0.1, r0=2.6, alpha=2.0, rlo=1.2)
    fec = {
        "name": "fec_eam",
        "note": "synthetic two-species Fe-C EAM table (cubic-knot form); Fe-Fe from fe_fs",
        "species": ["Fe", "C"],
        "mass": [55.845, 12.011],
        "emb_c": [1.0, 1.0],
        "pair": {
            "Fe-Fe": {"r": fe_knots, "a": list(map(float, fe_amp))},
            "Fe-C": {"r": fc_knots, "a": list(map(float, fec_amp))},
            "C-C": {"r": fc_knots, "a": list(map(float, cc_amp))},
        },
        "density": {
            "Fe<-Fe": {"R": fe_R, "A": fe_A},
            "C<-Fe": {"R": fe_R, "A": fe_A},
            "Fe<-C": {"R": [2.5, 3.3], "A": [2.0, 0.6]},
            "C<-C": {"R": [2.5, 3.3], "A": [2.0, 0.6]},
        },
    }
    for tab in (fe, fe15, cu, fec):
        with open(os.path.join(OUT, tab["name"] + ".json"), "w") as fh:
            json.dump(tab, fh, indent=1)
        print(tab["name"], tab.get("fit"))


if __name__ == "__main__":
    main()
