"""GPU parity of the third-order Gear predictor-corrector (paper, "Time
integration") against the oracle's Gear integrator: trajectories, forces and
energies of the global, LDS-brick and half-list kernels, batches, graph replay,
split calls and rigid atoms."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import announce, force_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


_REF = {}


def _oracle(orc, s, r, nsteps):
    key = (s.name, s.n_atoms, r, nsteps)
    if key not in _REF:
        sub = s.replica(r) if s.n_replicas > 1 else s
        rigid = bool(sub.rigid.any())
        _REF[key] = orc.run_gear(sub.pos, sub.vel, sub.species, sub.box[0], sub.periodic[0],
                                 orc.Potential(sub.potential), sub.dt_fs, nsteps,
                                 rigid=sub.rigid if rigid else None,
                                 rigid_velocity=sub.rigid_velocity[0] if rigid else None)
    return _REF[key]


def _check(en, r, ref, pos, f, precision):
    dx = np.max(np.abs(pos - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(f, ref.f) < 1e-8
        assert abs(en.pe[r] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])
        assert abs(en.ke[r] - ref.ke[-1]) <= 1e-8 * abs(ref.ke[-1]) + 1e-12
    else:
        assert dx < 1e-4
        assert abs(en.pe[r] + en.ke[r] - ref.pe[-1] - ref.ke[-1]) < 1e-5 * len(pos)


@pytest.mark.parametrize("precision,mode,kernel", [
    ("fp64", "full", 1), ("mixed", "full", 1), ("fp64", "half", 1), ("fp64", "full", 0), ("mixed", "full", 0),
])
def test_gear_trajectory_100_steps(md, orc, precision, mode, kernel):
    """bcc Fe, 2000 atoms, 100 Gear steps with list rebuilds every 10 (at the
    predicted positions) against the oracle."""
    s = inputs.workload("bcc2000")
    announce(f"gear trajectory bcc2000 {precision} {mode} kernel {kernel}")
    sim = md.Simulation(s, precision=precision, nbr_mode=mode, integrator="gear3")
    sim.set_option(md.MD_OPT_KERNEL, kernel)
    sim.step(100)
    en = sim.energy()
    ref = _oracle(orc, s, 0, 100)
    _check(en, 0, ref, sim.positions(), sim.forces(), precision)
    assert en.step == 100


def test_gear_split_calls_equal_one_call(md):
    """md_step(40) and md_step(1) + md_step(13) + md_step(26) agree: the Gear
    derivatives carry over between calls."""
    s = inputs.workload("bcc2000")
    announce("gear split calls")
    a = md.Simulation(s, integrator="gear3")
    a.step(40)
    b = md.Simulation(s, integrator="gear3")
    for n in (1, 13, 26):
        b.step(n)
    np.testing.assert_allclose(b.positions(), a.positions(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(b.velocities(), a.velocities(), rtol=0, atol=1e-13)
    assert b.energy().pe[0] == pytest.approx(a.energy().pe[0], rel=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gear_graph_replay_matches_eager(md, precision):
    """Gear steps replayed from HIP graphs equal the eager steps bitwise."""
    s = inputs.fec_replicas(3, nmin=600, nmax=2000, seed0=5500)
    announce(f"gear graph replay {precision}")
    out = []
    for use_graph in (0, 1):
        sim = md.Simulation(s, precision=precision, integrator="gear3")
        sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
        sim.step(60)
        out.append((sim.positions(), sim.velocities(), sim.forces()))
        if use_graph:
            assert sim.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 2
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_gear_batched_against_oracle_and_alone(md, orc):
    """Four Fe-C replicas: each against its own oracle run, and bitwise equal
    to the same replica run alone."""
    s = inputs.fec_replicas(4, nmin=250, nmax=1200, seed0=5600)
    announce("gear batched fec x4")
    sim = md.Simulation(s, integrator="gear3")
    sim.step(40)
    en = sim.energy()
    pos, f = sim.positions(), sim.forces()
    for r in range(s.n_replicas):
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        _check(en, r, _oracle(orc, s, r, 40), pos[a:b], f[a:b], "fp64")
        one = md.Simulation(s.replica(r), integrator="gear3")
        one.step(40)
        assert np.array_equal(one.positions(), pos[a:b])
        assert one.energy().pe[0] == en.pe[r]


def test_gear_piston_rigid_atoms(md, orc):
    """The rigid moving block under the Gear integrator: trajectory and the
    block's work (trapezoid rule) against the oracle."""
    s = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, piston_speed_a_per_fs=0.02, steps=0)
    announce("gear piston")
    sim = md.Simulation(s, integrator="gear3")
    sim.step(30)
    sim.step(30)
    en = sim.energy()
    ref = _oracle(orc, s, 0, 60)
    np.testing.assert_allclose(sim.positions(), ref.pos, rtol=0, atol=1e-8)
    assert en.piston_work[0] == pytest.approx(ref.work[-1], rel=1e-8, abs=1e-10)


def test_gear_energy_drifts_linearly_on_gpu(md):
    """10^4 FP64 Gear steps of bcc2000: the energy drift is linear (the drift
    rates of the two halves agree), as the paper reports for the
    predictor-corrector, and per atom it stays small."""
    s = inputs.workload("bcc2000")
    announce("gear drift 10k steps")
    sim = md.Simulation(s, integrator="gear3")
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    e = []
    for _ in range(100):
        sim.step(100)
        en = sim.energy()
        e.append(en.pe[0] + en.ke[0])
    e = np.array(e) / s.n_atoms
    t = np.arange(len(e))
    s1, s2 = np.polyfit(t[:50], e[:50], 1)[0], np.polyfit(t[50:], e[50:], 1)[0]
    announce(f"gear drift per 100 steps: {s1:.3e}, {s2:.3e} eV/atom")
    assert abs(s1 - s2) < 0.3 * max(abs(s1), abs(s2))
    assert abs(e[-1] - e[0]) < 1e-3


def test_gear_autotune_between_calls(md, orc):
    """md_autotune between Gear calls re-sorts the atoms; the Gear derivatives
    travel with them and the trajectory still follows the oracle."""
    s = inputs.workload("bcc2000")
    announce("gear autotune between calls")
    sim = md.Simulation(s, integrator="gear3")
    sim.step(20)
    sim.autotune(trials=1)
    sim.step(30)
    _check(sim.energy(), 0, _oracle(orc, s, 0, 50), sim.positions(), sim.forces(), "fp64")
