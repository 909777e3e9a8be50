"""GPU parity for the 15-spline iron potential (13 pair + 2 density knots), the
intermediate-complexity potential of the paper's lookup-table benchmark
("Parallel benchmarks"), against the FP64 CPU oracle.

Every evaluator and kernel family that can run it is compared element by
element on a displaced bcc crystal: the exact tables, the term-by-term knot
sums (16 + 4 knot variant, FP64 only) in the global-gather and the LDS-brick
kernels, the half list with atomics, and knots moved off every tabulation
grid (tables with split bins, and the knot sums).  Tolerances as in the other
parity tests, for both precisions.
"""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import TOL, force_error
from tests.test_gpu_parity import _check_snapshot, _oracle_snapshot

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _fe15(displace=0.07, seed=31, n=10):
    return inputs.bcc_fe(n, temperature=600.0, seed=seed, displace=displace, potential="fe15_fs",
                         pot_seed=3, name="bcc_fe15")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fe15_tables(md, orc, precision):
    s = _fe15()
    for kernel in (1, 0):
        sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: kernel})
        assert sim.get_option(md.MD_OPT_EVALUATOR) == 0
    _check_snapshot(md, orc, s, precision, nbr_mode="half")


def test_fe15_knot_sums(md, orc):
    """The term-by-term sums, FP64 only; mixed precision refuses them."""
    s = _fe15(seed=32)
    for kernel in (1, 0):
        _check_snapshot(md, orc, s, "fp64", options={md.MD_OPT_KERNEL: kernel, md.MD_OPT_EVALUATOR: 1})
    _check_snapshot(md, orc, s, "fp64", options={md.MD_OPT_EVALUATOR: 1}, nbr_mode="half")
    sim = md.Simulation(s, precision="mixed")
    with pytest.raises(md.MDError) as e:
        sim.set_option(md.MD_OPT_EVALUATOR, 1)
    assert e.value.code == md.MD_ERR_ARG


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fe15_off_grid_knots(md, orc, precision):
    """Pair knots moved by irrational fractions of a bin: no common grid, so
    the tables keep each knot that falls inside a bin as its own term."""
    s = _fe15(seed=33)
    pot = dict(s.potential)
    pot["pair_r"] = pot["pair_r"] + 1e-3 * np.sqrt(2.0) * np.arange(13)
    s.potential = pot
    for kernel in (1, 0):
        sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: kernel})
        assert sim.get_option(md.MD_OPT_EVALUATOR) == 0
    _check_snapshot(md, orc, s, precision, nbr_mode="half")
    if precision == "fp64":
        _check_snapshot(md, orc, s, precision, options={md.MD_OPT_EVALUATOR: 1})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fe15_autotune_then_parity(md, orc, precision):
    s = _fe15(seed=34)
    sim = md.Simulation(s, precision=precision)
    choice = sim.autotune(trials=2)
    if precision == "mixed":
        assert choice["evaluator"] == 0
    sim.eam_forces(want_energy=True)
    ref = _oracle_snapshot(orc, s)
    assert force_error(sim.forces(), ref.f) <= TOL[precision]["force"]


@pytest.mark.parametrize("evaluator", [0, 1])
def test_fe15_trajectory_100_steps(md, orc, evaluator):
    """100 FP64 velocity-Verlet steps with list rebuilds every 10 steps, tables
    and knot sums, against the oracle's brute-force trajectory (positions within
    1e-8 A, as for the 6 + 2 knot potential)."""
    s = inputs.bcc_fe(10, temperature=300.0, seed=35, potential="fe15_fs", pot_seed=3, skin=0.4,
                      name="bcc_fe15_nve")
    sim = md.Simulation(s, precision="fp64")
    sim.set_option(md.MD_OPT_EVALUATOR, evaluator)
    sim.step(100)
    en = sim.energy()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 100)
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert force_error(sim.forces(), ref.f) < 1e-8
    assert abs(en.pe[0] - ref.pe[-1]) < 1e-10 * abs(ref.pe[-1])
    assert en.step == 100
