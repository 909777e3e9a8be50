"""GPU parity of the LDS-brick pair kernels (MD_OPT_KERNEL = 2): brick lists
that keep each pair of two own atoms once, the other atom's share summed in
64-bit fixed point in LDS, against the FP64 oracle.  Same tolerances as the
other parity tests; the fixed-point sums are order independent, so graph replay
and batched runs are compared bitwise."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import announce, force_error
from tests.test_gpu_parity import _check_snapshot

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dims,lanes,block", [(0, 1, 1024), (444, 2, 1024), (222, 1, 512), (432, 2, 512),
                                              (111, 1, 256)])
def test_pair_bricks_snapshot(md, orc, precision, dims, lanes, block):
    """Displaced bcc with vacancies: forces, per-atom energies and the virial
    for brick shapes from one cell to 4 x 4 x 4, one or two lanes per atom."""
    s = inputs.bcc_fe(12, temperature=600.0, seed=91, vacancy_frac=0.01, displace=0.07, name="bcc_pairs")
    sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 2, md.MD_OPT_BRICK_DIMS: dims,
                                                          md.MD_OPT_LANES_PER_ATOM: lanes,
                                                          md.MD_OPT_BRICK_BLOCK: block})
    assert sim.get_option(md.MD_OPT_KERNEL) == 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_bricks_two_species_and_rigid(md, orc, precision):
    """Two species with distinct embedding constants (the other atom's density
    share uses its own density function), and a free-axis slab with rigid atoms
    (rigid pairs stay out of the virial)."""
    s = inputs.fec_replicas(3, nmin=600, nmax=1500, seed0=4750)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(75).random(s.pos.shape) - 1)
    pot = dict(s.potential)
    pot["emb_c"] = np.array([1.0, 0.7])
    s.potential = pot
    _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 2})
    s3 = inputs.fcc_piston(nx=5, ny=5, nz=8, piston_cells=2, steps=0)
    s3.pos = s3.pos + 0.03 * (2 * np.random.default_rng(76).random(s3.pos.shape) - 1)
    _check_snapshot(md, orc, s3, precision, options={md.MD_OPT_KERNEL: 2})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_bricks_fallbacks(md, orc, precision):
    """Bricks whose halo exceeds the staging area, or with more own atoms than
    one round of lanes, keep full rows and run as the full-list bricks: same
    results."""
    s = inputs.fec_replicas(2, nmin=800, nmax=1500, seed0=4650)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(65).random(s.pos.shape) - 1)
    sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 2, md.MD_OPT_HALO_CAP: 64})
    assert sim.get_option(md.MD_OPT_HALO_OVERFLOWS) > 0
    _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 2, md.MD_OPT_BRICK_DIMS: 444,
                                                    md.MD_OPT_BRICK_BLOCK: 64})


def test_pair_list_holds_each_inner_pair_once(md):
    """The pair list together with the pairs' mirror images is the full list."""
    s = inputs.bcc_fe(9, temperature=600.0, seed=92, displace=0.08)
    full = md.Simulation(s)
    full.set_option(md.MD_OPT_KERNEL, 0)
    full.build_neighbours()
    cf, lf = full.neighbours()
    pairs = md.Simulation(s)
    pairs.set_option(md.MD_OPT_KERNEL, 2)
    pairs.build_neighbours()
    cp, lp = pairs.neighbours()
    full_set = {(i, int(j)) for i in range(s.n_atoms) for j in lf[i, : cf[i]]}
    listed = [(i, int(j)) for i in range(s.n_atoms) for j in lp[i, : cp[i]]]
    assert len(set(listed)) == len(listed)
    both = set(listed) | {(j, i) for i, j in listed}
    assert both == full_set
    assert int(cp.sum()) < 0.9 * int(cf.sum())  # inner pairs once (small bricks here)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_bricks_trajectory(md, orc, precision):
    """100 velocity-Verlet steps with rebuilds every 10 against the oracle's
    trajectory (FP64 positions within 1e-8 A)."""
    s = inputs.workload("bcc2000")
    announce(f"pair bricks trajectory {precision}")
    sim = md.Simulation(s, precision=precision)
    sim.set_option(md.MD_OPT_KERNEL, 2)
    sim.step(100)
    en = sim.energy()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 100)
    dx = np.max(np.abs(sim.positions() - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(sim.forces(), ref.f) < 1e-8
        assert abs(en.pe[0] - ref.pe[-1]) < 1e-10 * abs(ref.pe[-1])
    else:
        assert dx < 1e-4
        assert abs(en.pe[0] + en.ke[0] - ref.pe[-1] - ref.ke[-1]) < 1e-5 * s.n_atoms


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_bricks_bitwise_reproducible(md, precision):
    """The fixed-point shares make the sums order independent: graph replay
    equals eager execution, and a replica in a batch equals the same replica
    alone, bit for bit."""
    s = inputs.fec_replicas(3, nmin=300, nmax=900, seed0=4950)
    eager = md.Simulation(s, precision=precision)
    graph = md.Simulation(s, precision=precision)
    for sim in (eager, graph):
        sim.set_option(md.MD_OPT_KERNEL, 2)
    graph.set_option(md.MD_OPT_USE_GRAPH, 1)
    for nsteps in (47, 31, 60):
        eager.step(nsteps)
        graph.step(nsteps)
        e1, e2 = eager.energy(), graph.energy()
        assert np.array_equal(eager.positions(), graph.positions())
        assert np.array_equal(eager.forces(), graph.forces())
        assert np.array_equal(e1.pe, e2.pe) and np.array_equal(e1.virial, e2.virial)
    assert graph.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 2
    pos, f = eager.positions(), eager.forces()
    for r in range(s.n_replicas):
        one = md.Simulation(s.replica(r), precision=precision)
        one.set_option(md.MD_OPT_KERNEL, 2)
        one.step(138)
        one.energy()
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        assert np.array_equal(one.positions(), pos[a:b])
        assert np.array_equal(one.forces(), f[a:b])
