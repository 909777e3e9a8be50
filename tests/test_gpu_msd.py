"""GPU parity of the mean square displacement per replica and species
(paper, "Self-diffusion in iron"; unwrapped positions, "Boundary
conditions") against the oracle's plain average."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _with_empty_replica(s):
    """s with an empty replica inserted after its first one."""
    off = np.concatenate([s.atom_offset[:2], s.atom_offset[1:]])
    ins = lambda a: np.concatenate([a[:1], a[:1], a[1:]])  # noqa: E731
    return inputs.System(
        name=s.name + "+empty", pos=s.pos, vel=s.vel, species=s.species, rigid=s.rigid, atom_offset=off,
        box=ins(s.box), origin=ins(s.origin), periodic=ins(s.periodic), rigid_velocity=ins(s.rigid_velocity),
        potential=s.potential, dt_fs=s.dt_fs, skin=s.skin, rebuild_every=s.rebuild_every, steps=0,
        temperature=ins(s.temperature), max_neighbours=s.max_neighbours,
    )


def test_msd_of_caller_positions(md, orc):
    """Seeded displacements written into the state arrays (several box lengths
    on some atoms, a separate spread for carbon) against the oracle, in a
    batch with an empty replica; counts exact."""
    s = _with_empty_replica(inputs.fec_replicas(3, nmin=1500, nmax=5000, seed0=4700))
    announce("msd of caller positions, fec x3 + empty")
    sim = md.Simulation(s)
    rng = np.random.default_rng(11)
    disp = rng.normal(0.0, 0.7, s.pos.shape)
    disp[s.species == 1] *= 3.0
    jump = rng.integers(-3, 4, s.pos.shape) * (rng.random(s.pos.shape) < 0.05)
    box_of_atom = np.repeat(s.box, np.diff(s.atom_offset), axis=0)
    new = s.pos + disp + jump * box_of_atom
    sim.set_state(pos=new)
    m, c = sim.msd()
    m_ref, c_ref = orc.msd(new, s.pos, s.species, s.atom_offset, 2)
    assert np.array_equal(c, c_ref)
    assert c[1].sum() == 0 and np.all(m[1] == 0.0)
    np.testing.assert_allclose(m, m_ref, rtol=1e-13, atol=0)
    sim.msd_origin()
    m0, _ = sim.msd()
    assert np.all(m0 == 0.0)


def test_msd_after_trajectory(md, orc):
    """100 FP64 steps of four Fe-C replicas: the MSD of the library's
    trajectory against the MSD of the oracle's, replica by replica."""
    s = inputs.fec_replicas(4, nmin=250, nmax=1200, seed0=4800)
    announce("msd after 100 steps, fec x4")
    sim = md.Simulation(s)
    sim.step(100)
    m, c = sim.msd()
    for r in range(s.n_replicas):
        sub = s.replica(r)
        ref = orc.run_verlet(sub.pos, sub.vel, sub.species, sub.box[0], sub.periodic[0],
                             orc.Potential(sub.potential), sub.dt_fs, 100)
        m_ref, c_ref = orc.msd(ref.pos, sub.pos, sub.species, sub.atom_offset, 2)
        assert np.array_equal(c[r], c_ref[0])
        np.testing.assert_allclose(m[r], m_ref[0], rtol=1e-7, atol=1e-12)
        assert m[r, 0] > 1e-3


def test_msd_ballistic_gas_across_boundaries(md):
    """Atoms farther apart than the cutoff, all moving at one velocity,
    cross the periodic box twice over 8000 steps: the library's unwrapped
    positions give MSD = |v|^2 t^2."""
    g = np.arange(4) * 7.0 + 1.0
    pos = np.array([[x, y, z] for x in g for y in g for z in g])
    v = np.array([0.008, -0.005, 0.004])
    base = inputs.workload("bcc2000")
    n = len(pos)
    s = inputs.System(
        name="ballistic", pos=pos, vel=np.tile(v, (n, 1)), species=np.zeros(n, np.uint8),
        rigid=np.zeros(n, np.uint8), atom_offset=np.array([0, n], np.int64), box=np.array([[28.0] * 3]),
        origin=np.zeros((1, 3)), periodic=np.ones((1, 3), np.uint8), rigid_velocity=np.zeros((1, 3)),
        potential=base.potential, dt_fs=1.0, skin=0.3, rebuild_every=10, steps=0, temperature=np.zeros(1),
        max_neighbours=16,
    )
    announce("msd ballistic gas, 8000 steps")
    sim = md.Simulation(s)
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    sim.step(8000)
    m, c = sim.msd()
    assert c[0, 0] == n
    assert np.max(np.abs(sim.positions() - pos)) > 2 * 28.0
    assert m[0, 0] == pytest.approx((v @ v) * 8000.0**2, rel=1e-11)


def test_msd_rigid_atoms_left_out(md, orc):
    """The moving piston's atoms are not averaged: the MSD of the mobile atoms
    after 60 steps against the oracle's piston trajectory."""
    s = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, piston_speed_a_per_fs=0.02, steps=0)
    announce("msd piston")
    sim = md.Simulation(s)
    sim.step(60)
    m, c = sim.msd()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 60,
                         rigid=s.rigid, rigid_velocity=s.rigid_velocity[0])
    m_ref, c_ref = orc.msd(ref.pos, s.pos, s.species, s.atom_offset, 1, rigid=s.rigid)
    assert c[0, 0] == c_ref[0, 0] == int((s.rigid == 0).sum())
    np.testing.assert_allclose(m, m_ref, rtol=1e-7, atol=1e-12)


def test_msd_batched_equals_one_by_one(md):
    """A replica's MSD in a batch is bitwise its MSD alone (fixed-order sums)."""
    s = inputs.fec_replicas(3, nmin=300, nmax=20000, seed0=4900)
    announce("msd batched vs one-by-one")
    sim = md.Simulation(s)
    sim.step(20)
    m, _ = sim.msd()
    for r in range(s.n_replicas):
        one = md.Simulation(s.replica(r))
        one.step(20)
        m1, _ = one.msd()
        assert np.array_equal(m1[0], m[r])


def test_msd_vacancy_workload_nvt(md, orc):
    """The self-diffusion workload at its replica shape (1999-atom bcc Fe with
    a vacancy) under the thermostat at 900 and 2000 K: per-replica MSD after
    100 FP64 steps against the oracle's NVT trajectory."""
    s = inputs.vacancy_replicas(temperatures=(900, 2000), per_temperature=1)
    kb = 8.617333262e-5
    q = np.array([(3 * 1999 - 3) * kb * t * 100.0**2 for t in s.temperature])
    announce("msd vacancy workload nvt")
    sim = md.Simulation(s, nh_temperature=s.temperature, nh_mass=q)
    sim.step(100)
    m, _ = sim.msd()
    for r in range(s.n_replicas):
        sub = s.replica(r)
        ref = orc.run_nh(sub.pos, sub.vel, sub.species, sub.box[0], sub.periodic[0], orc.Potential(sub.potential),
                         sub.dt_fs, 100, float(s.temperature[r]), float(q[r]))
        m_ref, _ = orc.msd(ref.pos, sub.pos, sub.species, sub.atom_offset, 1)
        np.testing.assert_allclose(m[r], m_ref[0], rtol=1e-7, atol=1e-12)
    assert m[1, 0] > m[0, 0]
