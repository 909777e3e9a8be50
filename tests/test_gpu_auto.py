"""GPU tests of the automatic list rebuild (MD_OPT_AUTO_REBUILD; paper, "The
Neighbourlist calculation": a list of r_c + skin stays complete while no atom
moves more than skin/2 from its position at the build).  Hot systems with a
0.2 A skin, where a fixed update period fails the skin guard, against the FP64
oracle's brute-force trajectories; the list's completeness at the current
positions; per-replica rebuilds (a replica in a batch runs bitwise as alone);
graph replay, split calls, the thermostat, Gear, half lists and sheared
cells; and at the benchmark's sizes, where the gated build kernels stride over
more slots and link cells than their capped grids hold, every atom against a
fresh build at the final positions."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import TOL, announce, energy_error, force_error

pytestmark = pytest.mark.gpu

SKIN = 0.2


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _hot(seed=31, temperature=1200.0):
    """2000-atom bcc Fe at 1200 K from the perfect lattice, 0.2 A skin."""
    return inputs.bcc_fe(10, temperature=temperature, seed=seed, skin=SKIN, rebuild_every=1000,
                         name=f"bcc2000_hot{seed}")


def _auto(md, s, **kw):
    sim = md.Simulation(s, **kw)
    sim.set_option(md.MD_OPT_AUTO_REBUILD, 1)
    return sim


_REF = {}


def _verlet(orc, s, nsteps):
    key = (s.name, s.n_atoms, nsteps)
    if key not in _REF:
        _REF[key] = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential),
                                   s.dt_fs, nsteps)
    return _REF[key]


def _check(en, ref, pos, f, precision, n_atoms, r=0):
    dx = np.max(np.abs(pos - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(f, ref.f) < 1e-8
        assert abs(en.pe[r] - ref.pe[-1]) < 1e-10 * abs(ref.pe[-1])
        assert abs(en.ke[r] - ref.ke[-1]) < 1e-8 * abs(ref.ke[-1])
    else:
        assert dx < 1e-4
        assert abs(en.pe[r] + en.ke[r] - ref.pe[-1] - ref.ke[-1]) < 1e-5 * n_atoms


def test_fixed_period_fails_where_auto_holds(md):
    """The control: with the same 0.2 A skin a 50-step update period trips the
    skin guard at its first scheduled build."""
    s = _hot()
    sim = md.Simulation(s, rebuild_every=50)
    sim.step(60)
    with pytest.raises(md.MDError) as e:
        sim.energy()
    assert e.value.code == md.MD_ERR_SKIN


@pytest.mark.parametrize("precision,mode", [("fp64", "full"), ("mixed", "full"), ("fp64", "half")])
def test_auto_rebuild_trajectory(md, orc, precision, mode):
    """100 velocity-Verlet steps at 1200 K with a 0.2 A skin against the
    oracle's brute-force trajectory (FP64: positions within 1e-8 A); the check
    triggers several rebuilds and never a skin error."""
    s = _hot()
    announce(f"auto rebuild trajectory {precision} {mode}")
    sim = _auto(md, s, precision=precision, nbr_mode=mode)
    sim.step(100)
    en = sim.energy()
    builds = sim.get_option(md.MD_OPT_N_BUILDS)
    assert 5 <= builds <= 60, builds
    _check(en, _verlet(orc, s, 100), sim.positions(), sim.forces(), precision, s.n_atoms)
    assert en.step == 100


def _pairs_within(pos, box, r):
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.rint(d / box)
    r2 = np.einsum("ijk,ijk->ij", d, d)
    np.fill_diagonal(r2, np.inf)
    i, j = np.nonzero(r2 < r * r)
    return set(zip(i.tolist(), j.tolist()))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_auto_rebuild_list_complete(md, orc, precision):
    """After 70 steps the list (read in caller numbering) holds every pair now
    closer than r_c, and only pairs closer than r_c + skin + the two atoms'
    allowed displacements."""
    s = _hot(seed=33)
    announce(f"auto rebuild list completeness {precision}")
    sim = _auto(md, s, precision=precision)
    sim.step(70)
    sim.energy()
    counts, lst = sim.neighbours()
    listed = {(i, int(j)) for i in range(s.n_atoms) for j in lst[i, : counts[i]]}
    rc = orc.cutoff(orc.Potential(s.potential))
    pos = sim.positions()
    assert _pairs_within(pos, s.box[0], rc) <= listed
    assert listed <= _pairs_within(pos, s.box[0], rc + 2 * SKIN)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_auto_rebuild_batched_equals_alone(md, precision):
    """Three Fe-C replicas at 300 to 1200 K: each replica rebuilds on its own
    atoms' displacements, so in the batch it runs bitwise as alone; the hot
    replica rebuilds more often than the cold one."""
    s = inputs.fec_replicas(3, nmin=500, nmax=1200, tmin=300.0, tmax=1200.0, seed0=5200, skin=0.3)
    announce(f"auto rebuild batched {precision}")
    batch = _auto(md, s, precision=precision)
    batch.step(80)
    eb = batch.energy()
    pos, f = batch.positions(), batch.forces()
    builds = []
    for r in range(s.n_replicas):
        one = _auto(md, s.replica(r), precision=precision)
        one.step(80)
        e1 = one.energy()
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        assert np.array_equal(one.positions(), pos[a:b])
        assert np.array_equal(one.forces(), f[a:b])
        assert e1.pe[0] == eb.pe[r] and e1.ke[0] == eb.ke[r]
        builds.append(one.get_option(md.MD_OPT_N_BUILDS))
    assert max(builds) > min(builds), builds
    assert batch.get_option(md.MD_OPT_N_BUILDS) >= max(builds)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_auto_rebuild_graph_equals_eager(md, precision):
    """Graph replay (the check and the gated build kernels captured with every
    step) equals eager execution bit for bit, over calls of 48, 47, 31 and 60
    steps (the second call resumes on a graph boundary, where the check of
    the first step is not yet done)."""
    s = inputs.fec_replicas(2, nmin=400, nmax=900, tmin=900.0, tmax=1200.0, seed0=5300, skin=0.25)
    announce(f"auto rebuild graph {precision}")
    eager = _auto(md, s, precision=precision)
    graph = _auto(md, s, precision=precision)
    graph.set_option(md.MD_OPT_USE_GRAPH, 1)
    for nsteps in (48, 47, 31, 60):
        eager.step(nsteps)
        graph.step(nsteps)
        e1, e2 = eager.energy(), graph.energy()
        assert np.array_equal(eager.positions(), graph.positions())
        assert np.array_equal(eager.velocities(), graph.velocities())
        assert np.array_equal(eager.forces(), graph.forces())
        assert np.array_equal(e1.pe, e2.pe) and np.array_equal(e1.virial, e2.virial)
    assert graph.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 8
    assert graph.get_option(md.MD_OPT_N_BUILDS) == eager.get_option(md.MD_OPT_N_BUILDS) > 3


def test_auto_rebuild_split_calls_and_moved_atoms(md, orc):
    """Calls of 20, 45 and 35 steps equal one 100-step call bit for bit; after
    the caller moves atoms by 0.5 A (md_state_changed) the next evaluation
    rebuilds first and matches the oracle's forces at the new positions."""
    s = _hot(seed=35)
    announce("auto rebuild split calls")
    one = _auto(md, s)
    one.step(100)
    e_one = one.energy()
    split = _auto(md, s)
    for n in (20, 45, 35):
        split.step(n)
    e_split = split.energy()
    assert np.array_equal(split.positions(), one.positions())
    assert np.array_equal(split.forces(), one.forces())
    assert e_split.pe[0] == e_one.pe[0]
    pos = split.positions()
    rng = np.random.default_rng(36)
    moved = rng.choice(s.n_atoms, 40, replace=False)
    pos[moved] += 0.5 * rng.standard_normal((40, 3)) / np.sqrt(3)
    split.set_state(pos=pos)
    split.eam_forces(True)
    en = split.energy()
    ref = orc.forces(pos, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential))
    assert force_error(split.forces(), ref.f) < 1e-10
    assert abs(en.pe[0] - ref.pe) < 1e-12 * abs(ref.pe)


def test_auto_rebuild_thermostat_and_gear(md, orc):
    """The Nose-Hoover and Gear integrators with automatic rebuilds (Gear's
    check on the predicted positions) against the oracle's runs."""
    s = _hot(seed=37)
    announce("auto rebuild nvt and gear")
    kb = 8.617333262e-5
    q = (3 * s.n_atoms - 3) * kb * 900.0 * 50.0**2
    nvt = _auto(md, s, nh_temperature=[900.0], nh_mass=[q])
    nvt.step(60)
    en = nvt.energy()
    ref = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 60,
                     900.0, q)
    assert nvt.get_option(md.MD_OPT_N_BUILDS) >= 3
    assert np.max(np.abs(nvt.positions() - ref.pos)) < 1e-8
    assert abs(en.nh_pi[0] - ref.pi[-1]) <= 1e-8 * abs(ref.pi[-1]) + 1e-14
    gear = _auto(md, s, integrator="gear3")
    gear.step(60)
    en = gear.energy()
    ref = orc.run_gear(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 60)
    assert gear.get_option(md.MD_OPT_N_BUILDS) >= 3
    assert np.max(np.abs(gear.positions() - ref.pos)) < 1e-8
    assert force_error(gear.forces(), ref.f) < 1e-8
    assert abs(en.pe[0] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_auto_rebuild_sheared_cell(md, orc, precision):
    """A hot crystal in a sheared cell (atoms re-wrapped across slanted faces
    by the gated builds) against the oracle's run with the cell held."""
    s = inputs.bcc_fe(7, temperature=1200.0, seed=39, displace=0.06, skin=SKIN, rebuild_every=1000,
                      name="strained_hot")
    strain = np.array([[1.0, 0.04, -0.03], [0.02, 0.99, 0.05], [-0.04, 0.03, 1.01]])
    h = strain @ np.diag(s.box[0])
    s.pos = s.pos @ strain.T
    announce(f"auto rebuild sheared cell {precision}")
    sim = _auto(md, s, precision=precision, box_matrix=h)
    sim.step(80)
    en = sim.energy()
    ref = orc.run_prt(s.pos, s.vel, s.species, h, orc.Potential(s.potential), s.dt_fs, 80, 0.0, 0.0,
                      origin=s.origin[0])
    assert sim.get_option(md.MD_OPT_N_BUILDS) >= 3
    _check(en, ref, sim.positions(), sim.forces(), precision, s.n_atoms)


def test_auto_rebuild_piston_free_axis(md, orc):
    """A rigid piston driven at 0.02 A/fs into a slab with a free z axis: the
    moving rigid atoms trigger the rebuilds; trajectory and piston work against
    the oracle."""
    s = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, piston_speed_a_per_fs=0.02, steps=0)
    s.skin = SKIN
    announce("auto rebuild piston")
    sim = _auto(md, s)
    sim.step(60)
    en = sim.energy()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 60,
                         rigid=s.rigid, rigid_velocity=s.rigid_velocity[0])
    assert sim.get_option(md.MD_OPT_N_BUILDS) >= 5  # 0.6 A of piston travel (dt 0.5 fs) over a 0.1 A guard
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert en.piston_work[0] == pytest.approx(ref.work[-1], rel=1e-8, abs=1e-10)


def test_auto_rebuild_thermostatted_batch(md, orc):
    """Per-replica Nose-Hoover thermostats on a batch with per-replica rebuilds:
    each replica against the oracle's NVT run, and bitwise as alone."""
    s = inputs.fec_replicas(2, nmin=300, nmax=700, tmin=600.0, tmax=1200.0, seed0=5400, skin=0.3)
    kb = 8.617333262e-5
    targets = [800.0, 1000.0]
    q = []
    for r in range(s.n_replicas):
        n = int(s.atom_offset[r + 1] - s.atom_offset[r])
        q.append((3 * n - 3) * kb * targets[r] * 50.0**2)
    announce("auto rebuild thermostatted batch")
    batch = _auto(md, s, nh_temperature=targets, nh_mass=q)
    batch.step(50)
    eb = batch.energy()
    pos = batch.positions()
    for r in range(s.n_replicas):
        sub = s.replica(r)
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        ref = orc.run_nh(sub.pos, sub.vel, sub.species, sub.box[0], sub.periodic[0], orc.Potential(sub.potential),
                         sub.dt_fs, 50, targets[r], q[r])
        assert np.max(np.abs(pos[a:b] - ref.pos)) < 1e-8
        assert abs(eb.nh_pi[r] - ref.pi[-1]) <= 1e-8 * abs(ref.pi[-1]) + 1e-14
        one = _auto(md, sub, nh_temperature=targets[r:r + 1], nh_mass=q[r:r + 1])
        one.step(50)
        one.energy()
        assert np.array_equal(one.positions(), pos[a:b])


def _fresh_fp64(md, s, pos, vel, **kw):
    """Forces and per-atom energies of a new FP64 context on the given state:
    its list, link cells and slot order come from these positions alone
    (the scheduled build, no automatic rebuild)."""
    import copy

    t = copy.copy(s)
    t.pos, t.vel = pos, vel
    sim = md.Simulation(t, precision="fp64", **kw)
    sim.eam_forces(want_energy=True)
    return sim.forces(), sim.atom_energies()


@pytest.mark.parametrize("precision,variant", [("fp64", "full"), ("mixed", "full"), ("fp64", "half"),
                                               ("mixed", "sheared")])
def test_auto_rebuild_full_size_crystal(md, orc, precision, variant):
    """The benchmark crystal (80^3 bcc cells, 1% vacancies, 1,013,760 atoms,
    ~130k link cells) at 1200 K with a 0.2 A skin and graph replay; the full
    list, the half list with atomics, and a sheared cell (the looping list
    kernel with edge-vector shifts): after 40 steps every atom's force and
    energy match a fresh FP64 build at the final positions to the contract,
    and sampled atoms match the oracle."""
    s = inputs.bcc_fe(80, temperature=1200.0, vacancy_frac=0.01, seed=2, skin=SKIN, rebuild_every=1000,
                      name="bcc1m_hot")
    kw, ref_kw = {}, {}
    if variant == "half":
        kw["nbr_mode"] = "half"
    if variant == "sheared":
        strain = np.array([[1.0, 0.03, -0.02], [0.01, 0.99, 0.04], [-0.03, 0.02, 1.01]])
        h = strain @ np.diag(s.box[0])
        s.pos = s.pos @ strain.T
        kw["box_matrix"] = ref_kw["box_matrix"] = h
    announce(f"auto rebuild bcc1m at 1200 K {precision} {variant}")
    sim = _auto(md, s, precision=precision, **kw)
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    sim.step(40)
    sim.energy()
    builds = sim.get_option(md.MD_OPT_N_BUILDS)
    pos, f, e = sim.positions(), sim.forces(), sim.atom_energies()
    f_ref, e_ref = _fresh_fp64(md, s, pos, sim.velocities(), **ref_kw)
    tol = TOL[precision]
    ferr, eerr = force_error(f, f_ref), energy_error(e, e_ref)
    sample = np.random.default_rng(4).choice(s.n_atoms, 16, replace=False)
    pot = orc.Potential(s.potential)
    if variant == "sheared":
        ref = orc.forces_sampled_tri(pos, s.species, kw["box_matrix"], pot, sample)
    else:
        ref = orc.forces_sampled(pos, s.species, s.box[0], s.periodic[0], pot, sample)
    rms = np.sqrt(np.mean(np.sum(f_ref**2, 1)))
    oerr = np.max(np.linalg.norm(f[sample] - ref.f, axis=1)) / rms
    announce(f"  {builds} builds, force err {ferr:.2e}, energy err {eerr:.2e}, oracle sample {oerr:.2e}")
    assert builds >= 4
    assert ferr <= tol["force"] and eerr <= tol["energy"]
    assert oerr <= tol["force"]


def test_auto_rebuild_full_size_batch(md):
    """The Fe-C batch (256 replicas, 2.1 M atoms) in mixed precision with a
    0.4 A skin and graph replay, as the benchmark's automatic-rebuild leg
    runs it: the hot replicas rebuild on their own, and after 20 steps every
    atom matches a fresh FP64 build at the final positions."""
    s = inputs.workload("fec256", skin=0.4)
    announce("auto rebuild fec256 mixed")
    sim = _auto(md, s, precision="mixed")
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    sim.step(20)
    sim.energy()
    builds = sim.get_option(md.MD_OPT_N_BUILDS)
    f, e = sim.forces(), sim.atom_energies()
    f_ref, e_ref = _fresh_fp64(md, s, sim.positions(), sim.velocities())
    ferr, eerr = force_error(f, f_ref), energy_error(e, e_ref)
    announce(f"  {builds} builds, force err {ferr:.2e}, energy err {eerr:.2e}")
    assert builds >= 3
    assert ferr <= TOL["mixed"]["force"] and eerr <= TOL["mixed"]["energy"]


def test_auto_rebuild_wide_list(md):
    """The looping list kernel with 64-bit list addresses: a list allocation
    above 4 GiB (128,000 atoms with room for 8,400 entries each, ~17,000 link
    cells) agrees bit for bit with the default capacity over 30 graph-replayed
    steps with automatic rebuilds at 1200 K."""
    s = inputs.bcc_fe(40, temperature=1200.0, seed=44, skin=SKIN, rebuild_every=1000, name="bcc_wide_hot")
    assert s.n_atoms * 16 * ((8400 + 7) // 4) >= 1 << 32
    announce("auto rebuild, list above 4 GiB")
    out = []
    for cap in (48, 8400):
        sim = _auto(md, s, max_neighbours=cap)
        sim.set_option(md.MD_OPT_USE_GRAPH, 1)
        sim.step(30)
        e = sim.energy()
        out.append((sim.positions(), sim.forces(), e.pe, sim.get_option(md.MD_OPT_N_BUILDS)))
        del sim
    assert out[0][3] == out[1][3] >= 3
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)


def test_auto_rebuild_full_size_gear(md):
    """Gear's predictor-corrector state (acceleration and its derivative)
    carried through the looping rebuilds of the 1,013,760-atom crystal at
    1200 K: 40 graph-replayed steps with automatic rebuilds against the same
    run rebuilt at every step (the two differ only in summation order)."""
    import copy

    s = inputs.bcc_fe(80, temperature=1200.0, vacancy_frac=0.01, seed=2, skin=SKIN, rebuild_every=1000,
                      name="bcc1m_hot")
    announce("auto rebuild bcc1m at 1200 K, Gear")
    auto = _auto(md, s, integrator="gear3")
    auto.set_option(md.MD_OPT_USE_GRAPH, 1)
    auto.step(40)
    auto.energy()
    t = copy.copy(s)
    t.rebuild_every = 1
    every = md.Simulation(t, integrator="gear3")
    every.set_option(md.MD_OPT_USE_GRAPH, 1)
    every.step(40)
    every.energy()
    builds = auto.get_option(md.MD_OPT_N_BUILDS)
    dx = np.max(np.abs(auto.positions() - every.positions()))
    ferr = force_error(auto.forces(), every.forces())
    announce(f"  {builds} builds, position diff {dx:.2e} A, force diff {ferr:.2e}")
    assert 4 <= builds < every.get_option(md.MD_OPT_N_BUILDS)
    assert dx < 1e-9 and ferr < 1e-9


@pytest.mark.parametrize("use_graph", [0, 1])
def test_auto_rebuild_energy_ring(md, orc, use_graph):
    """Energies of every step (MD_OPT_ENERGY_EVERY = 1) with automatic
    rebuilds, over 100 steps in calls of 7, 61 and 32, eager and
    graph-replayed: each entry carries its step index and matches the
    oracle's potential and kinetic energy of that step."""
    s = _hot(seed=41)
    announce(f"auto rebuild energy ring graph={use_graph}")
    sim = _auto(md, s, precision="fp64", energy_ring=128)
    sim.set_option(md.MD_OPT_ENERGY_EVERY, 1)
    sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    hist = []
    for n in (7, 61, 32):
        sim.step(n)
        hist += sim.energy_history()
    ref = _verlet(orc, s, 100)
    assert [h.step for h in hist] == list(range(1, 101))
    pe = np.array([h.pe[0] for h in hist])
    ke = np.array([h.ke[0] for h in hist])
    assert np.max(np.abs(pe - ref.pe[1:]) / np.abs(ref.pe[1:])) < 1e-11
    assert np.max(np.abs(ke - ref.ke[1:]) / np.abs(ref.ke[1:])) < 1e-11
    sim.energy()  # (automatic builds are counted as of the last md_energy)
    assert sim.get_option(md.MD_OPT_N_BUILDS) >= 3
