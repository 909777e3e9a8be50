"""GPU parity of the Parrinello-Rahman barostat on an orthorhombic box (paper,
"Barostat NPTp") against the oracle's NPH integrator: trajectories, box edges
and barostat energy, batches at different pressures, graph replay, split
calls, statistics and the compression limit."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import announce, force_error

pytestmark = pytest.mark.gpu

W_BOX = 2.0e4  # eV fs^2 / A^2: a box period of a few hundred fs at these sizes


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _crystal(cells=6, a=2.84, seed=7):
    # a = 2.84 A sits off this potential's equilibrium, so the box moves; the
    # 0.6 A skin leaves the barostat's guards (0.4 skin per atom, 0.2 skin of
    # strain over the list radius) room at 600 K
    s = inputs.bcc_fe(cells, a=a, temperature=600.0, seed=seed, displace=0.02, skin=0.6, name=f"pr{cells}_{seed}")
    s.max_neighbours = 80  # a compressed box brings the fourth shell inside the list radius
    return s


def _oracle(orc, s, r, nsteps, p_gpa, w):
    sub = s.replica(r) if s.n_replicas > 1 else s
    return orc.run_pr(sub.pos, sub.vel, sub.species, sub.box[0], orc.Potential(sub.potential), sub.dt_fs, nsteps,
                      p_gpa, w, origin=sub.origin[0])


def _check(en, r, ref, pos, f, precision):
    dx = np.max(np.abs(pos - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(f, ref.f) < 1e-8
        assert np.max(np.abs(en.box[r] - ref.box[-1])) < 1e-10 * ref.box[-1].max()
        assert abs(en.pe[r] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])
        assert abs(en.ke[r] - ref.ke[-1]) <= 1e-8 * abs(ref.ke[-1])
        assert abs(en.pr_energy[r] - ref.baro[-1]) <= 1e-9 * abs(ref.baro[-1])
    else:
        assert dx < 1e-4
        assert np.max(np.abs(en.box[r] - ref.box[-1])) < 1e-5
        h_gpu = en.pe[r] + en.ke[r] + en.pr_energy[r]
        h_ref = ref.pe[-1] + ref.ke[-1] + ref.baro[-1]
        assert abs(h_gpu - h_ref) < 1e-5 * len(pos)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pr_trajectory_100_steps(md, orc, precision):
    """432-atom bcc Fe off its equilibrium lattice at zero pressure: 100
    barostatted steps with list rebuilds every 10 against the oracle."""
    s = _crystal()
    announce(f"pr trajectory {precision}")
    sim = md.Simulation(s, precision=precision, pr_pressure_gpa=[0.0], pr_mass=[W_BOX])
    sim.step(100)
    en = sim.energy()
    ref = _oracle(orc, s, 0, 100, 0.0, W_BOX)
    assert np.max(np.abs(ref.box[-1] - s.box[0])) > 1e-3  # the box moved
    _check(en, 0, ref, sim.positions(), sim.forces(), precision)
    assert abs(en.volume[0] - np.prod(ref.box[-1])) < 1e-9 * en.volume[0]


def test_pr_batched_pressures(md, orc):
    """Three replicas of different sizes, each at its own pressure and box
    mass, against the oracle one by one; and bitwise equal to each replica
    alone."""
    parts = [_crystal(cells, seed=11 + k) for k, cells in enumerate((6, 7, 8))]
    pos = np.concatenate([p.pos for p in parts])
    vel = np.concatenate([p.vel for p in parts])
    off = np.concatenate([[0], np.cumsum([p.n_atoms for p in parts])]).astype(np.int64)
    s = inputs.System(
        name="pr_batch", pos=pos, vel=vel, species=np.zeros(len(pos), np.uint8), rigid=np.zeros(len(pos), np.uint8),
        atom_offset=off, box=np.array([p.box[0] for p in parts]), origin=np.zeros((3, 3)),
        periodic=np.ones((3, 3), np.uint8), rigid_velocity=np.zeros((3, 3)), potential=parts[0].potential,
        dt_fs=1.0, skin=0.6, rebuild_every=10, steps=0, temperature=np.full(3, 600.0), max_neighbours=80,
    )
    pressures = np.array([0.0, 2.0, 5.0])
    masses = np.array([0.5, 1.0, 2.0]) * W_BOX
    announce("pr batched pressures")
    sim = md.Simulation(s, pr_pressure_gpa=pressures, pr_mass=masses)
    sim.step(60)
    en = sim.energy()
    p_all, f_all = sim.positions(), sim.forces()
    for r in range(3):
        a, b = int(off[r]), int(off[r + 1])
        _check(en, r, _oracle(orc, s, r, 60, pressures[r], masses[r]), p_all[a:b], f_all[a:b], "fp64")
        one = md.Simulation(s.replica(r), pr_pressure_gpa=pressures[r:r + 1], pr_mass=masses[r:r + 1])
        one.step(60)
        e1 = one.energy()
        assert np.array_equal(one.positions(), p_all[a:b])
        assert np.array_equal(e1.box[0], en.box[r]) and e1.pe[0] == en.pe[r]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pr_graph_replay_matches_eager(md, precision):
    """Barostatted middle steps replayed from HIP graphs equal the eager ones
    bitwise (the box lives on the device, so the replays see it move)."""
    s = _crystal(7)
    announce(f"pr graph replay {precision}")
    out = []
    for use_graph in (0, 1):
        sim = md.Simulation(s, precision=precision, pr_pressure_gpa=[1.0], pr_mass=[W_BOX])
        sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
        sim.step(60)
        e = sim.energy()
        out.append((sim.positions(), sim.velocities(), e.box.copy(), e.pr_energy.copy()))
        if use_graph:
            assert sim.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 2
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_pr_split_calls_equal_one_call(md):
    """md_step(40) and md_step(1) + md_step(13) + md_step(26) agree: the box
    state carries over and the two box half kicks at a call boundary compose."""
    s = _crystal()
    announce("pr split calls")
    a = md.Simulation(s, pr_pressure_gpa=[0.0], pr_mass=[W_BOX])
    a.step(40)
    b = md.Simulation(s, pr_pressure_gpa=[0.0], pr_mass=[W_BOX])
    for n in (1, 13, 26):
        b.step(n)
    ea, eb = a.energy(), b.energy()
    np.testing.assert_allclose(b.positions(), a.positions(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(eb.box, ea.box, rtol=1e-13, atol=0)
    assert eb.pr_energy[0] == pytest.approx(ea.pr_energy[0], rel=1e-11)


def test_pr_conserved_quantity_and_mean_pressure(md):
    """6000 FP64 steps of 2000 atoms at 3 GPa: PE + KE + barostat energy stays
    in a band a thousand times narrower than the swing of PE + KE, and the
    pressure averaged over the last 4000 steps is the target."""
    s = inputs.bcc_fe(10, a=2.84, temperature=600.0, seed=21, displace=0.02, skin=0.6)
    s.max_neighbours = 80
    announce("pr statistics 2000 atoms 6000 steps")
    sim = md.Simulation(s, pr_pressure_gpa=[3.0], pr_mass=[4.0 * W_BOX])
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    h, u, p = [], [], []
    for k in range(120):
        sim.step(50)
        e = sim.energy()
        h.append(e.pe[0] + e.ke[0] + e.pr_energy[0])
        u.append(e.pe[0] + e.ke[0])
        if k >= 40:
            p.append(e.pressure_gpa[0])
    h, u, p = np.array(h), np.array(u), np.array(p)
    announce(f"band {np.ptp(h):.3e} eV, swing {np.ptp(u):.3e} eV, mean pressure {p.mean():.3f} GPa")
    assert np.ptp(h) < 2e-3 * np.ptp(u)
    assert abs(p.mean() - 3.0) < 0.2


def test_pr_compression_beyond_the_grid_is_reported(md):
    """A pressure far above what the crystal holds compresses the box past the
    room its link-cell grid leaves (cells of 4.70 A for a 4.4 A list radius):
    MD_ERR_BOX, not a silently incomplete list.  The list is rebuilt every step,
    so the strain between builds stays under its own guard."""
    s = inputs.bcc_fe(5, a=2.818, temperature=300.0, seed=5)
    announce("pr compression limit")
    sim = md.Simulation(s, rebuild_every=1, max_neighbours=160, pr_pressure_gpa=[200.0], pr_mass=[4.0e4])
    with pytest.raises(md.MDError) as e:
        for _ in range(50):
            sim.step(2)
            sim.energy()
    assert e.value.code == md.MD_ERR_BOX
    assert "barostat" in str(e.value)


def test_pr_refuses_rigid_atoms(md):
    s = inputs.fcc_piston(nx=6, ny=6, nz=8, piston_cells=2, steps=0)
    s.periodic[:] = 1
    s.box[0, 2] = 60.0
    with pytest.raises(md.MDError) as e:
        md.Simulation(s, pr_pressure_gpa=[0.0], pr_mass=[W_BOX])
    assert e.value.code == md.MD_ERR_ARG


def _npt_oracle(orc, s, r, nsteps, p_gpa, w, t, q):
    sub = s.replica(r) if s.n_replicas > 1 else s
    return orc.run_npt(sub.pos, sub.vel, sub.species, sub.box[0], orc.Potential(sub.potential), sub.dt_fs, nsteps,
                       p_gpa, w, t, q, origin=sub.origin[0])


def test_npt_trajectory_against_oracle(md, orc):
    """Barostat and thermostat together (NPT): 100 FP64 steps of 432 atoms at
    2 GPa and 900 K against the oracle's NPT integrator, including the
    thermostat's momentum and energy."""
    s = _crystal()
    q = (3 * s.n_atoms - 3) * 8.617333262e-5 * 900.0 * 50.0**2
    announce("npt trajectory")
    sim = md.Simulation(s, pr_pressure_gpa=[2.0], pr_mass=[W_BOX], nh_temperature=[900.0], nh_mass=[q])
    sim.step(100)
    en = sim.energy()
    ref = _npt_oracle(orc, s, 0, 100, 2.0, W_BOX, 900.0, q)
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert np.max(np.abs(en.box[0] - ref.box[-1])) < 1e-10 * ref.box[-1].max()
    assert abs(en.pe[0] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])
    assert abs(en.ke[0] - ref.ke[-1]) <= 1e-8 * abs(ref.ke[-1])
    assert abs(en.nh_pi[0] - ref.pi[-1]) <= 1e-8 * abs(ref.pi[-1]) + 1e-14
    assert abs(en.nh_energy[0] - ref.nh_energy[-1]) <= 1e-8 * abs(ref.nh_energy[-1]) + 1e-10
    assert abs(en.pr_energy[0] - ref.baro[-1]) <= 1e-9 * abs(ref.baro[-1])
    assert abs(ref.pi[-1]) > 1e-5 and np.max(np.abs(ref.box[-1] - s.box[0])) > 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_npt_graph_replay_and_split_calls(md, precision):
    """NPT steps replayed from graphs equal the eager ones bitwise; split calls
    agree with one call."""
    s = _crystal(7)
    q = (3 * s.n_atoms - 3) * 8.617333262e-5 * 700.0 * 50.0**2
    kw = dict(precision=precision, pr_pressure_gpa=[1.0], pr_mass=[W_BOX], nh_temperature=[700.0], nh_mass=[q])
    announce(f"npt graph replay {precision}")
    out = []
    for use_graph in (0, 1):
        sim = md.Simulation(s, **kw)
        sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
        sim.step(60)
        e = sim.energy()
        out.append((sim.positions(), e.box.copy(), e.nh_pi.copy()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    split = md.Simulation(s, **kw)
    for n in (1, 22, 37):
        split.step(n)
    np.testing.assert_allclose(split.positions(), out[0][0], rtol=0, atol=1e-9 if precision == "fp64" else 1e-6)


def test_pr_empty_replica_keeps_its_box(md, orc):
    """An empty replica beside a crystal: its box stays put (no internal
    pressure resists the external one, and no atom needs the box to move),
    while the crystal's replica follows the oracle."""
    c = _crystal()
    n = c.n_atoms
    s = inputs.System(
        name="pr_empty", pos=c.pos, vel=c.vel, species=c.species, rigid=c.rigid,
        atom_offset=np.array([0, 0, n], np.int64), box=np.array([[20.0] * 3, c.box[0]]), origin=np.zeros((2, 3)),
        periodic=np.ones((2, 3), np.uint8), rigid_velocity=np.zeros((2, 3)), potential=c.potential, dt_fs=1.0,
        skin=0.6, rebuild_every=10, steps=0, temperature=np.array([0.0, 600.0]), max_neighbours=80,
    )
    announce("pr empty replica")
    sim = md.Simulation(s, pr_pressure_gpa=[3.0, 0.0], pr_mass=[W_BOX, W_BOX])
    sim.step(40)
    en = sim.energy()
    assert np.array_equal(en.box[0], [20.0, 20.0, 20.0])
    ref = _oracle(orc, c, 0, 40, 0.0, W_BOX)
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert np.max(np.abs(en.box[1] - ref.box[-1])) < 1e-10 * ref.box[-1].max()


def test_pr_options_and_autotune_keep_the_box(md, orc):
    """Changing a kernel option between calls re-uploads the replica
    descriptors; under the barostat that upload keeps the box the device has
    reached (not the configured one).  md_autotune in between changes nothing
    of the state either: the split run still follows the oracle."""
    s = _crystal()
    announce("pr options and autotune between calls")
    sim = md.Simulation(s, pr_pressure_gpa=[1.0], pr_mass=[W_BOX])
    sim.step(30)
    box_mid = sim.energy().box[0].copy()
    assert np.max(np.abs(box_mid - s.box[0])) > 1e-3
    sim.set_option(md.MD_OPT_COMPACT, 0)
    sim.set_option(md.MD_OPT_BRICK_BLOCK, 512)
    assert np.array_equal(sim.energy().box[0], box_mid)
    sim.autotune(trials=1)
    sim.step(30)
    en = sim.energy()
    ref = _oracle(orc, s, 0, 60, 1.0, W_BOX)
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert np.max(np.abs(en.box[0] - ref.box[-1])) < 1e-10 * ref.box[-1].max()
