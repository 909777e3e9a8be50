"""GPU parity of sheared cells (box matrices) and of the Parrinello-Rahman
barostat on the full box matrix with an external stress (paper, "Barostat
NPTp") against the oracle: forces in sheared cells, trajectories with a fixed
and with a moving cell, batches, graph replay, split calls, the thermostat
together with the barostat, and the conserved quantity and mean stress of a
long run."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import TOL, announce, energy_error, force_error

pytestmark = pytest.mark.gpu

W_BOX = 1.0e5  # eV fs^2 / A^2: box periods of about a picosecond at these sizes
UNIMODULAR = np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])  # edges a, b, c + a


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _skewed(cells=7, temperature=300.0, seed=7, displace=0.02, skin=0.3):
    """bcc Fe in the cell [a, b, c + a] of the cube: the cube's periodic
    system, in a cell with non-orthogonal edges."""
    s = inputs.bcc_fe(cells, a=2.87, temperature=temperature, seed=seed, displace=displace, skin=skin,
                      name=f"skew{cells}_{seed}")
    return s, np.diag(s.box[0]) @ UNIMODULAR


def _moving(cells=8, seed=7, kind="skewed"):
    """Cells for the barostat: a 0.6 A skin leaves its guards (0.4 skin per
    atom, 0.2 skin of strain over the list radius per rebuild period) room;
    the narrowest width of the 8-cell skewed cell holds three link cells with
    15% to spare; compression brings the fourth shell into the list."""
    if kind == "strained":
        s, h = _strained(cells, seed)
        s.skin = 0.6
    else:
        s, h = _skewed(cells, seed=seed, skin=0.6)
        if kind == "cube":
            h = np.diag(s.box[0])
    s.max_neighbours = 80
    return s, h


def _strained(cells=7, seed=9):
    """A crystal mapped by a general (not upper-triangular) homogeneous
    strain into the matching cell, with random displacements."""
    s = inputs.bcc_fe(cells, a=2.87, temperature=300.0, seed=seed, displace=0.06, name=f"strained{cells}_{seed}")
    f = np.array([[1.0, 0.04, -0.03], [0.02, 0.99, 0.05], [-0.04, 0.03, 1.01]])
    h = f @ np.diag(s.box[0])
    s.pos = s.pos @ f.T
    return s, h


def _stress(p=1.0, xy=0.5, yz=-0.3):
    s = p * np.eye(3)
    s[0, 1] = s[1, 0] = xy
    s[1, 2] = s[2, 1] = yz
    return s


def _prt(orc, s, h, nsteps, p=0.0, w=0.0, stress=None, t_target=0.0, q=0.0):
    return orc.run_prt(s.pos, s.vel, s.species, h, orc.Potential(s.potential), s.dt_fs, nsteps, p, w,
                       stress_gpa=stress, origin=s.origin[0], t_target=t_target, q_ev_fs2=q)


def _check(en, r, ref, pos, f, precision, barostat=True):
    dx = np.max(np.abs(pos - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(f, ref.f) < 1e-8
        assert np.max(np.abs(en.h[r] - ref.h[-1])) < 1e-10 * np.abs(ref.h[-1]).max()
        assert abs(en.pe[r] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])
        assert abs(en.ke[r] - ref.ke[-1]) <= 1e-8 * abs(ref.ke[-1])
        if barostat:
            assert abs(en.pr_energy[r] - ref.baro[-1]) <= 1e-9 * abs(ref.baro[-1]) + 1e-9
    else:
        assert dx < 1e-4
        assert np.max(np.abs(en.h[r] - ref.h[-1])) < 1e-5
        tot = en.pe[r] + en.ke[r] + (en.pr_energy[r] if barostat else 0.0)
        tot_ref = ref.pe[-1] + ref.ke[-1] + (ref.baro[-1] if barostat else 0.0)
        assert abs(tot - tot_ref) < 1e-5 * len(pos)


@pytest.mark.parametrize("cell", ["skewed", "strained"])
@pytest.mark.parametrize("precision,mode", [("fp64", "full"), ("mixed", "full"), ("fp64", "half")])
def test_sheared_cell_forces(md, orc, cell, precision, mode):
    """Forces, per-atom energies and the virial tensor in a sheared cell
    against the oracle's shortest-image brute force."""
    s, h = _skewed(displace=0.08) if cell == "skewed" else _strained()
    announce(f"sheared cell forces {cell} {precision} {mode}")
    sim = md.Simulation(s, precision=precision, nbr_mode=mode, box_matrix=h)
    sim.eam_forces(True)
    en = sim.energy()
    ref = orc.forces_tri(s.pos, s.species, h, orc.Potential(s.potential))
    tol = TOL[precision]
    assert force_error(sim.forces(), ref.f) < tol["force"]
    assert energy_error(sim.atom_energies(), ref.e_atom) < tol["energy"]
    assert abs(en.pe[0] - ref.pe) <= 1e-12 * abs(ref.pe) * (1e5 if precision == "mixed" else 1)
    assert np.max(np.abs(en.virial[0] - ref.virial)) < (1e-9 if precision == "fp64" else 1e-4) * np.abs(ref.virial).max()
    assert np.allclose(en.h[0], h, rtol=0, atol=0)
    assert en.volume[0] == pytest.approx(abs(np.linalg.det(h)), rel=1e-14)


@pytest.mark.parametrize("precision,mode", [("fp64", "full"), ("mixed", "full"), ("fp64", "half")])
def test_sheared_cell_nve_trajectory(md, orc, precision, mode):
    """100 velocity-Verlet steps in a fixed sheared cell with list rebuilds
    every 10 (atoms cross the slanted faces) against the oracle's run with the
    box held."""
    s, h = _strained()
    announce(f"sheared cell nve {precision} {mode}")
    sim = md.Simulation(s, precision=precision, nbr_mode=mode, box_matrix=h)
    sim.step(100)
    ref = _prt(orc, s, h, 100)
    _check(sim.energy(), 0, ref, sim.positions(), sim.forces(), precision, barostat=False)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("integrator", ["verlet", "gear3", "nvt"])
def test_skewed_cell_is_the_cube(md, orc, integrator, precision):
    """The cell [a, b, c + a] holds the cube's periodic system, so every
    integrator in it follows the oracle's run of the cube (velocity Verlet,
    Gear, Nose-Hoover); mixed precision carries sheared-cell compact records
    through each integrator's passes."""
    s, h = _skewed()
    pot = orc.Potential(s.potential)
    announce(f"skewed cell = cube, {integrator} {precision}")
    if integrator == "nvt":
        q = (3 * s.n_atoms - 3) * orc.boltzmann_ev() * 500.0 * 50.0**2
        sim = md.Simulation(s, precision=precision, box_matrix=h, nh_temperature=[500.0], nh_mass=[q])
        ref = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, s.dt_fs, 60, 500.0, q)
    elif integrator == "gear3":
        sim = md.Simulation(s, precision=precision, box_matrix=h, integrator="gear3")
        ref = orc.run_gear(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, s.dt_fs, 60)
    else:
        sim = md.Simulation(s, precision=precision, box_matrix=h)
        ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, s.dt_fs, 60)
    sim.step(60)
    en = sim.energy()
    if precision == "mixed":
        assert sim.get_option(md.MD_OPT_COMPACT) == 1
        assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-4
        assert abs(en.pe[0] + en.ke[0] - ref.pe[-1] - ref.ke[-1]) < 1e-5 * s.n_atoms
        return
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert abs(en.pe[0] - ref.pe[-1]) <= 1e-10 * abs(ref.pe[-1])
    if integrator == "nvt":
        assert en.nh_pi[0] == pytest.approx(ref.pi[-1], rel=1e-8, abs=1e-14)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prt_trajectory_100_steps(md, orc, precision):
    """The full-matrix barostat under pressure and shear stress in the skewed
    cell (1024 atoms): 100 steps against the oracle (positions, box matrix,
    energies)."""
    s, h = _moving()
    announce(f"full-matrix barostat trajectory {precision}")
    sim = md.Simulation(s, precision=precision, box_matrix=h, pr_pressure_gpa=[1.0], pr_mass=[W_BOX],
                        pr_stress_gpa=_stress())
    sim.step(100)
    en = sim.energy()
    ref = _prt(orc, s, h, 100, 1.0, W_BOX, _stress())
    assert np.abs(ref.h[-1] - h).max() > 1e-3  # the cell moved
    assert abs(ref.h[-1][1, 0]) > 1e-4  # and sheared off its starting shape
    _check(en, 0, ref, sim.positions(), sim.forces(), precision)
    assert en.volume[0] == pytest.approx(abs(np.linalg.det(en.h[0])), rel=1e-13)


def test_prt_from_the_cube(md, orc):
    """An external stress alone (no box matrix) starts the full-matrix
    barostat from the orthorhombic box."""
    s, _ = _moving(kind="cube")
    announce("full-matrix barostat from the cube")
    sim = md.Simulation(s, pr_pressure_gpa=[0.5], pr_mass=[W_BOX], pr_stress_gpa=_stress(0.5, 0.8, 0.0))
    sim.step(80)
    ref = _prt(orc, s, np.diag(s.box[0]), 80, 0.5, W_BOX, _stress(0.5, 0.8, 0.0))
    assert abs(ref.h[-1][0, 1]) > 1e-4
    _check(sim.energy(), 0, ref, sim.positions(), sim.forces(), "fp64")


def test_prt_batched_against_oracle_and_alone(md, orc):
    """Three replicas (skewed, strained and cubic cells) under different
    pressures, stresses and box masses, each against its own oracle run and
    bitwise equal to the replica alone."""
    parts = [_moving(8, 21), _moving(7, 22, "strained"), _moving(8, 23, "cube")]
    hs = [p[1] for p in parts]
    sys_ = [p[0] for p in parts]
    pos = np.concatenate([p.pos for p in sys_])
    vel = np.concatenate([p.vel for p in sys_])
    off = np.concatenate([[0], np.cumsum([p.n_atoms for p in sys_])]).astype(np.int64)
    s = inputs.System(
        name="prt_batch", pos=pos, vel=vel, species=np.zeros(len(pos), np.uint8), rigid=np.zeros(len(pos), np.uint8),
        atom_offset=off, box=np.array([p.box[0] for p in sys_]), origin=np.zeros((3, 3)),
        periodic=np.ones((3, 3), np.uint8), rigid_velocity=np.zeros((3, 3)), potential=sys_[0].potential,
        dt_fs=1.0, skin=0.6, rebuild_every=10, steps=0, temperature=np.full(3, 300.0), max_neighbours=80,
    )
    pressures = np.array([0.0, 1.0, 2.0])
    masses = np.array([0.5, 1.0, 2.0]) * W_BOX
    stresses = np.array([_stress(0.0, 0.4, 0.0), _stress(1.0, -0.3, 0.2), _stress(2.0, 0.0, 0.6)])
    announce("full-matrix barostat batched")
    sim = md.Simulation(s, box_matrix=np.array(hs), pr_pressure_gpa=pressures, pr_mass=masses,
                        pr_stress_gpa=stresses)
    sim.step(60)
    en = sim.energy()
    p_all, f_all = sim.positions(), sim.forces()
    for r in range(3):
        a, b = int(off[r]), int(off[r + 1])
        ref = _prt(orc, s.replica(r), hs[r], 60, pressures[r], masses[r], stresses[r])
        _check(en, r, ref, p_all[a:b], f_all[a:b], "fp64")
        one = md.Simulation(s.replica(r), box_matrix=hs[r], pr_pressure_gpa=pressures[r:r + 1],
                            pr_mass=masses[r:r + 1], pr_stress_gpa=stresses[r])
        one.step(60)
        e1 = one.energy()
        assert np.array_equal(one.positions(), p_all[a:b])
        assert np.array_equal(e1.h[0], en.h[r]) and e1.pe[0] == en.pe[r]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prt_graph_replay_matches_eager(md, precision):
    """Full-matrix barostat steps replayed from HIP graphs equal the eager
    ones bitwise."""
    s, h = _moving()
    announce(f"full-matrix barostat graph replay {precision}")
    out = []
    for use_graph in (0, 1):
        sim = md.Simulation(s, precision=precision, box_matrix=h, pr_pressure_gpa=[1.0], pr_mass=[W_BOX],
                            pr_stress_gpa=_stress())
        sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
        sim.step(60)
        e = sim.energy()
        out.append((sim.positions(), sim.velocities(), e.h.copy(), e.pr_energy.copy()))
        if use_graph:
            assert sim.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 2
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_prt_split_calls_equal_one_call(md):
    """md_step(40) and md_step(1) + md_step(13) + md_step(26) agree."""
    s, h = _moving()
    announce("full-matrix barostat split calls")
    kw = dict(box_matrix=h, pr_pressure_gpa=[1.0], pr_mass=[W_BOX], pr_stress_gpa=_stress())
    a = md.Simulation(s, **kw)
    a.step(40)
    b = md.Simulation(s, **kw)
    for n in (1, 13, 26):
        b.step(n)
    ea, eb = a.energy(), b.energy()
    np.testing.assert_allclose(b.positions(), a.positions(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(eb.h, ea.h, rtol=1e-13, atol=1e-13)
    assert eb.pr_energy[0] == pytest.approx(ea.pr_energy[0], rel=1e-11)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prt_with_thermostat(md, orc, precision):
    """NPT on the full box matrix: 100 steps at 1 GPa with shear stress and
    600 K against the oracle (positions, box, energies, thermostat)."""
    s, h = _moving()
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 600.0 * 50.0**2
    announce(f"full-matrix NPT {precision}")
    sim = md.Simulation(s, precision=precision, box_matrix=h, pr_pressure_gpa=[1.0], pr_mass=[W_BOX],
                        pr_stress_gpa=_stress(), nh_temperature=[600.0], nh_mass=[q])
    sim.step(100)
    en = sim.energy()
    ref = _prt(orc, s, h, 100, 1.0, W_BOX, _stress(), 600.0, q)
    if precision == "fp64":
        _check(en, 0, ref, sim.positions(), sim.forces(), precision)
        assert en.nh_pi[0] == pytest.approx(ref.pi[-1], rel=1e-8, abs=1e-14)
        assert en.nh_energy[0] == pytest.approx(ref.nh_energy[-1], rel=1e-8, abs=1e-12)
    else:
        assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-4
        tot = en.pe[0] + en.ke[0] + en.pr_energy[0] + en.nh_energy[0]
        tot_ref = ref.pe[-1] + ref.ke[-1] + ref.baro[-1] + ref.nh_energy[-1]
        assert abs(tot - tot_ref) < 1e-5 * s.n_atoms


def test_prt_conserved_quantity_and_mean_stress(md):
    """3000 FP64 steps of 1024 atoms in the skewed cell at 1 GPa with shear
    stress (graphs on): the conserved quantity stays in a band a thousand times
    narrower than the swing of PE + KE, and the time-averaged internal stress
    carries the load P + (Omega0 / Omega) F (S - P) F^T, F = h h0^-1 (off
    the diagonal the kinetic tensor averages to zero; on it to 2 KE / 3)."""
    s, h0 = _moving()
    stress = _stress()
    announce("full-matrix barostat 3000 steps")
    sim = md.Simulation(s, box_matrix=h0, pr_pressure_gpa=[1.0], pr_mass=[W_BOX], pr_stress_gpa=stress)
    sim.set_option(md.MD_OPT_USE_GRAPH, 1)
    tot, swing, vir, ke, hs, vol = [], [], [], [], [], []
    for _ in range(150):
        sim.step(20)
        e = sim.energy()
        tot.append(e.pe[0] + e.ke[0] + e.pr_energy[0])
        swing.append(e.pe[0] + e.ke[0])
        vir.append(e.virial[0])
        ke.append(e.ke[0])
        hs.append(e.h[0])
        vol.append(e.volume[0])
    tot, swing = np.array(tot), np.array(swing)
    announce(f"band {np.ptp(tot):.3e} eV, swing {np.ptp(swing):.3e} eV")
    assert np.ptp(tot) < 2e-3 * np.ptp(swing)
    late = slice(50, None)
    conv = 160.217653
    v = np.array(vir)[late]
    k = np.array(ke)[late]
    om = np.array(vol)[late]
    pi = np.zeros((3, 3))
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for c, (i, j) in enumerate(idx):
        val = np.mean((v[:, c] + (2.0 * k / 3.0 if i == j else 0.0)) / om) * conv
        pi[i, j] = pi[j, i] = val
    hm = np.array(hs)[late].mean(0)
    f = hm @ np.linalg.inv(h0)
    load = np.eye(3) + abs(np.linalg.det(h0)) / abs(np.linalg.det(hm)) * f @ (stress - np.eye(3)) @ f.T
    announce(f"mean stress {np.round(pi, 3).tolist()} load {np.round(load, 3).tolist()}")
    assert np.max(np.abs(pi - load)) < 0.1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prt_options_and_autotune_keep_the_cell(md, orc, precision):
    """Option changes between calls re-upload the replica descriptors; under
    the full-matrix barostat that upload keeps the cell the device has reached
    (box matrix, inverse, strain map, record units).  md_autotune in between
    changes nothing of the state: the split run still follows the oracle."""
    s, h = _moving()
    announce(f"full-matrix barostat options and autotune between calls {precision}")
    kw = dict(box_matrix=h, pr_pressure_gpa=[1.0], pr_mass=[W_BOX], pr_stress_gpa=_stress())
    sim = md.Simulation(s, precision=precision, **kw)
    sim.step(30)
    h_mid = sim.energy().h[0].copy()
    assert np.max(np.abs(h_mid - h)) > 1e-4
    sim.set_option(md.MD_OPT_BRICK_BLOCK, 512)
    assert np.array_equal(sim.energy().h[0], h_mid)
    sim.autotune(trials=1)
    sim.step(30)
    en = sim.energy()
    ref = _prt(orc, s, h, 60, 1.0, W_BOX, _stress())
    if precision == "fp64":
        assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
        assert np.max(np.abs(en.h[0] - ref.h[-1])) < 1e-10 * np.abs(ref.h[-1]).max()
    else:
        assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-4
        assert np.max(np.abs(en.h[0] - ref.h[-1])) < 1e-5


def test_sheared_cell_unwrapped_images(md):
    """Positions given several edge vectors away from the cell (unwrapped, as
    the paper keeps them) give the same forces, and the caller's positions stay
    unwrapped: after 30 steps each shifted atom sits at its unshifted twin plus
    the same lattice vector."""
    s, h = _strained()
    rng = np.random.default_rng(3)
    k = rng.integers(-3, 4, size=(s.n_atoms, 3)).astype(float)
    shift = k @ h.T
    announce("sheared cell unwrapped images")
    a = md.Simulation(s, box_matrix=h)
    a.step(30)
    moved = inputs.System(**{**s.__dict__, "pos": s.pos + shift})
    b = md.Simulation(moved, box_matrix=h)
    b.step(30)
    np.testing.assert_allclose(b.forces(), a.forces(), rtol=0, atol=1e-9)
    np.testing.assert_allclose(b.positions() - shift, a.positions(), rtol=0, atol=1e-9)
    assert b.energy().pe[0] == pytest.approx(a.energy().pe[0], rel=1e-12)


def test_prt_compression_beyond_the_grid_is_reported(md):
    """Under a pressure far above what the crystal holds the sheared cell
    narrows past the room of its link-cell grid (three cells of 4.74 A across
    its narrowest width for a 4.4 A list radius): MD_ERR_BOX, not a silently
    incomplete list.  The list is rebuilt every step, so the strain between
    builds stays under its own guard."""
    s, h = _skewed()
    announce("full-matrix barostat compression limit")
    # W = 4e5: the oracle's cell reaches the limit near step 30 while the strain per step
    # stays under the guard (with W = 4e4 the strain guard trips first, MD_ERR_SKIN)
    sim = md.Simulation(s, box_matrix=h, rebuild_every=1, max_neighbours=160, pr_pressure_gpa=[200.0],
                        pr_mass=[4.0e5])
    with pytest.raises(md.MDError) as e:
        for _ in range(50):
            sim.step(2)
            sim.energy()
    assert e.value.code == md.MD_ERR_BOX


def test_prt_empty_replica_keeps_its_cell(md, orc):
    """An empty sheared replica beside a crystal under the full-matrix
    barostat: the empty cell stays put (nothing inside resists the load or
    needs the cell to move) while the crystal follows the oracle."""
    c, h = _moving()
    n = c.n_atoms
    h_empty = np.array([[24.0, 0.0, 6.0], [0.0, 24.0, 0.0], [0.0, 0.0, 24.0]])
    s = inputs.System(
        name="prt_empty", pos=c.pos, vel=c.vel, species=c.species, rigid=c.rigid,
        atom_offset=np.array([0, 0, n], np.int64), box=np.array([[24.0] * 3, c.box[0]]), origin=np.zeros((2, 3)),
        periodic=np.ones((2, 3), np.uint8), rigid_velocity=np.zeros((2, 3)), potential=c.potential, dt_fs=1.0,
        skin=0.6, rebuild_every=10, steps=0, temperature=np.array([0.0, 300.0]), max_neighbours=80,
    )
    announce("full-matrix barostat empty replica")
    sim = md.Simulation(s, box_matrix=np.array([h_empty, h]), pr_pressure_gpa=[3.0, 1.0], pr_mass=[W_BOX, W_BOX],
                        pr_stress_gpa=np.array([_stress(3.0, 1.0, 0.0), _stress()]))
    sim.step(40)
    en = sim.energy()
    assert np.array_equal(en.h[0], h_empty)
    ref = _prt(orc, c, h, 40, 1.0, W_BOX, _stress())
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert np.max(np.abs(en.h[1] - ref.h[-1])) < 1e-10 * np.abs(ref.h[-1]).max()
