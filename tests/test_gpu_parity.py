"""GPU parity: the HIP path through the C-ABI against the FP64 CPU oracle.

Every case compares element by element on the same seeded inputs, at sizes the
oracle finishes in seconds that still span many link cells, a ragged last
wavefront and several replicas.  Tolerances: forces max|df|/rms|f| <= 1e-10
(FP64) / 1e-5 (mixed); per-atom energies relative <= 1e-12 / 1e-7.
"""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs
from tests.gpu_helpers import TOL, announce, energy_error, force_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _oracle_snapshot(orc, s, r=0):
    sub = s.replica(r) if s.n_replicas > 1 else s
    pot = orc.Potential(sub.potential)
    return orc.forces(sub.pos, sub.species, sub.box[0], sub.periodic[0], pot,
                      rigid=sub.rigid if sub.rigid.any() else None)


def _check_snapshot(md, orc, s, precision, options=None, check_energy=True, virial_rel=None, force_tol=None,
                    **kw):
    """virial_rel: bound on the virial error relative to the larger of |PE| and
    the largest diagonal virial term (default: the energy tolerance).  The
    virial, like PE, is a sum over pairs of pair terms, so its rounding error
    scales with theirs; near zero pressure its own value cancels to a small
    fraction of them and is no scale for a relative error.  force_tol: bound
    on the force error (default the precision's tolerance)."""
    announce(f"snapshot {s.name} N={s.n_atoms} R={s.n_replicas} {precision} {kw} {options}")
    sim = md.Simulation(s, precision=precision, **kw)
    for opt, val in (options or {}).items():
        sim.set_option(opt, val)
    sim.eam_forces(want_energy=True)
    en = sim.energy()
    f = sim.forces()
    e = sim.atom_energies()
    tol = TOL[precision]
    for r in range(s.n_replicas):
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        if b == a:
            assert en.pe[r] == 0.0
            continue
        ref = _oracle_snapshot(orc, s, r)
        ftol = tol["force"] if force_tol is None else force_tol
        assert force_error(f[a:b], ref.f) <= ftol, (r, force_error(f[a:b], ref.f))
        if not check_energy:
            continue
        assert energy_error(e[a:b], ref.e_atom) <= tol["energy"], (r, energy_error(e[a:b], ref.e_atom))
        assert abs(en.pe[r] - ref.pe) <= tol["energy"] * abs(ref.pe)
        wscale = max(abs(ref.pe), np.abs(ref.virial[:3]).max())
        vrel = tol["energy"] if virial_rel is None else virial_rel
        assert np.max(np.abs(en.virial[r] - ref.virial)) <= vrel * wscale, (r, en.virial[r] - ref.virial)
    return sim


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bcc2000_snapshot(md, orc, precision):
    s = inputs.bcc_fe(10, temperature=300.0, seed=1, displace=0.05, name="bcc2000_dsp")
    _check_snapshot(md, orc, s, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vacancy_600K_snapshot(md, orc, precision):
    s = inputs.bcc_fe(9, temperature=600.0, seed=2, vacancy_frac=0.01, displace=0.08, name="bcc_vac")
    _check_snapshot(md, orc, s, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_species_fec_snapshot(md, orc, precision):
    s = inputs.fec_replicas(3, nmin=300, nmax=1500, seed0=4100)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(9).random(s.pos.shape) - 1)
    _check_snapshot(md, orc, s, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_liquid_boxes_snapshot(md, orc, precision):
    """Boxes under three link cells per axis (128..300 atoms): the stencil
    must visit each neighbouring cell once."""
    s = inputs.liquid_replicas(4, nmin=128, nmax=300, seed0=5100)
    _check_snapshot(md, orc, s, precision, max_neighbours=96)


@pytest.mark.parametrize("workload", ["bcc", "fec"])
def test_explicit_knot_evaluator(md, orc, workload):
    """The term-by-term knot sums (the paper's explicit evaluation) agree with
    the oracle in FP64.  They are FP64 only: in FP32 their knot terms cancel
    against each other and miss the mixed energy tolerance, so mixed precision
    refuses them."""
    if workload == "bcc":
        s = inputs.bcc_fe(8, temperature=300.0, seed=6, displace=0.06)
    else:
        s = inputs.fec_replicas(2, nmin=300, nmax=800, seed0=4300)
        s.pos = s.pos + 0.04 * (2 * np.random.default_rng(5).random(s.pos.shape) - 1)
    _check_snapshot(md, orc, s, "fp64", options={md.MD_OPT_EVALUATOR: 1})
    sim = md.Simulation(s, precision="mixed")
    with pytest.raises(md.MDError) as e:
        sim.set_option(md.MD_OPT_EVALUATOR, 1)
    assert e.value.code == md.MD_ERR_ARG


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_printed_ni_al_pair_knots(md, orc, precision):
    """The pair coefficients the paper prints ("Available potentials", Ni/Al),
    knots 2.96061 .. 4.35174 A on no common grid, with the iron density
    functions, on a displaced bcc crystal: the tables with split bins meet the
    contract in both precisions (global, brick and half-list kernels)."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ni_al_atvf.json")))
    s = inputs.bcc_fe(7, temperature=300.0, seed=61, displace=0.06, name="bcc_ni_al_pair")
    pot = dict(s.potential)
    pot["pair_a"] = np.array(g["pair_a"]).reshape(1, 1, 4)
    pot["pair_r"] = np.array(g["pair_r"]).reshape(1, 1, 4)
    s.potential = pot
    for kernel in (1, 0):
        sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: kernel})
        assert sim.get_option(md.MD_OPT_EVALUATOR) == 0
    _check_snapshot(md, orc, s, precision, nbr_mode="half")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_species_distinct_embedding(md, orc, precision):
    """Fe-C replicas with F_a = -c_a sqrt(rho) and c = (1.0, 0.7) ("Theoretical
    background": the embedding belongs to the site atom's species), on the
    global, brick and half-list kernels."""
    s = inputs.fec_replicas(3, nmin=300, nmax=1500, seed0=4700)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(47).random(s.pos.shape) - 1)
    pot = dict(s.potential)
    pot["emb_c"] = np.array([1.0, 0.7])
    s.potential = pot
    for kernel in (1, 0):
        _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: kernel})
    _check_snapshot(md, orc, s, precision, nbr_mode="half")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_global_gather_path(md, orc, precision):
    """The one-thread-per-atom global-gather kernels (int32 list with periodic
    shift codes, compact records in mixed mode) on single- and two-species
    systems."""
    s = inputs.bcc_fe(8, temperature=600.0, seed=8, displace=0.07)
    _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 1})
    s2 = inputs.fec_replicas(2, nmin=300, nmax=900, seed0=4400)
    s2.pos = s2.pos + 0.04 * (2 * np.random.default_rng(7).random(s2.pos.shape) - 1)
    sim = _check_snapshot(md, orc, s2, precision, options={md.MD_OPT_KERNEL: 1})
    assert sim.get_option(md.MD_OPT_COMPACT) == (precision == "mixed")
    if precision == "mixed":  # the FP64 position records in mixed precision
        sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 1, md.MD_OPT_COMPACT: 0})
        assert sim.get_option(md.MD_OPT_COMPACT) == 0
        _check_snapshot(md, orc, s2, precision, options={md.MD_OPT_KERNEL: 1, md.MD_OPT_COMPACT: 0})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_half_list_atomics(md, orc, precision):
    """Half list with FP64 atomics (each pair evaluated once): parity with the
    oracle on one species, two species and a free-axis piston with rigid atoms
    (whose mutual pairs stay out of the virial)."""
    s = inputs.bcc_fe(8, temperature=600.0, seed=21, displace=0.07)
    _check_snapshot(md, orc, s, precision, nbr_mode="half")
    s2 = inputs.fec_replicas(2, nmin=300, nmax=900, seed0=4700)
    s2.pos = s2.pos + 0.04 * (2 * np.random.default_rng(21).random(s2.pos.shape) - 1)
    _check_snapshot(md, orc, s2, precision, nbr_mode="half")
    s3 = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, steps=0)
    s3.pos = s3.pos + 0.03 * (2 * np.random.default_rng(22).random(s3.pos.shape) - 1)
    _check_snapshot(md, orc, s3, precision, nbr_mode="half")


def test_half_list_matches_full(md):
    """FP64: half list + atomics and full list agree to rounding (only the
    summation order differs); the half list holds every pair exactly once."""
    s = inputs.fec_replicas(2, nmin=500, nmax=1200, seed0=4800)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(23).random(s.pos.shape) - 1)
    out = {}
    for mode in ("full", "half"):
        sim = md.Simulation(s, nbr_mode=mode)
        sim.eam_forces(want_energy=True)
        en = sim.energy()
        out[mode] = (sim.forces(), sim.atom_energies(), en, sim.neighbours())
    (ff, ef, enf, (cf, lf)), (fh, eh, enh, (ch, lh)) = out["full"], out["half"]
    assert force_error(fh, ff) < 1e-12
    assert energy_error(eh, ef) < 1e-13
    assert np.allclose(enh.virial, enf.virial, rtol=1e-12, atol=1e-10)
    assert int(ch.sum()) * 2 == int(cf.sum())
    full_pairs = {(i, int(j)) for i in range(s.n_atoms) for j in lf[i, : cf[i]]}
    half_pairs = [(i, int(j)) for i in range(s.n_atoms) for j in lh[i, : ch[i]]]
    assert len(set(half_pairs)) == len(half_pairs)
    assert {(min(a, b), max(a, b)) for a, b in half_pairs} == {(min(a, b), max(a, b)) for a, b in full_pairs}


@pytest.mark.parametrize("precision,mode,kernel", [("fp64", "full", 1), ("mixed", "full", 1),
                                                   ("fp64", "full", 0), ("mixed", "half", 1)])
def test_graph_replay_matches_eager(md, precision, mode, kernel):
    """md_step with captured-graph replay gives bitwise the eager results
    (global and LDS-brick kernels, full and half lists; the half list's FP64
    atomics make its sums order dependent, so it is compared to rounding).
    The graphs are replayed over several calls, with the program's own eager
    work and synchronisations in between, and every call is compared."""
    s = inputs.fec_replicas(3, nmin=300, nmax=900, seed0=4900)
    eager = md.Simulation(s, precision=precision, nbr_mode=mode)
    graph = md.Simulation(s, precision=precision, nbr_mode=mode)
    for sim in (eager, graph):
        sim.set_option(md.MD_OPT_KERNEL, kernel)
    graph.set_option(md.MD_OPT_USE_GRAPH, 1)
    if mode == "half":
        for nsteps in (47, 31):
            eager.step(nsteps)
            graph.step(nsteps)
            e1, e2 = eager.energy(), graph.energy()
            assert np.max(np.abs(eager.positions() - graph.positions())) < 1e-9
            assert np.allclose(e1.pe, e2.pe, rtol=1e-10)
        assert graph.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 2
        return
    for nsteps in (47, 31, 60, 5):
        eager.step(nsteps)
        graph.step(nsteps)
        e1, e2 = eager.energy(), graph.energy()
        assert np.array_equal(eager.positions(), graph.positions())
        assert np.array_equal(eager.velocities(), graph.velocities())
        assert np.array_equal(eager.forces(), graph.forces())
        assert np.array_equal(e1.pe, e2.pe) and np.array_equal(e1.virial, e2.virial)
        assert graph.get_option(md.MD_OPT_N_BUILDS) == eager.get_option(md.MD_OPT_N_BUILDS)
    assert graph.get_option(md.MD_OPT_GRAPH_LAUNCHES) >= 4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_then_parity(md, orc, precision):
    """md_autotune leaves positions and velocities untouched and the chosen
    configuration keeps oracle parity; mixed precision keeps the tables (its
    FP32 knot sums miss the energy tolerance)."""
    s = inputs.fec_replicas(2, nmin=600, nmax=1200, seed0=5000)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(24).random(s.pos.shape) - 1)
    sim = md.Simulation(s, precision=precision)
    x0, v0 = sim.positions(), sim.velocities()
    choice = sim.autotune(trials=2)
    assert choice["kernel"] in (0, 1, 2) and choice["step_us"] > 0 and choice["evaluator"] in (0, 1)
    if precision == "mixed":
        assert choice["evaluator"] == 0
    assert np.array_equal(sim.positions(), x0) and np.array_equal(sim.velocities(), v0)
    sim.eam_forces(want_energy=True)
    sim.energy()
    for r in range(s.n_replicas):
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        ref = _oracle_snapshot(orc, s, r)
        assert force_error(sim.forces()[a:b], ref.f) <= TOL[precision]["force"]


@pytest.mark.parametrize("dims", [111, 211, 222, 432, 444])
def test_brick_shapes(md, orc, dims):
    """Every brick shape stages the same neighbourhoods: parity for 1x1x1 up to
    4x4x4 cells per brick (edge bricks partial: 9 cells per axis)."""
    s = inputs.bcc_fe(12, temperature=600.0, seed=9, displace=0.07)
    _check_snapshot(md, orc, s, "fp64", options={md.MD_OPT_KERNEL: 0, md.MD_OPT_BRICK_DIMS: dims})


@pytest.mark.parametrize("lanes,block", [(1, 256), (2, 512), (4, 1024), (4, 128)])
def test_brick_lanes_and_blocks(md, orc, lanes, block):
    """Lanes sharing one atom's list and workgroup sizes: same results (two
    species exercise the staged type bytes)."""
    s = inputs.fec_replicas(2, nmin=600, nmax=1400, seed0=4500)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(11).random(s.pos.shape) - 1)
    for prec in ("fp64", "mixed"):
        _check_snapshot(md, orc, s, prec, options={md.MD_OPT_KERNEL: 0, md.MD_OPT_LANES_PER_ATOM: lanes, md.MD_OPT_BRICK_BLOCK: block})


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_brick_global_fallback(md, orc, precision):
    """Bricks whose halo exceeds the LDS staging area read their neighbours
    from global memory through the same halo order: identical results."""
    s = inputs.fec_replicas(2, nmin=800, nmax=1500, seed0=4600)
    s.pos = s.pos + 0.04 * (2 * np.random.default_rng(12).random(s.pos.shape) - 1)
    sim = _check_snapshot(md, orc, s, precision, options={md.MD_OPT_KERNEL: 0, md.MD_OPT_HALO_CAP: 64})
    assert sim.get_option(md.MD_OPT_HALO_OVERFLOWS) > 0


def test_free_axis_piston_snapshot(md, orc):
    s = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, steps=0)
    s.pos = s.pos + 0.03 * (2 * np.random.default_rng(3).random(s.pos.shape) - 1)
    _check_snapshot(md, orc, s, "fp64")


def test_neighbour_list_complete(md, orc):
    """Every pair closer than r_c is listed and every entry is closer than
    r_c + skin (brute-force pair set in numpy)."""
    s = inputs.bcc_fe(8, temperature=600.0, seed=4, displace=0.1)
    sim = md.Simulation(s)
    sim.build_neighbours()
    counts, lst = sim.neighbours()
    pos = s.pos
    L = s.box[0]
    d = pos[None, :, :] - pos[:, None, :]
    d -= L * np.rint(d / L)
    r = np.linalg.norm(d, axis=2)
    np.fill_diagonal(r, np.inf)
    rc = orc.cutoff(orc.Potential(s.potential))
    for i in range(s.n_atoms):
        listed = set(lst[i, : counts[i]].tolist())
        assert len(listed) == counts[i]
        must = set(np.nonzero(r[i] < rc)[0].tolist())
        assert must <= listed
        assert all(r[i, j] < rc + s.skin for j in listed)


def test_list_above_4gib(md):
    """A list whose allocation exceeds 4 GiB (128,000 atoms with room for 8,400
    entries each) is written with 64-bit addresses instead of 32-bit buffer
    offsets: the same entries in the same order, so 12 steps (one rebuild) agree
    bit for bit with the default capacity."""
    s = inputs.bcc_fe(40, temperature=300.0, seed=44, name="bcc_wide")
    assert s.n_atoms * 16 * ((8400 + 7) // 4) >= 1 << 32
    announce("list above 4 GiB")
    out = []
    for cap in (48, 8400):
        sim = md.Simulation(s, max_neighbours=cap)
        sim.set_option(md.MD_OPT_KERNEL, 1)
        sim.step(12)
        e = sim.energy()
        out.append((sim.positions(), sim.forces(), e.pe))
        del sim
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_large_list_above_4gib(md):
    """64-bit list addresses at an ordinary capacity: 5,488,000 atoms with room
    for 192 entries each pass 4 GiB and agree bit for bit, over 12 steps with
    one rebuild, with the default capacity."""
    s = inputs.bcc_fe(140, temperature=300.0, seed=45, name="bcc_wide_large")
    assert s.n_atoms * 16 * ((192 + 7) // 4) >= 1 << 32
    announce("large list above 4 GiB")
    out = []
    for cap in (48, 192):
        sim = md.Simulation(s, max_neighbours=cap, want_e_atom=False)
        sim.set_option(md.MD_OPT_KERNEL, 1)
        sim.step(12)
        e = sim.energy()
        out.append((sim.positions(), sim.forces(), e.pe))
        del sim
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision,mode", [("fp64", "full"), ("mixed", "full"), ("fp64", "half")])
def test_trajectory_100_steps(md, orc, precision, mode):
    """100 velocity-Verlet steps with list rebuilds every 10 steps against the
    oracle's brute-force trajectory (FP64: positions within 1e-8 A)."""
    s = inputs.workload("bcc2000")
    announce(f"trajectory bcc2000 {precision} {mode}")
    sim = md.Simulation(s, precision=precision, nbr_mode=mode)
    sim.step(100)
    en = sim.energy()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 100)
    dx = np.max(np.abs(sim.positions() - ref.pos))
    if precision == "fp64":
        assert dx < 1e-8
        assert force_error(sim.forces(), ref.f) < 1e-8
        assert abs(en.pe[0] - ref.pe[-1]) < 1e-10 * abs(ref.pe[-1])
        assert abs(en.ke[0] - ref.ke[-1]) < 1e-8 * abs(ref.ke[-1])
    else:
        assert dx < 1e-4
        assert abs(en.pe[0] + en.ke[0] - ref.pe[-1] - ref.ke[-1]) < 1e-5 * s.n_atoms
    assert en.step == 100


def test_piston_trajectory(md, orc):
    """Rigid moving block, free z axis: trajectory and work against the oracle."""
    s = inputs.fcc_piston(nx=4, ny=4, nz=8, piston_cells=2, piston_speed_a_per_fs=0.02, steps=0)
    announce("piston trajectory")
    sim = md.Simulation(s)
    sim.step(60)
    en = sim.energy()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 60,
                         rigid=s.rigid, rigid_velocity=s.rigid_velocity[0])
    assert np.max(np.abs(sim.positions() - ref.pos)) < 1e-8
    assert en.piston_work[0] == pytest.approx(ref.work[-1], rel=1e-8, abs=1e-10)
    assert en.n_mobile[0] == int((s.rigid == 0).sum())


def test_batched_equals_one_by_one(md):
    """Replica r run inside a batch gives bitwise the same FP64 state as the
    same replica run alone."""
    s = inputs.fec_replicas(4, nmin=250, nmax=1200, seed0=4200)
    announce("batched vs one-by-one")
    sim = md.Simulation(s)
    sim.step(25)
    en = sim.energy()
    pos, f = sim.positions(), sim.forces()
    for r in range(s.n_replicas):
        one = md.Simulation(s.replica(r))
        one.step(25)
        e1 = one.energy()
        a, b = int(s.atom_offset[r]), int(s.atom_offset[r + 1])
        assert np.array_equal(one.positions(), pos[a:b])
        assert np.array_equal(one.forces(), f[a:b])
        assert e1.pe[0] == en.pe[r] and e1.ke[0] == en.ke[r]


def test_empty_and_tiny_replicas(md, orc):
    """An empty replica and a two-atom replica inside a batch."""
    base = inputs.liquid_replicas(2, nmin=150, nmax=200, seed0=5200)
    dimer_pos = np.array([[5.0, 5.0, 5.0], [7.3, 5.0, 5.0]])
    pos = np.concatenate([base.pos[: base.atom_offset[1]], dimer_pos, base.pos[base.atom_offset[1]:]])
    vel = np.zeros_like(pos)
    n0 = int(base.atom_offset[1])
    n2 = int(base.atom_offset[2] - base.atom_offset[1])
    off = np.array([0, n0, n0, n0 + 2, n0 + 2 + n2], np.int64)
    box = np.array([base.box[0], [20.0] * 3, [20.0] * 3, base.box[1]])
    s = inputs.System(
        name="mixed_batch", pos=pos, vel=vel, species=np.zeros(len(pos), np.uint8), rigid=np.zeros(len(pos), np.uint8),
        atom_offset=off, box=box, origin=np.zeros((4, 3)), periodic=np.ones((4, 3), np.uint8),
        rigid_velocity=np.zeros((4, 3)), potential=base.potential, dt_fs=1.0, skin=0.5, rebuild_every=5, steps=0,
        temperature=np.zeros(4), max_neighbours=96,
    )
    _check_snapshot(md, orc, s, "fp64")
