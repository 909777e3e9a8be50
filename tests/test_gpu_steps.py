"""GPU tests of the md_step call structure: a call that continues from the
previous one (no reload and no force pass at entry), md_state_changed, and the
per-step energies of the device ring (paper, "Thermodynamic Quantities"),
against the FP64 oracle's trajectory."""
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


def _crystal(seed=71):
    return inputs.bcc_fe(10, temperature=300.0, seed=seed, name="bcc2000_steps")


@pytest.mark.parametrize("precision,kernel", [("fp64", 1), ("fp64", 0), ("mixed", 1)])
def test_resumed_calls_equal_one_call(md, precision, kernel):
    """Three calls of 10, 25 and 15 steps give bitwise the state of one 50-step
    call, and the continuing calls run no force pass at entry (counted with
    MD_OPT_TIMING, which keeps the continuation)."""
    announce(f"resume {precision} kernel {kernel}")
    s = _crystal()
    one = md.Simulation(s, precision=precision)
    one.set_option(md.MD_OPT_KERNEL, kernel)
    one.step(50)
    e_one = one.energy()
    split = md.Simulation(s, precision=precision)
    split.set_option(md.MD_OPT_KERNEL, kernel)
    split.step(10)
    split.set_option(md.MD_OPT_TIMING, 1)
    split.kernel_times(reset=True)
    split.step(25)
    kt = split.kernel_times(reset=True)
    split.energy()
    split.step(15)
    e_split = split.energy()
    # 25 density passes (a fresh start would run 26); the force group also
    # counts the opening kick that starts the continued call
    assert kt["density"][1] == 25 and kt["force"][1] == 26, kt
    assert np.array_equal(split.positions(), one.positions())
    assert np.array_equal(split.velocities(), one.velocities())
    assert np.array_equal(split.forces(), one.forces())
    assert e_split.pe[0] == e_one.pe[0] and e_split.ke[0] == e_one.ke[0] and e_split.step == 50


def test_state_changed_reloads_and_reverses(md):
    """After reversing the velocities through the bound arrays (set_state calls
    md_state_changed), the next call reloads the state and recomputes the
    forces: 40 FP64 steps forward and 40 back return to the start (velocity
    Verlet is time reversible)."""
    s = _crystal(seed=72)
    sim = md.Simulation(s, precision="fp64")
    sim.step(40)
    sim.energy()
    sim.set_state(vel=-sim.velocities())
    sim.step(40)
    sim.energy()
    assert np.max(np.abs(sim.positions() - s.pos)) < 1e-10
    assert np.max(np.abs(sim.velocities() + s.vel)) < 1e-12


@pytest.mark.parametrize("use_graph", [0, 1])
def test_energy_ring_against_oracle(md, orc, use_graph):
    """Energies of every step (MD_OPT_ENERGY_EVERY = 1) over 100 steps in calls
    of 7, 61 and 32 steps, eager and graph-replayed: each entry carries its step
    index and matches the oracle's potential and kinetic energy of that step."""
    announce(f"energy ring graph={use_graph}")
    s = _crystal(seed=73)
    sim = md.Simulation(s, precision="fp64", energy_ring=128)
    sim.set_option(md.MD_OPT_ENERGY_EVERY, 1)
    sim.set_option(md.MD_OPT_USE_GRAPH, use_graph)
    hist = []
    for n in (7, 61, 32):
        sim.step(n)
        hist += sim.energy_history()
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 100)
    assert [h.step for h in hist] == list(range(1, 101))
    pe = np.array([h.pe[0] for h in hist])
    ke = np.array([h.ke[0] for h in hist])
    assert np.max(np.abs(pe - ref.pe[1:]) / np.abs(ref.pe[1:])) < 1e-11
    assert np.max(np.abs(ke - ref.ke[1:]) / np.abs(ref.ke[1:])) < 1e-11
    assert all(np.isfinite(h.pressure_gpa[0]) and h.volume[0] > 0 for h in hist)
    if use_graph:
        assert sim.get_option(md.MD_OPT_GRAPH_LAUNCHES) > 0


def test_energy_ring_keeps_the_latest(md):
    """Every third step into a ring of 4 entries over 30 steps: the history
    returns the last four sampled steps; a second read returns nothing new;
    batched replicas get one record each per entry."""
    s = inputs.fec_replicas(3, nmin=300, nmax=900, seed0=4900)
    sim = md.Simulation(s, precision="mixed", energy_ring=4)
    sim.set_option(md.MD_OPT_ENERGY_EVERY, 3)
    sim.step(30)
    hist = sim.energy_history()
    assert [h.step for h in hist] == [21, 24, 27, 30]
    assert all(h.pe.shape == (3,) for h in hist)
    last = sim.energy()
    assert np.array_equal(hist[-1].pe, last.pe) and np.array_equal(hist[-1].ke, last.ke)
    assert sim.energy_history() == []


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_neighbour_chunk_is_bitwise_neutral(md, orc, precision):
    """The global kernels with 2, 4 or 8 neighbour records in flight add the
    same terms in the same order: 30 steps with energies every step (the
    energy-step variant is chunked too) agree bit for bit, on the oracle's
    trajectory."""
    announce(f"neighbour chunk {precision}")
    s = inputs.bcc_fe(10, temperature=600.0, seed=74, vacancy_frac=0.01, displace=0.05, name="bcc_chunk")
    runs = []
    for nch in (4, 2, 8):
        sim = md.Simulation(s, precision=precision, energy_ring=64)
        sim.set_option(md.MD_OPT_KERNEL, 1)
        sim.set_option(md.MD_OPT_NEIGHBOUR_CHUNK, nch)
        sim.set_option(md.MD_OPT_ENERGY_EVERY, 1)
        sim.step(30)
        hist = sim.energy_history()
        runs.append((sim.positions(), sim.velocities(), sim.forces(), np.array([h.pe[0] for h in hist])))
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], orc.Potential(s.potential), s.dt_fs, 30)
    assert np.max(np.abs(runs[0][0] - ref.pos)) < (1e-8 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_energy_ring_batched_equals_alone(md, precision):
    """Per-step energies of the global kernels are summed per wavefront in the
    force pass (a wavefront never straddles two replicas): every ring entry of
    a replica inside a batch equals, bit for bit, that of the replica run alone,
    and matches the sums of the per-atom path within rounding."""
    s = inputs.fec_replicas(3, nmin=300, nmax=900, seed0=4960)
    batch = md.Simulation(s, precision=precision, energy_ring=64)
    batch.set_option(md.MD_OPT_KERNEL, 1)
    batch.set_option(md.MD_OPT_ENERGY_EVERY, 1)
    batch.step(25)
    hist = batch.energy_history()
    for r in range(s.n_replicas):
        one = md.Simulation(s.replica(r), precision=precision, energy_ring=64)
        one.set_option(md.MD_OPT_KERNEL, 1)
        one.set_option(md.MD_OPT_ENERGY_EVERY, 1)
        one.step(25)
        h1 = one.energy_history()
        assert [h.step for h in h1] == [h.step for h in hist]
        for a, b in zip(h1, hist):
            assert a.pe[0] == b.pe[r] and a.ke[0] == b.ke[r] and np.array_equal(a.virial[0], b.virial[r])
    # the brick kernels keep the per-atom energy path: same totals within rounding
    brick = md.Simulation(s, precision=precision, energy_ring=64)
    brick.set_option(md.MD_OPT_KERNEL, 0)
    brick.set_option(md.MD_OPT_ENERGY_EVERY, 1)
    brick.step(25)
    hb = brick.energy_history()
    tol = 1e-10 if precision == "fp64" else 1e-6
    for a, b in zip(hb, hist):
        assert np.all(np.abs(a.pe - b.pe) <= tol * np.abs(a.pe))
        assert np.all(np.abs(a.ke - b.ke) <= tol * np.abs(a.ke))
