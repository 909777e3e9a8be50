"""md_msd_static, the entry point that allocates nothing (its partial sums and
results live in a static device array of the library), against md_msd on the
same bound state: two calls in a row, the second on a smaller system, both
bitwise equal to md_msd."""
import numpy as np
import pytest

from paper_1107_2619_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def md():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2619_amd import md as _md

    return _md


def _static_msd(md, sim):
    """md_msd_static through the C ABI (the binding only marshals)."""
    return sim.msd_static()


def test_static_scratch_matches_workspace(md):
    big = inputs.fec_replicas(5, nmin=1500, nmax=4000, seed0=6100)
    small = inputs.fec_replicas(2, nmin=300, nmax=500, seed0=6200)
    for s in (big, small):  # the second call reuses the scratch the first one filled
        sim = md.Simulation(s, precision="fp64")
        sim.step(30)
        ref, ref_cnt = sim.msd()
        out, cnt = _static_msd(md, sim)
        assert np.array_equal(out, ref) and np.array_equal(cnt, ref_cnt)
        assert np.all(cnt.sum(1) == np.diff(s.atom_offset)) and np.all(out[cnt > 0] > 0)


def test_static_scratch_size_limit(md):
    """A batch whose partial sums exceed the static scratch (8000 dimers in
    open boxes: 18 doubles per replica against 2^17) is refused."""
    R = 8000
    pos = np.tile(np.array([[5.0, 5.0, 5.0], [7.4, 5.0, 5.0]]), (R, 1))
    base = inputs.workload("bcc2000")
    s = inputs.System(
        name="dimers", pos=pos, vel=np.zeros_like(pos), species=np.zeros(2 * R, np.uint8),
        rigid=np.zeros(2 * R, np.uint8), atom_offset=np.arange(0, 2 * R + 1, 2, dtype=np.int64),
        box=np.full((R, 3), 12.0), origin=np.zeros((R, 3)), periodic=np.zeros((R, 3), np.uint8),
        rigid_velocity=np.zeros((R, 3)), potential=base.potential, dt_fs=1.0, skin=0.3, rebuild_every=10, steps=0,
        temperature=np.zeros(R), max_neighbours=8,
    )
    sim = md.Simulation(s, precision="fp64")
    with pytest.raises(md.MDError) as e:
        _static_msd(md, sim)
    assert e.value.code == md.MD_ERR_ARG and "scratch" in str(e.value)
