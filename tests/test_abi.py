"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and md_create validates its arguments on the host (no device
work happens before md_bind)."""
import os
import re

import numpy as np
import pytest

from paper_1107_2619_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def md():
    from paper_1107_2619_amd import md as _md

    try:
        _md.library()
    except ImportError:
        pytest.fail("libmdeam.so is not built (run python -m paper_1107_2619_amd.build)")
    return _md


def _declared():
    text = open(os.path.join(ROOT, "include", "md.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(md_\w+)\s*\(", text, re.M)))


def test_header_symbols_exported(md):
    lib = md.library()
    declared = _declared()
    assert declared == sorted(md.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def _ctx(md, **over):
    s = inputs.workload("bcc2000")
    kw = dict(skin=0.3, max_neighbours=48)
    kw.update(over)
    pot = over.pop("potential", None) or s.potential
    kw.pop("potential", None)
    box = kw.pop("box", s.box)
    per = kw.pop("periodic", s.periodic)
    off = kw.pop("atom_offset", s.atom_offset)
    return md.Context(pot, off, box, per, **kw)


def test_create_ok_and_workspace(md):
    c = _ctx(md)
    assert c.workspace_bytes() > 2000 * 48 * 4


def test_box_too_small(md):
    with pytest.raises(md.MDError) as e:
        _ctx(md, box=[[8.7, 28.7, 28.7]])
    assert e.value.code == md.MD_ERR_BOX
    # a free axis may be small
    _ctx(md, box=[[8.7, 28.7, 28.7]], periodic=[[0, 1, 1]])


@pytest.mark.parametrize(
    "field,value,code",
    [("max_neighbours", 0, -1), ("rebuild_every", 0, -1), ("precision", 7, -1), ("nbr_mode", 3, -1),
     ("lanes_per_atom", 3, -1), ("lanes_per_atom", 8, -1), ("skin", -0.1, -1), ("dt_fs", 0.0, -1)],
)
def test_config_validation(md, field, value, code):
    with pytest.raises(md.MDError) as e:
        _ctx(md, **{field: value})
    assert e.value.code == code


def test_potential_validation(md):
    s = inputs.workload("bcc2000")
    bad = dict(s.potential)
    bad["dens_A"] = -np.abs(bad["dens_A"])
    with pytest.raises(md.MDError) as e:
        _ctx(md, potential=bad)
    assert e.value.code == md.MD_ERR_POTENTIAL
    pot2 = inputs.perturbed_potential("fec_eam", 1)
    pot2["pair_a"][0, 1, 0] += 1.0  # break the pair symmetry
    with pytest.raises(md.MDError) as e:
        _ctx(md, potential=pot2)
    assert e.value.code == md.MD_ERR_POTENTIAL
    heavy = dict(s.potential)
    heavy["mass"] = np.array([0.0])
    with pytest.raises(md.MDError):
        _ctx(md, potential=heavy)


def _fe_knots(npk, ndk, step, ns=1):
    """A one- or two-species table with npk pair and ndk density knots spaced
    ``step`` apart below 4.1 A (amplitudes of no physical meaning)."""
    pr = 4.1 - step * np.arange(npk)[::-1]
    dr = 4.1 - step * np.arange(ndk)[::-1]
    return {
        "pair_a": np.tile(np.linspace(0.5, -0.1, npk), (ns, ns, 1)),
        "pair_r": np.tile(pr, (ns, ns, 1)),
        "dens_A": np.tile(np.linspace(1.0, 2.0, ndk), (ns, ns, 1)),
        "dens_R": np.tile(dr, (ns, ns, 1)),
        "emb_c": np.ones(ns),
        "mass": np.full(ns, 55.845),
    }


def test_knot_limits_and_evaluators(md):
    """Up to 16 knots per function (the paper's benchmark iron potential is a
    sum of 15 cubic splines, "Parallel benchmarks").  The exact tables take any
    knot placement (knots off the bin grid become split terms inside their
    bin); the term-by-term sums, FP64 only, cover 8 + 8 knots, or 16 pair and
    4 density knots for one species.  Mixed precision refuses the knot sums."""
    fe15 = inputs.perturbed_potential("fe15_fs", 3)
    assert fe15["pair_a"].shape[2] == 13 and fe15["dens_A"].shape[2] == 2
    c = _ctx(md, potential=fe15)
    assert c.get_option(md.MD_OPT_EVALUATOR) == 0
    c.set_option(md.MD_OPT_EVALUATOR, 1)
    assert c.get_option(md.MD_OPT_EVALUATOR) == 1
    # 16 on-grid pair knots and 8 density knots: tables only
    c = _ctx(md, potential=_fe_knots(16, 8, 0.1))
    assert c.get_option(md.MD_OPT_EVALUATOR) == 0
    with pytest.raises(md.MDError) as e:
        c.set_option(md.MD_OPT_EVALUATOR, 1)
    assert e.value.code == md.MD_ERR_ARG
    # off-grid knots (step 0.1234 A): tables with split bins, and the 16 + 4 knot sums
    c = _ctx(md, potential=_fe_knots(16, 4, 0.1234))
    assert c.get_option(md.MD_OPT_EVALUATOR) == 0
    c.set_option(md.MD_OPT_EVALUATOR, 1)
    assert c.get_option(md.MD_OPT_EVALUATOR) == 1
    # off-grid with 5 density knots, or two species with 9 pair knots: tables only
    for pot in (_fe_knots(16, 5, 0.1234), _fe_knots(9, 2, 0.1234, ns=2)):
        c = _ctx(md, potential=pot)
        assert c.get_option(md.MD_OPT_EVALUATOR) == 0
        with pytest.raises(md.MDError) as e:
            c.set_option(md.MD_OPT_EVALUATOR, 1)
        assert e.value.code == md.MD_ERR_ARG
    # the printed Ni/Al pair knots (no common grid) in mixed precision: the tables
    g = _golden_ni_al()
    nial = _fe_knots(4, 2, 0.3)
    nial["pair_a"] = np.array(g["pair_a"]).reshape(1, 1, 4)
    nial["pair_r"] = np.array(g["pair_r"]).reshape(1, 1, 4)
    c = _ctx(md, potential=nial, precision="mixed")
    assert c.get_option(md.MD_OPT_EVALUATOR) == 0
    with pytest.raises(md.MDError) as e:
        c.set_option(md.MD_OPT_EVALUATOR, 1)
    assert e.value.code == md.MD_ERR_ARG and "FP64 only" in str(e.value)
    # two knots of one function closer than the finest bin (4.1 / 4096 A): no
    # tables, so FP64 takes the knot sums and mixed precision refuses the potential
    close = _fe_knots(6, 2, 0.3)
    close["pair_r"][0, 0, 0] = 2.6 + 1e-4 * np.sqrt(2.0)
    close["pair_r"][0, 0, 1] = 2.6 + 2e-4 * np.sqrt(3.0)
    c = _ctx(md, potential=close)
    assert c.get_option(md.MD_OPT_EVALUATOR) == 1
    with pytest.raises(md.MDError) as e:
        _ctx(md, potential=close, precision="mixed")
    assert e.value.code == md.MD_ERR_POTENTIAL
    # on the grid the two-species 9-knot table is accepted (tables)
    c = _ctx(md, potential=_fe_knots(9, 2, 0.1, ns=2))
    assert c.get_option(md.MD_OPT_EVALUATOR) == 0
    # 17 knots exceed the limit
    with pytest.raises(md.MDError) as e:
        _ctx(md, potential=_fe_knots(17, 2, 0.1))
    assert e.value.code == md.MD_ERR_POTENTIAL and "1..16" in str(e.value)


def _golden_ni_al():
    import json

    with open(os.path.join(ROOT, "tests", "golden", "ni_al_atvf.json")) as fh:
        return json.load(fh)


def test_atom_offset_validation(md):
    with pytest.raises(md.MDError):
        _ctx(md, atom_offset=[1, 2000])
    with pytest.raises(md.MDError):
        md.Context(inputs.workload("bcc2000").potential, [0, 10, 5], [[28.7] * 3] * 2, [[1, 1, 1]] * 2)


def test_small_boxes_get_at_least_one_cell(md):
    s = inputs.liquid_replicas(3, nmin=128, nmax=140, seed0=5300)
    c = md.Context(s.potential, s.atom_offset, s.box, s.periodic, skin=0.5, max_neighbours=96)
    assert c.workspace_bytes() > 0


def test_size_limits_rejected_on_host(md):
    """More atom slots than a list entry can index (2^25), and link-cell grids
    beyond the supported count, are refused before any device work."""
    s = inputs.workload("bcc2000")
    n = (1 << 25) + 1
    with pytest.raises(md.MDError) as e:
        md.Context(s.potential, [0, n], [[300.0] * 3], [[1, 1, 1]], skin=0.3, max_neighbours=48)
    assert e.value.code == md.MD_ERR_ARG and "too large" in str(e.value)
    # one atom slot short of the limit is accepted (no device memory is touched)
    md.Context(s.potential, [0, (1 << 25) - 64], [[300.0] * 3], [[1, 1, 1]], skin=0.3, max_neighbours=48)


def test_options_round_trip_on_host(md):
    c = _ctx(md)
    for opt, val in ((md.MD_OPT_USE_GRAPH, 1), (md.MD_OPT_KERNEL, 0), (md.MD_OPT_COMPACT, 0),
                     (md.MD_OPT_LANES_PER_ATOM, 2)):
        c.set_option(opt, val)
        assert c.get_option(opt) == val
    with pytest.raises(md.MDError):
        c.set_option(md.MD_OPT_USE_GRAPH, 2)
    with pytest.raises(md.MDError):
        c.set_option(999, 1)


def test_thermostat_validation(md):
    """Thermostat arguments: both or neither, T >= 0 and Q > 0, per replica."""
    _ctx(md, nh_temperature=[300.0], nh_mass=[50.0])
    _ctx(md, nh_temperature=[0.0], nh_mass=[1e-3])
    for kw in (dict(nh_temperature=[300.0]), dict(nh_mass=[50.0]), dict(nh_temperature=[-1.0], nh_mass=[50.0]),
               dict(nh_temperature=[300.0], nh_mass=[0.0]), dict(nh_temperature=[np.nan], nh_mass=[50.0]),
               dict(nh_temperature=[300.0], nh_mass=[np.inf])):
        with pytest.raises(md.MDError) as e:
            _ctx(md, **kw)
        assert e.value.code == md.MD_ERR_ARG


def test_msd_needs_a_bound_state(md):
    """md_msd and md_msd_origin refuse an unbound context before any device work."""
    c = _ctx(md)
    out = np.zeros(1)
    assert c.lib.md_msd(c.handle, out.ctypes.data, None, None) == md.MD_ERR_STATE
    assert c.lib.md_msd_origin(c.handle, None) == md.MD_ERR_STATE
    assert c.lib.md_msd(c.handle, None, None, None) == md.MD_ERR_ARG
    assert c.lib.md_msd(None, out.ctypes.data, None, None) == md.MD_ERR_ARG


def test_integrator_validation(md):
    """MD_GEAR3 is accepted alone; an unknown integrator, and Gear with the
    thermostat, are refused on the host."""
    _ctx(md, integrator="gear3")
    with pytest.raises(md.MDError) as e:
        _ctx(md, integrator=5)
    assert e.value.code == md.MD_ERR_ARG
    with pytest.raises(md.MDError) as e:
        _ctx(md, integrator="gear3", nh_temperature=[300.0], nh_mass=[50.0])
    assert e.value.code == md.MD_ERR_ARG
    assert _ctx(md, integrator="gear3").workspace_bytes() > _ctx(md).workspace_bytes()


def test_barostat_validation(md):
    """The barostat's arguments and preconditions are checked on the host."""
    s = inputs.bcc_fe(6, a=2.90)
    base = dict(skin=0.3, max_neighbours=48)
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, pr_pressure_gpa=[1.0], pr_mass=[1e4], **base)
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, pr_pressure_gpa=[1.0], pr_mass=[1e4],
               nh_temperature=[300.0], nh_mass=[50.0], **base)  # NPT
    bad = [
        dict(pr_pressure_gpa=[1.0]), dict(pr_mass=[1e4]),
        dict(pr_pressure_gpa=[np.nan], pr_mass=[1e4]), dict(pr_pressure_gpa=[1.0], pr_mass=[0.0]),
        dict(pr_pressure_gpa=[1.0], pr_mass=[1e4], integrator="gear3"),
        dict(pr_pressure_gpa=[1.0], pr_mass=[1e4], nbr_mode="half"),
    ]
    for kw in bad:
        with pytest.raises(md.MDError) as e:
            md.Context(s.potential, s.atom_offset, s.box, s.periodic, **base, **kw)
        assert e.value.code == md.MD_ERR_ARG, kw
    # a free axis, and a box of fewer than three link cells with the 5% margin
    with pytest.raises(md.MDError):
        md.Context(s.potential, s.atom_offset, s.box, [[1, 1, 0]], pr_pressure_gpa=[1.0], pr_mass=[1e4], **base)
    small = inputs.bcc_fe(4, a=2.90)
    with pytest.raises(md.MDError) as e:
        md.Context(small.potential, small.atom_offset, small.box, small.periodic, pr_pressure_gpa=[1.0], pr_mass=[1e4],
                   **base)
    assert e.value.code == md.MD_ERR_BOX


def test_box_matrix_validation(md):
    """Box matrices and the external stress are checked on the host: every axis
    periodic, a positive determinant, three link cells between each pair of
    faces, a symmetric stress that comes with the barostat."""
    s = inputs.bcc_fe(7, a=2.87)
    L = s.box[0][0]
    skew = np.diag([L] * 3) @ np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])  # widths L/sqrt2, L, L
    base = dict(skin=0.3, max_neighbours=48)
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, box_matrix=skew, **base)
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, box_matrix=skew, nbr_mode="half", **base)
    stress = np.eye(3)
    stress[0, 1] = stress[1, 0] = 0.5
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, box_matrix=skew, pr_pressure_gpa=[1.0],
               pr_mass=[1e4], pr_stress_gpa=stress, **base)
    md.Context(s.potential, s.atom_offset, s.box, s.periodic, pr_pressure_gpa=[1.0], pr_mass=[1e4],
               pr_stress_gpa=stress, **base)  # full-matrix barostat from the cube
    lopsided = stress.copy()
    lopsided[0, 1] = 0.7
    cases = [
        (dict(box_matrix=skew, pr_stress_gpa=stress), md.MD_ERR_ARG),  # stress without barostat
        (dict(box_matrix=skew, pr_pressure_gpa=[1.0], pr_mass=[1e4], pr_stress_gpa=lopsided), md.MD_ERR_ARG),
        (dict(box_matrix=skew, pr_pressure_gpa=[1.0], pr_mass=[1e4], nbr_mode="half"), md.MD_ERR_ARG),
        (dict(box_matrix=skew * np.array([1.0, 1.0, -1.0])), md.MD_ERR_BOX),  # left-handed
        (dict(box_matrix=np.diag([L] * 3) @ np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])),
         md.MD_ERR_BOX),  # width L/sqrt5 = 8.99 A: two link cells
    ]
    for kw, code in cases:
        with pytest.raises(md.MDError) as e:
            md.Context(s.potential, s.atom_offset, s.box, s.periodic, **base, **kw)
        assert e.value.code == code, kw
    with pytest.raises(md.MDError) as e:
        md.Context(s.potential, s.atom_offset, s.box, [[1, 1, 0]], box_matrix=skew, **base)
    assert e.value.code == md.MD_ERR_ARG


def test_energy_ring_options(md):
    """The per-step energy ring sizes the workspace (set before md_bind); the
    schedule is for velocity-Verlet NVE runs."""
    c = _ctx(md)
    base = c.workspace_bytes()
    c.set_option(md.MD_OPT_ENERGY_RING, 1000)
    assert c.get_option(md.MD_OPT_ENERGY_RING) == 1000
    assert c.workspace_bytes() >= base + 1000 * 12 * 8 - 256
    c.set_option(md.MD_OPT_ENERGY_EVERY, 5)
    assert c.get_option(md.MD_OPT_ENERGY_EVERY) == 5
    for opt, val in ((md.MD_OPT_ENERGY_RING, -1), (md.MD_OPT_ENERGY_EVERY, -2)):
        with pytest.raises(md.MDError) as e:
            c.set_option(opt, val)
        assert e.value.code == md.MD_ERR_ARG
    nvt = _ctx(md, nh_temperature=[300.0], nh_mass=[1e4])
    with pytest.raises(md.MDError) as e:
        nvt.set_option(md.MD_OPT_ENERGY_EVERY, 1)
    assert e.value.code == md.MD_ERR_ARG


def test_neighbour_chunk_option(md):
    """The neighbour chunk of the global kernels takes 2, 4 or 8 (default 4)."""
    c = _ctx(md)
    assert c.get_option(md.MD_OPT_NEIGHBOUR_CHUNK) == 4
    for v in (2, 8, 4):
        c.set_option(md.MD_OPT_NEIGHBOUR_CHUNK, v)
        assert c.get_option(md.MD_OPT_NEIGHBOUR_CHUNK) == v
    for v in (0, 3, 16):
        with pytest.raises(md.MDError) as e:
            c.set_option(md.MD_OPT_NEIGHBOUR_CHUNK, v)
        assert e.value.code == md.MD_ERR_ARG


def test_auto_rebuild_option(md):
    """Automatic rebuilds: 0 or 1 (default 0); the global kernels then run
    whatever MD_OPT_KERNEL says; refused under the barostat."""
    c = _ctx(md)
    assert c.get_option(md.MD_OPT_AUTO_REBUILD) == 0
    c.set_option(md.MD_OPT_KERNEL, 0)
    assert c.get_option(md.MD_OPT_KERNEL) == 0
    c.set_option(md.MD_OPT_AUTO_REBUILD, 1)
    assert c.get_option(md.MD_OPT_AUTO_REBUILD) == 1
    assert c.get_option(md.MD_OPT_KERNEL) == 1
    c.set_option(md.MD_OPT_AUTO_REBUILD, 0)
    assert c.get_option(md.MD_OPT_KERNEL) == 0
    for v in (-1, 2):
        with pytest.raises(md.MDError) as e:
            c.set_option(md.MD_OPT_AUTO_REBUILD, v)
        assert e.value.code == md.MD_ERR_ARG
    s = inputs.bcc_fe(6, a=2.90)
    pr = md.Context(s.potential, s.atom_offset, s.box, s.periodic, skin=0.3, max_neighbours=48,
                    pr_pressure_gpa=[1.0], pr_mass=[1e4])
    with pytest.raises(md.MDError) as e:
        pr.set_option(md.MD_OPT_AUTO_REBUILD, 1)
    assert e.value.code == md.MD_ERR_ARG
    pr.set_option(md.MD_OPT_AUTO_REBUILD, 0)
