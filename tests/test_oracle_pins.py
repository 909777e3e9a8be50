"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form, an
invariant, a limiting case, a library routine or a finite difference, chosen so
that a dropped term, a wrong sign or index, or a transposed operand fails at
least one of them.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import pdist

from paper_1107_2619_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GPA = 160.217653


# ----------------------------------------------------------------------------- units
def test_time_unit_matches_paper(orc):
    """Paper, "Units": the derived time unit is about 1.018e-14 s."""
    t0 = orc.time_unit_fs() * 1e-15
    assert abs(t0 - 1.018e-14) < 0.0005e-14


def test_constants_shared_by_inputs_and_oracle(orc):
    # value-identical constants on the two sides (the inputs module draws velocities)
    assert orc.time_unit_fs() == pytest.approx(inputs.TIME_UNIT_FS, rel=1e-15)
    assert orc.boltzmann_ev() == inputs.KB_EV


# ----------------------------------------------------------------------------- knot evaluator
def _golden_ni_al():
    with open(os.path.join(GOLDEN, "ni_al_atvf.json")) as fh:
        return json.load(fh)


def test_knot_sum_vanishes_beyond_largest_knot(orc):
    g = _golden_ni_al()
    for r in (g["rmax"], g["rmax"] + 1e-9, 4.5, 7.0):
        v, d = orc.knot_sum(g["pair_a"], g["pair_r"], r)
        assert v == 0.0 and d == 0.0


def test_knot_sum_outermost_interval_is_single_monomial(orc):
    """Between the two largest printed knots only the outermost term is on."""
    g = _golden_ni_al()
    a, rk = np.array(g["pair_a"]), np.array(g["pair_r"])
    order = np.argsort(rk)[::-1]
    k0, k1 = order[0], order[1]
    for r in np.linspace(rk[k1] + 1e-3, rk[k0] - 1e-3, 7):
        v, _ = orc.knot_sum(a, rk, r)
        assert v / (rk[k0] - r) ** 3 == pytest.approx(a[k0], rel=1e-12)


def test_knot_sum_piecewise_cubic_third_derivative(orc):
    """On each interval the function is a cubic whose r^3 coefficient is
    -(sum of the amplitudes of the knots still switched on)."""
    g = _golden_ni_al()
    a, rk = np.array(g["pair_a"]), np.array(g["pair_r"])
    edges = np.concatenate([[1.5], np.sort(rk)])
    for lo, hi in zip(edges[:-1], edges[1:]):
        rs = np.linspace(lo + 0.01 * (hi - lo), hi - 0.01 * (hi - lo), 9)
        vs = np.array([orc.knot_sum(a, rk, r)[0] for r in rs])
        c = np.polyfit(rs, vs, 3)
        assert np.max(np.abs(np.polyval(c, rs) - vs)) < 1e-10
        active = rk > 0.5 * (lo + hi)
        assert c[0] == pytest.approx(-a[active].sum(), rel=1e-6, abs=1e-9)


def test_knot_sum_c2_at_knots_and_derivative(orc):
    """Value, slope and curvature are continuous at every knot (one-sided cubic
    fits agree there); the third derivative jumps by 6 a_k at r_k.  The
    returned derivative equals a Richardson-extrapolated central difference."""
    g = _golden_ni_al()
    a, rk = np.array(g["pair_a"]), np.array(g["pair_r"])
    f = lambda x: orc.knot_sum(a, rk, x)[0]  # noqa: E731
    edges = np.concatenate([[1.5], np.sort(rk), [5.0]])
    for q in range(1, len(edges) - 1):
        k = edges[q]
        lo, hi = edges[q - 1], edges[q + 1]
        left = np.polyfit(np.linspace(lo + 0.05 * (k - lo), k - 0.05 * (k - lo), 9),
                          [f(x) for x in np.linspace(lo + 0.05 * (k - lo), k - 0.05 * (k - lo), 9)], 3)
        right = np.polyfit(np.linspace(k + 0.05 * (hi - k), hi - 0.05 * (hi - k), 9),
                           [f(x) for x in np.linspace(k + 0.05 * (hi - k), hi - 0.05 * (hi - k), 9)], 3)
        for order in range(3):
            dl = np.polyval(np.polyder(left, order) if order else left, k)
            dr = np.polyval(np.polyder(right, order) if order else right, k)
            assert abs(dl - dr) < 1e-7 * (1 + abs(dl))
        jump = 6 * (right[0] - left[0])
        amp = a[np.argmin(np.abs(rk - k))]
        assert jump == pytest.approx(6 * amp, rel=1e-6)
    for r in (2.5, 2.86, 3.0, 3.5, 4.0, 4.3):
        h = 1e-4
        d1 = (f(r + h) - f(r - h)) / (2 * h)
        d2 = (f(r + h / 2) - f(r - h / 2)) / h
        rich = (4 * d2 - d1) / 3
        assert orc.knot_sum(a, rk, r)[1] == pytest.approx(rich, rel=1e-9, abs=1e-12)


def test_knot_sum_printed_ni_al_values(orc):
    """The printed Ni/Al pair coefficients ("Available potentials") evaluated at
    fixed radii, values worked out by hand from the printed numbers (stored in
    the fixture with their derivation)."""
    g = _golden_ni_al()
    for r, (v_ref, d_ref) in g["values"].items():
        v, d = orc.knot_sum(g["pair_a"], g["pair_r"], float(r))
        assert v == pytest.approx(v_ref, abs=2e-12), r
        assert d == pytest.approx(d_ref, abs=2e-12), r


# ----------------------------------------------------------------------------- embedding
def _with_emb_c(arr, c):
    out = dict(arr)
    out["emb_c"] = np.asarray(c, np.float64)
    return out


def test_embedding_constant_is_per_species(orc, fec_pot):
    """F_a(rho) = -c_a sqrt(rho): the constant belongs to the site atom's species
    ("Theoretical background", the Finnis-Sinclair square root)."""
    c = [1.0, 0.7]
    pot = orc.Potential(_with_emb_c(inputs.perturbed_potential("fec_eam", 1), c))
    for a in (0, 1):
        for rho in (0.25, 1.0, 3.7):
            F, dF = orc.embed(pot, a, rho)
            assert F == pytest.approx(-c[a] * math.sqrt(rho), rel=1e-15)
            assert dF == pytest.approx(-c[a] / (2.0 * math.sqrt(rho)), rel=1e-15)


def test_two_species_dimer_with_distinct_embedding(orc):
    """A 0-1 dimer in open space: E = phi_01(r) - c_0 sqrt(rho_01(r)) - c_1 sqrt(rho_10(r)),
    the embedding of each atom taken with its own constant; the bond force is the
    derivative of that sum, which a centred difference of the closed form gives."""
    c = [1.0, 0.7]
    pot = orc.Potential(_with_emb_c(inputs.perturbed_potential("fec_eam", 1), c))
    big = [100.0] * 3
    for r in (1.9, 2.3, 2.8):
        def closed(x):
            return (orc.pair(pot, 0, 1, x)[0] - c[0] * math.sqrt(orc.density(pot, 0, 1, x)[0])
                    - c[1] * math.sqrt(orc.density(pot, 1, 0, x)[0]))
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        res = orc.forces(pos, np.array([0, 1], np.uint8), big, [0, 0, 0], pot)
        assert res.pe == pytest.approx(closed(r), rel=1e-14)
        h = 1e-4
        d1 = (closed(r + h) - closed(r - h)) / (2 * h)
        d2 = (closed(r + h / 2) - closed(r - h / 2)) / h
        g = (4 * d2 - d1) / 3  # dE/dr; the force on atom 1 is -g along +x
        assert res.f[1, 0] == pytest.approx(-g, rel=1e-8)
        assert res.f[0, 0] == pytest.approx(g, rel=1e-8)
        assert res.e_atom[0] == pytest.approx(0.5 * orc.pair(pot, 0, 1, r)[0]
                                              - c[0] * math.sqrt(orc.density(pot, 0, 1, r)[0]), rel=1e-14)


# ----------------------------------------------------------------------------- lattices
def _bcc_shells(a):
    return [(a * math.sqrt(3) / 2, 8), (a, 6), (a * math.sqrt(2), 12), (a * math.sqrt(11) / 2, 24),
            (a * math.sqrt(3), 8), (2 * a, 6)]


def _fcc_shells(a):
    return [(a / math.sqrt(2), 12), (a, 6), (a * math.sqrt(1.5), 24), (a * math.sqrt(2), 12),
            (a * math.sqrt(2.5), 24), (a * math.sqrt(3), 8)]


@pytest.mark.parametrize("a", [2.75, 2.80, 2.87, 2.95, 3.02])
def test_bcc_perfect_lattice_closed_form(orc, fe_pot, a):
    """Every atom of an ideal bcc crystal has e = 1/2 sum_s n_s phi(d_s) +
    F(sum_s n_s rho(d_s)) over the neighbour shells; forces vanish by
    inversion symmetry."""
    n = 4
    pos = inputs.bcc(n, n, n, a)
    sp = np.zeros(len(pos), np.uint8)
    res = orc.forces(pos, sp, [n * a] * 3, [1, 1, 1], fe_pot)
    rho = sum(m * orc.density(fe_pot, 0, 0, d)[0] for d, m in _bcc_shells(a))
    e = 0.5 * sum(m * orc.pair(fe_pot, 0, 0, d)[0] for d, m in _bcc_shells(a)) + orc.embed(fe_pot, 0, rho)[0]
    assert np.allclose(res.rho, rho, rtol=1e-13, atol=0)
    assert np.allclose(res.e_atom, e, rtol=1e-13, atol=0)
    assert res.pe == pytest.approx(len(pos) * e, rel=1e-13)
    assert np.max(np.abs(res.f)) <= 1e-12


def test_fcc_perfect_lattice_closed_form(orc):
    pot = orc.Potential(inputs.perturbed_potential("cu_fs", 3))
    a, n = 3.615, 3
    pos = inputs.fcc(n, n, n, a)
    res = orc.forces(pos, np.zeros(len(pos), np.uint8), [n * a] * 3, [1, 1, 1], pot)
    rho = sum(m * orc.density(pot, 0, 0, d)[0] for d, m in _fcc_shells(a))
    e = 0.5 * sum(m * orc.pair(pot, 0, 0, d)[0] for d, m in _fcc_shells(a)) + orc.embed(pot, 0, rho)[0]
    assert np.allclose(res.e_atom, e, rtol=1e-13, atol=0)
    assert np.max(np.abs(res.f)) <= 1e-12


@pytest.mark.parametrize("emb_c", [None, (1.0, 0.7)])
def test_b2_two_species_closed_form(orc, fec_pot, emb_c):
    """Ordered CsCl-type crystal of species 0 at cube corners and species 1 at
    centres: the first shell of each atom is the other species, the next two
    its own.  Pins the [site, neighbour] index order of the density and the
    per-species embedding (an asymmetric EAM density, "Theoretical background"):
    with distinct constants c_a the embedding term is written out as
    -c_a sqrt(rho) from the potential's own numbers."""
    if emb_c is not None:
        fec_pot = orc.Potential(_with_emb_c(inputs.perturbed_potential("fec_eam", 1), emb_c))
    c = fec_pot.emb_c
    a, n = 2.87, 4
    corners = inputs.bcc(n, n, n, a)[0::2]
    centres = inputs.bcc(n, n, n, a)[1::2]
    pos = np.concatenate([corners, centres])
    sp = np.concatenate([np.zeros(len(corners)), np.ones(len(centres))]).astype(np.uint8)
    res = orc.forces(pos, sp, [n * a] * 3, [1, 1, 1], fec_pot)
    d1, d2, d3 = a * math.sqrt(3) / 2, a, a * math.sqrt(2)
    for s, o in ((0, 1), (1, 0)):
        rho = 8 * orc.density(fec_pot, s, o, d1)[0] + 6 * orc.density(fec_pot, s, s, d2)[0] + \
            12 * orc.density(fec_pot, s, s, d3)[0]
        e = 0.5 * (8 * orc.pair(fec_pot, s, o, d1)[0] + 6 * orc.pair(fec_pot, s, s, d2)[0] +
                   12 * orc.pair(fec_pot, s, s, d3)[0]) - c[s] * math.sqrt(rho)
        assert np.allclose(res.rho[sp == s], rho, rtol=1e-13)
        assert np.allclose(res.e_atom[sp == s], e, rtol=1e-13)
    # the two densities really differ, so a transposed index would be caught
    assert abs(orc.density(fec_pot, 0, 1, d1)[0] - orc.density(fec_pot, 1, 0, d1)[0]) > 1e-3
    assert np.max(np.abs(res.f)) <= 1e-12


# ----------------------------------------------------------------------------- forces
def _displaced_bcc(n, a, amp, rng):
    pos = inputs.bcc(n, n, n, a)
    return pos + amp * (2 * rng.random(pos.shape) - 1)


def _fd_forces(orc, pos, sp, box, per, pot, atoms, h=2e-3):
    out = np.zeros((len(atoms), 3))
    for q, i in enumerate(atoms):
        for c in range(3):
            def e_at(s):
                p = pos.copy()
                p[i, c] += s
                return orc.energy(p, sp, box, per, pot)
            d1 = (e_at(h) - e_at(-h)) / (2 * h)
            d2 = (e_at(h / 2) - e_at(-h / 2)) / h
            out[q, c] = -(4 * d2 - d1) / 3
    return out


def test_forces_are_minus_energy_gradient_fe(orc, fe_pot, rng):
    pos = _displaced_bcc(4, 2.87, 0.12, rng)
    sp = np.zeros(len(pos), np.uint8)
    box, per = [4 * 2.87] * 3, [1, 1, 1]
    res = orc.forces(pos, sp, box, per, fe_pot)
    atoms = [0, 17, 63, 127]
    fd = _fd_forces(orc, pos, sp, box, per, fe_pot, atoms)
    scale = np.sqrt(np.mean(np.sum(res.f**2, 1)))
    assert np.max(np.abs(fd - res.f[atoms])) / scale < 1e-8
    assert res.pe == pytest.approx(orc.energy(pos, sp, box, per, fe_pot), rel=1e-13)


def test_forces_are_minus_energy_gradient_two_species_free_axis(orc, fec_pot, rng):
    """Two species with asymmetric densities, one free axis."""
    pos = _displaced_bcc(4, 2.87, 0.1, rng)
    sp = (rng.random(len(pos)) < 0.3).astype(np.uint8)
    box, per = [4 * 2.87, 4 * 2.87, 4 * 2.87], [1, 1, 0]
    res = orc.forces(pos, sp, box, per, fec_pot)
    atoms = [i for i in range(len(pos)) if sp[i] == 1][:2] + [i for i in range(len(pos)) if sp[i] == 0][:2]
    fd = _fd_forces(orc, pos, sp, box, per, fec_pot, atoms)
    scale = np.sqrt(np.mean(np.sum(res.f**2, 1)))
    assert np.max(np.abs(fd - res.f[atoms])) / scale < 1e-8


def test_net_force_vanishes(orc, fec_pot, rng):
    pos = _displaced_bcc(4, 2.87, 0.15, rng)
    sp = (rng.random(len(pos)) < 0.2).astype(np.uint8)
    res = orc.forces(pos, sp, [4 * 2.87] * 3, [1, 1, 1], fec_pot)
    assert np.max(np.abs(res.f.sum(0))) < 1e-11 * np.abs(res.f).max() * len(pos)


def test_dimer(orc, fe_pot):
    """Two atoms in open space: E = phi(r) + 2 F(rho(r)), equal and opposite
    forces along the bond with magnitude |phi' + 2 F'(rho) rho'|."""
    big = [100.0, 100.0, 100.0]
    for r in (2.0, 2.4, 2.9, 3.4, 3.9):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r / math.sqrt(3)] * 3])
        sp = np.zeros(2, np.uint8)
        res = orc.forces(pos, sp, big, [0, 0, 0], fe_pot)
        rho, drho = orc.density(fe_pot, 0, 0, r)
        phi, dphi = orc.pair(fe_pot, 0, 0, r)
        F, dF = orc.embed(fe_pot, 0, rho)
        assert res.pe == pytest.approx(phi + 2 * F, rel=1e-14)
        g = dphi + 2 * dF * drho
        unit = (pos[1] - pos[0]) / r
        assert np.allclose(res.f[0], g * unit, rtol=1e-13, atol=1e-15)
        assert np.allclose(res.f[1], -g * unit, rtol=1e-13, atol=1e-15)


def test_isolated_atom_has_no_energy(orc, fe_pot):
    pos = np.array([[5.0, 5.0, 5.0], [20.0, 20.0, 20.0]])
    res = orc.forces(pos, np.zeros(2, np.uint8), [40.0] * 3, [0, 0, 0], fe_pot)
    assert res.pe == 0.0 and np.all(res.f == 0.0) and np.all(res.rho == 0.0)


def test_pair_only_limit_matches_pdist(orc, rng):
    """With F = 0 the model is a plain pair potential (paper: Morse or
    Lennard-Jones cast into the EAM form by setting F = 0): the energy is the
    sum of phi over all unordered pairs, distances from scipy's pdist."""
    arr = inputs.perturbed_potential("fe_fs", 7)
    arr["emb_c"] = np.zeros(1)
    pot = orc.Potential(arr)
    pos = rng.random((60, 3)) * 9.0 + 20.0  # a free cluster
    res = orc.forces(pos, np.zeros(60, np.uint8), [100.0] * 3, [0, 0, 0], pot)
    d = pdist(pos)
    ref = sum(orc.pair(pot, 0, 0, r)[0] for r in d)
    assert res.pe == pytest.approx(ref, rel=1e-12)


# ----------------------------------------------------------------------------- virial
def test_virial_trace_is_minus_volume_derivative(orc, fe_pot):
    """On the ideal lattice P = W/(3V) = -dE/dV (T = 0)."""
    for a in (2.80, 2.87, 2.95):
        n = 4
        pos = inputs.bcc(n, n, n, a)
        sp = np.zeros(len(pos), np.uint8)
        res = orc.forces(pos, sp, [n * a] * 3, [1, 1, 1], fe_pot)
        h = 1e-5
        e = lambda s: orc.energy(pos * (1 + s), sp, [n * a * (1 + s)] * 3, [1, 1, 1], fe_pot)  # noqa: E731
        vol = (n * a) ** 3
        dEdV = (e(h) - e(-h)) / (2 * h) / (3 * vol)
        p_virial = (res.virial[0] + res.virial[1] + res.virial[2]) / (3 * vol)
        assert p_virial == pytest.approx(-dEdV, rel=1e-7, abs=1e-10)


def test_virial_tensor_is_minus_strain_derivative_cluster(orc, fec_pot, rng):
    """For a free cluster, W_ab = -dE/d(eps_ab) under the homogeneous strain
    x -> (1 + eps) x, for all six components."""
    pos = _displaced_bcc(3, 2.87, 0.1, rng) + 30.0
    sp = (rng.random(len(pos)) < 0.25).astype(np.uint8)
    box, per = [100.0] * 3, [0, 0, 0]
    res = orc.forces(pos, sp, box, per, fec_pot)
    comps = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    h = 1e-5
    centre = pos.mean(0)
    for c, (p, q) in enumerate(comps):
        def e_at(s):
            eps = np.zeros((3, 3))
            eps[p, q] += s / (1 if p == q else 2)
            eps[q, p] += 0 if p == q else s / 2
            return orc.energy(centre + (pos - centre) @ (np.eye(3) + eps).T, sp, box, per, fec_pot)
        dE = (e_at(h) - e_at(-h)) / (2 * h)
        assert res.virial[c] == pytest.approx(-dE, rel=1e-6, abs=1e-8)


def test_virial_skips_fixed_pairs(orc, fe_pot, rng):
    """Paper, "Fixed atoms": the stress ignores forces between fixed atoms."""
    pos = _displaced_bcc(4, 2.87, 0.1, rng)
    sp = np.zeros(len(pos), np.uint8)
    rigid = np.zeros(len(pos), np.uint8)
    rigid[:40] = 1
    box = [4 * 2.87] * 3
    full = orc.forces(pos, sp, box, [1, 1, 1], fe_pot)
    part = orc.forces(pos, sp, box, [1, 1, 1], fe_pot, rigid=rigid)
    assert np.array_equal(full.f, part.f)
    assert not np.allclose(full.virial, part.virial)
    all_rigid = orc.forces(pos, sp, box, [1, 1, 1], fe_pot, rigid=np.ones(len(pos), np.uint8))
    assert np.all(all_rigid.virial == 0.0)


# ----------------------------------------------------------------------------- invariances
def test_translation_image_and_permutation_invariance(orc, fec_pot, rng):
    pos = _displaced_bcc(4, 2.87, 0.12, rng)
    sp = (rng.random(len(pos)) < 0.2).astype(np.uint8)
    L = 4 * 2.87
    box, per = [L] * 3, [1, 1, 1]
    ref = orc.forces(pos, sp, box, per, fec_pot)
    scale = np.abs(ref.f).max()
    t = orc.forces(pos + np.array([3.3, -17.1, 0.77]), sp, box, per, fec_pot)
    assert np.max(np.abs(t.f - ref.f)) < 1e-10 * scale
    assert np.allclose(t.e_atom, ref.e_atom, rtol=1e-12)
    shifted = pos.copy()
    shifted[5] += np.array([L, -2 * L, 3 * L])  # unwrapped positions
    s = orc.forces(shifted, sp, box, per, fec_pot)
    assert np.max(np.abs(s.f - ref.f)) < 1e-10 * scale
    perm = rng.permutation(len(pos))
    p = orc.forces(pos[perm], sp[perm], box, per, fec_pot)
    assert np.max(np.abs(p.f - ref.f[perm])) < 1e-12 * scale
    assert np.allclose(p.e_atom, ref.e_atom[perm], rtol=1e-13)


def test_box_too_small_is_rejected(orc, fe_pot):
    pos = inputs.bcc(2, 2, 2, 2.87)
    with pytest.raises(ValueError):
        orc.forces(pos, np.zeros(len(pos), np.uint8), [5.74] * 3, [1, 1, 1], fe_pot)


def test_sampled_mode_matches_full(orc, fec_pot, rng):
    pos = _displaced_bcc(5, 2.87, 0.1, rng)
    sp = (rng.random(len(pos)) < 0.2).astype(np.uint8)
    box, per = [5 * 2.87] * 3, [1, 1, 1]
    full = orc.forces(pos, sp, box, per, fec_pot)
    idx = rng.choice(len(pos), 20, replace=False)
    sm = orc.forces_sampled(pos, sp, box, per, fec_pot, idx)
    assert np.max(np.abs(sm.f - full.f[idx])) < 1e-12 * np.abs(full.f).max()
    assert np.allclose(sm.e_atom, full.e_atom[idx], rtol=1e-13)
    assert np.allclose(sm.rho, full.rho[idx], rtol=1e-13)


# ----------------------------------------------------------------------------- integrator
def _small_md(seed=3, n=4, T=300.0):
    return inputs.bcc_fe(n, temperature=T, seed=seed, displace=0.05, dt_fs=1.0)


def test_momentum_conserved(orc):
    s = _small_md()
    pot = orc.Potential(s.potential)
    m = s.potential["mass"][s.species]
    p0 = (m[:, None] * s.vel).sum(0)
    assert np.max(np.abs(p0)) < 1e-12
    r = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 50)
    p1 = (m[:, None] * r.vel).sum(0)
    assert np.max(np.abs(p1)) < 1e-11


def test_verlet_time_reversible(orc):
    """Velocity Verlet is time-reversible (paper, "Time integration")."""
    s = _small_md()
    pot = orc.Potential(s.potential)
    fwd = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100)
    back = orc.run_verlet(fwd.pos, -fwd.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100)
    assert np.max(np.abs(back.pos - s.pos)) < 1e-10
    assert np.max(np.abs(back.vel + s.vel)) < 1e-10


def test_verlet_second_order(orc):
    """Global error of the trajectory falls as dt^2."""
    s = _small_md(T=600.0)
    pot = orc.Potential(s.potential)
    t_end = 20.0
    ref = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 0.125, int(t_end / 0.125))
    errs = []
    for dt in (1.0, 0.5):
        r = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, dt, int(t_end / dt))
        errs.append(np.max(np.abs(r.pos - ref.pos)))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_nve_energy_bounded_without_drift(orc):
    """NVE velocity Verlet: total energy fluctuates within a bounded band with
    no secular drift (paper, "Integration error")."""
    s = _small_md(T=600.0)
    pot = orc.Potential(s.potential)
    r = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 2000)
    e = (r.pe + r.ke) / s.n_atoms
    de = e - e[0]
    assert np.max(np.abs(de)) < 2e-4
    slope = np.polyfit(np.arange(len(e)), e, 1)[0]
    assert abs(slope) * len(e) < 2e-5
    # a genuine exchange between kinetic and potential energy took place
    assert np.std(r.ke / s.n_atoms) > 50 * np.std(e)


def test_piston_work_energy_balance(orc):
    """A rigid block moving at a prescribed velocity ("Fixed atoms") does work
    W = -integral of sum_{block} f.v_p dt, and E_tot(t) - E_tot(0) = W."""
    s = inputs.fcc_piston(nx=3, ny=3, nz=6, piston_cells=1, piston_speed_a_per_fs=0.02, steps=0)
    pot = orc.Potential(s.potential)
    r = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 0.5, 400,
                       rigid=s.rigid, rigid_velocity=s.rigid_velocity[0])
    e = r.pe + r.ke
    assert abs(r.work[-1]) > 0.05  # the piston really did work
    assert np.max(np.abs(e - e[0] - r.work)) < 2e-3 * abs(r.work).max()
    zr = r.pos[s.rigid == 1, 2] - s.pos[s.rigid == 1, 2]
    assert np.allclose(zr, 400 * 0.5 * 0.02, rtol=1e-12)


def test_temperature_degrees_of_freedom(orc):
    """3N-3 degrees of freedom once momentum is fixed (paper, NVTp section);
    3N when a moving rigid block breaks momentum conservation."""
    kb = orc.boltzmann_ev()
    assert orc.temperature(0.5 * 99 * kb * 300.0, 34, False) == pytest.approx(300.0, rel=1e-14)
    assert orc.temperature(0.5 * 102 * kb * 300.0, 34, True) == pytest.approx(300.0, rel=1e-14)


# --- Nose-Hoover NVT (paper, "Thermostat NVTp") -------------------------------

def _nh_system():
    from paper_1107_2619_amd import inputs

    s = inputs.bcc_fe(4, temperature=600.0, seed=7, displace=0.02)
    return s


def test_nh_large_thermostat_mass_is_nve(orc):
    """Q -> infinity decouples the thermostat: the NVE trajectory."""
    s = _nh_system()
    pot = orc.Potential(s.potential)
    v = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100)
    n = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100, 300.0, 1e15)
    assert np.max(np.abs(v.pos - n.pos)) < 1e-9
    assert np.max(np.abs(n.pi)) < 1e-12


def test_nh_extended_energy_conserved(orc):
    """PE + KE + Q pi^2/2 + g k_B T xi is a constant of the motion: over 2000
    steps it stays within a band a thousand times narrower than the swing of
    PE + KE that the thermostat drives (600 K start, 300 K target)."""
    s = _nh_system()
    pot = orc.Potential(s.potential)
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 300.0 * 50.0**2
    r = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 2000, 300.0, q)
    h = r.pe + r.ke + r.nh_energy
    assert np.ptp(h) < 1e-3 * np.ptp(r.pe + r.ke)
    assert np.ptp(h) / s.n_atoms < 2e-5


def test_nh_fixed_point_is_the_target_temperature(orc):
    """The time-averaged temperature (2 KE / g k_B) settles at the target: the
    reading of the thermostat equation with the full kinetic term (the halved
    term as printed would settle at twice the target)."""
    s = _nh_system()
    pot = orc.Potential(s.potential)
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 300.0 * 50.0**2
    r = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 3000, 300.0, q)
    t = 2.0 * r.ke[1000:] / (g * orc.boltzmann_ev())
    assert abs(t.mean() - 300.0) < 15.0


def test_nh_time_reversible(orc):
    """Reversing velocities and the thermostat momentum retraces the path."""
    s = _nh_system()
    pot = orc.Potential(s.potential)
    q = (3 * s.n_atoms - 3) * orc.boltzmann_ev() * 300.0 * 50.0**2
    a = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100, 300.0, q)
    assert abs(a.pi[-1]) > 1e-6
    b = orc.run_nh(a.pos, -a.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100, 300.0, q, pi0=-a.pi[-1])
    assert np.max(np.abs(b.pos - s.pos)) < 1e-10
    assert np.max(np.abs(b.vel + s.vel)) < 1e-12
    assert abs(b.pi[-1]) < 1e-14


# --- Mean square displacement and diffusion ("Self-diffusion in iron") -------

def test_msd_worked_example(orc):
    """Three atoms displaced by 1, 2 and 3 A along different axes: MSD 14/3 A^2;
    split by species, (1 + 4) / 2 and 9; a rigid atom is left out."""
    p0 = np.zeros((3, 3))
    p = np.array([[1.0, 0, 0], [0, 2.0, 0], [0, 0, 3.0]])
    m, c = orc.msd(p, p0, [0, 0, 0], [0, 3], 1)
    assert m[0, 0] == pytest.approx(14.0 / 3.0, rel=1e-15) and c[0, 0] == 3
    m, c = orc.msd(p, p0, [0, 0, 1], [0, 3], 2)
    assert m[0].tolist() == [2.5, 9.0] and c[0].tolist() == [2, 1]
    m, c = orc.msd(p, p0, [0, 0, 0], [0, 3], 2, rigid=[0, 1, 0])
    assert m[0].tolist() == [5.0, 0.0] and c[0].tolist() == [2, 0]


def test_msd_uniform_translation_and_permutation(orc, rng):
    """A rigid translation d of every atom gives |d|^2 in every replica and
    species; reordering atoms inside a replica changes nothing."""
    n = 300
    p0 = rng.uniform(0, 20, (n, 3))
    sp = rng.integers(0, 2, n)
    off = [0, 100, 100, 300]
    d = np.array([0.3, -1.7, 2.2])
    m, c = orc.msd(p0 + d, p0, sp, off, 2)
    nonempty = c > 0
    assert np.allclose(m[nonempty], d @ d, rtol=1e-14) and np.all(m[~nonempty] == 0.0)
    assert c[1].sum() == 0
    p = p0 + rng.normal(0, 0.5, (n, 3))
    perm = np.concatenate([rng.permutation(100), 100 + rng.permutation(200)])
    m1, _ = orc.msd(p, p0, sp, off, 2)
    m2, _ = orc.msd(p[perm], p0[perm], sp[perm], off, 2)
    assert np.allclose(m1, m2, rtol=1e-13)


def test_msd_ballistic_across_periodic_boundaries(orc):
    """Isolated atoms (beyond the cutoff of each other) fly in straight lines
    through the periodic box several times: the oracle's trajectory stays
    unwrapped, so the MSD is |v|^2 t^2."""
    from paper_1107_2619_amd import inputs

    pot = orc.Potential(inputs.perturbed_potential("fe_fs", 1))
    g = np.arange(4) * 7.0 + 1.0
    pos = np.array([[x, y, z] for x in g for y in g for z in g])
    v = np.array([0.031, -0.017, 0.024])
    vel = np.tile(v, (len(pos), 1))
    r = orc.run_verlet(pos, vel, np.zeros(len(pos), np.uint8), [28.0] * 3, [1, 1, 1], pot, 1.0, 2000)
    m, _ = orc.msd(r.pos, pos, np.zeros(len(pos)), [0, len(pos)], 1)
    assert np.max(np.abs(r.pos - pos)) > 2 * 28.0
    assert m[0, 0] == pytest.approx((v @ v) * 2000.0**2, rel=1e-12)


def test_diffusion_of_a_random_walk(orc):
    """Gaussian random walks with per-axis step variance s^2 per dt have
    MSD(n) = 3 n s^2, so D = s^2 / (2 dt); the estimate from 4000 seeded
    walkers over 400 steps lands within 3%."""
    rng = np.random.default_rng(77)
    s, dt, n_w, n_t = 0.1, 2.0, 4000, 400
    steps = rng.normal(0.0, s, (n_t, n_w, 3))
    paths = np.cumsum(steps, 0)
    t = dt * np.arange(1, n_t + 1)
    msd_t = np.array([orc.msd(paths[k], np.zeros((n_w, 3)), np.zeros(n_w), [0, n_w], 1)[0][0, 0]
                      for k in range(0, n_t, 20)])
    d = orc.diffusion_coefficient(t[::20], msd_t)
    assert d == pytest.approx(s * s / (2 * dt), rel=0.03)


# --- Third-order Gear predictor-corrector ("Time integration") ----------------

def _dimer_reference(orc, pot, mass, r0, w0, times):
    """Separation of a free dimer by an independent high-order integrator
    (scipy's DOP853 at tight tolerance) on the oracle's pinned forces."""
    from scipy.integrate import solve_ivp

    box, per = [50.0] * 3, [0, 0, 0]
    conv = 1.0 / orc.time_unit_fs() ** 2  # (eV/A)/amu -> A/fs^2

    def rhs(_t, y):
        f = orc.forces(np.array([[10.0, 10, 10], [10.0 + y[0], 10, 10]]), [0, 0], box, per, pot).f
        return [y[1], 2.0 * f[1, 0] / mass * conv]

    return solve_ivp(rhs, (0.0, max(times)), [r0, w0], method="DOP853", rtol=1e-13, atol=1e-14,
                     t_eval=times).y[0]


def test_gear_dimer_converges_and_beats_verlet(orc):
    """The paper prefers the predictor-corrector for trajectory accuracy: on a
    vibrating dimer its separation error at 1, 0.5 and 0.25 fs is a fraction of
    velocity Verlet's and shrinks with the step."""
    from paper_1107_2619_amd import inputs

    raw = inputs.perturbed_potential("fe_fs", 1)
    pot = orc.Potential(raw)
    r0, w0 = 2.3, 0.004
    times = [40.0, 80.0, 120.0, 160.0, 200.0]
    ref = _dimer_reference(orc, pot, raw["mass"][0], r0, w0, times)
    pos = np.array([[10.0, 10, 10], [10.0 + r0, 10, 10]])
    vel = np.array([[-w0 / 2, 0, 0], [w0 / 2, 0, 0]])
    errs = {}
    for dt in (1.0, 0.5, 0.25):
        eg = ev = 0.0
        for t, rr in zip(times, ref):
            n = int(round(t / dt))
            g = orc.run_gear(pos, vel, [0, 0], [50.0] * 3, [0, 0, 0], pot, dt, n)
            v = orc.run_verlet(pos, vel, [0, 0], [50.0] * 3, [0, 0, 0], pot, dt, n)
            eg = max(eg, abs(g.pos[1, 0] - g.pos[0, 0] - rr))
            ev = max(ev, abs(v.pos[1, 0] - v.pos[0, 0] - rr))
        errs[dt] = eg
        assert eg < 0.2 * ev
    assert errs[1.0] < 3e-5 and errs[0.5] < 0.5 * errs[1.0] and errs[0.25] < 0.5 * errs[0.5]


def test_gear_free_flight_is_exact(orc):
    """Atoms out of each other's range move on straight lines."""
    from paper_1107_2619_amd import inputs

    pot = orc.Potential(inputs.perturbed_potential("fe_fs", 1))
    g = np.arange(3) * 9.0 + 1.0
    pos = np.array([[x, y, z] for x in g for y in g for z in g])
    rng = np.random.default_rng(5)
    vel = rng.normal(0, 0.002, (1, 3)).repeat(len(pos), 0)
    r = orc.run_gear(pos, vel, np.zeros(len(pos)), [27.0] * 3, [1, 1, 1], pot, 1.0, 300)
    assert np.allclose(r.pos, pos + 300.0 * vel, rtol=0, atol=1e-11)
    assert np.allclose(r.vel, vel, rtol=0, atol=1e-15)
    assert np.all(r.pe == 0.0)


def test_gear_piston_work_energy_balance(orc):
    """The rigid block's work (trapezoid rule over the force evaluations)
    balances the mobile atoms' energy change, as for Verlet."""
    from paper_1107_2619_amd import inputs

    s = inputs.fcc_piston(nx=3, ny=3, nz=6, piston_cells=1, piston_speed_a_per_fs=0.02, steps=0)
    pot = orc.Potential(s.potential)
    r = orc.run_gear(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 0.5, 400,
                     rigid=s.rigid, rigid_velocity=s.rigid_velocity[0])
    e = r.pe + r.ke
    assert abs(r.work[-1]) > 0.05
    assert np.max(np.abs(e - e[0] - r.work)) < 5e-4 * abs(r.work).max()
    zr = r.pos[s.rigid == 1, 2] - s.pos[s.rigid == 1, 2]
    assert np.allclose(zr, 400 * 0.5 * 0.02, rtol=1e-12)


def test_gear_energy_drifts_linearly(orc):
    """In NVE the predictor-corrector's energy drifts linearly with the number
    of steps ("Integration error"), where Verlet's stays bounded: the drift
    rates over two halves of 8000 steps agree, and exceed Verlet's rate by far."""
    s = _nh_system()
    pot = orc.Potential(s.potential)
    g = orc.run_gear(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 8000)
    v = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 8000)
    t = np.arange(8001)
    eg, ev = g.pe + g.ke, v.pe + v.ke
    s1 = np.polyfit(t[:4000], eg[:4000], 1)[0]
    s2 = np.polyfit(t[4000:], eg[4000:], 1)[0]
    sv = np.polyfit(t, ev, 1)[0]
    assert abs(s1 - s2) < 0.2 * abs(s1)
    assert abs(s1) > 5.0 * abs(sv)


# --- Parrinello-Rahman barostat, orthorhombic box ("Barostat NPTp") ----------

def _pr_system():
    from paper_1107_2619_amd import inputs

    return inputs.bcc_fe(4, a=2.90, temperature=600.0, seed=7, displace=0.02)


def test_pr_infinite_box_mass_is_nve(orc):
    """W -> infinity freezes the box: the NVE trajectory."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    v = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 200)
    r = orc.run_pr(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 200, 0.0, 1e30)
    assert np.max(np.abs(v.pos - r.pos)) < 1e-10
    assert np.all(r.box == s.box[0])


def test_pr_cold_lattice_box_against_independent_integrator(orc):
    """A perfect lattice at rest stays a scaled lattice, so the box alone obeys
    W d2L/dt2 = (Omega / L)(pi(L) - P) with pi from the (pinned) virial: scipy's
    DOP853 integrates that equation independently.  The barostat run follows it
    with second-order error in the step, and all three edges stay equal."""
    from scipy.integrate import solve_ivp

    from paper_1107_2619_amd import inputs

    lat = inputs.bcc_fe(4, a=2.90, temperature=0.0, seed=7)
    pot = orc.Potential(lat.potential)
    L0, w = lat.box[0][0], 1e4
    conv = orc.pressure_unit_gpa()
    p_ext = 1.5  # GPa

    def rhs(_t, y):
        vir = orc.forces(lat.pos * (y[0] / L0), lat.species, [y[0]] * 3, [1, 1, 1], pot).virial
        return [y[1], y[0] ** 2 * (vir[0] / y[0] ** 3 - p_ext / conv) / w]

    times = [100.0, 200.0, 300.0, 400.0]
    ref = solve_ivp(rhs, (0.0, 400.0), [L0, 0.0], method="DOP853", rtol=1e-12, atol=1e-13, t_eval=times).y[0]
    assert np.ptp(ref) > 0.2  # the box really moves
    errs = []
    for dt in (1.0, 0.5):
        e = 0.0
        for t, rr in zip(times, ref):
            r = orc.run_pr(lat.pos, np.zeros_like(lat.pos), lat.species, lat.box[0], pot, dt, int(t / dt), p_ext, w)
            assert np.ptp(r.box[-1]) < 1e-9
            e = max(e, abs(r.box[-1, 0] - rr))
        errs.append(e)
    assert errs[0] < 1e-3 and 3.0 < errs[0] / errs[1] < 5.0


def test_pr_conserved_quantity(orc):
    """PE + KE + P Omega + W |dL/dt|^2 / 2 stays within a band a thousand times
    narrower than the swing of PE + KE, and the band shrinks as dt^2."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    bands = []
    for dt in (1.0, 0.5):
        r = orc.run_pr(s.pos, s.vel, s.species, s.box[0], pot, dt, int(2000 / dt), 0.0, 1e4)
        h = r.pe + r.ke + r.baro
        bands.append(np.ptp(h))
        assert np.ptp(h) < 2e-3 * np.ptp(r.pe + r.ke)
    assert bands[1] < 0.35 * bands[0]


def test_pr_mean_pressure_is_the_target(orc):
    """The box settles where the time-averaged internal pressure equals the
    external one (a sign error in the box force would run away instead)."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    for p_ext in (0.0, 5.0):
        r = orc.run_pr(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 6000, p_ext, 1e4)
        assert abs(r.pressure[2000:].mean() - p_ext) < 0.15


def test_pr_time_reversible(orc):
    """Reversing the velocities and the box velocity retraces the path."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    a = orc.run_pr(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 200, 0.0, 1e4)
    assert np.max(np.abs(a.ldot[-1])) > 1e-5
    b = orc.run_pr(a.pos, -a.vel, s.species, a.box[-1], pot, 1.0, 200, 0.0, 1e4, ldot0=-a.ldot[-1])
    assert np.max(np.abs(b.pos - s.pos)) < 1e-10
    assert np.max(np.abs(b.box[-1] - s.box[0])) < 1e-11
    assert np.max(np.abs(b.ldot[-1])) < 1e-13


# --- Barostat with thermostat (NPT, "Barostat NPTp") --------------------------

def test_npt_limits_are_nph_and_nvt(orc):
    """Q -> infinity gives the barostat alone, W -> infinity the thermostat
    alone, trajectory for trajectory."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 500.0 * 50.0**2
    a = orc.run_npt(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 200, 1.0, 1e4, 500.0, 1e30)
    b = orc.run_pr(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 200, 1.0, 1e4)
    assert np.max(np.abs(a.pos - b.pos)) < 1e-10 and np.max(np.abs(a.box - b.box)) < 1e-12
    c = orc.run_npt(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 200, 1.0, 1e30, 500.0, q)
    d = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 200, 500.0, q)
    assert np.max(np.abs(c.pos - d.pos)) < 1e-10 and abs(c.pi[-1] - d.pi[-1]) < 1e-14


def test_npt_conserved_quantity_and_averages(orc):
    """PE + KE + barostat and thermostat energies stay within a band a
    thousand times narrower than the swing of PE + KE; the time-averaged
    pressure and temperature settle at their targets."""
    s = _pr_system()
    pot = orc.Potential(s.potential)
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 500.0 * 50.0**2
    r = orc.run_npt(s.pos, s.vel, s.species, s.box[0], pot, 1.0, 6000, 2.0, 1e4, 500.0, q)
    h = r.pe + r.ke + r.baro + r.nh_energy
    assert np.ptp(h) < 2e-3 * np.ptp(r.pe + r.ke)
    assert abs(r.pressure[2000:].mean() - 2.0) < 0.15
    t = 2.0 * r.ke[2000:] / (g * orc.boltzmann_ev())
    assert abs(t.mean() - 500.0) < 15.0


# --- Box matrix: sheared cells and Parrinello-Rahman with nine box degrees of
# freedom ("Barostat NPTp") ----------------------------------------------------

_UNIMODULAR = np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])  # c' = c + a


def _skewed_crystal(n=7, temperature=300.0, displace=0.02):
    """A bcc crystal of n^3 cells described by the cell [a, b, c + a]: the same
    periodic system as the cube, in a cell whose edges are not orthogonal."""
    s = inputs.bcc_fe(n, a=2.87, temperature=temperature, seed=7, displace=displace)
    return s, np.diag(s.box[0]) @ _UNIMODULAR


def test_sheared_cell_equals_cube(orc, fec_pot, rng):
    """A cell spanning the same lattice of images gives the cube's forces,
    energies and virial."""
    s = inputs.bcc_fe(6, a=2.87, temperature=0.0, seed=7, displace=0.08)
    sp = (rng.random(s.n_atoms) < 0.2).astype(np.uint8)
    ref = orc.forces(s.pos, sp, s.box[0], [1, 1, 1], fec_pot)
    for u in (_UNIMODULAR, _UNIMODULAR.T):
        t = orc.forces_tri(s.pos, sp, np.diag(s.box[0]) @ u, fec_pot)
        assert np.max(np.abs(t.f - ref.f)) < 1e-12
        assert np.max(np.abs(t.e_atom - ref.e_atom)) < 1e-12
        assert np.max(np.abs(t.virial - ref.virial)) < 1e-10


def test_sheared_cell_rotation_covariance(orc, fe_pot, rng):
    """Rotating atoms and cell together rotates the forces and the virial
    tensor and leaves every per-atom energy unchanged."""
    s, h = _skewed_crystal(6, 0.0, 0.08)
    ref = orc.forces_tri(s.pos, s.species, h, fe_pot)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    t = orc.forces_tri(s.pos @ q.T, s.species, q @ h, fe_pot)
    scale = np.abs(ref.f).max()
    assert np.max(np.abs(t.f - ref.f @ q.T)) < 1e-12 * scale * 100
    assert np.max(np.abs(t.e_atom - ref.e_atom)) < 1e-12
    w = lambda v: np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])  # noqa: E731
    assert np.max(np.abs(w(t.virial) - q @ w(ref.virial) @ q.T)) < 1e-9


def test_sheared_cell_shortest_image_by_enumeration(orc, fec_pot):
    """Against a plain enumeration of the periodic images (-2..2 lattice
    vectors per edge) in a strongly sheared cell: every pair in range, the
    densities, energies and forces."""
    h = np.array([[9.2, 3.1, 2.4], [0.4, 9.6, -2.7], [-0.6, 0.9, 10.1]])
    gen = np.random.default_rng(5)
    frac = gen.random((24, 3))
    pos = frac @ h.T + gen.normal(scale=0.3, size=(24, 3))
    sp = (gen.random(24) < 0.3).astype(np.uint8)
    res = orc.forces_tri(pos, sp, h, fec_pot)
    rc = orc.cutoff(fec_pot)
    shifts = np.array([[i, j, k] for i in range(-2, 3) for j in range(-2, 3) for k in range(-2, 3)]) @ h.T
    n = len(pos)
    pairs = []
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = pos[j] + shifts - pos[i]
            r = np.sqrt((d * d).sum(1))
            hit = np.nonzero(r < rc)[0]
            assert len(hit) <= 1
            for k in hit:
                pairs.append((i, j, d[k], r[k]))
    rho = np.zeros(n)
    for i, j, d, r in pairs:
        rho[i] += orc.density(fec_pot, sp[i], sp[j], r)[0]
    dF = np.array([orc.embed(fec_pot, sp[i], rho[i])[1] for i in range(n)])
    e = np.array([orc.embed(fec_pot, sp[i], rho[i])[0] for i in range(n)])
    f = np.zeros((n, 3))
    for i, j, d, r in pairs:
        phi, dphi = orc.pair(fec_pot, sp[i], sp[j], r)
        g = dphi + dF[i] * orc.density(fec_pot, sp[i], sp[j], r)[1] + dF[j] * orc.density(fec_pot, sp[j], sp[i], r)[1]
        f[i] += g * d / r
        e[i] += 0.5 * phi
    assert len(pairs) > 100
    assert np.allclose(res.rho, rho, rtol=1e-13, atol=1e-14)
    assert np.allclose(res.e_atom, e, rtol=1e-12, atol=1e-13)
    assert np.max(np.abs(res.f - f)) < 1e-12


def test_virial_tensor_is_box_derivative(orc, fec_pot, rng):
    """-dU/dh at fixed fractional coordinates equals W h^-T (the virial tensor
    times the inverse transposed cell), all nine components of a sheared
    cell: the driving term of the box equation."""
    s = inputs.bcc_fe(4, a=2.87, temperature=0.0, seed=7, displace=0.1)
    h = np.diag(s.box[0]) @ np.array([[1.0, 0.05, 0.03], [0.0, 1.0, 0.04], [0.0, 0.0, 1.0]])
    pos = s.pos @ (h @ np.diag(1.0 / s.box[0])).T
    sp = (rng.random(s.n_atoms) < 0.25).astype(np.uint8)
    res = orc.forces_tri(pos, sp, h, fec_pot)
    v = res.virial
    w = np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]])
    want = w @ np.linalg.inv(h).T
    frac = pos @ np.linalg.inv(h).T

    def u(dh):
        hh = h + dh
        return orc.forces_tri(frac @ hh.T, sp, hh, fec_pot).pe

    step = 1e-4
    got = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = 1.0
            d1 = (u(step * e) - u(-step * e)) / (2 * step)
            d2 = (u(0.5 * step * e) - u(-0.5 * step * e)) / step
            got[a, b] = -(4 * d2 - d1) / 3
    assert np.abs(want).max() > 1.0 and abs(want[0, 1]) > 0.1
    assert np.max(np.abs(got - want)) < 1e-6 * np.abs(want).max()


def test_sheared_fixed_cell_is_the_cube_run(orc):
    """With the box held (W = 0) the run in the sheared cell is the velocity
    Verlet run of the cube, step for step."""
    s, h = _skewed_crystal(6)
    pot = orc.Potential(s.potential)
    a = orc.run_verlet(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 60)
    b = orc.run_prt(s.pos, s.vel, s.species, h, pot, 1.0, 60)
    assert np.max(np.abs(a.pos - b.pos)) < 1e-12
    assert np.max(np.abs(a.pe - b.pe)) < 1e-9
    assert np.all(b.h == h)


def test_prt_cold_lattice_box_against_independent_integrator(orc):
    """A strained perfect lattice at rest stays a lattice, so the box alone
    obeys W h'' = (pi(h) - P) Omega h^-T - h Sigma with pi from the (pinned)
    virial tensor: scipy's DOP853 integrates those nine equations
    independently, under pressure and a deviatoric stress.  The run follows it
    with second-order error in the step."""
    from scipy.integrate import solve_ivp

    lat = inputs.bcc_fe(4, a=2.90, temperature=0.0, seed=7)
    pot = orc.Potential(lat.potential)
    h0 = np.diag(lat.box[0]) @ np.array([[1.0, 0.05, 0.03], [0.0, 1.0, 0.04], [0.0, 0.0, 1.0]])
    frac = lat.pos @ np.diag(1.0 / lat.box[0])
    w, conv, p_ext = 1e4, orc.pressure_unit_gpa(), 1.0
    stress = p_ext * np.eye(3) + np.array([[0.3, 0.8, 0.0], [0.8, -0.2, -0.5], [0.0, -0.5, 0.0]])
    om0 = abs(np.linalg.det(h0))
    sig = om0 * np.linalg.inv(h0) @ ((stress - p_ext * np.eye(3)) / conv) @ np.linalg.inv(h0).T

    def rhs(_t, y):
        h, hd = y[:9].reshape(3, 3), y[9:]
        v = orc.forces_tri(frac @ h.T, lat.species, h, pot).virial
        om = abs(np.linalg.det(h))
        pi = np.array([[v[0], v[3], v[4]], [v[3], v[1], v[5]], [v[4], v[5], v[2]]]) / om
        acc = ((pi - p_ext / conv * np.eye(3)) @ (om * np.linalg.inv(h).T) - h @ sig) / w
        return np.concatenate([hd, acc.reshape(9)])

    times = [100.0, 200.0, 300.0]
    ref = solve_ivp(rhs, (0.0, 300.0), np.concatenate([h0.reshape(9), np.zeros(9)]), method="DOP853",
                    rtol=1e-11, atol=1e-12, t_eval=times).y[:9].T.reshape(-1, 3, 3)
    assert np.ptp(ref[:, 0, 1]) > 0.05  # the shear really moves
    errs = []
    for dt in (1.0, 0.5):
        e = 0.0
        for t, rr in zip(times, ref):
            r = orc.run_prt(lat.pos @ (h0 @ np.diag(1.0 / lat.box[0])).T, np.zeros_like(lat.pos), lat.species, h0,
                            pot, dt, int(t / dt), p_ext, w, stress_gpa=stress)
            e = max(e, np.abs(r.h[-1] - rr).max())
        errs.append(e)
    assert errs[0] < 1e-2 and 3.0 < errs[0] / errs[1] < 5.0


def _prt_stress():
    s = 1.0 * np.eye(3)
    s[0, 1] = s[1, 0] = 0.5
    s[1, 2] = s[2, 1] = -0.3
    return s


def test_prt_conserved_quantity(orc):
    """PE + KE + P Omega + W tr(h'^T h')/2 + Omega0 tr((S - P) eps) stays in a
    band a thousand times narrower than the swing of PE + KE in a sheared cell
    under shear stress, and the band shrinks as dt^2."""
    s, h = _skewed_crystal()
    pot = orc.Potential(s.potential)
    bands = []
    for dt in (1.0, 0.5):
        r = orc.run_prt(s.pos, s.vel, s.species, h, pot, dt, int(1000 / dt), 1.0, 3e4, stress_gpa=_prt_stress())
        tot = r.pe + r.ke + r.baro
        bands.append(np.ptp(tot))
        assert np.ptp(tot) < 2e-3 * np.ptp(r.pe + r.ke)
        assert np.abs(r.h[-1] - h).max() > 0.1  # the cell really deforms
    assert bands[1] < 0.35 * bands[0]


def test_prt_mean_stress_balances_the_load(orc):
    """The cell settles where the time-averaged internal stress equals the
    load carried to the current cell, P + (Omega0 / Omega) F (S - P) F^T with
    F = h h0^-1 (the box equation at rest); a sign or transposition error in
    the stress term would not settle there."""
    s, h0 = _skewed_crystal()
    pot = orc.Potential(s.potential)
    stress = _prt_stress()
    r = orc.run_prt(s.pos, s.vel, s.species, h0, pot, 1.0, 3000, 1.0, 3e4, stress_gpa=stress)
    st = r.stress[1000:].mean(0)
    pi = np.array([[st[0], st[3], st[4]], [st[3], st[1], st[5]], [st[4], st[5], st[2]]])
    hm = r.h[1000:].mean(0)
    f = hm @ np.linalg.inv(h0)
    load = np.eye(3) + abs(np.linalg.det(h0)) / abs(np.linalg.det(hm)) * f @ (stress - np.eye(3)) @ f.T
    assert np.max(np.abs(pi - load)) < 0.05
    assert abs(pi[0, 1] - 0.5) < 0.1 and abs(pi[1, 2] + 0.3) < 0.1


def test_prt_time_reversible(orc):
    """Reversing the velocities and the box velocity (same reference cell for
    the strain) retraces the path."""
    s, h = _skewed_crystal(6)
    pot = orc.Potential(s.potential)
    a = orc.run_prt(s.pos, s.vel, s.species, h, pot, 1.0, 150, 1.0, 1e4, stress_gpa=_prt_stress())
    assert np.max(np.abs(a.hdot[-1])) > 1e-4
    b = orc.run_prt(a.pos, -a.vel, s.species, a.h[-1], pot, 1.0, 150, 1.0, 1e4, stress_gpa=_prt_stress(),
                    hdot0=-a.hdot[-1], h_ref=h)
    assert np.max(np.abs(b.pos - s.pos)) < 1e-9
    assert np.max(np.abs(b.h[-1] - h)) < 1e-11
    assert np.max(np.abs(b.hdot[-1])) < 1e-13
    assert abs(b.baro[-1] - a.baro[0]) < 1e-9


def test_prt_with_thermostat_limits(orc):
    """Q -> infinity gives the barostat alone; W -> infinity the thermostat
    alone in the fixed sheared cell, which is the cube's thermostat run."""
    s, h = _skewed_crystal(6)
    pot = orc.Potential(s.potential)
    g = 3 * s.n_atoms - 3
    q = g * orc.boltzmann_ev() * 500.0 * 50.0**2
    a = orc.run_prt(s.pos, s.vel, s.species, h, pot, 1.0, 100, 1.0, 1e4, stress_gpa=_prt_stress(), t_target=500.0,
                    q_ev_fs2=1e30)
    b = orc.run_prt(s.pos, s.vel, s.species, h, pot, 1.0, 100, 1.0, 1e4, stress_gpa=_prt_stress())
    assert np.max(np.abs(a.pos - b.pos)) < 1e-10 and np.max(np.abs(a.h - b.h)) < 1e-12
    c = orc.run_prt(s.pos, s.vel, s.species, h, pot, 1.0, 100, 0.0, 0.0, t_target=500.0, q_ev_fs2=q)
    d = orc.run_nh(s.pos, s.vel, s.species, s.box[0], s.periodic[0], pot, 1.0, 100, 500.0, q)
    assert np.max(np.abs(c.pos - d.pos)) < 1e-10 and abs(c.pi[-1] - d.pi[-1]) < 1e-14


def test_sheared_sampled_mode_matches_full(orc, fec_pot, rng):
    """The sampled evaluation in a sheared cell gives the full evaluation's
    rows for the sampled atoms (a strained crystal, two species)."""
    s = inputs.bcc_fe(6, a=2.87, temperature=0.0, seed=7, displace=0.1)
    f = np.array([[1.0, 0.04, -0.03], [0.02, 0.99, 0.05], [-0.04, 0.03, 1.01]])
    h = f @ np.diag(s.box[0])
    pos = s.pos @ f.T
    sp = (rng.random(s.n_atoms) < 0.2).astype(np.uint8)
    full = orc.forces_tri(pos, sp, h, fec_pot)
    sample = rng.choice(s.n_atoms, 40, replace=False)
    part = orc.forces_sampled_tri(pos, sp, h, fec_pot, sample)
    assert np.max(np.abs(part.f - full.f[sample])) < 1e-12
    assert np.max(np.abs(part.e_atom - full.e_atom[sample])) < 1e-12
    assert np.max(np.abs(part.rho - full.rho[sample])) < 1e-13
