"""Pins of the 1D oracle against the paper and the mathematics (CPU)."""
import json
import os

import numpy as np
import pytest

import tninputs
from oracle import gates, imps
from tests import pins

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# --- gates (Sec. V A, Eq. (iMPO1)) ------------------------------------------

def test_interaction_split_closed_form():
    # exp(d sz sz) = cosh d I I + sinh d sz sz: the SVD split must be exactly that
    d = 0.01
    L, R = gates.split_interaction(1.0, d)
    assert L.shape[0] == 2
    np.testing.assert_allclose(L[0], np.sqrt(np.cosh(d)) * np.eye(2), atol=1e-15)
    np.testing.assert_allclose(L[1], np.sqrt(np.sinh(d)) * pins.SZ, atol=1e-15)
    np.testing.assert_allclose(R, L, atol=1e-15)


def test_impo_ring_equals_trotter_product():
    # contract the iMPO on a 6-site ring and compare with the dense gate product
    n, J, h, dt = 6, 1.0, 0.7, 0.13
    g = gates.impo(J, h, dt)                       # [a][b][s][s']
    # ring contraction: operator[s1..sn, s1'..sn'] = Tr_kappa prod g
    op = g.transpose(0, 2, 3, 1)                   # [a][s][s'][b]
    acc = op
    for _ in range(n - 1):
        acc = np.einsum("a...b,bstc->a...stc", acc, op)
    acc = np.einsum("a...a->...", acc)             # trace over the closing kappa bond
    perm = [2 * i for i in range(n)] + [2 * i + 1 for i in range(n)]
    dense = acc.transpose(perm).reshape(2 ** n, 2 ** n)
    bonds = [(i, (i + 1) % n) for i in range(n)]
    ref = pins.trotter_product(n, bonds, h, dt, J)
    np.testing.assert_allclose(dense, ref, atol=1e-13)


def test_trotter_error_is_third_order():
    n, h = 8, 1.0
    bonds = [(i, (i + 1) % n) for i in range(n)]
    H = pins.tfim_hamiltonian(n, bonds, h)
    from scipy.linalg import expm
    errs = []
    for dt in (0.04, 0.02):
        errs.append(np.linalg.norm(pins.trotter_product(n, bonds, h, dt) - expm(-dt * H), 2))
    ratio = errs[0] / errs[1]
    assert 7.0 < ratio < 9.0


# --- transfer-matrix fixed points (Sec. III A, Eq. (iMPSDM1)) ----------------

def _dense_tm(kets, bras):
    n = kets[0].shape[0]
    E = np.eye(n * n)
    for k, b in zip(kets, bras):
        e = np.zeros((n * n, n * n))
        for a in range(n):
            for a2 in range(n):
                for c in range(n):
                    for c2 in range(n):
                        e[a * n + a2, c * n + c2] = sum(k[a, s, c] * b[a2, s, c2]
                                                        for s in range(k.shape[1]))
        E = E @ e
    return E


@pytest.mark.parametrize("mixed", [False, True])
def test_tm_fixed_point_brute_force(mixed):
    rng = np.random.default_rng(3)
    kets = [rng.standard_normal((3, 2, 3)) for _ in range(2)]
    bras = [rng.standard_normal((3, 2, 3)) for _ in range(2)] if mixed else kets
    try:
        vl, vr, eta = imps.tm_fixed_point(kets, bras)
    except ValueError:
        pytest.skip("complex dominant eigenvalue for this seed")
    E = _dense_tm(kets, bras)
    w, v = np.linalg.eig(E)
    i = int(np.argmax(np.abs(w)))
    assert abs(eta - w[i].real) < 1e-12 * abs(w[i])
    # left: x E = eta x ; right: E y = eta y
    np.testing.assert_allclose(vl.ravel() @ E, eta * vl.ravel(), atol=1e-12)
    np.testing.assert_allclose(E @ vr.ravel(), eta * vr.ravel(), atol=1e-11)
    assert abs(np.sum(vl * vr) - 1) < 1e-12


def _canonical_state(seed=0, chi=8):
    ga, _, gb, _ = tninputs.imps_two_site(seed, chi)
    sites, _ = imps.run_itebd([ga, gb], 1.0, 1.0, 0.05, chi, 30)
    return sites


def test_canonical_form_constraints_and_tm_route():
    # the paper's local iteration reaches the canonical constraints, and its
    # Schmidt values agree with the transfer-matrix route (Orus-Vidal)
    sites = _canonical_state()
    a1, lam, Qc, Pc = imps.canonicalize_a_form(sites)
    gams = imps.to_gamma_lambda(a1, lam)
    assert imps.canonical_residual(gams, lam) < 1e-10
    for b in (0, 1):
        vl, vr = imps.bond_fixed_points(sites, b)
        _, _, s = imps.truncation_pq(vl, vr, sites[0].shape[0])
        np.testing.assert_allclose(np.sort(lam[b])[::-1], s / np.linalg.norm(s), atol=1e-10)
    # A1 = Qc A Pc represents the same state: same energy
    assert abs(imps.energy_per_site(a1, 1.0, 1.0) - imps.energy_per_site(sites, 1.0, 1.0)) < 1e-12


def test_canonical_fixed_points_are_lambda():
    # in the A form a canonical iMPS has both TM fixed points equal to lambda
    sites = _canonical_state()
    a1, lam, _, _ = imps.canonicalize_a_form(sites)
    vl, vr = imps.bond_fixed_points(a1, 0)
    d = np.diag(lam[0])
    np.testing.assert_allclose(vl / np.trace(vl), d / np.trace(d), atol=1e-10)
    np.testing.assert_allclose(vr / np.trace(vr), d / np.trace(d), atol=1e-10)


def _rand_orth(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def _gauged(a, V):
    # site 0 sits between bond 1 (left) and bond 0 (right)
    return [np.einsum("ia,asb,jb->isj", V[1], a[0], V[0]),
            np.einsum("ia,asb,jb->isj", V[0], a[1], V[1])]


def test_gauge_fix_direct_known_answer():
    rng = np.random.default_rng(11)
    a, _, _, _ = imps.canonicalize_a_form(_canonical_state())
    V = [_rand_orth(rng, 8), _rand_orth(rng, 8)]
    U, F = imps.gauge_fix_direct(a, _gauged(a, V))
    assert abs(F - 1) < 1e-12
    # (U0, U1) and (-U0, -U1) are the same gauge on a two-site cell
    sgn = np.sign(np.sum(U[0] * V[0]))
    for b in (0, 1):
        np.testing.assert_allclose(sgn * U[b], V[b], atol=1e-9)


def test_gauge_fix_iterative_converges_to_known_answer():
    rng = np.random.default_rng(12)
    a, _, _, _ = imps.canonicalize_a_form(_canonical_state())
    V = [_rand_orth(rng, 8), _rand_orth(rng, 8)]
    start = [imps.polar_orthogonal(v + 0.2 * rng.standard_normal(v.shape)) for v in V]
    U, F, _ = imps.gauge_fix(a, _gauged(a, V), U0=start, tol=1e-14)
    # the alternating iteration converges linearly; directions with small
    # Schmidt weight are pinned only weakly by the fidelity
    assert abs(F - 1) < 1e-10
    sgn = np.sign(np.sum(U[0] * V[0]))
    for b in (0, 1):
        np.testing.assert_allclose(sgn * U[b], V[b], atol=1e-6)


# --- iTEBD energies --------------------------------------------------------

def test_paper_exact_energy_value():
    # the paper's printed exact energy per link at h = 1.05
    g = GOLD["tfim1d_h1.05_energy_per_link"]
    assert abs(pins.tfim1d_energy(1.05) - g["value"]) < 0.5e-6


def test_recycled_with_one_step_equals_plain():
    # N_Re = 1: every step rebuilds the environment, so the recycled
    # trajectory equals the plain one up to gauge
    ga, _, gb, _ = tninputs.imps_two_site(2, 8)
    sites, _ = imps.run_itebd([ga, gb], 1.0, 1.0, 0.02, 8, 20)
    g = gates.impo(1.0, 1.0, 0.02)
    a, b = sites, sites
    for _ in range(5):
        a, _, _, _, _ = imps.itebd_plain_step(a, g, 8)
        b, _, _, _, _ = imps.recycle_build(b, g, 8)
        assert abs(imps.energy_per_site(a, 1, 1) - imps.energy_per_site(b, 1, 1)) < 1e-10


def test_zero_field_energy_is_minus_one():
    ga, _, gb, _ = tninputs.imps_two_site(0, 4)
    sites, _ = imps.run_itebd([ga, gb], 1.0, 0.0, 0.1, 4, 300)
    assert abs(imps.energy_per_site(sites, 1.0, 0.0) + 1.0) < 1e-10


def test_offcritical_energy_matches_closed_form():
    # h = 0.5: gapped, chi = 8 saturates; the residual is the O(dt^2) Trotter
    # error of the second-order split
    ga, _, gb, _ = tninputs.imps_two_site(0, 8)
    sites, _ = imps.run_itebd([ga, gb], 1.0, 0.5, 0.01, 8, 1500)
    e = imps.energy_per_site(sites, 1.0, 0.5)
    assert abs(e - pins.tfim1d_energy(0.5)) < 2e-5


@pytest.mark.slow
def test_critical_chain_recycled_reaches_exact_energy():
    # two-site iMPS, chi=16, dt=0.01, h=1: energy against -4/pi
    ga, _, gb, _ = tninputs.imps_two_site(0, 16)
    sites, _ = imps.run_itebd([ga, gb], 1.0, 1.0, 0.01, 16, 300)
    sites, _ = imps.run_itebd(sites, 1.0, 1.0, 0.01, 16, 1700, n_re=20)
    e = imps.energy_per_site(sites, 1.0, 1.0)
    assert abs(e + 4 / np.pi) < 2e-4


# --- N_Re -> infinity (Sec. V C, the limit lines of Fig. 19) -------------------

def _after_plain(chi, h, dt, nplain, seed=0):
    ga, _, gb, _ = tninputs.imps_two_site(seed, chi)
    sites = [ga / np.linalg.norm(ga), gb / np.linalg.norm(gb)]
    g = gates.impo(1.0, h, dt)
    for _ in range(nplain):
        sites, _, _, _, _ = imps.itebd_plain_step(sites, g, chi)
    return sites, g


def test_recycle_limit_is_the_limit_of_recycling():
    # the dominant eigenvector of each site's renormalized gate is a fixed
    # point of the map, and repeated recycling (A <- G A, normalised)
    # converges to it
    chi = 8
    sites, g = _after_plain(chi, 1.05, 0.05, 50)
    new, (Lf, Rf), _, _, _ = imps.recycle_build(sites, g, chi)
    lim, lams, ratios = imps.recycle_limit(Lf, Rf, g, new)
    assert max(ratios) < 1
    for X in (0, 1):
        G = imps.renormalized_gate_matrix(Lf, Rf, g, X)
        r = G @ lim[X].ravel() - lams[X] * lim[X].ravel()
        assert np.abs(r).max() < 1e-12 * lams[X]
    cur = new
    for _ in range(5000):
        cur = imps.apply_renormalized(Lf, Rf, g, cur)
    for X in (0, 1):
        assert np.abs(cur[X] - lim[X]).max() < 1e-10


def test_recycle_limit_keeps_the_plain_fixed_point():
    # at a converged state of plain iTEBD the truncated gated state is the
    # state itself up to gauge, so the recycling limit leaves its energy
    chi, h = 4, 2.0
    sites, g = _after_plain(chi, h, 0.05, 600)
    e0 = imps.energy_per_site(sites, 1.0, h)
    s1, _, _, _, _ = imps.itebd_plain_step(sites, g, chi)
    assert abs(imps.energy_per_site(s1, 1.0, h) - e0) < 1e-13
    new, (Lf, Rf), _, _, F = imps.recycle_build(sites, g, chi)
    assert F > 1 - 1e-12
    lim, _, _ = imps.recycle_limit(Lf, Rf, g, new)
    assert abs(imps.energy_per_site(lim, 1.0, h) - e0) < 1e-10


def test_recycle_limit_trajectory_reaches_the_plain_energy():
    # the N_Re -> infinity scheme converges in a few environment steps to the
    # state plain iTEBD reaches after hundreds of steps
    chi, h, dt = 4, 2.0, 0.05
    ref, _ = _after_plain(chi, h, dt, 600)
    e_ref = imps.energy_per_site(ref, 1.0, h)
    sites, _ = _after_plain(chi, h, dt, 3)
    _, log = imps.run_itebd(sites, 1.0, h, dt, chi, 12, n_re=None, energy_every=1)
    assert abs(log[-1][1] - e_ref) < 1e-9
    assert abs(log[0][1] - e_ref) > 1e-2
