"""Pins of the 2D oracle (CTMRG, RDMs, canonical form, gauge fix, ALS)."""
import numpy as np
import pytest

import tninputs
from oracle import ctmrg, fu, gates, grad, peps
from tests import pins

ZZ = np.kron(pins.SZ, pins.SZ)


def _env(cell, chi, D, seed=0, positive=True):
    return tninputs.ctm_env(seed, cell.Lx * cell.Ly, chi, D, positive=positive)


# --- gates (Sec. VI A, Fig. 20) --------------------------------------------

def test_ipepo_equals_trotter_product_on_torus():
    # 3x2 torus: contract the iPEPO network and compare with the dense product
    Lx, Ly, J, h, dt = 3, 2, 1.0, 0.9, 0.11
    g = gates.ipepo(J, h, dt)                     # [l][r][d][u][s][s']
    n = Lx * Ly
    idx = lambda x, y: (y % Ly) * Lx + (x % Lx)
    # each bond gets its own einsum letter
    letters = iter("ABCDEFGHIJKLMNOPQRSTUVWXYZ")
    hb = {(x, y): next(letters) for x in range(Lx) for y in range(Ly)}   # right bond of (x,y)
    vb = {(x, y): next(letters) for x in range(Lx) for y in range(Ly)}   # down bond of (x,y)
    outs = "abcdefghijkl"
    specs, ops = [], []
    for y in range(Ly):
        for x in range(Lx):
            p = idx(x, y)
            l, r = hb[((x - 1) % Lx, y)], hb[(x, y)]
            d, u = vb[(x, y)], vb[(x, (y - 1) % Ly)]
            specs.append(l + r + d + u + outs[p] + outs[n + p])
            ops.append(g)
    res = np.einsum(",".join(specs) + "->" + outs[:2 * n], *ops, optimize=True)
    dense = res.reshape(2 ** n, 2 ** n)
    bonds = [(idx(x, y), idx(x + 1, y)) for x in range(Lx) for y in range(Ly)]
    bonds += [(idx(x, y), idx(x, y + 1)) for x in range(Lx) for y in range(Ly)]
    ref = pins.trotter_product(n, bonds, h, dt, J)
    np.testing.assert_allclose(dense, ref, atol=1e-12)


# --- CTMRG against the classical Ising model ---------------------------------

@pytest.mark.parametrize("cellspec", [tninputs.SINGLE_SITE, tninputs.CHECKERBOARD])
def test_ctmrg_ising_disordered_onsager(cellspec):
    Lx, Ly, sites = cellspec
    cell = ctmrg.Cell(Lx, Ly, sites)
    beta, chi = 0.3, 16
    A = pins.ising_peps(beta)
    C, T = _env(cell, chi, 2, positive=True)
    C, T, it, delta = ctmrg.ctmrg(cell, [A, A], C, T, chi, max_iter=80, tol=1e-12)
    _, rh, rv = peps.rdms(cell, [A, A], C, T)
    ref = pins.onsager_nn(beta)
    for p in range(Lx * Ly):
        assert abs(np.trace(rh[p] @ ZZ) - ref) < 1e-9
        assert abs(np.trace(rv[p] @ ZZ) - ref) < 1e-9


@pytest.mark.parametrize("cellspec", [tninputs.SINGLE_SITE, tninputs.CHECKERBOARD])
def test_ctmrg_anisotropic_ising(cellspec):
    # different couplings on horizontal and vertical bonds: catches any mix-up
    # of leg orientation or move direction, which the isotropic model hides
    Lx, Ly, sites = cellspec
    cell = ctmrg.Cell(Lx, Ly, sites)
    bh, bv, chi = 0.35, 0.15, 16
    A = pins.ising_peps_aniso(bh, bv)
    C, T = _env(cell, chi, 2)
    C, T, _, _ = ctmrg.ctmrg(cell, [A, A], C, T, chi, max_iter=80, tol=1e-12)
    _, rh, rv = peps.rdms(cell, [A, A], C, T)
    ch, cv = pins.onsager_nn_aniso(bh, bv)
    assert abs(ch - cv) > 0.05
    for p in range(Lx * Ly):
        assert abs(np.trace(rh[p] @ ZZ) - ch) < 1e-9
        assert abs(np.trace(rv[p] @ ZZ) - cv) < 1e-9


def test_ctmrg_ising_ordered_yang():
    cell = ctmrg.Cell(1, 1, [0])
    beta, chi = 0.6, 16
    A = pins.ising_peps(beta)
    # up-polarised boundary: the spin-up product boundary plus a small
    # positive random part
    from scipy.linalg import sqrtm
    W = np.array([[np.exp(beta / 2), np.exp(-beta / 2)], [np.exp(-beta / 2), np.exp(beta / 2)]])
    v = np.real(sqrtm(W))[0]
    C, T = _env(cell, chi, 2, positive=True)
    C, T = 1e-3 * C, 1e-3 * T
    C[..., 0, 0] += 1.0
    T[..., 0, :, :, 0] += np.outer(v, v)
    C, T, _, _ = ctmrg.ctmrg(cell, [A], C, T, chi, max_iter=250, tol=1e-14)
    m = abs(peps.magnetization_z(cell, [A], C, T))
    assert abs(m - pins.yang_m(beta)) < 1e-9
    r1, rh, _ = peps.rdms(cell, [A], C, T)
    assert abs(np.trace(rh[0] @ ZZ) - pins.onsager_nn(beta)) < 1e-9


def test_product_state_exact():
    # D = 1 product state cos(t)|0> + sin(t)|1>: exact at chi = 1
    t, h = 0.37, 2.0
    A = np.array([np.cos(t), np.sin(t)]).reshape(2, 1, 1, 1, 1)
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    C, T = _env(cell, 1, 1, positive=True)
    C, T, _, _ = ctmrg.ctmrg(cell, [A, A], C, T, 1, max_iter=5)
    e = peps.energy_per_site(cell, [A, A], C, T, 1.0, h)
    mz, mx = np.cos(2 * t), np.sin(2 * t)
    assert abs(e - (-2 * mz ** 2 - h * mx)) < 1e-14


def test_rotation_four_times_is_identity():
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    A, B = tninputs.ipeps_sites(1, 2, 2)
    C, T = _env(cell, 5, 2, positive=False)
    c, t, CC, TT = cell, [A, B], C, T
    for _ in range(4):
        c, t, CC, TT = ctmrg.rotate_ccw(c, t, CC, TT)
    assert c.sites == cell.sites
    np.testing.assert_array_equal(CC, C)
    np.testing.assert_array_equal(TT, T)
    np.testing.assert_array_equal(t[0], A)


def _ipeps_state(D=2, seed=0):
    """A random checkerboard state (N(0,1) site tensors)."""
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    return cell, tninputs.ipeps_sites(seed, 2, D)


def test_observables_gauge_invariant_and_rdms_valid():
    cell, sites = _ipeps_state()
    chi = 12
    # a ket <-> bra symmetric starting boundary keeps the environment, and
    # hence every reduced density matrix, symmetric
    C, T = _env(cell, chi, 2)
    C1, T1, _, _ = ctmrg.ctmrg(cell, sites, C, T, chi, max_iter=60, tol=1e-12)
    e1 = peps.energy_per_site(cell, sites, C1, T1, 1.0, 3.0)
    rho1, rh, rv = peps.rdms(cell, sites, C1, T1)
    for r in rho1 + rh + rv:
        np.testing.assert_allclose(r, r.T, atol=1e-12)
        assert np.min(np.linalg.eigvalsh(0.5 * (r + r.T))) > -1e-12
        assert abs(np.trace(r) - 1) < 1e-14
    # random invertible gauge on each of the four links (Sec. IV: B = M K A M^-1 K^-1)
    rng = np.random.default_rng(4)
    links, _ = peps.cell_links(cell)
    # an orthogonal gauge is an exact symmetry of finite-chi CTMRG; a general
    # invertible one only up to the truncation error
    for kind, tol in (("orthogonal", 1e-10), ("invertible", 1e-4)):
        if kind == "orthogonal":
            M = [np.linalg.qr(rng.standard_normal((2, 2)))[0] for _ in links]
        else:
            M = [np.eye(2) + 0.3 * rng.standard_normal((2, 2)) for _ in links]
        Minv = [np.linalg.inv(m) for m in M]
        g2 = peps.truncate(sites, links, M, Minv)      # a1^T a2 = (M^T a1)^T (M^-1 a2)
        C2, T2, _, _ = ctmrg.ctmrg(cell, g2, C, T, chi, max_iter=60, tol=1e-12)
        e2 = peps.energy_per_site(cell, g2, C2, T2, 1.0, 3.0)
        assert abs(e1 - e2) < tol, kind


# --- canonical form and gauge fixing (Sec. IV) --------------------------------

def test_ipeps_canonical_constraints():
    cell, sites = _ipeps_state(D=3)
    a1, lams, Pc, Qc, it = peps.canonicalize_a_form(cell, sites)
    links, leg_link = peps.cell_links(cell)
    # recover Gamma from the A form and check Eqs. (17)-(20)
    gams = []
    for s, a in enumerate(a1):
        t = a
        for leg, ax in peps.LEGS.items():
            lam = lams[leg_link[s][leg]]
            shape = [1] * 5
            shape[ax] = lam.size
            t = t / np.sqrt(lam).reshape(shape)
        gams.append(t)
    assert peps.canonical_residual(cell, gams, lams) < 1e-10


def test_ipeps_gauge_fix_known_answer():
    cell, sites = _ipeps_state(D=3)
    a, _, _, _, _ = peps.canonicalize_a_form(cell, sites)
    links, _ = peps.cell_links(cell)
    rng = np.random.default_rng(7)
    V = []
    for _ in links:
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        V.append(q * np.sign(np.diag(r)))
    new = peps.truncate(a, links, [v.T for v in V], V)
    from oracle.imps import polar_orthogonal
    start = [polar_orthogonal(v + 0.1 * rng.standard_normal(v.shape)) for v in V]
    U, F, _ = peps.gauge_fix(cell, a, new, U0=start, tol=1e-14)
    assert abs(F - 1) < 1e-10


# --- ALS (Eqs. (var), (var1)) ---------------------------------------------------

def _factorized_env(rng, n):
    Lh = rng.standard_normal((n, n))
    Rh = rng.standard_normal((n, n))
    L, R = Lh @ Lh.T, Rh @ Rh.T
    N = np.einsum("ia,jb->ijab", L, R)
    return N, L, R


def test_als_factorized_environment_is_eckart_young():
    # N = L (x) R: f = ||L^1/2 (I - PQ) R^1/2||^2, minimum = sum of the
    # discarded squared singular values of L^1/2 R^1/2
    rng = np.random.default_rng(1)
    n, D = 8, 3
    N, L, R = _factorized_env(rng, n)
    from scipy.linalg import sqrtm
    s = np.linalg.svd(np.real(sqrtm(L)) @ np.real(sqrtm(R)), compute_uv=False)
    fmin = float(np.sum(s[D:] ** 2))
    P0 = rng.standard_normal((n, D))
    Q0 = rng.standard_normal((D, n))
    P, Q, f, sweeps, hist = fu.als(N, P0, Q0, tol=1e-15, max_sweeps=500)
    assert abs(f - fmin) < 1e-9 * fmin
    # cost never increases over sweeps (alternating exact minimisation)
    assert all(b <= a + 1e-10 * abs(a) for a, b in zip(hist, hist[1:]))


def test_als_full_rank_target_is_exact():
    rng = np.random.default_rng(2)
    n = 6
    N, _, _ = _factorized_env(rng, n)
    P, Q, f, _, _ = fu.als(N, rng.standard_normal((n, n)), rng.standard_normal((n, n)))
    _, t = fu.cost(N, P, Q)
    assert abs(f) < 1e-10 * t


def test_full_update_product_state_mean_field():
    # D = 1 full update (chi = 1 is exact for a product state) approaches the
    # mean-field energy -2 - h^2/8 for h < 4 as dt -> 0
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    rng = np.random.default_rng(0)
    A = rng.standard_normal((2, 1, 1, 1, 1))
    B = rng.standard_normal((2, 1, 1, 1, 1))
    sites, log = fu.run_fu(cell, [A, B], 1.0, 3.0, 0.02, 1, 1, 200)
    assert abs(log[-1][1] - (-2 - 9 / 8)) < 2e-3


# --- energy-gradient oracle ---------------------------------------------------

def test_energy_is_scale_invariant():
    # E(cA) = E(A) exactly, so the directional derivative along A vanishes
    A = tninputs.ipeps_sites(0, 1, 2)[0]
    C0, T0 = tninputs.ctm_env(1, 1, 6, 2)
    e1 = grad.energy_after(A, C0, T0, 6, 4, 1.0, 3.0)
    e2 = grad.energy_after(1.7 * A, C0, T0, 6, 4, 1.0, 3.0)
    assert abs(e1 - e2) < 1e-12
    d = grad.fd_directional(A, C0, T0, 6, 4, 1.0, 3.0, [A / np.linalg.norm(A)])
    # rounding through the SVDs of the iterations sets the difference floor
    assert abs(d[0]) < 1e-6
