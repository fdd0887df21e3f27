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
    # the canonical spectra are non-degenerate, so the gauge is unique: U = V
    for u, v in zip(U, V):
        np.testing.assert_allclose(u, v, atol=1e-8)


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


# --- the 2x2 block of Sec. VI B (Fig. 21): networks and the joint cost ---------

def _qmat(beta):
    W = np.array([[np.exp(beta / 2), np.exp(-beta / 2)], [np.exp(-beta / 2), np.exp(beta / 2)]])
    from scipy.linalg import sqrtm
    return np.real(sqrtm(W))


def test_block_network_onsager():
    # Ising PEPS A = prod Q_{s,leg}: on a link, sum_ij Q_{s1 i} O_ij Q_{s2 j}
    # = (Q O Q^T)_{s1 s2}; O = Q^-1 sz Q puts sz on the first end (ket layer),
    # O' = Q sz Q^-1 on the second end (bra layer).  The block's network with
    # the slot cut, closed by (O, O'), over the closed block, is then
    # <s s>_nn along the slot's direction (Onsager); anisotropic couplings
    # tell horizontal slots from vertical ones and any swap of the two ends
    # gives 1 instead
    bh, bv, chi = 0.35, 0.15, 16
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    A = pins.ising_peps_aniso(bh, bv)
    C, T = _env(cell, chi, 2)
    C, T, _, _ = ctmrg.ctmrg(cell, [A, A], C, T, chi, max_iter=80, tol=1e-12)
    ch, cv = pins.onsager_nn_aniso(bh, bv)
    t = {X: A for X in ("TL", "TR", "BR", "BL")}
    E = fu.block_corners(cell, C, T, t, t)
    Z = fu.block_closed(E)
    for slot in range(4):
        horiz = fu.SLOTS[slot][2] == "r"
        Qm = _qmat(bh if horiz else bv)
        O = np.linalg.solve(Qm, pins.SZ @ Qm)
        O2 = Qm @ pins.SZ @ np.linalg.inv(Qm)
        N = fu.block_open(E, slot)
        assert abs(np.einsum("ijab,ij,ab->", N, np.eye(2), np.eye(2)) / Z - 1) < 1e-12
        val = np.einsum("ijab,ij,ab->", N, O, O2) / Z
        assert abs(val - (ch if horiz else cv)) < 1e-9, slot


def test_block_network_product_state_factorizes():
    # D = 1 with a scalar environment: the open network of a slot is the
    # Gram matrix of the first end's open leg times that of the second end's
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    rng = np.random.default_rng(3)
    sites = [rng.standard_normal((2, 1, 1, 1, 1)) for _ in range(2)]
    th = [gates.apply_ipepo(gates.ipepo(1.0, 3.0, 0.1), a) for a in sites]
    P, Q = fu.su_truncation(cell, th, 1)
    C, T = np.ones((4, 4, 1, 1)), np.ones((4, 4, 1, 1, 1, 1))
    for slot, (_, e1, l1, e2, l2) in enumerate(fu.SLOTS):
        N, M = fu.bond_environment(cell, th, P, Q, P, Q, C, T, slot)
        t = fu.block_tensors(cell, th, P, Q, P, Q, slot)
        g1 = np.moveaxis(t[e1], peps.LEGS[l1], 0).reshape(2, -1)
        g2 = np.moveaxis(t[e2], peps.LEGS[l2], 0).reshape(2, -1)
        ref = np.einsum("ia,jb->ijab", g1 @ g1.T, g2 @ g2.T)
        c = np.sum(N * ref) / np.sum(ref * ref)
        np.testing.assert_allclose(N, c * ref, atol=1e-14 * np.abs(N).max())


def _block_problem(D=2, chi=6, seed=0):
    """A gated state one full-update step from the seeded start, its
    pre-truncation and the converged environment of the pre-truncated state."""
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    g = gates.ipepo(1.0, 3.0, 0.01)
    sites = [s / np.linalg.norm(s) for s in tninputs.ipeps_sites(seed, 2, D)]
    C, T = _env(cell, chi, D)
    out = fu.fu_env_step(cell, sites, g, D, chi, C, T)
    th = [gates.apply_ipepo(g, a) for a in out["sites"]]
    P, Q = fu.su_truncation(cell, th, D)
    links, _ = peps.cell_links(cell)
    C, T, _, _ = ctmrg.ctmrg(cell, peps.truncate(th, links, P, Q), out["C"], out["T"], chi,
                             100, 1e-10)
    return cell, th, P, Q, C, T


def test_block_truncation_joint_cost():
    cell, th, P, Q, C, T = _block_problem()
    tn = abs(fu.block_norm(cell, th, P, Q, C, T))
    P1, Q1, f, passes, sweeps, hist = fu.fu_truncate(cell, th, P, Q, C, T, 1e-15, 300, 1)
    assert passes < 300
    # every update minimises the one cost f(zeta) exactly in its variable:
    # f never increases (Sec. VI B, block coordinate descent)
    assert all(b <= a + 1e-13 * tn for a, b in zip(hist, hist[1:]))
    assert f < hist[0]
    # f is one function of zeta: the four slots' environments give one value
    sg = np.sign(fu.block_norm(cell, th, P, Q, C, T))
    fs = []
    for k in range(4):
        N, M = fu.bond_environment(cell, th, P, Q, P1, Q1, C, T, k)
        fs.append(fu.cost(sg * N, P1[k], Q1[k], np.einsum("ijaa->ij", sg * M), tn)[0])
    assert max(fs) - min(fs) < 1e-12 * tn
    assert abs(fs[0] - f) < 1e-12 * tn
    # converged: one more cycle leaves f where it is; the truncations move
    # only along the directions f weighs least, by the square root of what
    # the cost still changes (f is quadratic at its minimum)
    P2, Q2, f2, _, _, _ = fu.fu_truncate(cell, th, P, Q, C, T, 0.0, 1, 1, P1, Q1)
    assert abs(f2 - f) < 1e-14 * tn
    for b in range(4):
        assert np.abs(P2[b] @ Q2[b] - P1[b] @ Q1[b]).max() < 1e-6


def test_block_truncation_full_rank_is_exact():
    # keeping the full bond kappa D, PQ = I is feasible and f reaches 0
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    g = gates.ipepo(1.0, 3.0, 0.05)
    sites = tninputs.ipeps_sites(4, 2, 1)
    th = [gates.apply_ipepo(g, a) for a in sites]
    Dk = th[0].shape[1]
    P, Q = fu.su_truncation(cell, th, Dk)
    links, _ = peps.cell_links(cell)
    C, T = _env(cell, 4, Dk)
    C, T, _, _ = ctmrg.ctmrg(cell, peps.truncate(th, links, P, Q), C, T, 4, 60, 1e-10)
    rng = np.random.default_rng(5)
    P0 = [p + 0.2 * rng.standard_normal(p.shape) for p in P]
    Q0 = [q + 0.2 * rng.standard_normal(q.shape) for q in Q]
    tn = abs(fu.block_norm(cell, th, P, Q, C, T))
    _, _, f, _, _, hist = fu.fu_truncate(cell, th, P, Q, C, T, 1e-15, 50, 1)
    assert hist[0] < 1e-12 * tn        # the pre-truncation itself is exact here
    P1, Q1, f, _, _, hist = fu.fu_truncate(cell, th, P, Q, C, T, 1e-15, 100, 1, P0, Q0)
    # from a perturbed start of the internal links
    assert hist[0] > 1e-2 * tn
    assert f < 1e-13 * tn


def test_recycling_with_one_step_is_plain_2d():
    # N_Re = 1 through the recycling branch: the renormalized gate applied
    # once is the full-update step in another gauge, so every energy of the
    # trajectory is the plain one
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    D, chi = 2, 6
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_sites(2, 2, D)]
    C, T = tninputs.ctm_env(3, 4, chi, D, positive=True)
    _, log_p = fu.run_fu(cell, A, 1.0, 3.0, 0.01, D, chi, 3, n_re=1, C=C, T=T)
    _, log_r = fu.run_fu(cell, A, 1.0, 3.0, 0.01, D, chi, 3, n_re=1, C=C, T=T,
                         force_recycle=True)
    assert [r for _, _, r in log_r] == [True] * 3
    for (_, ep, _), (_, er, _) in zip(log_p, log_r):
        assert abs(ep - er) < 1e-10 * abs(ep)


def test_recycle_fidelity_near_one_for_slow_evolution():
    # a short time step changes the state little: the gauge fix of the
    # canonical truncated state against the canonical A_0 reaches F ~ 1
    cell = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    D, chi, dt = 2, 6, 1e-4
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_sites(2, 2, D)]
    a0 = peps.canonicalize_a_form(cell, A)[0]
    C, T = tninputs.ctm_env(3, 4, chi, D, positive=True)
    out = fu.fu_env_step(cell, a0, gates.ipepo(1.0, 3.0, dt), D, chi, C, T)
    _, _, _, F = fu.recycle_build(cell, a0, out, 2)
    assert F > 1 - 1e-6


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


def test_one_site_truncation_is_the_slot_mean_of_the_checkerboard():
    # The one-site cell (Sec. VI B): its block holds the horizontal link in
    # the top and bottom slots and the vertical link in the left and right
    # ones, and each link gets the mean of its two slots' (P, Q).  The
    # checkerboard with B = A and the one-site environment on every position
    # is the same block with one link per slot, so its four results, averaged
    # over the slots of each one-site link, must give the one-site result.
    c1 = ctmrg.Cell(1, 1, [0])
    cb = ctmrg.Cell(2, 2, [0, 1, 1, 0])
    g = gates.ipepo(1.0, 3.0, 0.01)
    D, chi = 2, 6
    a = tninputs.ipeps_sites(7, 1, D)[0]
    th = [gates.apply_ipepo(g, a / np.linalg.norm(a))]
    P, Q = fu.su_truncation(c1, th, D)
    links1, _ = peps.cell_links(c1)
    C, T = _env(c1, chi, D, seed=1)
    C, T, _, _ = ctmrg.ctmrg(c1, peps.truncate(th, links1, P, Q), C, T, chi, 100, 1e-10)
    P1, Q1, f1, _, _, _ = fu.fu_truncate(c1, th, P, Q, C, T, 0.0, 3, 1)
    linksb, _ = peps.cell_links(cb)
    onesite = [0 if leg == "r" else 1 for _, leg, _, _ in linksb]
    Pb, Qb, fb, _, _, _ = fu.fu_truncate(cb, [th[0], th[0]], [P[m] for m in onesite],
                                         [Q[m] for m in onesite], np.repeat(C, 4, axis=0),
                                         np.repeat(T, 4, axis=0), 0.0, 3, 1)
    assert abs(fb - f1) < 1e-12 * abs(fu.block_norm(c1, th, P, Q, C, T))
    for link in (0, 1):
        ks = [b for b in range(4) if onesite[b] == link]
        assert len(ks) == 2
        np.testing.assert_allclose(sum(Pb[b] for b in ks) / 2, P1[link], atol=1e-12)
        np.testing.assert_allclose(sum(Qb[b] for b in ks) / 2, Q1[link], atol=1e-12)


def test_untruncated_environment_equals_an_orthogonal_pretruncation():
    # The form without pre-truncation (Sec. VI B, closing cost remark): the
    # environment of Theta itself and identities on the block's outer legs.
    # An orthogonal gauge O per link (O on the first end, O^T on the second)
    # is a pre-truncation that keeps the state; CTMRG is covariant under it,
    # so the truncation from the environment of the gauged Theta with
    # (O, O^T) on the outer legs must equal the untruncated form, while the
    # wrong orientation (O on both ends) must not.
    c1 = ctmrg.Cell(1, 1, [0])
    g = gates.ipepo(1.0, 3.0, 0.01)
    D, chi = 2, 6
    a = tninputs.ipeps_sites(7, 1, D)[0]
    th = [gates.apply_ipepo(g, a / np.linalg.norm(a))]
    Dk = th[0].shape[1]
    links, _ = peps.cell_links(c1)
    P0, Q0 = fu.su_truncation(c1, th, D)
    rng = np.random.default_rng(3)
    O = []
    for _ in links:
        q, r = np.linalg.qr(rng.standard_normal((Dk, Dk)))
        O.append(q * np.sign(np.diag(r)))
    Ot = [o.T for o in O]
    eye = [np.eye(Dk) for _ in links]
    Ca, Ta = _env(c1, chi, Dk, seed=1)
    C1, T1, _, d1 = ctmrg.ctmrg(c1, th, Ca, Ta, chi, 200, 1e-12)
    C2, T2, _, d2 = ctmrg.ctmrg(c1, peps.truncate(th, links, O, Ot), Ca, Ta, chi, 200, 1e-12)
    assert d1 < 1e-12 and d2 < 1e-12
    r1 = fu.fu_truncate(c1, th, eye, eye, C1, T1, 0.0, 2, 1, P0=P0, Q0=Q0)
    r2 = fu.fu_truncate(c1, th, O, Ot, C2, T2, 0.0, 2, 1, P0=P0, Q0=Q0)
    t1 = abs(fu.block_norm(c1, th, eye, eye, C1, T1))
    t2 = abs(fu.block_norm(c1, th, O, Ot, C2, T2))
    # the two environments agree to the CTMRG tolerance
    assert abs(r1[2] / t1 - r2[2] / t2) < 1e-9 * r1[2] / t1
    for b in range(len(links)):
        assert np.abs(r1[0][b] @ r1[1][b] - r2[0][b] @ r2[1][b]).max() < 1e-9
    r3 = fu.fu_truncate(c1, th, O, O, C2, T2, 0.0, 1, 1, P0=P0, Q0=Q0)
    assert max(np.abs(r1[0][b] @ r1[1][b] - r3[0][b] @ r3[1][b]).max() for b in (0, 1)) > 0.1


def test_torus_ed_brackets():
    # the 4x4 torus ED that brackets 2D energies loosely (finite size): its
    # own limits (h = 0: -2 exactly; h >> J: -h - J^2 / (2 h) from second-order
    # perturbation, two bonds per site, the next order J^4 / h^3 coming from
    # the plaquettes: 5e-6 at h = 50), the 4x4 values at h = 3.0, 3.05, and
    # the variational bound it sets for product states (mean field -2 - h^2/8)
    assert abs(pins.tfim2d_torus_ed(3, 3, 0.0) + 2.0) < 1e-12
    h = 50.0
    assert abs(pins.tfim2d_torus_ed(4, 4, h) - (-h - 1.0 / (2 * h))) < 1e-5
    e3 = pins.tfim2d_torus_ed(4, 4, 3.0)
    assert abs(e3 + 3.215508) < 1e-6
    assert abs(pins.tfim2d_torus_ed(4, 4, 3.05) + 3.259021) < 1e-6
    assert e3 < -2 - 3.0 ** 2 / 8


def test_simple_update_limits():
    # no interaction: the gate is a product of one-site gates, the state
    # goes to the x-polarised product state, E = -h
    oc = ctmrg.Cell(1, 1, [0])
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_near_product(0, 1, 1)]
    s = fu.run_su(oc, A, 0.0, 3.0, 0.05, 1, 200)
    C, T = _env(oc, 1, 1, seed=1)
    C, T, _, _ = ctmrg.ctmrg(oc, s, C, T, 1, 10, 1e-12)
    assert abs(peps.energy_per_site(oc, s, C, T, 0.0, 3.0) + 3.0) < 1e-12
    # D = 1: the simple update tends to the mean-field product state,
    # E = -2 - h^2 / 8, with a Trotter error that falls as dt^2
    errs = []
    for dt in (0.02, 0.01):
        s = fu.run_su(oc, A, 1.0, 3.0, dt, 1, int(4 / dt))
        C, T = _env(oc, 1, 1, seed=1)
        C, T, _, _ = ctmrg.ctmrg(oc, s, C, T, 1, 10, 1e-12)
        errs.append(peps.energy_per_site(oc, s, C, T, 1.0, 3.0) - (-2 - 3.0 ** 2 / 8))
    assert 0 < errs[1] < 1e-4 and errs[0] / errs[1] > 3
