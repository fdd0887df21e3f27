"""Full update with environment recycling for an iPEPS (Sec. VI B, VI C).

Oracle (test infrastructure only).

Readings taken where the paper is silent or describes a one-site cell:
* unit cell: the checkerboard [[A, B], [B, A]] with four inequivalent links
  (or any cell whose legs map to distinct links); no averaging of P and Q
  over equivalent links;
* pre-truncation before the environment is computed (the paper uses the
  simple update): Theta is brought to canonical form (Sec. IV A) and each
  link keeps its D largest Schmidt values;
* the bond environment N of a link is the CTM network around the two sites
  of that link, with Theta^ (Theta with every other leg truncated by the
  current (P, Q)) on both sites and the link's ket and bra legs open:
  N[i, j, i', j'] with i, j the ket legs of the first and second site and
  i', j' the bra legs; N is symmetrised in (ket <-> bra) and its overall
  sign, which the normalised boundary leaves free, is taken with
  <I|N|I> > 0;
* ALS (Eqs. (var), (var1)): with Q fixed, P = R^{-1} S where
  R[(i c),(i' c')] = sum_{j j'} Q[c,j] N[i,j,i',j'] Q[c',j'] and
  S[(i c)] = sum_{j i'} Q[c,j] N[i,j,i',i']; then Q likewise; after each
  pair the pair is balanced through the SVD of P Q; solves use
  R + 1e-14 tr(R) I;
* the links are updated in cell order (r, d, l, u for the checkerboard),
  each with its N rebuilt from the current zeta, and the whole cycle is
  repeated until the cost of every link, traced from one cycle to the next,
  changes by less than tol <I|N|I> (Sec. VI B: the cycle over r, d, l, u
  is iterated until every tensor of zeta is converged, recognised from the
  cost of Eq. (var)); each visit makes ``max_sweeps`` ALS sweeps on its
  link (1 is the literal order of the section: one P and one Q update per
  link per cycle);
* recycling (Sec. VI C): the state A_0 that the renormalized gate is
  applied to is in canonical form (A form) -- the section assumes it, and
  the gauge fix U relates two canonical states; the environment step brings
  A_0 to canonical form first;
* energies are measured at environment steps, for the pre-truncated state
  the environment was computed for.
"""
from __future__ import annotations

import numpy as np

from . import gates
from .ctmrg import Cell, ctmrg, rotate_ccw
from .imps import polar_orthogonal
from .peps import (LEGS, PATH_HALF, apply_leg, canonical_pq, canonicalize, canonicalize_a_form,
                   cell_links, energy_per_site, gauge_fix, truncate)


# ---------------------------------------------------------------------------
# pre-truncation (simple-update style)
# ---------------------------------------------------------------------------

def su_truncation(cell, thetas, D, tol=1e-14, max_iter=1000):
    """(P, Q) per link from the canonical form of Theta: the first D columns
    of Pc and rows of Qc (``canonical_pq``: bond kappa*D), i.e. the D
    largest Schmidt values of every link are kept."""
    _, lams, _, TR, TL = canonicalize(cell, thetas, None, tol, max_iter)
    Pc, Qc = canonical_pq(TR, TL, lams)
    return [p[:, :D].copy() for p in Pc], [q[:D, :].copy() for q in Qc]


# ---------------------------------------------------------------------------
# bond environment: the 2x2 block B of Fig. 21(a)
# ---------------------------------------------------------------------------

# Slots of the block's four internal links, in the order they are visited:
# (name, first end, its leg, second end, its leg); block positions TL, TR,
# BR, BL.  The first end carries P, the second Q (A~ = Q Theta P).
SLOTS = (("top", "TL", "r", "TR", "l"),
         ("left", "TL", "d", "BL", "u"),
         ("bottom", "BL", "r", "BR", "l"),
         ("right", "TR", "d", "BR", "u"))
# internal legs of each block position, the rest face the environment
INTERNAL = {"TL": ("r", "d"), "TR": ("l", "d"), "BR": ("l", "u"), "BL": ("r", "u")}


def block_positions(cell, x0=0, y0=0):
    """Cell positions of the block with its top-left site at (x0, y0)."""
    return {"TL": cell.pos(x0, y0), "TR": cell.pos(x0 + 1, y0),
            "BR": cell.pos(x0 + 1, y0 + 1), "BL": cell.pos(x0, y0 + 1)}


def block_slot_links(cell):
    """Cell link of each slot of the block at the origin; raises if some
    link of the cell is not inside the block (the truncation of such a cell
    is not one block's variational problem)."""
    links, leg_link = cell_links(cell)
    pos = block_positions(cell)
    out = []
    for _, e1, l1, e2, l2 in SLOTS:
        s1, s2 = cell.sites[pos[e1]], cell.sites[pos[e2]]
        b = leg_link[s1][l1]
        assert leg_link[s2][l2] == b and links[b][0] == s1 and links[b][2] == s2
        out.append(b)
    if sorted(set(out)) != list(range(len(links))):
        raise ValueError("the 2x2 block does not hold every link of this cell")
    return out


def _trunc_leg(t, site, leg, b, links, P, Q):
    """Truncate ``leg`` of ``site``'s tensor with link b's P (first end) or
    Q (second end)."""
    s1, l1, _, _ = links[b]
    return apply_leg(t, leg, P[b].T if (site == s1 and leg == l1) else Q[b])


def block_tensors(cell, thetas, Psu, Qsu, Pz, Qz, open_slot):
    """Site tensors of the four block positions: the legs facing the
    environment truncated by the pre-truncation (Psu, Qsu) that the
    environment was computed for; internal legs by the slot's current
    (Pz[slot], Qz[slot]) when Pz is given, untruncated when Pz is None; the
    open slot's legs untruncated."""
    links, leg_link = cell_links(cell)
    pos = block_positions(cell)
    slot_of = {}
    for k, (_, e1, l1, e2, l2) in enumerate(SLOTS):
        slot_of[(e1, l1)] = k
        slot_of[(e2, l2)] = k
    out = {}
    for X, p in pos.items():
        s = cell.sites[p]
        t = thetas[s]
        for leg in LEGS:
            b = leg_link[s][leg]
            if leg not in INTERNAL[X]:
                t = _trunc_leg(t, s, leg, b, links, Psu, Qsu)
                continue
            k = slot_of[(X, leg)]
            if k == open_slot or Pz is None:
                continue
            first = SLOTS[k][1] == X
            t = apply_leg(t, leg, Pz[k].T if first else Qz[k])
        out[X] = t
    return out


def block_corners(cell, C, T, kets, bras):
    """The four enlarged corners of the block (environment tensors of the
    block's positions, Sec. VI B): each carries its two boundary legs and
    the ket and bra index of its two internal legs.
      E_TL[t, rk, rb, dk, db, x]   t: to T1 of TR, x: to T4 of BL
      E_TR[t, lk, lb, dk, db, f]   f: to T2 of BR
      E_BR[f, uk, ub, lk, lb, y]   y: to T3 of BL
      E_BL[y, rk, rb, uk, ub, x]"""
    P = block_positions(cell)
    tl, tr, br, bl = P["TL"], P["TR"], P["BR"], P["BL"]
    E = {}
    E["TL"] = np.einsum("gh,huUt,xlLg,slrdu,sLRDU->trRdDx", C[tl, 0], T[tl, 0], T[tl, 3],
                        kets["TL"], bras["TL"], optimize=True)
    E["TR"] = np.einsum("tuUh,he,erRf,slrdu,sLRDU->tlLdDf", T[tr, 0], C[tr, 1], T[tr, 1],
                        kets["TR"], bras["TR"], optimize=True)
    E["BR"] = np.einsum("frRg,gh,hdDy,slrdu,sLRDU->fuUlLy", T[br, 1], C[br, 2], T[br, 2],
                        kets["BR"], bras["BR"], optimize=True)
    E["BL"] = np.einsum("ydDg,ge,elLx,slrdu,sLRDU->yrRuUx", T[bl, 2], C[bl, 3], T[bl, 3],
                        kets["BL"], bras["BL"], optimize=True)
    return E


# The ring of enlarged corners, one index letter per leg: top link (a, A at
# TL; c, C at TR), right link (e, E at TR; g, G at BR), bottom link (h, H at
# BR; k, K at BL), left link (b, B at TL; m, M at BL); boundary legs t, f,
# y, x.  Closing a link identifies its two letters; the open slot keeps both
# ends and lists them as (first ket, second ket, first bra, second bra).
_OPEN = {0: "taAbBx,tcCeEf,feEhHy,yhHbBx->acAC",
         1: "taAbBx,taAeEf,feEhHy,yhHmMx->bmBM",
         2: "taAbBx,taAeEf,feEhHy,ykKbBx->khKH",
         3: "taAbBx,taAeEf,fgGhHy,yhHbBx->egEG"}


def block_open(E, slot):
    """Contract the ring of enlarged corners with slot ``slot`` cut:
    N[i, j, i', j'] with i, j the ket index of its first and second end and
    i', j' the bra index."""
    return np.einsum(_OPEN[slot], E["TL"], E["TR"], E["BR"], E["BL"], optimize=True)


def block_closed(E):
    """The closed ring: the block's norm network."""
    return float(np.einsum("taAbBx,taAeEf,feEhHy,yhHbBx->", E["TL"], E["TR"], E["BR"], E["BL"],
                           optimize=True))


def block_norm(cell, thetas, Psu, Qsu, C, T):
    """<Psi_g|Psi_g> of the block: every internal link untruncated."""
    t = block_tensors(cell, thetas, Psu, Qsu, None, None, -1)
    return block_closed(block_corners(cell, C, T, t, t))


def bond_environment(cell, thetas, Psu, Qsu, Pz, Qz, C, T, slot):
    """The two environments of slot ``slot`` (see module docstring):
    N[i, j, i', j'] with the other internal links truncated by zeta in both
    layers, symmetrised in ket <-> bra, and M[i, j, i', j'] with zeta in the
    ket layer and the untruncated bra layer of Psi_g.  Both unnormalised,
    in the sign of the raw network."""
    kz = block_tensors(cell, thetas, Psu, Qsu, Pz, Qz, slot)
    kg = block_tensors(cell, thetas, Psu, Qsu, None, None, slot)
    N = block_open(block_corners(cell, C, T, kz, kz), slot)
    M = block_open(block_corners(cell, C, T, kz, kg), slot)
    n = N.shape[0]
    N2 = N.reshape(n * n, n * n)
    N = (0.5 * (N2 + N2.T)).reshape(n, n, n, n)
    return N, M


# ---------------------------------------------------------------------------
# ALS (Eqs. (var), (var1))
# ---------------------------------------------------------------------------

def cost(N, P, Q, tb=None, t=None):
    """f = <Psi_g|Psi_g> - 2 <Psi_g|Psi_zeta> + <Psi_zeta|Psi_zeta> (Eq. (var),
    real case) as a function of one link's (P, Q): <PQ|N|PQ> is the last
    term, sum_ij (PQ)_ij tb_ij the middle one and t the first.  Without tb
    and t, the first two come from N itself (tb_ij = sum_a N[i, j, a, a],
    t = <I|N|I>): the cost of a single link whose environment is N.
    Returns (f, t)."""
    n = N.shape[0]
    I = np.eye(n)
    O = P @ Q
    if tb is None:
        tb = np.einsum("ijaa->ij", N)
    if t is None:
        t = float(np.einsum("ijab,ij,ab->", N, I, I))
    c = float(np.sum(O * tb))
    q = float(np.einsum("ijab,ij,ab->", N, O, O))
    return float(t - 2 * c + q), float(t)


def _solve(R, S):
    """Solve (R + 1e-14 tr(R) I) x = S; R is the positive semi-definite
    quadratic form of Eq. (var1), its trace the scale of the regulariser."""
    n = R.shape[0]
    reg = 1e-14 * np.trace(R)
    return np.linalg.solve(R + reg * np.eye(n), S)


def _svd_signfix(m):
    """SVD with each left singular vector's first entry within 1e-8 of its
    largest magnitude made positive (the right vector flips with it)."""
    u, s, vt = np.linalg.svd(m)
    for i in range(u.shape[1]):
        a = np.abs(u[:, i])
        j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
        if u[j, i] < 0:
            u[:, i] = -u[:, i]
            vt[i, :] = -vt[i, :]
    return u, s, vt


def als(N, P, Q, tol=1e-12, max_sweeps=50, tb=None, t=None):
    """Alternating least squares on one link (Eq. (var1)): P = R^-1 S with Q
    fixed, then Q with P fixed, then the pair balanced through the SVD of
    P Q (which leaves P Q, hence f, unchanged); ``cost`` explains N, tb, t.
    Stops when a sweep changes f by less than tol t.  Returns (P, Q, f,
    sweeps, history) with history the cost at the start and after every
    half step."""
    n, D = P.shape
    if tb is None:
        tb = np.einsum("ijaa->ij", N)             # sum_i' N[i,j,i',i']
    f, t = cost(N, P, Q, tb, t)
    hist = [f]
    sw = 0
    for sw in range(1, max_sweeps + 1):
        # P with Q fixed
        R = np.einsum("cj,ijak,dk->icad", Q, N, Q).reshape(n * D, n * D)
        S = np.einsum("cj,ij->ic", Q, tb).reshape(n * D)
        P = _solve(0.5 * (R + R.T), S).reshape(n, D)
        hist.append(cost(N, P, Q, tb, t)[0])
        # Q with P fixed
        R = np.einsum("ic,ijak,ad->cjdk", P, N, P).reshape(D * n, D * n)
        S = np.einsum("ic,ij->cj", P, tb).reshape(D * n)
        Q = _solve(0.5 * (R + R.T), S).reshape(D, n)
        # balance the pair
        u, s, vt = _svd_signfix(P @ Q)
        sq = np.sqrt(s[:D])
        P, Q = u[:, :D] * sq[None, :], sq[:, None] * vt[:D]
        fn, _ = cost(N, P, Q, tb, t)
        hist.append(fn)
        done = abs(fn - f) < tol * abs(t)
        f = fn
        if done:
            break
    return P, Q, f, sw, hist


# ---------------------------------------------------------------------------
# the truncation of all links (Sec. VI B)
# ---------------------------------------------------------------------------

def fu_truncate(cell, thetas, Psu, Qsu, C, T, tol=1e-12, max_passes=50, max_sweeps=1,
                P0=None, Q0=None):
    """Minimise the block cost f(zeta) of Eq. (var) over zeta = (P, Q) of
    the block's four internal links (Sec. VI B), starting from (P0, Q0) per
    link (default: the pre-truncation (Psu, Qsu), which also truncates the
    legs facing the environment throughout): cycles over the slots top, left, bottom,
    right; each visit builds the slot's two environments from the current
    zeta and makes ``max_sweeps`` ALS sweeps (1: one P and one Q update per
    link per cycle, the section's order); the cycles stop when one changes f
    by less than tol <Psi_g|Psi_g>, or after ``max_passes``.  A link that
    several slots hold (a one-site cell) gets the mean of their (P, Q).
    Returns (P, Q, f, passes, sweeps, history) with history f at the start
    and after every half step."""
    links, _ = cell_links(cell)
    slot_link = block_slot_links(cell)
    Pz = [(Psu if P0 is None else P0)[b].copy() for b in slot_link]
    Qz = [(Qsu if Q0 is None else Q0)[b].copy() for b in slot_link]
    tn = block_norm(cell, thetas, Psu, Qsu, C, T)
    # the normalised boundary fixes the networks only up to a common sign:
    # take the one with <Psi_g|Psi_g> > 0
    sg = 1.0 if tn > 0 else -1.0
    tn = abs(tn)
    history, sweeps, passes = [], 0, 0
    f_prev = None
    for passes in range(1, max_passes + 1):
        for k in range(len(SLOTS)):
            N, M = bond_environment(cell, thetas, Psu, Qsu, Pz, Qz, C, T, k)
            N, M = sg * N, sg * M
            Pz[k], Qz[k], f, sw, h = als(N, Pz[k], Qz[k], tol, max_sweeps,
                                         tb=np.einsum("ijaa->ij", M), t=tn)
            if not history:
                history.append(h[0])
                f_prev = h[0]
            history.extend(h[1:])
            sweeps += sw
        done = abs(f - f_prev) < tol * tn
        f_prev = f
        if done:
            break
    P, Q = [], []
    for b in range(len(links)):
        ks = [k for k, lb in enumerate(slot_link) if lb == b]
        P.append(sum(Pz[k] for k in ks) / len(ks))
        Q.append(sum(Qz[k] for k in ks) / len(ks))
    return P, Q, f_prev, passes, sweeps, history


# ---------------------------------------------------------------------------
# drivers
# ---------------------------------------------------------------------------

def fu_env_step(cell, sites, g, D, chi, C, T, ctm_tol=1e-10, ctm_max=100, J=1.0, h=3.0,
                als_tol=1e-12, als_passes=50, als_sweeps=1, pretruncate=True):
    """One full-update step with a freshly computed environment: Theta = g A,
    pre-truncation, CTMRG (warm-started from C, T), energy, the ALS cycles
    over all links, A~ = Q Theta P.  Returns a dict.

    ``pretruncate=False`` is the form without the pre-truncation (Sec. VI B,
    the cost remark closing the section): the environment is that of Theta
    itself, bond kappa D (C, T of that bond; cost O(chi^3 D^6 kappa^6)), the
    block's outer legs stay untruncated, and the energy is Theta's; the ALS
    still starts from the simple-update truncation."""
    links, _ = cell_links(cell)
    thetas = [gates.apply_ipepo(g, a) for a in sites]
    P, Q = su_truncation(cell, thetas, D)
    if pretruncate:
        Pe, Qe = P, Q
        pre = truncate(thetas, links, P, Q)
    else:
        Dk = thetas[0].shape[1]
        Pe = [np.eye(Dk) for _ in links]
        Qe = [np.eye(Dk) for _ in links]
        pre = thetas
    C, T, iters, delta = ctmrg(cell, pre, C, T, chi, ctm_max, ctm_tol)
    E = energy_per_site(cell, pre, C, T, J, h)
    P, Q, f, passes, sweeps, _ = fu_truncate(cell, thetas, Pe, Qe, C, T, als_tol, als_passes,
                                             als_sweeps, P0=P, Q0=Q)
    new = truncate(thetas, links, P, Q)
    return dict(sites=new, thetas=thetas, P=P, Q=Q, C=C, T=T, energy=E,
                ctm_iters=iters, ctm_delta=delta, cost=f, als_passes=passes,
                als_sweeps=sweeps)


def run_su(cell, sites, J, h, dt, D, nsteps, tol=1e-14, max_iter=1000):
    """The simple update (Sec. VI A, the scheme the section contrasts with
    the full update): each step applies the iPEPO gate and truncates every
    link by the canonical form of Theta, keeping its D largest Schmidt
    values (``su_truncation``); no environment.  Returns the sites."""
    links, _ = cell_links(cell)
    g = gates.ipepo(J, h, dt)
    sites = [s / np.linalg.norm(s) for s in sites]
    for _ in range(nsteps):
        thetas = [gates.apply_ipepo(g, a) for a in sites]
        P, Q = su_truncation(cell, thetas, D, tol, max_iter)
        sites = [t / np.linalg.norm(t) for t in truncate(thetas, links, P, Q)]
    return sites


def gauge_start(P, Q, Pc, Qc, kappa):
    """Start of the gauge fix inside the recycling step (Sec. VI C): for a
    small time step the renormalized gate is close to the identity, so the
    kappa = 0 block of the composite truncation maps the old bond basis onto
    the new one; both ends' blocks, each normalised, are added and the
    orthogonal polar factor is taken."""
    U0 = []
    for b in range(len(P)):
        b1 = (P[b] @ Pc[b])[0::kappa, :].T
        b2 = (Qc[b] @ Q[b])[:, 0::kappa]
        U0.append(polar_orthogonal(b1 / np.linalg.norm(b1) + b2 / np.linalg.norm(b2)))
    return U0


def renormalized_gate(P, Q, Pc, Qc, U):
    """Per-link factors of G (Sec. VI C step (iii), read as
    G = U^T (Qc Q) g (P Pc) U per link): Rf = P Pc U on the first leg,
    Lf = U^T Qc Q on the second leg."""
    Rf = [P[b] @ Pc[b] @ U[b] for b in range(len(P))]
    Lf = [U[b].T @ Qc[b] @ Q[b] for b in range(len(P))]
    return Rf, Lf


def recycle_build(cell, a0, out, kappa, gauge_tol=1e-12):
    """Steps (i)-(iii) of Sec. VI C for the canonical state a0 and the
    full-update step ``out`` computed from it: canonical form of A~ (A~_1,
    Pc, Qc), the gauge U with A~_1 ~ U a0 U^T, and the renormalized gate's
    factors.  Returns (Rf, Lf, U, F)."""
    a1, _, Pc, Qc, _ = canonicalize_a_form(cell, out["sites"])
    U0 = gauge_start(out["P"], out["Q"], Pc, Qc, kappa)
    U, F, _ = gauge_fix(cell, a0, a1, tol=gauge_tol, U0=U0)
    Rf, Lf = renormalized_gate(out["P"], out["Q"], Pc, Qc, U)
    return Rf, Lf, U, F


def run_fu(cell, sites, J, h, dt, D, chi, nsteps, n_re=1, n_warm=0, C=None, T=None,
           ctm_tol=1e-10, ctm_max=100, seed_env=0, callback=None, min_fidelity=None,
           force_recycle=False, als_tol=1e-12, als_passes=50, als_sweeps=1, pretruncate=True):
    """Imaginary-time evolution of an iPEPS by full update, the environment
    recomputed every ``n_re`` steps after ``n_warm`` plain steps and the
    renormalized gate applied in between (Sec. VI C).  A recycling step
    first brings A_0 to canonical form.  With ``min_fidelity``, a recycling
    step whose gauge fix ends below it takes the plain step instead (the new
    state is too far from A_0 for G to stand in for the environment).
    ``force_recycle`` takes the recycling branch even for n_re = 1, where it
    must reproduce the plain trajectory (the renormalized gate applied once
    is the full-update step in another gauge).  ``pretruncate=False``
    computes every environment for Theta itself (``fu_env_step``; C, T then
    have bond kappa D).  Returns (sites, log) with log entries (step,
    energy_per_site, recycled) at environment steps."""
    links, _ = cell_links(cell)
    g = gates.ipepo(J, h, dt)
    kappa = g.shape[0]
    sites = [s / np.linalg.norm(s) for s in sites]
    npos = cell.Lx * cell.Ly
    if C is None:
        import tninputs
        C, T = tninputs.ctm_env(seed_env, npos, chi, D if pretruncate else kappa * D,
                                positive=True)
    log = []
    step = 0
    while step < nsteps:
        recycle = step >= n_warm and (n_re > 1 or force_recycle)
        if recycle:
            sites = canonicalize_a_form(cell, sites)[0]
        out = fu_env_step(cell, sites, g, D, chi, C, T, ctm_tol, ctm_max, J, h, als_tol,
                          als_passes, als_sweeps, pretruncate)
        C, T = out["C"], out["T"]
        F = None
        if recycle:
            Rf, Lf, U, F = recycle_build(cell, sites, out, kappa)
            if min_fidelity is not None and F < min_fidelity:
                recycle = False
        out["fidelity"] = F
        log.append((step + 1, out["energy"], recycle))
        if callback:
            callback(step, out)
        if not recycle:
            sites = out["sites"]
            step += 1
            continue
        sites = truncate(out["thetas"], links, Rf, Lf)
        step += 1
        for _ in range(n_re - 1):
            if step >= nsteps:
                break
            sites = truncate([gates.apply_ipepo(g, a) for a in sites], links, Rf, Lf)
            step += 1
    return sites, log
