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
  R + 1e-14 tr(R) I; one pass over the links in cell order (r, d, l, u for
  the checkerboard), each link iterated until |df|/f_0 < tol;
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
# bond environment
# ---------------------------------------------------------------------------

def theta_hat(cell, thetas, P, Q, site, open_leg):
    """Theta of ``site`` with every leg except ``open_leg`` truncated."""
    links, leg_link = cell_links(cell)
    t = thetas[site]
    for leg in LEGS:
        if leg == open_leg:
            continue
        b = leg_link[site][leg]
        s1, l1, s2, l2 = links[b]
        if site == s1 and leg == l1:
            t = apply_leg(t, leg, P[b].T)
        else:
            t = apply_leg(t, leg, Q[b])
    return t


def _find_h(cell, s1, s2):
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            if cell.sites[cell.pos(x, y)] == s1 and cell.sites[cell.pos(x + 1, y)] == s2:
                return x, y
    raise ValueError("link not found")


def _n_horizontal(cell, C, T, x, y, ket1, ket2):
    p, q = cell.pos(x, y), cell.pos(x + 1, y)
    L = np.einsum("gh,hpqt,eijg,fe,bmnf,sikmp,sjlnq->tklb",
                  C[p, 0], T[p, 0], T[p, 3], C[p, 3], T[p, 2], ket1, ket1, optimize=PATH_HALF)
    R = np.einsum("tpqh,he,eklf,fg,gmnb,sikmp,sjlnq->tijb",
                  T[q, 0], C[q, 1], T[q, 1], C[q, 2], T[q, 2], ket2, ket2, optimize=PATH_HALF)
    return np.einsum("tkKb,tiIb->kiKI", L, R, optimize=True)


def bond_environment(cell, thetas, P, Q, C, T, b):
    """N[i, j, i', j'] of link b (see module docstring); the environment C,
    T belongs to the pre-truncated state on ``cell``."""
    links, _ = cell_links(cell)
    s1, l1, s2, l2 = links[b]
    t1 = theta_hat(cell, thetas, P, Q, s1, l1)
    t2 = theta_hat(cell, thetas, P, Q, s2, l2)
    if l1 == "r":
        x, y = _find_h(cell, s1, s2)
        N = _n_horizontal(cell, C, T, x, y, t1, t2)
    else:
        # a vertical link is horizontal in the lattice rotated by 90 degrees
        rc, rt, rC, rT = rotate_ccw(cell, [t1, t2], C, T)
        x, y = None, None
        for yy in range(cell.Ly):
            for xx in range(cell.Lx):
                if cell.sites[cell.pos(xx, yy)] == s1 and cell.sites[cell.pos(xx, yy + 1)] == s2:
                    x, y = xx, yy
                    break
            if x is not None:
                break
        if x is None:
            raise ValueError("link not found")
        N = _n_horizontal(rc, rC, rT, y, -x, rt[0], rt[1])
    n = N.shape[0]
    N2 = N.reshape(n * n, n * n)
    N = (0.5 * (N2 + N2.T)).reshape(n, n, n, n)
    # the boundary fixes N only up to an overall factor (its tensors are
    # normalised, their sign is free): take the sign with <I|N|I> > 0
    if np.einsum("iiaa->", N) < 0:
        N = -N
    return N


# ---------------------------------------------------------------------------
# ALS (Eqs. (var), (var1))
# ---------------------------------------------------------------------------

def cost(N, P, Q):
    """f = <I|N|I> - 2 <PQ|N|I> + <PQ|N|PQ> (Eq. (var), real case)."""
    n = N.shape[0]
    I = np.eye(n)
    O = P @ Q
    t = np.einsum("ijab,ij,ab->", N, I, I)
    c = np.einsum("ijab,ij,ab->", N, O, I)
    q = np.einsum("ijab,ij,ab->", N, O, O)
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


def als(N, P, Q, tol=1e-12, max_sweeps=50):
    """Alternating least squares for one link.  Returns (P, Q, f, sweeps,
    history) with history the cost after each sweep."""
    n, D = P.shape
    trace_b = np.einsum("ijaa->ij", N)            # sum_i' N[i,j,i',i']
    f, f0 = cost(N, P, Q)
    hist = [f]
    sw = 0
    for sw in range(1, max_sweeps + 1):
        # P with Q fixed
        R = np.einsum("cj,ijak,dk->icad", Q, N, Q).reshape(n * D, n * D)
        S = np.einsum("cj,ij->ic", Q, trace_b).reshape(n * D)
        P = _solve(0.5 * (R + R.T), S).reshape(n, D)
        # Q with P fixed
        R = np.einsum("ic,ijak,ad->cjdk", P, N, P).reshape(D * n, D * n)
        S = np.einsum("ic,ij->cj", P, trace_b).reshape(D * n)
        Q = _solve(0.5 * (R + R.T), S).reshape(D, n)
        # balance the pair
        u, s, vt = _svd_signfix(P @ Q)
        sq = np.sqrt(s[:D])
        P, Q = u[:, :D] * sq[None, :], sq[:, None] * vt[:D]
        fn, _ = cost(N, P, Q)
        hist.append(fn)
        done = abs(fn - f) < tol * abs(f0)
        f = fn
        if done:
            break
    return P, Q, f, sw, hist


# ---------------------------------------------------------------------------
# drivers
# ---------------------------------------------------------------------------

def fu_env_step(cell, sites, g, D, chi, C, T, ctm_tol=1e-10, ctm_max=100, J=1.0, h=3.0,
                als_tol=1e-12, als_max=50):
    """One full-update step with a freshly computed environment: Theta = g A,
    pre-truncation, CTMRG (warm-started from C, T), energy, ALS on every link,
    A~ = Q Theta P.  Returns a dict."""
    links, _ = cell_links(cell)
    thetas = [gates.apply_ipepo(g, a) for a in sites]
    P, Q = su_truncation(cell, thetas, D)
    pre = truncate(thetas, links, P, Q)
    C, T, iters, delta = ctmrg(cell, pre, C, T, chi, ctm_max, ctm_tol)
    E = energy_per_site(cell, pre, C, T, J, h)
    costs = []
    for b in range(len(links)):
        N = bond_environment(cell, thetas, P, Q, C, T, b)
        P[b], Q[b], f, _, _ = als(N, P[b], Q[b], als_tol, als_max)
        costs.append(f)
    new = truncate(thetas, links, P, Q)
    return dict(sites=new, thetas=thetas, P=P, Q=Q, C=C, T=T, energy=E,
                ctm_iters=iters, ctm_delta=delta, costs=costs)


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


def run_fu(cell, sites, J, h, dt, D, chi, nsteps, n_re=1, n_warm=0, C=None, T=None,
           ctm_tol=1e-10, ctm_max=100, seed_env=0, callback=None):
    """Imaginary-time evolution of an iPEPS by full update, the environment
    recomputed every ``n_re`` steps after ``n_warm`` plain steps and the
    renormalized gate applied in between (Sec. VI C).  Returns (sites, log)
    with log entries (step, energy_per_site) at environment steps."""
    links, _ = cell_links(cell)
    g = gates.ipepo(J, h, dt)
    sites = [s / np.linalg.norm(s) for s in sites]
    npos = cell.Lx * cell.Ly
    if C is None:
        import tninputs
        C, T = tninputs.ctm_env(seed_env, npos, chi, D, positive=True)
    log, fac = [], None
    step = 0
    while step < nsteps:
        warm = step < n_warm
        out = fu_env_step(cell, sites, g, D, chi, C, T, ctm_tol, ctm_max, J, h)
        C, T = out["C"], out["T"]
        log.append((step + 1, out["energy"]))
        if callback:
            callback(step, out)
        if warm or n_re == 1:
            sites = out["sites"]
            step += 1
            continue
        a1, _, Pc, Qc, _ = canonicalize_a_form(cell, out["sites"])
        U0 = gauge_start(out["P"], out["Q"], Pc, Qc, g.shape[0])
        U, _, _ = gauge_fix(cell, sites, a1, U0=U0)
        Rf, Lf = renormalized_gate(out["P"], out["Q"], Pc, Qc, U)
        a0 = sites
        sites = truncate(out["thetas"], links, Rf, Lf)
        step += 1
        for _ in range(n_re - 1):
            if step >= nsteps:
                break
            sites = truncate([gates.apply_ipepo(g, a) for a in sites], links, Rf, Lf)
            step += 1
        del a0
    return sites, log
