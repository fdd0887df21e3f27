"""iPEPS observables, canonical form and gauge fixing.

Oracle (test infrastructure only).

* Reduced density matrices and the TFIM energy from a CTM environment
  (Sec. VI D: energy per link, magnetisation m_z).  Reading taken for the
  units: energy per site = mean over positions of the bond energies of the
  position's right and down bonds plus its field energy; the paper's energy
  per link on the square lattice is that divided by 2.
* Canonical form of an iPEPS (Sec. IV A, Eqs. (17)-(20)) by the paper's
  iteration (steps (i)-(iii), Fig. 11), generalised to a unit cell with one
  bond spectrum per inequivalent link.  Reading taken for the missing
  figure: for a link between the r (or d) leg of site X and the l (or u) leg
  of site Y, V_1 is the Gram matrix of Gamma_X on that leg with the full
  lambda's on X's other three legs (left hand side of Eq. (17) or (19)),
  V_2 the Gram matrix of Gamma_Y on its leg with lambda's on Y's other legs
  (Eq. (18) or (20)); per link the 1D rule applies: V_1 = Y^T Y,
  V_2 = X X^T, SVD Y lambda X = U S V^T, Gamma_X <- Gamma_X Y^+ U on that
  leg, Gamma_Y <- V^T X^+ Gamma_Y, lambda <- S.  The printed step (ii) uses
  lambda_h for the vertical SVD; lambda_v is read.
* Gauge fixing (Sec. IV B, Eq. (25)): one orthogonal U per link applied to
  both of its legs, maximising the fidelity by alternating Procrustes steps.
* The A form puts sqrt(lambda) on all four legs (Sec. IV B).
"""
from __future__ import annotations

import numpy as np

from .ctmrg import Cell, rotate_ccw
from . import gates
from .imps import polar_orthogonal

CUT = 1e-14
# contraction orders: ring of the 3x3 network, and a half of the 2x4 network
PATH_RING = ["einsum_path", (0, 1), (0, 8), (4, 7), (4, 6), (4, 5), (0, 4), (0, 3),
             (0, 2), (0, 1)]
PATH_HALF = ["einsum_path", (0, 1), (0, 5), (2, 4), (2, 3), (0, 1), (0, 1)]
LEGS = {"l": 1, "r": 2, "d": 3, "u": 4}


# ---------------------------------------------------------------------------
# cell links
# ---------------------------------------------------------------------------

def cell_links(cell):
    """Inequivalent links of a unit cell, in first-seen order over positions
    (r link then d link of each position): list of (site1, leg1, site2,
    leg2) with leg1 in {r, d} and leg2 the matching {l, u}.  Also returns
    leg_link[site][leg] -> link index.  For the checkerboard this gives
    0: A.r-B.l, 1: A.d-B.u, 2: B.r-A.l, 3: B.d-A.u."""
    links, index = [], {}
    nsite = max(cell.sites) + 1
    leg_link = [dict() for _ in range(nsite)]
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            s = cell.sites[cell.pos(x, y)]
            for leg1, leg2, (dx, dy) in (("r", "l", (1, 0)), ("d", "u", (0, 1))):
                t = cell.sites[cell.pos(x + dx, y + dy)]
                key = (s, leg1, t)
                if key not in index:
                    index[key] = len(links)
                    links.append((s, leg1, t, leg2))
                b = index[key]
                for site, leg in ((s, leg1), (t, leg2)):
                    if leg_link[site].get(leg, b) != b:
                        raise ValueError("cell assigns two links to one leg")
                    leg_link[site][leg] = b
    return links, leg_link


def apply_leg(t, leg, m):
    """new[..., i, ...] = sum_a m[i, a] t[..., a, ...] on leg ``leg``."""
    ax = LEGS[leg]
    return np.moveaxis(np.tensordot(m, t, axes=([1], [ax])), 0, ax)


def truncate(thetas, links, P, Q):
    """Insert P_b on the first leg and Q_b on the second leg of every link
    (A~ = Q Theta P, Sec. VI B); returns normalised tensors."""
    out = [t.copy() for t in thetas]
    for b, (s1, l1, s2, l2) in enumerate(links):
        out[s1] = apply_leg(out[s1], l1, P[b].T)
        out[s2] = apply_leg(out[s2], l2, Q[b])
    return [o / np.linalg.norm(o) for o in out]


# ---------------------------------------------------------------------------
# reduced density matrices and energy
# ---------------------------------------------------------------------------

def rdm_one(C, T, p, a):
    """One-site density matrix at position p (3x3 CTM network)."""
    r = np.einsum("ab,bpqc,cd,dkle,ef,fmng,gh,hija,sikmp,Sjlnq->sS",
                  C[p, 0], T[p, 0], C[p, 1], T[p, 1], C[p, 2], T[p, 2],
                  C[p, 3], T[p, 3], a, a, optimize=PATH_RING)
    return r / np.trace(r)


def _half_left(C, T, p, ket, bra, open_phys):
    """Left half of a horizontal two-site network at position p: C1 T1 T4
    C4 T3 with the site; open legs (T1.b, [s, s'], rk, rb, T3.a)."""
    if open_phys:
        return np.einsum("gh,hpqt,eijg,fe,bmnf,sikmp,Sjlnq->tsSklb",
                         C[p, 0], T[p, 0], T[p, 3], C[p, 3], T[p, 2], ket, bra, optimize=PATH_HALF)
    return np.einsum("gh,hpqt,eijg,fe,bmnf,sikmp,sjlnq->tklb",
                     C[p, 0], T[p, 0], T[p, 3], C[p, 3], T[p, 2], ket, bra, optimize=PATH_HALF)


def _half_right(C, T, q, ket, bra, open_phys):
    """Right half at position q: T1 C2 T2 C3 T3 with the site; open legs
    (T1.a, [s, s'], lk, lb, T3.b)."""
    if open_phys:
        return np.einsum("tpqh,he,eklf,fg,gmnb,sikmp,Sjlnq->tsSijb",
                         T[q, 0], C[q, 1], T[q, 1], C[q, 2], T[q, 2], ket, bra, optimize=PATH_HALF)
    return np.einsum("tpqh,he,eklf,fg,gmnb,sikmp,sjlnq->tijb",
                     T[q, 0], C[q, 1], T[q, 1], C[q, 2], T[q, 2], ket, bra, optimize=PATH_HALF)


def rdm_two_h(cell, tensors, C, T, x, y):
    """Two-site density matrix of the horizontal pair (x,y)-(x+1,y), as a
    4x4 matrix on (s1 s2),(s1' s2')."""
    p, q = cell.pos(x, y), cell.pos(x + 1, y)
    a, b = tensors[cell.sites[p]], tensors[cell.sites[q]]
    L = _half_left(C, T, p, a, a, True)
    R = _half_right(C, T, q, b, b, True)
    r = np.einsum("tsSklb,tuUklb->suSU", L, R).reshape(4, 4)
    return r / np.trace(r)


def rdms(cell, tensors, C, T):
    """All RDMs: one-site rho1[p], horizontal rhoh[p] (p with its right
    neighbour) and vertical rhov[p] (p with the site below, top site first)."""
    npos = cell.Lx * cell.Ly
    rho1 = [rdm_one(C, T, p, tensors[cell.sites[p]]) for p in range(npos)]
    rhoh = [None] * npos
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            rhoh[cell.pos(x, y)] = rdm_two_h(cell, tensors, C, T, x, y)
    rc, rt, rC, rT = rotate_ccw(cell, tensors, C, T)
    rhov = [None] * npos
    for y in range(cell.Ly):
        for x in range(cell.Lx):
            # old (x, y) sits at new (y, -x); its lower neighbour at new (y+1, -x)
            rhov[cell.pos(x, y)] = rdm_two_h(rc, rt, rC, rT, y, -x)
    return rho1, rhoh, rhov


def energy_per_site(cell, tensors, C, T, J, h):
    """TFIM energy per site (Sec. VI A Hamiltonian); the paper's energy per
    link is this divided by 2."""
    zz = np.kron(gates.SZ, gates.SZ)
    rho1, rhoh, rhov = rdms(cell, tensors, C, T)
    npos = len(rho1)
    e = 0.0
    for p in range(npos):
        e += -J * np.trace(rhoh[p] @ zz) - J * np.trace(rhov[p] @ zz)
        e += -h * np.trace(rho1[p] @ gates.SX)
    return float(e / npos)


def magnetization_z(cell, tensors, C, T):
    """m_z = <sz> averaged over positions (Sec. VI D)."""
    npos = cell.Lx * cell.Ly
    return float(np.mean([np.trace(rdm_one(C, T, p, tensors[cell.sites[p]]) @ gates.SZ)
                          for p in range(npos)]))


# ---------------------------------------------------------------------------
# canonical form (Sec. IV A)
# ---------------------------------------------------------------------------

def _weighted(g, leg_link_s, lams, skip):
    """Gamma with the full lambda of each leg's link multiplied on every leg
    except ``skip``."""
    t = g
    for leg, ax in LEGS.items():
        if leg == skip:
            continue
        lam = lams[leg_link_s[leg]]
        shape = [1] * 5
        shape[ax] = lam.size
        t = t * lam.reshape(shape)
    return t


def _gram(t, leg):
    ax = LEGS[leg]
    m = np.moveaxis(t, ax, 0).reshape(t.shape[ax], -1)
    return m @ m.T


def _signfix_cols(u, vt=None):
    """Make the first entry within 1e-8 of each column's largest magnitude
    positive (flipping the matching row of vt)."""
    for i in range(u.shape[1]):
        a = np.abs(u[:, i])
        j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
        if u[j, i] < 0:
            u[:, i] = -u[:, i]
            if vt is not None:
                vt[i, :] = -vt[i, :]
    return u, vt


def _sqrt_factor(v):
    """v = F F^T with F = W sqrt(S); returns (F, pinv(F))."""
    v = 0.5 * (v + v.T)
    s, w = np.linalg.eigh(v)
    keep = s > CUT * s.max()
    sq = np.where(keep, np.sqrt(np.abs(s)), 0.0)
    isq = np.where(keep, 1.0 / np.where(keep, sq, 1.0), 0.0)
    return w * sq, (w * isq).T


def canonicalize(cell, gammas, lams=None, tol=1e-14, max_iter=1000):
    """Iterate the paper's canonicalization (Sec. IV A) on all links at once.

    Returns (gammas, lams, iters, TR, TL): TR[b] is the accumulated right
    transform of link b's first leg (Gamma_1 <- Gamma_1 TR on that leg) and
    TL[b] that of its second leg (Gamma_2 <- TL Gamma_2)."""
    links, leg_link = cell_links(cell)
    gammas = [g.copy() for g in gammas]
    dims = [gammas[s1].shape[LEGS[l1]] for (s1, l1, _, _) in links]
    if lams is None:
        lams = [np.full(n, 1.0 / np.sqrt(n)) for n in dims]
    lams = [l / np.linalg.norm(l) for l in lams]
    TR = [np.eye(n) for n in dims]
    TL = [np.eye(n) for n in dims]
    it = 0
    for it in range(1, max_iter + 1):
        upd, newl = [], []
        for b, (s1, l1, s2, l2) in enumerate(links):
            v1 = _gram(_weighted(gammas[s1], leg_link[s1], lams, l1), l1)
            v2 = _gram(_weighted(gammas[s2], leg_link[s2], lams, l2), l2)
            Yt, Ytinv = _sqrt_factor(v1)
            X, Xinv = _sqrt_factor(v2)
            u, s, vt = np.linalg.svd(Yt.T @ np.diag(lams[b]) @ X)
            # the sign rule acts on the transform itself, which does not
            # depend on the eigenbases chosen for V_1 and V_2
            r, l = _signfix_cols(Ytinv.T @ u, vt @ Xinv)
            upd.append((r, l))
            newl.append(s / np.linalg.norm(s))
        for b, (s1, l1, s2, l2) in enumerate(links):
            r, l = upd[b]
            gammas[s1] = apply_leg(gammas[s1], l1, r.T)
            gammas[s2] = apply_leg(gammas[s2], l2, l)
            TR[b] = TR[b] @ r
            TL[b] = l @ TL[b]
            # only the direction of the accumulated transforms matters
            TR[b] = TR[b] / np.linalg.norm(TR[b])
            TL[b] = TL[b] / np.linalg.norm(TL[b])
        delta = max(float(np.max(np.abs(newl[b] - lams[b]))) for b in range(len(links)))
        lams = newl
        gammas = [g / np.linalg.norm(g) for g in gammas]
        if delta < tol:
            break
    # the canonical gauge is unique up to the sign of each bond index: fix it
    # on the columns of the accumulated first-end transform (rows of the
    # second-end one flip with them), independently of the iteration's path
    for b, (s1, l1, s2, l2) in enumerate(links):
        before = TR[b].copy()
        TR[b], TL[b] = _signfix_cols(TR[b].copy(), TL[b].copy())
        sg = np.where(np.sum(before * TR[b], axis=0) < 0, -1.0, 1.0)
        gammas[s1] = apply_leg(gammas[s1], l1, np.diag(sg))
        gammas[s2] = apply_leg(gammas[s2], l2, np.diag(sg))
    return gammas, lams, it, TR, TL


def canonical_residual(cell, gammas, lams):
    """Largest deviation of the four constraint matrices of Eqs. (17)-(20)
    from a multiple of the identity, per unit trace."""
    links, leg_link = cell_links(cell)
    out = 0.0
    for s, g in enumerate(gammas):
        for leg in LEGS:
            m = _gram(_weighted(g, leg_link[s], lams, leg), leg)
            m = m / (np.trace(m) / m.shape[0])
            out = max(out, float(np.max(np.abs(m - np.eye(m.shape[0])))))
    return out


def a_form(cell, gammas, lams):
    """A = sqrt(lambda) on all four legs of Gamma, unit Frobenius norm."""
    links, leg_link = cell_links(cell)
    out = []
    for s, g in enumerate(gammas):
        t = g
        for leg, ax in LEGS.items():
            lam = np.sqrt(lams[leg_link[s][leg]])
            shape = [1] * 5
            shape[ax] = lam.size
            t = t * lam.reshape(shape)
        out.append(t / np.linalg.norm(t))
    return out


def canonical_pq(TR, TL, lams):
    """Pc = TR sqrt(lambda), Qc = sqrt(lambda) TL per link.  Without
    truncation the two are inverse up to a factor (the iteration keeps
    TR lambda TL proportional to the identity); the factor and the split of
    scale between them, which the normalisation of the sites removes, are
    fixed by Pc Qc = I and |Pc|_F = |Qc|_F."""
    Pc, Qc = [], []
    for b in range(len(TR)):
        p = TR[b] * np.sqrt(lams[b])[None, :]
        q = np.sqrt(lams[b])[:, None] * TL[b]
        m = np.sqrt(p.shape[0] / np.trace(p @ q))
        p, q = p * m, q * m
        r = np.sqrt(np.linalg.norm(q) / np.linalg.norm(p))
        Pc.append(p * r)
        Qc.append(q / r)
    return Pc, Qc


def canonicalize_a_form(cell, tensors, tol=1e-14, max_iter=1000):
    """Canonicalize A-form tensors (starting from flat lambdas) and return
    (A1, lams, Pc, Qc, iters) with A1 = Qc/Pc applied to ``tensors``: Pc[b]
    on link b's first leg (new = Pc^T old), Qc[b] on its second leg."""
    links, _ = cell_links(cell)
    g, lams, it, TR, TL = canonicalize(cell, tensors, None, tol, max_iter)
    Pc, Qc = canonical_pq(TR, TL, lams)
    a1 = truncate(tensors, links, Pc, Qc)
    return a1, lams, Pc, Qc, it


# ---------------------------------------------------------------------------
# gauge fixing (Sec. IV B)
# ---------------------------------------------------------------------------

def _apply_all(t, site, leg_link, U, skip=None):
    for leg in LEGS:
        if leg == skip:
            continue
        t = apply_leg(t, leg, U[leg_link[site][leg]])
    return t


def fidelity(cell, a_ref, a_new, U):
    links, leg_link = cell_links(cell)
    num = sum(np.sum(a_new[s] * _apply_all(a_ref[s], s, leg_link, U)) for s in range(len(a_ref)))
    den = sum(np.linalg.norm(a) * np.linalg.norm(b) for a, b in zip(a_ref, a_new))
    return float(num / den)


def gauge_fix(cell, a_ref, a_new, tol=1e-12, max_iter=1000, U0=None):
    """Find orthogonal U_b per link with a_new ~ U(a_ref) (U_b applied as
    new = U_b old on both legs of link b) by maximising the fidelity of
    Eq. (25): for each link in turn, with every other factor (including the
    other occurrence of U_b when both legs sit on one tensor, as in the
    paper's step (i)) held fixed, the fidelity is linear in U_b with
    coefficient K and the maximiser is U_b = W V^T from K = W S V^T.
    Returns (U, F, iters)."""
    links, leg_link = cell_links(cell)
    dims = [a_ref[s1].shape[LEGS[l1]] for (s1, l1, _, _) in links]

    def coeff(U, b):
        s1, l1, s2, l2 = links[b]
        K = np.zeros((dims[b], dims[b]))
        for site, leg in ((s1, l1), (s2, l2)):
            rest = _apply_all(a_ref[site], site, leg_link, U, skip=leg)
            ax = LEGS[leg]
            K += np.moveaxis(a_new[site], ax, 0).reshape(dims[b], -1) @ \
                np.moveaxis(rest, ax, 0).reshape(dims[b], -1).T
        return K

    U = [np.eye(n) for n in dims] if U0 is None else [u.copy() for u in U0]
    F = fidelity(cell, a_ref, a_new, U)
    it = 0
    for it in range(1, max_iter + 1):
        for b in range(len(links)):
            U[b] = polar_orthogonal(coeff(U, b))
        Fn = fidelity(cell, a_ref, a_new, U)
        done = abs(Fn - F) < tol
        F = Fn
        if done:
            break
    return U, F, it
