"""Directional corner transfer matrix renormalization group (CTMRG).

Oracle (test infrastructure only).

The paper computes the environment of the double-layer network a = sum_s
A^s (x) A^s with the corner transfer matrix method (Sec. VI B, Fig. 21(a):
four corners C1..C4 and edges around the sites) but does not state the
projector scheme.  Reading taken: directional CTMRG on an Lx x Ly unit cell
with four-corner projectors from the SVD of the product of the two halves of
the 2x2 block, one projector per row cut, the move for one column absorbing
it into the left boundary for all rows.

Conventions
-----------
* Positions p = y * Lx + x, x to the right, y downwards, periodic.
* Site tensors A[s][l][r][d][u].
* Per position: C[p][k] (k=0..3: C1 top-left, C2 top-right, C3
  bottom-right, C4 bottom-left) and T[p][k] (T1 top, T2 right, T3 bottom,
  T4 left).  Boundary legs are ordered clockwise around the ring C1 T1 C2
  T2 C3 T3 C4 T4: C_k[a][b] has a towards the previous tensor in that ring
  and b towards the next; T_k[a][ket][bra][b] likewise, with (ket, bra)
  hooking onto the site leg facing it.
* A composite leg crossing a cut is ordered (boundary chi, ket D, bra D).
* Moves: left, up, right, down.  The up/right/down moves are the left move
  of the lattice rotated counter-clockwise by 90, 180, 270 degrees.
* Every new corner and edge is scaled to unit Frobenius norm.
* Singular values below 1e-14 times the largest are dropped when forming
  S^{-1/2}; each kept left singular vector is sign-fixed so that its first
  entry within a relative 1e-8 of the largest magnitude is positive.
* Convergence: per corner the singular values normalised to unit l2 norm;
  delta = max over corners of the l2 change between iterations.
"""
from __future__ import annotations

import numpy as np

CUT = 1e-14
# pairwise contraction order for (corner, edge, edge, ket, bra) networks:
# corner with the first edge, then the second edge, then ket, then bra
PATH4 = ["einsum_path", (0, 1), (0, 3), (0, 2), (0, 1)]


class Cell:
    """Unit cell geometry: Lx x Ly positions, ``sites[p]`` is the site index
    at position p."""

    def __init__(self, Lx, Ly, sites):
        self.Lx, self.Ly = Lx, Ly
        self.sites = list(sites)
        assert len(self.sites) == Lx * Ly

    def pos(self, x, y):
        return (y % self.Ly) * self.Lx + (x % self.Lx)


def rotate_ccw(cell, tensors, C, T):
    """Rotate the lattice picture counter-clockwise by 90 degrees.

    New coordinates (x', y') = (y, -x); the new left leg is the old up leg,
    new right = old down, new down = old left, new up = old right; the new
    C_k / T_k of a position is the old C_{k+1} / T_{k+1}."""
    Lx, Ly = cell.Lx, cell.Ly
    ncell_sites = [0] * (Lx * Ly)
    nC = np.empty_like(C)
    nT = np.empty_like(T)
    for xn in range(Ly):
        for yn in range(Lx):
            x, y = (-yn) % Lx, xn
            p_old = y * Lx + x
            p_new = yn * Ly + xn
            ncell_sites[p_new] = cell.sites[p_old]
            for k in range(4):
                nC[p_new, k] = C[p_old, (k + 1) % 4]
                nT[p_new, k] = T[p_old, (k + 1) % 4]
    ntens = [a.transpose(0, 4, 3, 1, 2) for a in tensors]
    return Cell(Ly, Lx, ncell_sites), ntens, nC, nT


def _svd_signfix(m):
    """SVD with each left singular vector's sign fixed: the first entry whose
    magnitude is within a relative 1e-8 of the largest is made positive (the
    tolerance makes the rule independent of rounding when symmetric inputs
    give vectors whose largest entries come in +- pairs)."""
    u, s, vt = np.linalg.svd(m)
    for i in range(u.shape[1]):
        a = np.abs(u[:, i])
        j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
        if u[j, i] < 0:
            u[:, i] = -u[:, i]
            vt[i, :] = -vt[i, :]
    return u, s, vt


def enlarged_corners(cell, tensors, C, T, x, y):
    """The four enlarged corners of the 2x2 block whose top-left site is
    (x, y), as matrices between composite cut legs:

    UL[(T4.a, dk, db), (T1.b, rk, rb)]   at (x, y)
    UR[(T1.a, lk, lb), (T2.b, dk, db)]   at (x+1, y)
    DL[(T4.b, uk, ub), (T3.a, rk, rb)]   at (x, y+1)
    DR[(T3.b, lk, lb), (T2.a, uk, ub)]   at (x+1, y+1)
    """
    chi = C.shape[-1]
    tl, tr = cell.pos(x, y), cell.pos(x + 1, y)
    bl, br = cell.pos(x, y + 1), cell.pos(x + 1, y + 1)
    a_tl, a_tr = tensors[cell.sites[tl]], tensors[cell.sites[tr]]
    a_bl, a_br = tensors[cell.sites[bl]], tensors[cell.sites[br]]
    D = a_tl.shape[1]
    n = chi * D * D
    ul = np.einsum("gh,hpqB,aijg,sikmp,sjlnq->amnBkl",
                   C[tl, 0], T[tl, 0], T[tl, 3], a_tl, a_tl, optimize=PATH4).reshape(n, n)
    ur = np.einsum("he,apqh,eklB,sikmp,sjlnq->aijBmn",
                   C[tr, 1], T[tr, 0], T[tr, 1], a_tr, a_tr, optimize=PATH4).reshape(n, n)
    dl = np.einsum("gh,amng,hijB,sikmp,sjlnq->Bpqakl",
                   C[bl, 3], T[bl, 2], T[bl, 3], a_bl, a_bl, optimize=PATH4).reshape(n, n)
    dr = np.einsum("eg,akle,gmnB,sikmp,sjlnq->Bijapq",
                   C[br, 2], T[br, 1], T[br, 2], a_br, a_br, optimize=PATH4).reshape(n, n)
    return ul, ur, dl, dr


def projectors(ul, ur, dl, dr, chi):
    """Projector pair for the left part of the cut between the two rows of
    the block.  With R_u = UL UR, R_d = DL DR and the SVD
    R_u^T R_d = W S V^T truncated to chi:
    P = R_d V S^{-1/2} (attached to the upper side of the cut) and
    Pt = S^{-1/2} W^T R_u^T (attached to the lower side), so that
    R_u^T P Pt R_d = W_chi S_chi V_chi^T.

    Returns (P [n][chi], Pt [chi][n], S)."""
    ru = ul @ ur
    rd = dl @ dr
    m = ru.T @ rd
    w, s, vt = _svd_signfix(m)
    k = min(chi, s.size)
    sk = s[:k]
    keep = sk > CUT * s[0]
    isq = np.where(keep, 1.0 / np.sqrt(np.where(keep, sk, 1.0)), 0.0)
    P = (rd @ vt[:k].T) * isq[None, :]
    Pt = isq[:, None] * (w[:, :k].T @ ru.T)
    if k < chi:                      # pad with zero columns if n < chi
        P = np.pad(P, ((0, 0), (0, chi - k)))
        Pt = np.pad(Pt, ((0, chi - k), (0, 0)))
    return P, Pt, s


def _normalize(t):
    nrm = np.linalg.norm(t)
    return t / nrm if nrm > 0 else t


def left_move(cell, tensors, C, T, x, chi):
    """Absorb column x into the left boundary (all rows), producing the C1,
    T4 and C4 of column x+1.  Returns new (C, T) arrays and the singular
    value lists of the projector problems."""
    Ly = cell.Ly
    Ps, Pts, spectra = [None] * Ly, [None] * Ly, [None] * Ly
    for y in range(Ly):
        ul, ur, dl, dr = enlarged_corners(cell, tensors, C, T, x, y)
        Ps[y], Pts[y], spectra[y] = projectors(ul, ur, dl, dr, chi)
    Cn, Tn = C.copy(), T.copy()
    D = T.shape[3]
    for y in range(Ly):
        src = cell.pos(x, y)
        dst = cell.pos(x + 1, y)
        a = tensors[cell.sites[src]]
        # C1 of (x+1, y+1): C1 T1 of (x, y+1), down leg projected with P_y
        s1 = cell.pos(x, y + 1)
        d1 = cell.pos(x + 1, y + 1)
        ct = np.einsum("ag,gkbB->akbB", C[s1, 0], T[s1, 0]).reshape(chi * D * D, chi)
        Cn[d1, 0] = _normalize(Ps[y].T @ ct)
        # T4 of (x+1, y): Pt_{y-1} (T4 a a) P_y; the up leg (T4.b, uk, ub)
        # takes Pt of the cut above row y, the down leg (T4.a, dk, db) takes
        # P of the cut below it
        pt = Pts[(y - 1) % Ly].reshape(chi, chi, D, D)
        pp = Ps[y].reshape(chi, D, D, chi)
        t4 = np.einsum("cBpq,aijB,sikmp,sjlnq,amne->eklc",
                       pt, T[src, 3], a, a, pp, optimize=PATH4)
        Tn[dst, 3] = _normalize(t4)
        # C4 of (x+1, y): C4 T3 of (x, y), up leg projected with Pt_y
        z = np.einsum("akbg,gB->aBkb", T[src, 2], C[src, 3]).reshape(chi, chi * D * D)
        Cn[dst, 3] = _normalize(z @ Pts[y].T)
    return Cn, Tn, spectra


def corner_spectra(C):
    """Singular values of every corner, each normalised to unit l2 norm;
    shape [npos][4][chi]."""
    out = np.empty(C.shape[:3])
    for p in range(C.shape[0]):
        for k in range(4):
            s = np.linalg.svd(C[p, k], compute_uv=False)
            out[p, k] = s / np.linalg.norm(s)
    return out


def iteration(cell, tensors, C, T, chi):
    """One CTMRG iteration: left, up, right and down moves, each sweeping
    every column of the (rotated) cell in increasing x."""
    for _ in range(4):
        for x in range(cell.Lx):
            C, T, _ = left_move(cell, tensors, C, T, x, chi)
        cell, tensors, C, T = rotate_ccw(cell, tensors, C, T)
    return C, T


def ctmrg(cell, tensors, C, T, chi, max_iter=100, tol=1e-10):
    """Iterate until delta < tol (delta as in the module docstring), or
    until delta stalls: after 20 iterations, the best delta of the last 10
    is not below 0.9 times the best before them (reading taken where the
    paper is silent: a rate that slow, above 0.9895 per iteration, would not
    reach tol within hundreds of iterations, and a cut through a dense part
    of the projector spectrum keeps delta fluctuating without a trend).
    Returns (C, T, iters, delta)."""
    C = np.array(C, dtype=np.float64)
    T = np.array(T, dtype=np.float64)
    prev = corner_spectra(C)
    delta, it = np.inf, 0
    hist = []
    for it in range(1, max_iter + 1):
        C, T = iteration(cell, tensors, C, T, chi)
        cur = corner_spectra(C)
        delta = float(np.max(np.linalg.norm(cur - prev, axis=-1)))
        prev = cur
        hist.append(delta)
        if delta < tol:
            break
        if len(hist) >= 20 and min(hist[-10:]) > 0.9 * min(hist[:-10]):
            break
    return C, T, it, delta
