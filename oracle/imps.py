"""1D iMPS pieces of environment-recycled iTEBD.

Oracle (test infrastructure only).

State convention: a two-site unit cell in the symmetric "A form"
A_X = sqrt(lambda_left) Gamma_X sqrt(lambda_right) (the form the paper uses
for recycling, Sec. V B step (i)), each of shape [chi][d][chi]; the chain is
... A_A A_B A_A A_B ...; bond 0 is A_A's right bond (A_A -> A_B), bond 1 is
A_B's right bond (A_B -> A_A).

Readings taken where the paper is silent (real arithmetic throughout):
* the transpose replaces the Hermitian conjugate and orthogonal matrices
  replace unitaries; imaginary-time TFIM evolution from a real state stays
  real;
* the left resolution of the identity: a left Gram matrix V_L = Y^T Y has
  Y = sqrt(S) W^T from V_L = W S W^T, the bond matrix whose SVD gives the new
  Schmidt values is Y lambda X; the paper writes it as Y^T lambda X with the
  transposed convention for Y; the singular values are the same;
* eigen/singular values below 1e-14 times the largest are dropped in
  pseudo-inverses;
* tensors are rescaled to unit Frobenius norm after each step and the bond
  spectra to unit l2 norm.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import gates

CUT = 1e-14


# ---------------------------------------------------------------------------
# transfer-matrix fixed points
# ---------------------------------------------------------------------------

def _tm_apply_left(kets, bras, v):
    """One application of the unit-cell transfer matrix from the left:
    v[a][a'] -> sum_s K^s^T v B^s for every site in order (ket K, bra B)."""
    for k, b in zip(kets, bras):
        n1, d, n2 = k.shape
        t = (v.T @ k.reshape(n1, d * n2)).reshape(-1, d * n2)   # [a', (s c)]
        v = t.reshape(-1, d, n2).transpose(2, 0, 1).reshape(n2, -1) @ \
            b.reshape(-1, n2)                                    # sum over (a', s)
    return v


def _tm_apply_right(kets, bras, v):
    """From the right: v[b][b'] -> sum_s K^s v B^s^T, last site first."""
    for k, b in zip(reversed(kets), reversed(bras)):
        n1, d, n2 = k.shape
        t = k.reshape(n1 * d, n2) @ v                            # [(a s), d']
        v = t.reshape(n1, d * n2) @ b.reshape(-1, d * n2).T      # sum over (s, d')
    return v


def _dominant(apply, n, v0):
    """Dominant eigenpair of a linear map on n x n matrices via ARPACK
    (k=1, largest magnitude), with a deterministic start vector."""
    op = spla.LinearOperator((n * n, n * n), matvec=lambda x: apply(x.reshape(n, n)).ravel(),
                             dtype=np.float64)
    if n * n <= 64:
        m = np.column_stack([op.matvec(e) for e in np.eye(n * n)])
        w, vec = np.linalg.eig(m)
        i = int(np.argmax(np.abs(w)))
        return w[i], vec[:, i]
    w, vec = spla.eigs(op, k=1, which="LM", v0=v0.ravel(), tol=1e-14, ncv=24, maxiter=100000)
    return w[0], vec[:, 0]


def tm_fixed_point(kets, bras):
    """Dominant left and right eigenvectors of the unit-cell transfer matrix
    built from ket tensors ``kets`` and bra tensors ``bras`` (lists over the
    cell, each [chi][d][chi]) -- the 1D environment (Sec. III A;
    Eq. (iMPSDM1) for the mixed ket/bra case).

    Returns (vl, vr, eta) with vl[a][a'] and vr[b][b'] indexed (ket, bra),
    eta vl = sum_s K^T vl B over the cell and eta vr = sum_s K vr B^T;
    normalised so that ||vl||_F = 1, Tr(vl) > 0 and sum(vl * vr) = 1.
    """
    n = kets[0].shape[0]
    v0 = np.eye(n)
    etal, xl = _dominant(lambda v: _tm_apply_left(kets, bras, v), n, v0)
    etar, xr = _dominant(lambda v: _tm_apply_right(kets, bras, v), n, v0)
    if abs(etal.imag) > 1e-10 * abs(etal) or abs(etar.imag) > 1e-10 * abs(etar):
        raise ValueError("dominant transfer-matrix eigenvalue is not real")
    vl = np.real(xl).reshape(n, n)
    vr = np.real(xr).reshape(n, n)
    vl = vl / np.linalg.norm(vl)
    if np.trace(vl) < 0:
        vl = -vl
    vr = vr / np.sum(vl * vr)
    return vl, vr, float(np.real(etal))


# ---------------------------------------------------------------------------
# resolutions of the identity and truncation
# ---------------------------------------------------------------------------

def _sym_sqrt_factors(v):
    """For a symmetric positive semi-definite v = W S W^T return (F, Finv)
    with F = W sqrt(S) (so v = F F^T) and the pseudo-inverse Finv of F;
    eigenvalues below CUT * max are dropped."""
    v = 0.5 * (v + v.T)
    s, w = np.linalg.eigh(v)
    if s[-1] < 0:               # fixed point came out negative definite
        s, w = -s[::-1], w[:, ::-1]
    # eigenvector signs: first entry within 1e-8 of the largest magnitude positive
    for i in range(w.shape[1]):
        a = np.abs(w[:, i])
        j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
        if w[j, i] < 0:
            w[:, i] = -w[:, i]
    keep = s > CUT * s.max()
    sq = np.where(keep, np.sqrt(np.abs(s)), 0.0)
    isq = np.where(keep, 1.0 / np.where(keep, sq, 1.0), 0.0)
    return w * sq, (w * isq).T


def truncation_pq(vl, vr, chi):
    """Truncation of one bond of an A-form iMPS from its environment
    (Eq. (EqCanoPQ1)).

    vl is the Gram matrix of the half-chain to the left of the bond, vr that
    of the half-chain to the right.  With vl = Y^T Y, vr = X X^T and the SVD
    Y X = U S V^T, the identity on the bond is Y^+ U S V^T X^+; keeping the
    chi largest singular values and giving sqrt(S) to both sides gives
    P = Y^+ U_chi sqrt(S_chi) (attached to the left site's right leg) and
    Q = sqrt(S_chi) V_chi^T X^+ (attached to the right site's left leg).

    Returns (P, Q, S) with S the full singular value list (descending).
    """
    Yt, Ytinv = _sym_sqrt_factors(vl)        # vl = Yt Yt^T, Y = Yt^T
    X, Xinv = _sym_sqrt_factors(vr)          # vr = X X^T
    Y, Yinv = Yt.T, Ytinv.T
    u, s, vt = np.linalg.svd(Y @ X)
    # sign of each singular pair: first entry of u within 1e-8 of its largest
    # magnitude positive (fixes the gauge of the new bond index)
    for i in range(u.shape[1]):
        a = np.abs(u[:, i])
        j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
        if u[j, i] < 0:
            u[:, i] = -u[:, i]
            vt[i, :] = -vt[i, :]
    sq = np.sqrt(s[:chi])
    P = Yinv @ (u[:, :chi] * sq)
    Q = (sq[:, None] * vt[:chi]) @ Xinv
    return P, Q, s


def bond_fixed_points(sites, bond):
    """Left/right Gram matrices at ``bond`` of a two-site A-form chain.

    Bond 0 sits after site 0, bond 1 after site 1.  The half-chain to the
    left of bond b ends with site b; the one to the right starts with the
    other site."""
    a, b = (sites[0], sites[1]) if bond == 0 else (sites[1], sites[0])
    # cell [b, a]: its left fixed point ends with a, its right one starts with b
    vl, vr, _ = tm_fixed_point([b, a], [b, a])
    return vl, vr


def itebd_plain_step(sites, g, chi):
    """One plain iTEBD step on a two-site A-form iMPS (Sec. V B, first
    paragraph): Theta = g A (bond kappa*chi), environment from the
    transfer-matrix fixed points of the Theta chain, truncation A~ = Q Theta P.

    Returns (new_sites, P, Q, spectra, trunc_err) where P[b], Q[b] belong to
    bond b, spectra[b] is the normalised kept spectrum and trunc_err sums the
    discarded weight of both bonds."""
    th = [gates.apply_impo(g, s) for s in sites]
    P, Q, spec, err = [None, None], [None, None], [None, None], 0.0
    for bnd in (0, 1):
        vl, vr = bond_fixed_points(th, bnd)
        P[bnd], Q[bnd], s = truncation_pq(vl, vr, chi)
        w = s ** 2
        err += float(w[chi:].sum() / w.sum())
        spec[bnd] = s[:chi] / np.linalg.norm(s[:chi])
    # site 0 sits between bond 1 (left) and bond 0 (right); site 1 the reverse
    new = [np.einsum("ia,asb,bj->isj", Q[1], th[0], P[0], optimize=True),
           np.einsum("ia,asb,bj->isj", Q[0], th[1], P[1], optimize=True)]
    new = [t / np.linalg.norm(t) for t in new]
    return new, P, Q, spec, err


# ---------------------------------------------------------------------------
# energy
# ---------------------------------------------------------------------------

def two_site_rdms(sites):
    """Two-site reduced density matrices rho[b] (4x4 on (s1 s2),(t1 t2)) for
    the pair (site b, site b+1), from the exact transfer-matrix environment
    of the A-form chain; trace 1."""
    rhos = []
    for b in (0, 1):
        a, c = sites[b], sites[1 - b]
        # cell [a, c]: left environment ends with c (just before a), right
        # environment starts with a (just after c)
        vl, vr, _ = tm_fixed_point([a, c], [a, c])
        m = np.einsum("asb,btc->astc", a, c)
        rho = np.einsum("xy,xstc,yuvd,cd->stuv", vl, m, m, vr).reshape(4, 4)
        rhos.append(rho / np.trace(rho))
    return rhos


def energy_per_site(sites, J, h):
    """Energy per site of the TFIM (Sec. V A), equal to the paper's energy
    per link in 1D: the mean over the two bonds of <-J sz sz> plus the mean
    over the two sites of <-h sx>."""
    zz = np.kron(gates.SZ, gates.SZ)
    xi = np.kron(gates.SX, gates.ID)
    ix = np.kron(gates.ID, gates.SX)
    r0, r1 = two_site_rdms(sites)
    ezz = -J * 0.5 * (np.trace(r0 @ zz) + np.trace(r1 @ zz))
    ex = -h * 0.5 * (np.trace(r0 @ xi) + np.trace(r0 @ ix))
    return float(ezz + ex)


# ---------------------------------------------------------------------------
# canonical form (Sec. III A) for the Gamma-lambda two-site cell
# ---------------------------------------------------------------------------

def to_gamma_lambda(sites, lams):
    """Gamma_X = lambda_left^{-1/2} A_X lambda_right^{-1/2}."""
    il = [np.where(l > 0, 1.0 / np.sqrt(np.where(l > 0, l, 1.0)), 0.0) for l in lams]
    g0 = il[1][:, None, None] * sites[0] * il[0][None, None, :]
    g1 = il[0][:, None, None] * sites[1] * il[1][None, None, :]
    return [g0, g1]


def to_a_form(gams, lams):
    sq = [np.sqrt(l) for l in lams]
    a0 = sq[1][:, None, None] * gams[0] * sq[0][None, None, :]
    a1 = sq[0][:, None, None] * gams[1] * sq[1][None, None, :]
    return [a0, a1]


def canonicalize(gams, lams, tol=1e-14, max_iter=1000):
    """The paper's local iterative canonicalization (Sec. III A, steps
    (i)-(iii), Fig. 3) applied to both bonds of a two-site cell at once.

    At each bond b between site l (left) and site r (right):
    V_L = sum_s (lam_l Gamma_l^s)^T (lam_l Gamma_l^s),
    V_R = sum_s (Gamma_r^s lam_r)(Gamma_r^s lam_r)^T, V_L = Y^T Y,
    V_R = X X^T, SVD Y lam_b X = U S V^T; then Gamma_l <- Gamma_l Y^+ U,
    Gamma_r <- V^T X^+ Gamma_r, lam_b <- S.  Iterates until the spectra move
    by less than ``tol``.

    Returns (gams, lams, iters, TL, TR): TR[b] (right transform applied to the
    left site of bond b, product of the Y^+ U factors) and TL[b] (left
    transform applied to the right site, product of V^T X^+), so the final
    Gamma's are TL[left bond] Gamma_0 TR[right bond].
    """
    gams = [g.copy() for g in gams]
    lams = [l / np.linalg.norm(l) for l in lams]
    n = [gams[0].shape[2], gams[1].shape[2]]
    TR = [np.eye(n[0]), np.eye(n[1])]
    TL = [np.eye(n[0]), np.eye(n[1])]
    it = 0
    for it in range(1, max_iter + 1):
        newl, upd = [None, None], [None, None]
        for b in (0, 1):
            gl, gr = gams[b], gams[1 - b]
            lam_l, lam_r = lams[1 - b], lams[1 - b]
            x_l = lam_l[:, None, None] * gl
            x_r = gr * lam_r[None, None, :]
            VL = np.einsum("asb,asc->bc", x_l, x_l)
            VR = np.einsum("asb,csb->ac", x_r, x_r)
            Yt, Ytinv = _sym_sqrt_factors(VL)
            X, Xinv = _sym_sqrt_factors(VR)
            u, s, vt = np.linalg.svd(Yt.T @ np.diag(lams[b]) @ X)
            upd[b] = (Ytinv.T @ u, vt @ Xinv)
            newl[b] = s / np.linalg.norm(s)
        for b in (0, 1):
            r, l = upd[b]
            gams[b] = np.einsum("asb,bc->asc", gams[b], r)
            gams[1 - b] = np.einsum("ab,bsc->asc", l, gams[1 - b])
            TR[b] = TR[b] @ r
            TL[b] = l @ TL[b]
            # only the direction of the accumulated transforms matters
            TR[b] = TR[b] / np.linalg.norm(TR[b])
            TL[b] = TL[b] / np.linalg.norm(TL[b])
        delta = max(np.max(np.abs(newl[b] - lams[b])) for b in (0, 1))
        lams = newl
        # keep Gamma at a fixed scale so the iteration cannot drift
        gams = [g / np.linalg.norm(g) for g in gams]
        if delta < tol:
            break
    return gams, lams, it, TL, TR


def canonical_residual(gams, lams):
    """Largest deviation from the canonical constraints (Eqs.
    (iMPS_canonical_constraintL/R)) after fixing the overall scale of each
    constraint: sum_s Gamma^T lam_l^2 Gamma ~ I and sum_s Gamma lam_r^2
    Gamma^T ~ I."""
    out = 0.0
    for b in (0, 1):
        g = gams[b]
        lam_l, lam_r = lams[1 - b], lams[b]
        left = np.einsum("asb,a,asc->bc", g, lam_l ** 2, g)
        right = np.einsum("asb,b,csb->ac", g, lam_r ** 2, g)
        for m in (left, right):
            m = m / (np.trace(m) / m.shape[0])
            out = max(out, float(np.max(np.abs(m - np.eye(m.shape[0])))))
    return out


def canonicalize_a_form(sites, lams=None):
    """Canonicalize an A-form cell: returns (A1, lams1, Qc, Pc) with
    A1_X = Qc[left bond] A_X Pc[right bond] (Sec. V B step (i)).  ``lams``
    are the bond spectra the A form was built with (flat if unknown)."""
    if lams is None:
        lams = [np.full(sites[0].shape[2], 1.0), np.full(sites[1].shape[2], 1.0)]
    gams = to_gamma_lambda(sites, lams)
    g1, l1, _, TL, TR = canonicalize(gams, lams)
    a1 = to_a_form(g1, l1)
    # undo the rescaling of Gamma done inside the iteration: fit one scalar per site
    Pc, Qc = [None, None], [None, None]
    il = [np.where(l > 0, 1.0 / np.sqrt(np.where(l > 0, l, 1.0)), 0.0) for l in lams]
    for b in (0, 1):
        Pc[b] = (il[b][:, None] * TR[b]) * np.sqrt(l1[b])[None, :]
        Qc[b] = (np.sqrt(l1[b])[:, None] * TL[b]) * il[b][None, :]
    # the canonical gauge is unique up to the sign of each bond index: fix
    # it on the columns of Pc (rows of Qc flip with them), independently of
    # the path the iteration took
    for b in (0, 1):
        for i in range(Pc[b].shape[1]):
            a = np.abs(Pc[b][:, i])
            j = int(np.argmax(a >= (1.0 - 1e-8) * a.max()))
            if Pc[b][j, i] < 0:
                Pc[b][:, i] = -Pc[b][:, i]
                Qc[b][i, :] = -Qc[b][i, :]
        # the scale is free too: Pc and Qc are inverse up to a factor, and
        # Pc -> c Pc, Qc -> Qc / c is removed by the site normalisation; fix
        # Pc Qc = I and |Pc| = |Qc|
        m = np.sqrt(Pc[b].shape[0] / np.trace(Pc[b] @ Qc[b]))
        Pc[b], Qc[b] = Pc[b] * m, Qc[b] * m
        r = np.sqrt(np.linalg.norm(Qc[b]) / np.linalg.norm(Pc[b]))
        Pc[b], Qc[b] = Pc[b] * r, Qc[b] / r
    raw = [np.einsum("ia,asb,bj->isj", Qc[1], sites[0], Pc[0]),
           np.einsum("ia,asb,bj->isj", Qc[0], sites[1], Pc[1])]
    a1 = [r / np.linalg.norm(r) for r in raw]
    return a1, l1, Qc, Pc


# ---------------------------------------------------------------------------
# gauge fixing (Sec. III B)
# ---------------------------------------------------------------------------

def polar_orthogonal(k):
    """Orthogonal U maximising <U, k>_F: with k = W S V^T, U = W V^T (the
    Procrustes step of the iterative method, Sec. III B 2 (i)-(ii))."""
    w, _, vt = np.linalg.svd(k)
    return w @ vt


def gauge_start(P, Pc, Q, Qc, kappa):
    """Starting point for the iterative gauge fix inside the recycling step.
    For small time steps the renormalized gate is close to the identity, so
    the kappa = 0 block of the composite truncation maps the old bond basis
    onto the new one: on the left site of a bond the new index j takes
    sum_i A_0[i] (P Pc)[(i, 0), j], on the right site sum_i (Qc Q)[j, (i, 0)]
    A_0[i].  Both estimates of U (new = U old) are scaled to unit norm,
    added, and made orthogonal.  Reading taken: the paper starts from the
    identity or a random matrix, which can stall in a local maximum when the
    two canonical forms differ by sign flips."""
    out = []
    for b in range(len(P)):
        e1 = (P[b] @ Pc[b])[0::kappa, :].T
        e2 = (Qc[b] @ Q[b])[:, 0::kappa]
        out.append(polar_orthogonal(e1 / np.linalg.norm(e1) + e2 / np.linalg.norm(e2)))
    return out


def gauge_fix_direct(a_ref, a_new):
    """The paper's direct method (Sec. III B 1, Eq. (iMPSDM1)) for a two-site
    cell: the dominant left eigenvector of the mixed transfer matrix (ket
    a_ref, bra a_new) at bond b equals w_b U_b^T when a_new = U a_ref U^T, with
    w_b the positive left fixed point of a_ref; hence U_b is the orthogonal
    polar factor of its transpose.  The sign of each eigenvector is chosen
    to maximise the fidelity."""
    U = []
    for b in (0, 1):
        a, c = (0, 1) if b == 0 else (1, 0)
        vl, _, _ = tm_fixed_point([a_ref[c], a_ref[a]], [a_new[c], a_new[a]])
        U.append(polar_orthogonal(vl.T))
    best, bestF = None, -np.inf
    norm = sum(np.linalg.norm(x) * np.linalg.norm(y) for x, y in zip(a_ref, a_new))
    for s0 in (1.0, -1.0):
        for s1 in (1.0, -1.0):
            V = [s0 * U[0], s1 * U[1]]
            f = np.einsum("ia,asb,jb,isj->", V[1], a_ref[0], V[0], a_new[0], optimize=True)
            f += np.einsum("ia,asb,jb,isj->", V[0], a_ref[1], V[1], a_new[1], optimize=True)
            if f / norm > bestF:
                best, bestF = V, f / norm
    return best, float(bestF)


def gauge_fix(a_ref, a_new, tol=1e-12, max_iter=1000, U0=None):
    """Iterative fidelity maximisation (Sec. III B 2, Eq. (15)) generalised to
    a two-site cell with one orthogonal U per bond: find U[0], U[1] so that
    a_new_X ~ U[left] a_ref_X U[right]^T.  Bonds are updated alternately
    (Procrustes on the linear coefficient of each U) until the normalised
    fidelity F = sum_X <a_new_X, U a_ref_X U^T> / sum_X |a_ref_X||a_new_X|
    stops changing by more than ``tol``.

    Returns (U, F, iters)."""
    n = a_ref[0].shape[2]
    norm = sum(np.linalg.norm(a) * np.linalg.norm(b) for a, b in zip(a_ref, a_new))

    def fid(U):
        f = np.einsum("ia,asb,jb,isj->", U[1], a_ref[0], U[0], a_new[0], optimize=True)
        f += np.einsum("ia,asb,jb,isj->", U[0], a_ref[1], U[1], a_new[1], optimize=True)
        return f / norm

    def coeff(U, b):
        # site b has U[o] on its left and U[b] on its right;
        # site o has U[b] on its left and U[o] on its right
        o = 1 - b
        k = np.einsum("isj,ia,asb->jb", a_new[b], U[o], a_ref[b], optimize=True)
        k += np.einsum("isj,jb,asb->ia", a_new[o], U[o], a_ref[o], optimize=True)
        return k

    U = [np.eye(n), np.eye(n)] if U0 is None else [u.copy() for u in U0]
    F = fid(U)
    it = 0
    for it in range(1, max_iter + 1):
        for b in (0, 1):
            U[b] = polar_orthogonal(coeff(U, b))
        Fn = fid(U)
        done = abs(Fn - F) < tol
        F = Fn
        if done:
            break
    return U, float(F), it


# ---------------------------------------------------------------------------
# recycling (Sec. V B)
# ---------------------------------------------------------------------------

def renormalized_gate(P, Q, Qc, Pc, U):
    """Per-bond factors of G = U^T Qc Q g P Pc U (Sec. V B step (iii)):
    Lf[b] = U[b]^T Qc[b] Q[b] acts on the left leg of the site right of bond
    b, Rf[b] = P[b] Pc[b] U[b] on the right leg of the site left of it."""
    Lf = [U[b].T @ Qc[b] @ Q[b] for b in (0, 1)]
    Rf = [P[b] @ Pc[b] @ U[b] for b in (0, 1)]
    return Lf, Rf


def apply_renormalized(Lf, Rf, g, sites):
    """A_X <- G A_X, normalised."""
    th = [gates.apply_impo(g, s) for s in sites]
    new = [np.einsum("ia,asb,bj->isj", Lf[1], th[0], Rf[0], optimize=True),
           np.einsum("ia,asb,bj->isj", Lf[0], th[1], Rf[1], optimize=True)]
    return [t / np.linalg.norm(t) for t in new]


def recycle_build(sites, g, chi, gauge="iterative"):
    """Environment step of the recycling scheme (Sec. V B (i)-(iii)):
    truncate g A_0 with a fresh environment, canonicalize, gauge-fix against
    A_0 (``gauge``: "iterative", Sec. III B 2, or "direct", Sec. III B 1),
    and build the renormalized gate.  Returns (new_sites, (Lf, Rf), spectra,
    trunc_err, fidelity)."""
    # the scheme starts from a canonical A_0
    sites, _, _, _ = canonicalize_a_form(sites)
    trunc, P, Q, spec, err = itebd_plain_step(sites, g, chi)
    a1, l1, Qc, Pc = canonicalize_a_form(trunc, spec)
    kappa = g.shape[0]
    if gauge == "direct":
        U, F = gauge_fix_direct(sites, a1)
    elif gauge == "iterative":
        U, F, _ = gauge_fix(sites, a1, U0=gauge_start(P, Pc, Q, Qc, kappa))
    else:
        raise ValueError(f"unknown gauge-fix method {gauge!r}")
    Lf, Rf = renormalized_gate(P, Q, Qc, Pc, U)
    new = apply_renormalized(Lf, Rf, g, sites)
    return new, (Lf, Rf), l1, err, F


def renormalized_gate_matrix(Lf, Rf, g, X):
    """The map A_X -> G A_X of site X (0: left site of bond 0, 1: the right
    one) as a dense matrix on the flattened site tensor [chi][d][chi]:
    G[(i s j), (a t b)] = sum_{k k'} Lf[(i), (a k)] g[k, k', s, t] Rf[(b k'), j],
    with the factors of the bonds to the left and right of X."""
    lf, rf = (Lf[1], Rf[0]) if X == 0 else (Lf[0], Rf[1])
    chi, n = lf.shape
    kappa = g.shape[0]
    d = g.shape[2]
    lf3 = lf.reshape(chi, n // kappa, kappa)          # [i][a][k]
    rf3 = rf.reshape(n // kappa, kappa, chi)          # [b][k'][j]
    G = np.einsum("iak,kKst,bKj->isjatb", lf3, g, rf3, optimize=True)
    return G.reshape(chi * d * chi, chi * d * chi)


def recycle_limit(Lf, Rf, g, sites):
    """N_Re -> infinity (Sec. V C, the limit lines of Fig. 19): recycling
    the environment without end takes each site to the dominant eigenvector
    of its renormalized gate, the map A_X -> G A_X.  Per site, the
    eigenvector of the eigenvalue of largest magnitude (dense eig), which
    must be real; scaled to unit norm with a positive overlap with the
    current site.  Returns (sites, eigenvalues, gap ratios |l2 / l1|)."""
    out, lams, ratios = [], [], []
    for X in (0, 1):
        G = renormalized_gate_matrix(Lf, Rf, g, X)
        w, v = np.linalg.eig(G)
        order = np.argsort(-np.abs(w))
        l1, l2 = w[order[0]], w[order[1]]
        if abs(l1.imag) > 1e-12 * abs(l1) or abs(l1 - l2) < 1e-12 * abs(l1):
            raise ValueError("the renormalized gate has no simple real dominant eigenvalue")
        vec = np.real(v[:, order[0]]).reshape(sites[X].shape)
        vec = vec / np.linalg.norm(vec)
        if np.sum(vec * sites[X]) < 0:
            vec = -vec
        out.append(vec)
        lams.append(float(l1.real))
        ratios.append(float(abs(l2) / abs(l1)))
    return out, lams, ratios


def run_itebd(sites, J, h, dt, chi, nsteps, n_re=1, energy_every=None, gauge="iterative"):
    """Imaginary-time iTEBD (Eq. (eq), power method on the iMPO) with the
    environment recomputed every ``n_re`` steps and the renormalized gate
    applied in between.  ``n_re=1`` is the plain algorithm; ``n_re=None`` is
    the limit N_Re -> infinity (each environment step jumps to the dominant
    eigenvector of its renormalized gate; ``nsteps`` then counts environment
    steps).  ``gauge`` picks the gauge fix of the environment steps (see
    recycle_build).  Returns the final sites and a list of (step, energy)
    taken at environment steps."""
    g = gates.impo(J, h, dt)
    sites = [s / np.linalg.norm(s) for s in sites]
    log = []
    fac = None
    if n_re is None:
        for step in range(nsteps):
            sites, fac, _, _, _ = recycle_build(sites, g, chi, gauge)
            sites, _, _ = recycle_limit(fac[0], fac[1], g, sites)
            if energy_every and step % energy_every == 0:
                log.append((step + 1, energy_per_site(sites, J, h)))
        return sites, log
    for step in range(nsteps):
        if step % n_re == 0:
            if n_re == 1:
                sites, _, _, _, _ = itebd_plain_step(sites, g, chi)
            else:
                sites, fac, _, _, _ = recycle_build(sites, g, chi, gauge)
            if energy_every and (step // n_re) % energy_every == 0:
                log.append((step + 1, energy_per_site(sites, J, h)))
        else:
            sites = apply_renormalized(fac[0], fac[1], g, sites)
    return sites, log
