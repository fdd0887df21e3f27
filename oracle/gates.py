"""Trotter gates, iMPO and iPEPO for the transverse-field Ising model.

Oracle (test infrastructure only).

Hamiltonian (Sec. V A and Sec. VI A): H = -J sum sz sz - h sum sx.  The
second-order Suzuki-Trotter split puts half a field step on both sides of a
full interaction step; the field gate is g_F = exp(+delta h sx / 2) and the
interaction gate is g_I = exp(+delta J sz(x)sz).

The interaction gate is split by an SVD of its operator reshaping
(Eq. (iMPO1), Fig. 15; Fig. 20 in 2D) into kappa = 2 terms.  Reading taken
where the paper puts all of S on one side: the square root of each singular
value goes to both sides, and each left singular vector is sign-fixed so that
its largest-magnitude entry is positive.  The represented operator is the
same; only a diagonal gauge on the kappa leg changes.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
ID = np.eye(2)


def field_gate(h: float, dt: float) -> np.ndarray:
    """g_F = exp(-H_F dt/2) with H_F = -h sx (Sec. V A)."""
    return expm(0.5 * dt * h * SX)


def interaction_gate(J: float, dt: float) -> np.ndarray:
    """g_I = exp(-H_I dt) with H_I = -J sz(x)sz, as a 4x4 matrix on
    (s1 s2),(s1' s2')."""
    return expm(dt * J * np.kron(SZ, SZ))


def split_interaction(J: float, dt: float, tol: float = 1e-14):
    """Operator SVD of g_I (Eq. (iMPO1), Fig. 15(b)).

    Returns (L, R), each of shape [kappa][d][d], such that
    g_I = sum_k L[k] (x) R[k].  kappa counts the singular values above
    ``tol`` times the largest (2 for the Ising interaction)."""
    g = interaction_gate(J, dt).reshape(2, 2, 2, 2)          # s1 s2 s1' s2'
    m = g.transpose(0, 2, 1, 3).reshape(4, 4)                # (s1 s1'),(s2 s2')
    u, s, vt = np.linalg.svd(m)
    kappa = int(np.sum(s > tol * s[0]))
    L = np.empty((kappa, 2, 2))
    R = np.empty((kappa, 2, 2))
    for k in range(kappa):
        uk, vk = u[:, k], vt[k, :]
        i = int(np.argmax(np.abs(uk)))
        sgn = 1.0 if uk[i] > 0 else -1.0
        L[k] = (sgn * np.sqrt(s[k]) * uk).reshape(2, 2)
        R[k] = (sgn * np.sqrt(s[k]) * vk).reshape(2, 2)
    return L, R


def impo(J: float, h: float, dt: float) -> np.ndarray:
    """iMPO site tensor g[a][b][s][s'] (left kappa leg a, right kappa leg b,
    output s, input s'), g = g_F (R_a L_b) g_F (Eq. (iMPO1)): the site takes
    the right factor of the bond on its left and the left factor of the bond
    on its right."""
    gf = field_gate(h, dt)
    L, R = split_interaction(J, dt)
    kap = L.shape[0]
    g = np.empty((kap, kap, 2, 2))
    for a in range(kap):
        for b in range(kap):
            g[a, b] = gf @ R[a] @ L[b] @ gf
    return g


def ipepo(J: float, h: float, dt: float) -> np.ndarray:
    """iPEPO site tensor g[l][r][d][u][s][s'] (Sec. VI A, Fig. 20(d)).

    Horizontal bond (left site, right site) = sum_k L[k] (x) R[k]: the left
    site's r leg carries L, the right site's l leg carries R.  Vertical bond
    (top site, bottom site): the top site's d leg carries L, the bottom
    site's u leg carries R.  All factors act on the same site between the
    two half field gates."""
    gf = field_gate(h, dt)
    L, R = split_interaction(J, dt)
    kap = L.shape[0]
    g = np.empty((kap, kap, kap, kap, 2, 2))
    for l in range(kap):
        for r in range(kap):
            for d in range(kap):
                for u in range(kap):
                    g[l, r, d, u] = gf @ R[l] @ L[r] @ L[d] @ R[u] @ gf
    return g


def apply_impo(g: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Theta = g . Gamma for an iMPS site tensor [chi][d][chi]; the new bond
    index is (chi index, kappa index) with the kappa index fastest."""
    kap = g.shape[0]
    chi_l, d, chi_r = gamma.shape
    th = np.einsum("abst,itj->iasjb", g, gamma)
    return th.reshape(chi_l * kap, d, chi_r * kap)


def apply_ipepo(g: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Theta = g . A for an iPEPS site tensor [d][D][D][D][D] (s,l,r,d,u);
    every bond leg becomes (D index, kappa index), kappa fastest."""
    kap = g.shape[0]
    d, D1, D2, D3, D4 = A.shape
    th = np.einsum("abcest,tlrdu->slarbdcue", g, A)
    return th.reshape(d, D1 * kap, D2 * kap, D3 * kap, D4 * kap)
