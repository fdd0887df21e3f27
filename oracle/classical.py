"""The classical 2D Ising partition function by the power method on an iMPS,
with the environment recycled (Sec. I: the transfer matrix of a classical
model takes the place of the imaginary-time operator, and the recycling of
the environment carries over unchanged).

Oracle (test infrastructure only).

The model: square lattice, J = 1, inverse temperature beta,
Z = sum_s prod_<ij> exp(beta s_i s_j).  Its row-to-row transfer matrix,
with the vertical bonds between two rows and half of the horizontal bonds
of each row, is T(s', s) = prod_i exp(beta s'_i s_i)
exp(beta (s_i s_{i+1} + s'_i s'_{i+1}) / 2).  One vertical bond as a 2 x 2
matrix in (s', s) is c exp(K* sx) with c = sqrt(2 sinh 2 beta) and
tanh K* = exp(-2 beta) (the dual coupling), and a row's horizontal bonds
are the diagonal exp(beta sum sz sz).  So T = H^1/2 V H^1/2 has the
spectrum of c^L G with G = exp(K* sx / 2)^(x L) exp(beta sum sz sz)
exp(K* sx / 2)^(x L): the second-order gate of the transverse-field Ising
chain (Sec. V A) at dt J = beta, dt h = K*.  Its dominant eigenvector psi,
which the power method reaches, sits in the middle of a vertical bond.

Two quantities of the model follow from psi:
* ln Z per site = ln c + ln mu, mu the dominant eigenvalue of G per site,
  taken as the Rayleigh quotient (<psi|G|psi> / <psi|psi>)^(1/N): per
  two-site cell, the ratio of the dominant eigenvalues of the mixed
  transfer matrix of (G psi, psi) and of (psi, psi);
* <psi|sx|psi> = P(same) tanh K* + P(opposite) coth K* for the two spins
  of a vertical bond, since sx V^1/2 psi sits between the bond's halves
  and (sx exp(K* sx))_{s s'} / exp(K* sx)_{s s'} is tanh K* for s = s'
  and coth K* otherwise; with e = <s s'> of nearest neighbours this is
  ((1 + e) exp(-2 beta) + (1 - e) exp(2 beta)) / 2.
"""
from __future__ import annotations

import numpy as np

from . import gates, imps


def row_gate(beta):
    """(J, h, dt) of the transverse-field gate that the row transfer matrix
    is (up to the scale c per site): dt J = beta, dt h = K*."""
    return beta, float(np.arctanh(np.exp(-2.0 * beta))), 1.0


def log_scale(beta):
    """ln c per site, c = sqrt(2 sinh 2 beta)."""
    return 0.5 * np.log(2.0 * np.sinh(2.0 * beta))


def _cell_eigenvalue(kets, bras):
    """Dominant eigenvalue of the two-site transfer matrix sum_s K^s (x) B^s,
    kets and bras of possibly different bonds, by dense diagonalisation."""
    E = None
    for k, b in zip(kets, bras):
        e = np.einsum("asc,bsd->abcd", k, b)
        e = e.reshape(k.shape[0] * b.shape[0], k.shape[2] * b.shape[2])
        E = e if E is None else E @ e
    w = np.linalg.eigvals(E)
    lead = w[np.argmax(np.abs(w))]
    if abs(lead.imag) > 1e-10 * abs(lead) or lead.real <= 0:
        raise ValueError("the cell transfer matrix has no positive dominant eigenvalue")
    return float(lead.real)


def log_mu(sites, beta):
    """ln of the per-site Rayleigh quotient of G on the two-site iMPS."""
    J, h, dt = row_gate(beta)
    g = gates.impo(J, h, dt)
    gs = [gates.apply_impo(g, a) for a in sites]
    return 0.5 * (np.log(_cell_eigenvalue(gs, sites)) - np.log(_cell_eigenvalue(sites, sites)))


def log_z(sites, beta):
    """ln Z per site (= -beta f) from the converged iMPS."""
    return log_scale(beta) + log_mu(sites, beta)


def sigma_x(sites):
    """<psi|sx|psi>, the mean over the two sites."""
    return -imps.energy_per_site(sites, 0.0, 1.0)


def power_method(sites, beta, chi, nsteps, n_re=1, n_warm=0, gauge="iterative"):
    """``n_warm`` plain applications of the transfer matrix with the
    truncation of iTEBD, then ``nsteps`` more: plain with n_re = 1, the
    environment recycled otherwise, the limit N_Re -> infinity with
    n_re = None (nsteps then counts environment steps); ``gauge`` is the
    gauge fix of the recycling's environment steps ("iterative" or
    "direct").  Returns the sites."""
    J, h, dt = row_gate(beta)
    if n_warm:
        sites, _ = imps.run_itebd(sites, J, h, dt, chi, n_warm)
    out, _ = imps.run_itebd(sites, J, h, dt, chi, nsteps, n_re=n_re, gauge=gauge)
    return out
