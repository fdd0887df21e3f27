"""Closed forms and brute-force references used to pin the oracle.

These are textbook results, written here independently of ``oracle/``:
the exact 1D TFIM ground-state energy (Pfeuty), Onsager's nearest-neighbour
energy and Yang's spontaneous magnetisation of the 2D classical Ising
model, the Ising-PEPS construction whose norm is the classical partition
function, and dense exact diagonalisation of tiny spin systems.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate
from scipy.linalg import expm, sqrtm
from scipy.special import ellipk

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])

BETA_C = 0.5 * np.log(1.0 + np.sqrt(2.0))


def tfim1d_energy(h: float) -> float:
    """e(h) = -(1/pi) int_0^pi sqrt(1 + h^2 - 2 h cos k) dk (J = 1)."""
    val, _ = integrate.quad(lambda k: np.sqrt(1 + h * h - 2 * h * np.cos(k)), 0, np.pi,
                            epsabs=1e-14, epsrel=1e-14, limit=200)
    return -val / np.pi


def onsager_nn(beta: float) -> float:
    """<s_i s_j> for nearest neighbours of the square-lattice Ising model."""
    k = 2 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    u = -1 / np.tanh(2 * beta) * (1 + (2 / np.pi) * (2 * np.tanh(2 * beta) ** 2 - 1)
                                  * ellipk(k * k))
    return -u / 2


def yang_m(beta: float) -> float:
    return (1 - np.sinh(2 * beta) ** -4) ** 0.125 if beta > BETA_C else 0.0


def ising_peps(beta: float) -> np.ndarray:
    """D=2 iPEPS tensor whose norm network is the classical Ising partition
    function: A^s_{lrdu} = Q_{sl} Q_{sr} Q_{sd} Q_{su}, Q Q^T = exp(beta/2 s s')."""
    W = np.array([[np.exp(beta / 2), np.exp(-beta / 2)], [np.exp(-beta / 2), np.exp(beta / 2)]])
    Q = np.real(sqrtm(W))
    return np.einsum("sl,sr,sd,su->slrdu", Q, Q, Q, Q)


def ising_peps_aniso(beta_h: float, beta_v: float) -> np.ndarray:
    """Ising PEPS with coupling beta_h on horizontal (l, r) bonds and beta_v
    on vertical (d, u) bonds."""
    def q(b):
        W = np.array([[np.exp(b / 2), np.exp(-b / 2)], [np.exp(-b / 2), np.exp(b / 2)]])
        return np.real(sqrtm(W))
    Qh, Qv = q(beta_h), q(beta_v)
    return np.einsum("sl,sr,sd,su->slrdu", Qh, Qh, Qv, Qv)


def onsager_nn_aniso(K1: float, K2: float, n: int = 512):
    """Nearest-neighbour correlations (along direction 1, along direction 2)
    of the anisotropic square-lattice Ising model from Onsager's free energy
    -beta f = ln 2 + (1/8 pi^2) int int ln[cosh 2K1 cosh 2K2
    - sinh 2K1 cos t1 - sinh 2K2 cos t2], differentiated under the integral;
    periodic trapezoid rule (spectrally accurate away from criticality)."""
    t = 2 * np.pi * np.arange(n) / n
    c1, c2 = np.meshgrid(np.cos(t), np.cos(t), indexing="ij")
    den = np.cosh(2 * K1) * np.cosh(2 * K2) - np.sinh(2 * K1) * c1 - np.sinh(2 * K2) * c2
    d1 = (2 * np.sinh(2 * K1) * np.cosh(2 * K2) - 2 * np.cosh(2 * K1) * c1) / den
    d2 = (2 * np.cosh(2 * K1) * np.sinh(2 * K2) - 2 * np.cosh(2 * K2) * c2) / den
    return float(d1.mean() / 2), float(d2.mean() / 2)


def op_on(n: int, ops: dict) -> np.ndarray:
    """Dense operator on n spins with ops {site: 2x2}."""
    out = np.array([[1.0]])
    for i in range(n):
        out = np.kron(out, ops.get(i, np.eye(2)))
    return out


def tfim_hamiltonian(n: int, bonds, h: float, J: float = 1.0) -> np.ndarray:
    H = np.zeros((2 ** n, 2 ** n))
    for (i, j) in bonds:
        H -= J * op_on(n, {i: SZ, j: SZ})
    for i in range(n):
        H -= h * op_on(n, {i: SX})
    return H


def trotter_product(n: int, bonds, h: float, dt: float, J: float = 1.0) -> np.ndarray:
    """exp(-H_F dt/2) exp(-H_I dt) exp(-H_F dt/2), dense."""
    HF = np.zeros((2 ** n, 2 ** n))
    for i in range(n):
        HF -= h * op_on(n, {i: SX})
    HI = np.zeros((2 ** n, 2 ** n))
    for (i, j) in bonds:
        HI -= J * op_on(n, {i: SZ, j: SZ})
    half = expm(-0.5 * dt * HF)
    return half @ expm(-dt * HI) @ half


def onsager_free_energy(beta: float, n: int = 1024) -> float:
    """-beta f per site of the isotropic square-lattice Ising model (J = 1),
    Onsager: ln 2 + (1/8 pi^2) int int ln[cosh^2 2K - sinh 2K (cos t1 + cos t2)]
    over [0, 2 pi)^2; periodic trapezoid rule (spectrally accurate away from
    criticality)."""
    t = 2 * np.pi * np.arange(n) / n
    c1, c2 = np.meshgrid(np.cos(t), np.cos(t), indexing="ij")
    arg = np.cosh(2 * beta) ** 2 - np.sinh(2 * beta) * (c1 + c2)
    return float(np.log(2.0) + 0.5 * np.log(arg).mean())


def onsager_free_energy_1d(beta: float) -> float:
    """The same in its one-dimensional integral form:
    ln(2 cosh 2K) + (1/pi) int_0^{pi/2} ln[(1 + sqrt(1 - k^2 sin^2 p)) / 2] dp,
    k = 2 sinh 2K / cosh^2 2K."""
    k = 2 * np.sinh(2 * beta) / np.cosh(2 * beta) ** 2
    val, _ = integrate.quad(lambda p: np.log(0.5 * (1 + np.sqrt(1 - (k * np.sin(p)) ** 2))),
                            0, np.pi / 2, epsabs=1e-14, epsrel=1e-13, limit=200)
    return float(np.log(2 * np.cosh(2 * beta)) + val / np.pi)


def tfim2d_torus_ed(Lx: int, Ly: int, h: float, J: float = 1.0) -> float:
    """Ground-state energy per site of H = -J sum_<ij> sz sz - h sum sx on an
    Lx x Ly torus (each nearest-neighbour bond once), by sparse Lanczos."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh
    n = Lx * Ly
    dim = 2 ** n
    idx = np.arange(dim)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1      # bit i of state: site i
    z = 1 - 2 * bits                                           # sz eigenvalue per site
    site = lambda x, y: (y % Ly) * Lx + (x % Lx)
    bonds = [(site(x, y), site(x + 1, y)) for y in range(Ly) for x in range(Lx)]
    bonds += [(site(x, y), site(x, y + 1)) for y in range(Ly) for x in range(Lx)]
    diag = -J * sum(z[:, i] * z[:, j] for i, j in bonds).astype(np.float64)
    rows, cols = [idx], [idx]
    vals = [diag]
    for i in range(n):
        rows.append(idx)
        cols.append(idx ^ (1 << i))
        vals.append(np.full(dim, -h))
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim))
    w = eigsh(H, k=1, which="SA", tol=1e-12, return_eigenvectors=False)
    return float(w[0]) / n
