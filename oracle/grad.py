"""Energy of a single-site iPEPS after a fixed number of CTMRG iterations,
and its central finite-difference directional derivatives.

Oracle (test infrastructure only).  The energy function is
E(A) = energy per site of the TFIM (Sec. VI A) evaluated with the CTM
environment obtained by exactly ``n_iter`` CTMRG iterations (no convergence
test) started from a fixed environment (C0, T0) that does not depend on A.
"""
from __future__ import annotations

import numpy as np

from .ctmrg import Cell, iteration
from .peps import energy_per_site


def energy_after(A, C0, T0, chi, n_iter, J, h):
    cell = Cell(1, 1, [0])
    C, T = np.array(C0, dtype=np.float64), np.array(T0, dtype=np.float64)
    for _ in range(n_iter):
        C, T = iteration(cell, [A], C, T, chi)
    return energy_per_site(cell, [A], C, T, J, h)


def fd_directional(A, C0, T0, chi, n_iter, J, h, directions, step=1e-6):
    """Central differences (E(A + step v) - E(A - step v)) / (2 step) along
    each direction v."""
    out = []
    for v in directions:
        ep = energy_after(A + step * v, C0, T0, chi, n_iter, J, h)
        em = energy_after(A - step * v, C0, T0, chi, n_iter, J, h)
        out.append((ep - em) / (2 * step))
    return np.array(out)
