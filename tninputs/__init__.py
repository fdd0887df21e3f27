"""Seeded synthetic inputs shared by the CPU oracle, the GPU tests and the bench.

This module draws random numbers and arranges them into arrays of the shapes
the transverse-field Ising workloads use.  It holds none of the method's
arithmetic (no gates, contractions, factorizations or normalisations beyond
what is needed to describe a distribution), so both the oracle and the HIP
path can consume its output without sharing any computation.

Every generator uses ``numpy.random.default_rng(seed).standard_normal`` and
draws its arrays in the documented order, so a given seed always produces the
same tensors.

Layouts (all float64, C-contiguous):

* iMPS site tensor ``Gamma[chi][d][chi]`` (left bond, physical, right bond).
* iPEPS site tensor ``A[d][D][D][D][D]`` with legs (s, l, r, d, u).
* CTM corners ``C[pos][4][chi][chi]`` and edges ``T[pos][4][chi][D][D][chi]``;
  the four corners/edges of a position are C1..C4 / T1..T4 (top-left,
  top-right, bottom-right, bottom-left / top, right, bottom, left), each with
  its two boundary legs ordered clockwise around the boundary ring and the
  (ket, bra) leg pair of an edge in the middle.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "imps_two_site",
    "ipeps_sites",
    "ctm_env",
    "unit_directions",
    "CHECKERBOARD",
    "SINGLE_SITE",
]

# Position -> site index for a 2x2 checkerboard cell [[A, B], [B, A]] and a
# 1x1 cell, stored row-major over (y, x): index = y * Lx + x.
CHECKERBOARD = (2, 2, (0, 1, 1, 0))
SINGLE_SITE = (1, 1, (0,))


def imps_two_site(seed: int, chi: int, d: int = 2):
    """Two-site iMPS {Gamma_A, lambda_A, Gamma_B, lambda_B}.

    Draw order: Gamma_A then Gamma_B, each N(0,1) of shape [chi][d][chi].
    The bond vectors are flat, lambda = 1/sqrt(chi) (unit l2 norm).
    """
    rng = np.random.default_rng(seed)
    ga = rng.standard_normal((chi, d, chi))
    gb = rng.standard_normal((chi, d, chi))
    lam = np.full(chi, 1.0 / np.sqrt(chi))
    return ga, lam.copy(), gb, lam.copy()


def ipeps_sites(seed: int, nsite: int, D: int, d: int = 2):
    """``nsite`` iPEPS site tensors, N(0,1) of shape [d][D][D][D][D], drawn in
    site order (A, then B, ...)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((d, D, D, D, D)) for _ in range(nsite)]


def ipeps_near_product(seed: int, nsite: int, D: int, eps: float = 1e-2, d: int = 2):
    """A random product state with a small bond-D part: the N(0,1) tensors
    of bond 1 from ``seed`` (``ipeps_sites(seed, nsite, 1)``) on the index-0
    corner of each bond, plus ``eps`` times the N(0,1) bond-D tensors from
    ``seed + 1``.  Random bond-D tensors alone carry closed-loop
    correlations on their bonds that imaginary-time evolution does not
    remove; this start has none."""
    prod, noise = ipeps_sites(seed, nsite, 1, d), ipeps_sites(seed + 1, nsite, D, d)
    out = []
    for a, z in zip(prod, noise):
        t = eps * z
        t[:, 0, 0, 0, 0] += a[:, 0, 0, 0, 0]
        out.append(t)
    return out


def ctm_env(seed: int, npos: int, chi: int, D: int, positive: bool = False):
    """Random CTM environment for ``npos`` cell positions.

    Draw order: all corners C[pos][k] (pos-major, k = 0..3), then all edges
    T[pos][k].  Returns arrays of shape [npos][4][chi][chi] and
    [npos][4][chi][D][D][chi].  With ``positive`` the entries are the
    magnitudes of the draws and each edge is made symmetric under exchange
    of its (ket, bra) legs (the distribution of a boundary of a positive
    double-layer network).
    """
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((npos, 4, chi, chi))
    T = rng.standard_normal((npos, 4, chi, D, D, chi))
    if positive:
        C = np.abs(C)
        T = np.abs(T)
        T = 0.5 * (T + T.transpose(0, 1, 2, 4, 3, 5))
    return C, T


def unit_directions(seed: int, count: int, shape):
    """``count`` random directions in the space of arrays of ``shape``, each
    N(0,1) then scaled to unit Frobenius norm; shape [count, *shape]."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count,) + tuple(shape))
    n = np.sqrt((v.reshape(count, -1) ** 2).sum(axis=1))
    return v / n.reshape((count,) + (1,) * len(shape))
