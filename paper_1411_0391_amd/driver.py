"""Imaginary-time evolution drivers that compose the library's calls.

Only control flow lives here: every arithmetic step is a call into
``libitebd.so`` through :class:`paper_1411_0391_amd.Context`.

Full update with environment recycling (Sec. VI B, VI C of the paper):
each environment step applies the gate, pre-truncates the gated state by
its canonical form, converges the CTM environment (warm-started from the
previous one), measures the energy, truncates every link by ALS on its bond
environment, and -- in the recycling phase -- canonicalises the result,
fixes its gauge against the previous state and builds the renormalized gate
G, which then replaces the environment for the next ``n_re - 1`` steps.
"""
from __future__ import annotations

import time


def full_update(ctx, Lx, Ly, cell, sites, C, T, J, h, dt, nsteps, n_re=1, n_warm=0,
                ctm_tol=1e-10, ctm_max=100, als_tol=1e-12, als_passes=50, als_sweeps=1,
                canon_tol=1e-14, canon_max=1000, gauge_tol=1e-12, gauge_max=1000,
                min_fidelity=None, force_recycle=False, callback=None, pretruncate=True):
    """Evolve the iPEPS ``sites`` (device [nsite][d][D]^4) for ``nsteps``
    steps of size dt.  C, T (device) are the start environment and are
    updated in place.  Returns (sites, log) with log entries (step,
    energy_per_site, seconds since start, recycled, fidelity) at
    environment steps; the environment is recomputed every ``n_re`` steps
    after ``n_warm`` plain steps.  A recycling step first brings the state
    A_0 to canonical form (Sec. VI C assumes it).  With ``min_fidelity``, an
    environment step whose gauge fix ends below that fidelity (the new state
    is too far from the previous one for its gate to stand in for the
    environment) is not recycled: the evolution continues with the plain
    step.  ``force_recycle`` takes the recycling branch for n_re = 1 too.
    ``callback(step, info)`` gets, per environment step, a dict with the
    energy, whether it was recycled, the gauge-fix fidelity, the CTMRG
    iterations and final delta, the block cost over the block norm and the
    ALS cycles; a true return value ends the evolution there.
    ``pretruncate=False`` computes each environment for Theta itself, bond
    kappa D (C, T of that bond; the O(chi^3 D^6 kappa^6) form that the
    pre-truncation avoids, Sec. VI B): the truncation block's outer legs
    then carry identities, and the energy is Theta's."""
    import torch
    D = sites.shape[2]
    kappa = 2
    eye = None
    if not pretruncate:
        nlink = len(ctx.cell_links(Lx, Ly, sites.shape[0], cell))
        eye = torch.eye(kappa * D, dtype=torch.float64, device=sites.device)
        eye = eye.expand(nlink, kappa * D, kappa * D).contiguous()
    log = []
    t0 = time.perf_counter()
    step = 0
    while step < nsteps:
        recycle = step >= n_warm and (n_re > 1 or force_recycle)
        if recycle:
            sites, _, _, _, _, _ = ctx.ipeps_canonicalize(Lx, Ly, cell, sites, tol=canon_tol,
                                                          max_iter=canon_max)
        Th = ctx.ipeps_gate(sites, J, h, dt)
        _, _, Psu, Qsu, _, _ = ctx.ipeps_canonicalize(Lx, Ly, cell, Th, D_keep=D, tol=canon_tol,
                                                       max_iter=canon_max, a_out=False)
        if pretruncate:
            pre, Pe, Qe = ctx.ipeps_truncate(Lx, Ly, cell, Th, Psu, Qsu), Psu, Qsu
        else:
            pre, Pe, Qe = Th, eye, eye
        _, ctm_iters, ctm_delta = ctx.ctmrg_iterate(Lx, Ly, pre, cell, C, T, ctm_max, ctm_tol)
        E = ctx.ipeps_energy(Lx, Ly, pre, cell, C, T, J, h)
        P, Q = Psu.clone(), Qsu.clone()
        f, norm, passes, sweeps = ctx.bond_env_truncate(Lx, Ly, cell, Th, C, T, Pe, Qe, P, Q,
                                                        als_passes, als_sweeps, als_tol)
        new = ctx.ipeps_truncate(Lx, Ly, cell, Th, P, Q)
        F = None
        if recycle:
            a1, _, Pc, Qc, _, _ = ctx.ipeps_canonicalize(Lx, Ly, cell, new, tol=canon_tol,
                                                          max_iter=canon_max)
            U = ctx.fu_gauge_start(P, Q, Pc, Qc, kappa)
            F, _, _ = ctx.gauge_fix(Lx, Ly, cell, sites, a1, U, tol=gauge_tol,
                                    max_iter=gauge_max)
            if min_fidelity is not None and F < min_fidelity:
                recycle = False
        torch.cuda.current_stream().synchronize()
        log.append((step + 1, E, time.perf_counter() - t0, recycle, F))
        stop = False
        if callback:
            stop = bool(callback(step, dict(energy=E, recycled=recycle, fidelity=F,
                                            ctm_iters=ctm_iters, ctm_delta=ctm_delta,
                                            als_cost=f / norm, als_passes=passes,
                                            seconds=log[-1][2])))
        if not recycle:
            sites = new
            step += 1
        else:
            Rf, Lf = ctx.fu_renormalized_gate(P, Q, Pc, Qc, U)
            sites = ctx.ipeps_truncate(Lx, Ly, cell, Th, Rf, Lf)
            step += 1
            for _ in range(n_re - 1):
                if step >= nsteps or stop:
                    break
                sites = ctx.ipeps_truncate(Lx, Ly, cell, ctx.ipeps_gate(sites, J, h, dt), Rf,
                                           Lf)
                step += 1
        if stop:
            break
    return sites, log


def simple_update(ctx, Lx, Ly, cell, sites, J, h, dt, nsteps, canon_tol=1e-14, canon_max=1000):
    """The simple update (Sec. VI A): per step the iPEPO gate, then every
    link truncated to its D largest Schmidt values through the canonical
    form of Theta; no environment.  Returns the sites (device)."""
    D = sites.shape[2]
    for _ in range(nsteps):
        Th = ctx.ipeps_gate(sites, J, h, dt)
        _, _, P, Q, _, _ = ctx.ipeps_canonicalize(Lx, Ly, cell, Th, D_keep=D, tol=canon_tol,
                                                   max_iter=canon_max, a_out=False)
        sites = ctx.ipeps_truncate(Lx, Ly, cell, Th, P, Q)
    return sites
