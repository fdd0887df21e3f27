"""GPU parity of the CTMRG path against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import tninputs
from oracle import ctmrg as octm
from oracle import peps as opeps
from tests import pins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1411_0391_amd as tn  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = tn.Context()
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("M,N,K,ta,tb", [(64, 64, 16, False, False), (70, 33, 19, False, False),
                                         (130, 97, 200, True, False), (5, 129, 64, False, True),
                                         (257, 65, 33, True, True), (1, 1, 1, False, False),
                                         # split along K with a ragged last slice, on the
                                         # 96- and 128-wide tiles
                                         (300, 96, 1000, False, False), (200, 120, 333, True, False),
                                         (77, 90, 517, False, True), (64, 64, 4099, True, True),
                                         # short K: 32-column tiles, ragged in M, N and K
                                         (2592, 96, 96, False, False), (300, 100, 50, True, True),
                                         (65, 127, 20, False, True)])
def test_gemm_parity(ctx, M, N, K, ta, tb):
    rng = np.random.default_rng(M * 7 + N)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 1.5 * (A.T if ta else A) @ (B.T if tb else B) - 0.5 * C0
    C = dev(C0)
    ctx.gemm(dev(A), dev(B), C, ta=ta, tb=tb, alpha=1.5, beta=-0.5)
    np.testing.assert_allclose(host(C), ref, rtol=0, atol=1e-12 * max(1, np.abs(ref).max()))


def _setup(cellspec, D, chi, seed=0):
    Lx, Ly, cell = cellspec
    nsite = max(cell) + 1
    sites = tninputs.ipeps_sites(seed, nsite, D)
    C, T = tninputs.ctm_env(seed + 1, Lx * Ly, chi, D, positive=True)
    return Lx, Ly, list(cell), sites, C, T


@pytest.mark.parametrize("cellspec,D,chi,seed", [(tninputs.CHECKERBOARD, 2, 6, 4),
                                                 (tninputs.SINGLE_SITE, 3, 7, 0),
                                                 (tninputs.CHECKERBOARD, 3, 9, 0),
                                                 # the fused site absorption at D = 5 and 6
                                                 (tninputs.SINGLE_SITE, 5, 5, 0),
                                                 (tninputs.CHECKERBOARD, 6, 4, 0),
                                                 (tninputs.SINGLE_SITE, 6, 5, 0),
                                                 # D = 8: the two table contractions of
                                                 # the site layers (no fused kernel);
                                                 # chi = 5 takes the subspace projector SVD
                                                 (tninputs.SINGLE_SITE, 8, 5, 0),
                                                 (tninputs.CHECKERBOARD, 8, 4, 0)])
def test_single_left_move_parity(ctx, cellspec, D, chi, seed):
    Lx, Ly, cell, sites, C, T = _setup(cellspec, D, chi, seed=seed)
    ocell = octm.Cell(Lx, Ly, cell)
    Cr, Tr, spectra = octm.left_move(ocell, sites, C, T, 0, chi)
    gap = min(s[chi - 1] / s[chi] for s in spectra)
    assert gap > 1 + 1e-6, "test input has no gap at chi"
    # the new boundary tensors are compared entry by entry, so every kept
    # singular vector must be determined: a pair of kept values closer than
    # 1e-5 s_1 leaves its vectors (and C', T') fixed only to ~1e-16 / gap
    sep = min(np.min(np.abs(np.diff(s[:chi]))) / s[0] for s in spectra)
    assert sep > 1e-5, "test input has nearly degenerate kept singular values"
    Cg, Tg = dev(C), dev(T)
    ctx.ctmrg_moves(Lx, Ly, dev(np.stack(sites)), cell, Cg, Tg, 1, 0)
    # raw tensors: same sign convention on both sides
    np.testing.assert_allclose(host(Cg), Cr, atol=1e-10)
    np.testing.assert_allclose(host(Tg), Tr, atol=1e-10)


@pytest.fixture(scope="module")
def headline():
    """The measured workload: checkerboard, D = 6, chi = 72 (n = 2592), the
    bench's seeded sites and positive seeded boundary, and that boundary
    after one oracle iteration (8 moves)."""
    D, chi = 6, 72
    Lx, Ly, cell, sites, C0, T0 = _setup(tninputs.CHECKERBOARD, D, chi, seed=0)
    ocell = octm.Cell(Lx, Ly, cell)
    C, T = octm.iteration(ocell, sites, C0, T0, chi)
    return Lx, Ly, cell, ocell, sites, C0, T0, C, T, chi


def test_headline_move_parity(ctx, headline):
    """The bench's path at its own size: one left move from the oracle's
    warmed boundary, with the projector SVDs warm-started from the GPU's own
    iteration from the seeded start (as in the bench), then cold.  n = 2592
    takes the subspace projector SVD (split-K products, the Rayleigh-Ritz SVD
    on the side stream, plain steps).  The kept singular values of this
    boundary lie within 1e-6 s_1 of each other, so the comparison is gauge
    invariant: normalised corner spectra and reduced density matrices.  The
    kept subspace is fixed by the gap at the cut only to the rounding level
    n u s_1 / (s_chi - s_chi+1) in any FP64 SVD (LAPACK's included), and a
    direction of the cut enters the new boundary with weight s_chi / s_1: the
    bound is ten times that product, or 1e-10 if larger."""
    Lx, Ly, cell, ocell, sites, C0, T0, C, T, chi = headline
    n = chi * sites[0].shape[1] ** 2
    sd = dev(np.stack(sites))
    ctx.clear_cache()
    Cg, Tg = dev(C0), dev(T0)
    ctx.ctmrg_moves(Lx, Ly, sd, cell, Cg, Tg, 4 * Lx, 0)
    Cr, Tr, spectra = octm.left_move(ocell, sites, C, T, 0, chi)
    assert min(s[chi - 1] / s[chi] for s in spectra) > 1 + 1e-4
    cond = max(n * 1.11e-16 * s[0] / (s[chi - 1] - s[chi]) * s[chi - 1] / s[0] for s in spectra)
    tol = max(1e-10, 10 * cond)
    sr = octm.corner_spectra(Cr)
    r1 = opeps.rdm_one(Cr, Tr, 0, sites[cell[0]])
    rh = opeps.rdm_two_h(ocell, sites, Cr, Tr, 0, 0)
    for warm in (True, False):
        if not warm:
            ctx.clear_cache()
        Cg, Tg = dev(C), dev(T)
        ctx.prof_enable(True)
        ctx.ctmrg_moves(Lx, Ly, sd, cell, Cg, Tg, 1, 0)
        prof = ctx.prof_read()
        ctx.prof_enable(False)
        assert prof["svd_explicit"] == 0
        r1g, rhg, _ = ctx.ipeps_rdms(Lx, Ly, sd, cell, Cg, Tg)
        errs = (np.abs(octm.corner_spectra(host(Cg)) - sr).max(),
                np.abs(host(r1g)[0] - r1).max(), np.abs(host(rhg)[0] - rh).max())
        print(f"headline move (warm={warm}): spectra {errs[0]:.2e} rho1 {errs[1]:.2e} "
              f"rho_h {errs[2]:.2e}; bound {tol:.2e}; subspace iterations {prof['svd_iters']}, "
              f"stopped at the rounding floor {prof['svd_unconverged']}")
        assert max(errs) < tol, errs


def test_headline_boundary_converges_below_1e_12(ctx):
    """The measured workload's boundary (the bench's seeded sites and positive
    seeded boundary, D = 6, chi = 72), converged by the library to CTMRG
    delta < 1e-7 and then advanced one iteration per call: the change of the
    corner spectra must fall below 1e-12 and stay there.  The projector
    triplets are accurate to 1e-13 s_1; when the Rayleigh-Ritz basis was
    orthonormal only to the Jacobi tolerance (8 k u = 1.7e-13), delta stalled
    near 3e-10."""
    D, chi = 6, 72
    Lx, Ly, cell = tninputs.CHECKERBOARD
    cell = list(cell)
    sd = dev(np.stack(tninputs.ipeps_sites(0, 2, D)))
    C_h, T_h = tninputs.ctm_env(1, Lx * Ly, chi, D, positive=True)
    Cg, Tg = dev(C_h), dev(T_h)
    ctx.clear_cache()
    _, it, de = ctx.ctmrg_iterate(Lx, Ly, sd, cell, Cg, Tg, 100, 1e-7)
    assert de < 1e-7
    ds = [ctx.ctmrg_iterate(Lx, Ly, sd, cell, Cg, Tg, 1, 0.0)[2] for _ in range(24)]
    print(f"prepared in {it} iterations (delta {de:.1e}); then " +
          " ".join(f"{d:.1e}" for d in ds))
    assert max(ds[-10:]) < 1e-12, ds


def test_low_rank_projector_move_parity(ctx):
    """A nearly product state (seeded product tensors in D = 4 plus 1e-3 of
    N(0,1)): the projector problem at n = chi D^2 = 512 has far fewer
    independent directions than the subspace block (k = 48), so its
    Cholesky-QR must complete the block with random directions.  One left
    move against the oracle's.  Kept singular values reach down to ~2e-14
    s_1, where their vectors are rounding noise in any FP64 SVD and S^-1/2
    gives them unit weight in the new C and T: the tensors (and their
    spectra) are not fixed by the problem, the observables, which weight
    each direction by its singular value, are."""
    D, chi = 4, 32
    prod = tninputs.ipeps_sites(0, 2, 1)
    noise = tninputs.ipeps_sites(1, 2, D)
    sites = []
    for a, z in zip(prod, noise):
        t = 1e-3 * z
        t[:, 0, 0, 0, 0] += a[:, 0, 0, 0, 0]
        sites.append(t / np.linalg.norm(t))
    Lx, Ly, cell = tninputs.CHECKERBOARD
    cell = list(cell)
    C, T = tninputs.ctm_env(1, 4, chi, D, positive=True)
    ocell = octm.Cell(Lx, Ly, cell)
    Cr, Tr, spectra = octm.left_move(ocell, sites, C, T, 0, chi)
    assert max(s[1] / s[0] for s in spectra) < 1e-5      # one dominant direction
    Cg, Tg = dev(C), dev(T)
    sd = dev(np.stack(sites))
    ctx.clear_cache()
    ctx.ctmrg_moves(Lx, Ly, sd, cell, Cg, Tg, 1, 0)
    assert np.isfinite(host(Cg)).all() and np.isfinite(host(Tg)).all()
    r1g, rhg, _ = ctx.ipeps_rdms(Lx, Ly, sd, cell, Cg, Tg)
    np.testing.assert_allclose(host(r1g)[0], opeps.rdm_one(Cr, Tr, 0, sites[cell[0]]), atol=1e-10)
    np.testing.assert_allclose(host(rhg)[0], opeps.rdm_two_h(ocell, sites, Cr, Tr, 0, 0),
                               atol=1e-10)


def test_eight_row_cell_move_parity(ctx):
    """A left move of a 1 x 8 cell: eight row cuts batched into one projector
    SVD on the subspace path (n = chi D^2 = 288), whose Cholesky status for
    all row cuts is read back at every Rayleigh-Ritz step.  Gauge-invariant
    comparison (the kept values lie within 1e-7 s_1 of each other)."""
    cell = [0, 1, 0, 1, 0, 1, 0, 1]
    D, chi = 4, 18
    sites = tninputs.ipeps_sites(0, 2, D)
    C, T = tninputs.ctm_env(1, 8, chi, D, positive=True)
    ocell = octm.Cell(1, 8, cell)
    Cr, Tr, spectra = octm.left_move(ocell, sites, C, T, 0, chi)
    # a gap at the cut, and kept values far above the rounding floor of the
    # projector problem (a kept value near 1e-14 s_1 is noise on both sides)
    assert len(spectra) == 8 and min(s[chi - 1] / s[chi] for s in spectra) > 1 + 1e-2
    assert min(s[chi - 1] / s[0] for s in spectra) > 1e-9
    Cg, Tg = dev(C), dev(T)
    ctx.prof_enable(True)
    ctx.ctmrg_moves(1, 8, dev(np.stack(sites)), cell, Cg, Tg, 1, 0)
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    assert prof["svd_explicit"] == 0
    np.testing.assert_allclose(octm.corner_spectra(host(Cg)), octm.corner_spectra(Cr), atol=1e-10)
    r1g, _, _ = ctx.ipeps_rdms(1, 8, dev(np.stack(sites)), cell, Cg, Tg)
    for p in (0, 3, 7):
        np.testing.assert_allclose(host(r1g)[p], opeps.rdm_one(Cr, Tr, p, sites[cell[p]]),
                                   atol=1e-10)


@pytest.mark.parametrize("cellspec", [tninputs.CHECKERBOARD, tninputs.SINGLE_SITE])
def test_one_iteration_parity_all_directions(ctx, cellspec):
    D, chi = 2, 8
    Lx, Ly, cell, sites, C, T = _setup(cellspec, D, chi, seed=3)
    ocell = octm.Cell(Lx, Ly, cell)
    Cr, Tr = octm.iteration(ocell, sites, C, T, chi)
    Cg, Tg = dev(C), dev(T)
    ctx.ctmrg_moves(Lx, Ly, dev(np.stack(sites)), cell, Cg, Tg, 4 * Lx, 0)
    # gauge-invariant comparison: normalised corner spectra and RDMs
    sg = octm.corner_spectra(host(Cg))
    sr = octm.corner_spectra(Cr)
    np.testing.assert_allclose(sg, sr, atol=1e-10)
    r1g, rhg, rvg = ctx.ipeps_rdms(Lx, Ly, dev(np.stack(sites)), cell, Cg, Tg)
    r1, rh, rv = opeps.rdms(ocell, sites, Cr, Tr)
    np.testing.assert_allclose(host(r1g), np.stack(r1), atol=1e-10)
    np.testing.assert_allclose(host(rhg), np.stack(rh), atol=1e-10)
    np.testing.assert_allclose(host(rvg), np.stack(rv), atol=1e-10)


@pytest.mark.parametrize("cellspec", [tninputs.CHECKERBOARD, tninputs.SINGLE_SITE])
def test_rdms_parity_same_environment(ctx, cellspec):
    D, chi = 3, 7
    Lx, Ly, cell, sites, C, T = _setup(cellspec, D, chi, seed=5)
    ocell = octm.Cell(Lx, Ly, cell)
    r1g, rhg, rvg = ctx.ipeps_rdms(Lx, Ly, dev(np.stack(sites)), cell, dev(C), dev(T))
    r1, rh, rv = opeps.rdms(ocell, sites, C, T)
    np.testing.assert_allclose(host(r1g), np.stack(r1), atol=1e-12)
    np.testing.assert_allclose(host(rhg), np.stack(rh), atol=1e-12)
    np.testing.assert_allclose(host(rvg), np.stack(rv), atol=1e-12)


def test_ctmrg_converges_to_onsager(ctx):
    beta, chi = 0.3, 16
    A = pins.ising_peps(beta)
    Lx, Ly, cell = tninputs.CHECKERBOARD
    C, T = tninputs.ctm_env(0, 4, chi, 2, positive=True)
    Cg, Tg = dev(C), dev(T)
    sites = dev(np.stack([A, A]))
    # the corner-spectrum delta of this Z2-symmetric model stalls near 1e-9
    # at chi = 16 (near-degenerate pairs); the observables are the pin
    rc, it, delta = ctx.ctmrg_iterate(Lx, Ly, sites, list(cell), Cg, Tg, 80, 1e-12)
    assert delta < 1e-7
    _, rh, rv = ctx.ipeps_rdms(Lx, Ly, sites, list(cell), Cg, Tg)
    zz = np.kron(pins.SZ, pins.SZ)
    ref = pins.onsager_nn(beta)
    for p in range(4):
        assert abs(np.trace(host(rh)[p] @ zz) - ref) < 1e-9
        assert abs(np.trace(host(rv)[p] @ zz) - ref) < 1e-9


def test_converged_energy_parity(ctx):
    D, chi = 2, 10
    Lx, Ly, cell, sites, C, T = _setup(tninputs.CHECKERBOARD, D, chi, seed=0)
    ocell = octm.Cell(Lx, Ly, cell)
    Cr, Tr, itr, dr = octm.ctmrg(ocell, sites, C, T, chi, max_iter=60, tol=1e-11)
    er = opeps.energy_per_site(ocell, sites, Cr, Tr, 1.0, 3.0)
    Cg, Tg = dev(C), dev(T)
    sg = dev(np.stack(sites))
    rc, it, delta = ctx.ctmrg_iterate(Lx, Ly, sg, cell, Cg, Tg, 60, 1e-11)
    eg = ctx.ipeps_energy(Lx, Ly, sg, cell, Cg, Tg, 1.0, 3.0)
    assert it == itr
    assert abs(eg - er) < 1e-10 * abs(er)


@pytest.mark.parametrize("precision,u_in", [("fp32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("M,N,K,ta,tb", [(300, 200, 700, False, False), (2592, 96, 2592, True, False),
                                         (65, 130, 33, False, True)])
def test_reduced_precision_gemm(ctx, precision, u_in, M, N, K, ta, tb):
    """Operands rounded to fp32 / bf16, fp32 accumulation: elementwise error
    within (2 u_in + K u_fp32) (|A| |B|)."""
    rng = np.random.default_rng(M + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    Ae, Be = (A.T if ta else A), (B.T if tb else B)
    ref = Ae @ Be
    bound = (2 * u_in + K * 2.0 ** -24) * (np.abs(Ae) @ np.abs(Be))
    C = dev(np.zeros((M, N)))
    ctx.gemm(dev(A), dev(B), C, ta=ta, tb=tb, precision=precision)
    err = np.abs(host(C) - ref)
    assert (err <= bound).all(), float((err / bound).max())
    # and it is not silently FP64
    assert err.max() > 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_precision_form_converges_to_fp64_energy(ctx, precision):
    """Bulk contractions in fp32 / bf16 until their delta stalls, then FP64
    iterations to tol: the energy agrees with the oracle's converged FP64
    CTMRG to 1e-10 relative (stated tolerance of the precision form)."""
    D, chi = 3, 32
    Lx, Ly, cell, sites, C, T = _setup(tninputs.CHECKERBOARD, D, chi, seed=0)
    ocell = octm.Cell(Lx, Ly, cell)
    Cr, Tr, itr, dr = octm.ctmrg(ocell, sites, C, T, chi, max_iter=100, tol=1e-11)
    er = opeps.energy_per_site(ocell, sites, Cr, Tr, 1.0, 3.0)
    Cg, Tg = dev(C), dev(T)
    sg = dev(np.stack(sites))
    ctx.clear_cache()
    rc, it, delta = ctx.ctmrg_iterate(Lx, Ly, sg, cell, Cg, Tg, 100, 1e-10, precision=precision,
                                      n_polish=3)
    eg = ctx.ipeps_energy(Lx, Ly, sg, cell, Cg, Tg, 1.0, 3.0)
    assert rc == tn.TN_OK and delta < 1e-10
    assert abs(eg - er) < 1e-10 * abs(er)


def test_invalid_arguments_are_rejected(ctx):
    sites = dev(np.zeros((1, 2, 2, 2, 2, 2)))
    C, T = dev(np.zeros((1, 4, 4, 4))), dev(np.zeros((1, 4, 4, 2, 2, 4)))
    with pytest.raises(tn.TNError):
        ctx.ctmrg_moves(1, 1, sites, [3], C, T, 1)          # site index out of range
    with pytest.raises(tn.TNError):
        ctx.ctmrg_iterate(1, 1, sites, [0], C, T, 0, 1e-8)  # max_iter < 1
    with pytest.raises(tn.TNError):
        ctx.ctmrg_iterate(1, 1, sites, [0], C, T, 5, 1e-8, n_polish=-1)


@pytest.mark.parametrize("cellspec,D,chi", [(tninputs.CHECKERBOARD, 3, 32),
                                            (tninputs.SINGLE_SITE, 4, 20)])
def test_subspace_projector_path_parity(ctx, cellspec, D, chi):
    # n = chi D^2 > 256 takes the subspace-iteration projector SVD; after one
    # warm-up iteration the environment has a decaying spectrum as in use
    Lx, Ly, cell, sites, C, T = _setup(cellspec, D, chi, seed=7)
    ocell = octm.Cell(Lx, Ly, cell)
    C, T = octm.iteration(ocell, sites, C, T, chi)
    Cr, Tr, spectra = octm.left_move(ocell, sites, C, T, 0, chi)
    gap = min(s[chi - 1] / s[chi] for s in spectra)
    assert gap > 1 + 1e-6
    Cg, Tg = dev(C), dev(T)
    ctx.prof_enable(True)
    ctx.ctmrg_moves(Lx, Ly, dev(np.stack(sites)), cell, Cg, Tg, 1, 0)
    st = ctx.prof_read()
    ctx.prof_enable(False)
    assert st["svd_explicit"] == 0 and st["svd_calls"] == Ly
    np.testing.assert_allclose(host(Cg), Cr, atol=1e-9)
    np.testing.assert_allclose(host(Tg), Tr, atol=1e-9)


@pytest.mark.timeout(600)
def test_full_size_move_d8_chi128(ctx):
    """One left move of the large configuration: checkerboard, D = 8,
    chi = 128, so n = 8192 and a projector subspace of k = 160 (Cholesky and
    Jacobi with their work matrices beyond LDS).  The oracle needs minutes
    per move at this size (the SVD of an 8192 x 8192 matrix), so the checks
    are properties of the move: one subspace-iteration projector problem per
    row cut, finite output, unit Frobenius norm on every tensor the move
    writes (C1 of column x+1, row y+1; T4 and C4 of column x+1, row y) and
    every other tensor untouched."""
    D, chi = 8, 128
    Lx, Ly, cell, sites, C, T = _setup(tninputs.CHECKERBOARD, D, chi)
    ocell = octm.Cell(Lx, Ly, cell)
    written = set()
    for y in range(Ly):
        written.add((ocell.pos(1, y + 1), 0, "C"))
        written.add((ocell.pos(1, y), 3, "T"))
        written.add((ocell.pos(1, y), 3, "C"))
    Cg, Tg = dev(C), dev(T)
    ctx.prof_enable(True)
    ctx.prof_read()
    ctx.ctmrg_moves(Lx, Ly, dev(np.stack(sites)), cell, Cg, Tg, 1, 0)
    st = ctx.prof_read()
    ctx.prof_enable(False)
    print("projector problems", st["svd_calls"], "subspace iterations", st["svd_iters"])
    assert st["svd_calls"] == Ly and st["svd_explicit"] == 0
    Ch, Th = host(Cg), host(Tg)
    assert np.isfinite(Ch).all() and np.isfinite(Th).all()
    for p in range(Lx * Ly):
        for k in range(4):
            for name, new, old in (("C", Ch, C), ("T", Th, T)):
                if (p, k, name) in written:
                    assert abs(np.linalg.norm(new[p, k]) - 1.0) < 1e-12
                else:
                    np.testing.assert_array_equal(new[p, k], old[p, k])
