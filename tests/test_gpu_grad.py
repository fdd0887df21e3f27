"""GPU energy gradient: the hand-written reverse pass through CTMRG and the
energy (energy_grad) against the oracle's energy and its central finite
differences, plus exact invariants of E(A)."""
import time

import numpy as np
import pytest

import tninputs
from oracle import grad as ograd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1411_0391_amd as tn  # noqa: E402

J, H = 1.0, 3.0


@pytest.fixture(scope="module")
def ctx():
    c = tn.Context()
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def case(D, chi, seed=0):
    A = tninputs.ipeps_sites(seed, 1, D)[0]
    C0, T0 = tninputs.ctm_env(seed + 1, 1, chi, D)
    return A, C0, T0


def test_energy_and_gradient_match_the_oracle(ctx):
    D, chi, n_iter = 2, 6, 2
    A, C0, T0 = case(D, chi)
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=n_iter, ckpt_every=1)
    er = ograd.energy_after(A, C0, T0, chi, n_iter, J, H)
    print("E gpu", e, "oracle", er)
    assert abs(e - er) < 1e-10 * abs(er)
    dirs = tninputs.unit_directions(5, 8, A.shape)
    fd = ograd.fd_directional(A, C0, T0, chi, n_iter, J, H, dirs)
    gd = np.tensordot(dirs, host(g), axes=A.ndim)
    print("directional derivatives gpu", gd)
    print("oracle central differences ", fd)
    # E of this random state is steep (derivatives ~1e2) and its rounding
    # through the projectors' S^-1/2 limits the central differences to ~1e-7
    np.testing.assert_allclose(gd, fd, rtol=2e-6, atol=0)


@pytest.mark.parametrize("D,chi,n_iter", [(3, 14, 6), (4, 9, 3), (3, 15, 3)])
def test_steep_cases_with_small_steps(ctx, D, chi, n_iter):
    # random states where E(A) bends within 1e-6 of A (derivatives 1e3-1e5):
    # the central difference is linear only at steps near 1e-8 (at 1e-6 it is
    # off by up to 40%), and there it matches the reverse pass; (3, 15, 3) has
    # n = 135 and takes the GPU-wide SVD
    A, C0, T0 = case(D, chi)
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=n_iter, ckpt_every=2)
    dirs = tninputs.unit_directions(5, 1, A.shape)
    fd = ograd.fd_directional(A, C0, T0, chi, n_iter, J, H, dirs, step=1e-8)
    gd = np.tensordot(dirs, host(g), axes=A.ndim)
    print("gpu", gd, "central difference (step 1e-8)", fd)
    np.testing.assert_allclose(gd, fd, rtol=1e-4, atol=0)


def test_broadening_only_touches_near_degenerate_pairs(ctx):
    # the relative broadening 1e-12 changes the gradient only where two
    # singular values agree to ~1e-6; none do here
    A, C0, T0 = case(2, 8, seed=17)
    args = (dev(A), dev(C0[0]), dev(T0[0]), J, H)
    _, g0 = ctx.energy_grad(*args, n_iter=3, ckpt_every=2, broadening=0.0)
    _, g1 = ctx.energy_grad(*args, n_iter=3, ckpt_every=2, broadening=1e-12)
    g0, g1 = host(g0), host(g1)
    assert np.linalg.norm(g1 - g0) < 1e-8 * np.linalg.norm(g0)


def test_scale_invariance(ctx):
    # E(cA) = E(A): the gradient is orthogonal to A
    D, chi = 3, 9
    A, C0, T0 = case(D, chi, seed=3)
    e1, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=3, ckpt_every=2)
    e2, g2 = ctx.energy_grad(dev(2.5 * A), dev(C0[0]), dev(T0[0]), J, H, n_iter=3, ckpt_every=2)
    g, g2 = host(g), host(g2)
    assert abs(e1 - e2) < 1e-10 * abs(e1)
    assert abs(np.vdot(g, A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    # dE/d(cA) = dE/dA / c.  The two evaluations take different rounding
    # paths through three CTMRG iterations whose projectors carry S^-1/2;
    # their spread across builds is 1-1.5e-9 of max |g| for this steep state
    np.testing.assert_allclose(2.5 * g2, g, rtol=0, atol=1e-8 * np.abs(g).max())


def test_checkpointing_is_exact(ctx):
    D, chi, n_iter = 2, 8, 5
    A, C0, T0 = case(D, chi, seed=7)
    args = (dev(A), dev(C0[0]), dev(T0[0]), J, H)
    ref = None
    for ck in (1, 2, 3, 5, 9):
        e, g = ctx.energy_grad(*args, n_iter=n_iter, ckpt_every=ck)
        g = host(g)
        if ref is None:
            ref = (e, g)
        else:
            assert e == ref[0]
            np.testing.assert_allclose(g, ref[1], rtol=0, atol=1e-13 * np.abs(ref[1]).max())


def test_zero_iterations(ctx):
    # E of the starting environment itself: only the energy network is differentiated
    D, chi = 2, 6
    A, C0, T0 = case(D, chi, seed=11)
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=0, ckpt_every=1)
    er = ograd.energy_after(A, C0, T0, chi, 0, J, H)
    assert abs(e - er) < 1e-12 * abs(er)
    dirs = tninputs.unit_directions(2, 4, A.shape)
    fd = ograd.fd_directional(A, C0, T0, chi, 0, J, H, dirs)
    np.testing.assert_allclose(np.tensordot(dirs, host(g), axes=A.ndim), fd, rtol=1e-7,
                               atol=1e-8)


def test_autograd_function(ctx):
    D, chi = 2, 6
    A, C0, T0 = case(D, chi, seed=13)
    At = dev(A).requires_grad_(True)
    E = tn.energy(At, dev(C0[0]), dev(T0[0]), ctx, J, H, n_iter=2, ckpt_every=1)
    E.backward()
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=2, ckpt_every=1)
    assert float(E) == e
    np.testing.assert_array_equal(host(At.grad), host(g))


def test_bad_arguments(ctx):
    A, C0, T0 = case(2, 6)
    a, c, t = dev(A), dev(C0[0]), dev(T0[0])
    with pytest.raises(tn.TNError):
        ctx.energy_grad(a, c, t, J, H, n_iter=2, ckpt_every=0)
    with pytest.raises(tn.TNError):
        ctx.energy_grad(a, c, t, J, H, n_iter=-1)
    with pytest.raises(tn.TNError):
        ctx.energy_grad(a, c, t, J, H, n_iter=1, precision="bf16")
    # the FP32-bulk function has no gradient bound to state: rejected
    with pytest.raises(tn.TNError, match="FP64 only"):
        ctx.energy_grad(a, c, t, J, H, n_iter=1, precision="fp32")
    A3 = tninputs.ipeps_sites(0, 1, 2, d=3)[0]
    with pytest.raises(tn.TNError):
        ctx.energy_grad(dev(A3), c, t, J, H, n_iter=1)
    # n = chi D^2 above 512
    Ab, Cb, Tb = case(4, 33)
    with pytest.raises(tn.TNError):
        ctx.energy_grad(dev(Ab), dev(Cb[0]), dev(Tb[0]), J, H, n_iter=1)


@pytest.mark.timeout(900)
def test_single_site_d4_chi32(ctx):
    # the differentiation workload: D = 4, chi = 32 (n = 512), 20 iterations,
    # checkpoints every 5, against the oracle's energy and central differences
    # along seeded unit directions
    D, chi, n_iter = 4, 32, 20
    A, C0, T0 = case(D, chi, seed=21)
    t0 = time.perf_counter()
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=n_iter, ckpt_every=5)
    torch.cuda.synchronize()
    print(f"energy_grad D=4 chi=32, 20 iterations: {time.perf_counter() - t0:.2f} s, E = {e!r}")
    g = host(g)
    assert np.isfinite(g).all()
    assert abs(np.vdot(g, A)) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)
    er = ograd.energy_after(A, C0, T0, chi, n_iter, J, H)
    print("oracle E", er)
    assert abs(e - er) < 1e-10 * abs(er)
    # E(A) of this random state bends on the scale of 1e-5 and carries ~1e-13
    # of rounding: the central difference drifts by 3% between steps 1e-3 and
    # 1e-7; at 1e-7 it is linear to within its noise (~5e-7 absolute)
    dirs = tninputs.unit_directions(9, 2, A.shape)
    fd = ograd.fd_directional(A, C0, T0, chi, n_iter, J, H, dirs, step=1e-7)
    gd = np.tensordot(dirs, g, axes=A.ndim)
    print("directional derivatives gpu", gd)
    print("oracle central differences ", fd)
    np.testing.assert_allclose(gd, fd, rtol=3e-3, atol=0)


def _richardson(A, C0, T0, chi, n_iter, dirs, h):
    # central differences at h and 2h combined to cancel the h^2 term: the
    # error is O(h^4) plus rounding ~1e-16 |E| / h
    d1 = ograd.fd_directional(A, C0, T0, chi, n_iter, J, H, dirs, step=h)
    d2 = ograd.fd_directional(A, C0, T0, chi, n_iter, J, H, dirs, step=2 * h)
    return (4 * d1 - d2) / 3


def _smooth_case(D, chi):
    # a near-product state (bond-D part 0.3) and the positive seeded
    # boundary: E(A) is smooth on the scale of 1e-2 here, unlike the N(0,1)
    # states above, so Richardson-extrapolated differences at h = 1e-3 reach
    # ~1e-10 (measured: estimates from h = 2e-3, 1e-3, 5e-4 agree to 1e-10
    # relative, 2e-11 absolute on the smallest component)
    A = tninputs.ipeps_near_product(3, 1, D, eps=0.3)[0]
    C0, T0 = tninputs.ctm_env(4, 1, chi, D, positive=True)
    return A, C0, T0


@pytest.mark.timeout(600)
def test_gradient_along_64_directions(ctx):
    """64 seeded unit directions (D = 3, chi = 12, 6 iterations, n = 108):
    the adjoint's directional derivatives against Richardson-extrapolated
    central differences of the oracle's E, to 1e-7 relative."""
    D, chi, n_iter = 3, 12, 6
    A, C0, T0 = _smooth_case(D, chi)
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=n_iter, ckpt_every=2)
    assert abs(e - ograd.energy_after(A, C0, T0, chi, n_iter, J, H)) < 1e-10 * abs(e)
    dirs = tninputs.unit_directions(11, 64, A.shape)
    fd = _richardson(A, C0, T0, chi, n_iter, dirs, 1e-3)
    gd = np.tensordot(dirs, host(g), axes=A.ndim)
    err = np.abs(gd - fd)
    print("max relative deviation", float(np.max(err / np.maximum(np.abs(fd), 1e-2 * np.abs(fd).max()))))
    np.testing.assert_allclose(gd, fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())


@pytest.mark.timeout(900)
def test_d4_chi32_gradient_richardson(ctx):
    """The differentiation workload's size (D = 4, chi = 32, n = 512, 20
    iterations, checkpoints every 5) on a state where E is smooth: four
    seeded directions against Richardson-extrapolated central differences
    (each oracle evaluation takes ~8 s), to 1e-7 relative."""
    D, chi, n_iter = 4, 32, 20
    A, C0, T0 = _smooth_case(D, chi)
    e, g = ctx.energy_grad(dev(A), dev(C0[0]), dev(T0[0]), J, H, n_iter=n_iter, ckpt_every=5)
    assert abs(e - ograd.energy_after(A, C0, T0, chi, n_iter, J, H)) < 1e-10 * abs(e)
    dirs = tninputs.unit_directions(5, 4, A.shape)
    fd = _richardson(A, C0, T0, chi, n_iter, dirs, 1e-3)
    gd = np.tensordot(dirs, host(g), axes=A.ndim)
    print("gpu", gd, "richardson", fd)
    np.testing.assert_allclose(gd, fd, rtol=1e-7, atol=1e-9 * np.abs(fd).max())
