"""GPU parity of the small dense FP64 SVD against LAPACK (through the C ABI)."""
import numpy as np
import pytest

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


def _graded(rng, n, decades):
    q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -decades, n)
    return (q1 * s) @ q2.T, s


@pytest.mark.parametrize("m,n", [(96, 96), (130, 70), (33, 33), (7, 5), (1, 1),
                                 # batched, work matrix beyond LDS (global memory)
                                 (160, 160)])
def test_svd_random_parity(ctx, m, n):
    rng = np.random.default_rng(m + 7 * n)
    A = rng.standard_normal((3, m, n))
    U, S, V = ctx.svd(torch.from_numpy(A).cuda())
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    for b in range(3):
        ref = np.linalg.svd(A[b], compute_uv=False)
        np.testing.assert_allclose(S[b], ref, rtol=1e-12, atol=1e-13 * ref[0])
        np.testing.assert_allclose((U[b] * S[b]) @ V[b].T, A[b], atol=1e-12 * ref[0])
        np.testing.assert_allclose(U[b].T @ U[b], np.eye(n), atol=1e-12)
        np.testing.assert_allclose(V[b].T @ V[b], np.eye(n), atol=1e-12)


@pytest.mark.parametrize("m,n", [(300, 256), (512, 512), (200, 129)])
def test_svd_single_large_matrix(ctx, m, n):
    # one matrix with n > 128 runs across the GPU, one launch per round
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((1, m, n)) * np.logspace(0, -6, n)[None, None, :]
    U, S, V = ctx.svd(dev(A))
    U, S, V = host(U)[0], host(S)[0], host(V)[0]
    ref = np.linalg.svd(A[0], compute_uv=False)
    np.testing.assert_allclose(S, ref, rtol=1e-10, atol=1e-13 * ref[0])
    np.testing.assert_allclose((U * S) @ V.T, A[0], atol=1e-12 * ref[0])
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-9)


def test_svd_graded_high_relative_accuracy_and_sweeps(ctx):
    # A = B diag(d) with B well conditioned and d over 12 decades: one-sided
    # Jacobi resolves every singular value to high relative accuracy
    rng = np.random.default_rng(1)
    B = np.eye(96) + 0.1 * rng.standard_normal((96, 96))
    d = np.logspace(0, -12, 96)
    A = B * d[None, :]
    ref = np.linalg.svd(A, compute_uv=False)
    ctx.prof_enable(True)
    ctx.prof_read()
    _, S, _ = ctx.svd(torch.from_numpy(A[None]).cuda())
    st = ctx.prof_read()
    ctx.prof_enable(False)
    print("sweeps", st["jacobi_sweeps"])
    np.testing.assert_allclose(S.cpu().numpy()[0], ref, rtol=1e-9)
    assert st["jacobi_sweeps"] <= 15


def test_svd_near_diagonal_converges_fast(ctx):
    rng = np.random.default_rng(2)
    s = np.logspace(0, -10, 96)
    A = np.triu(np.diag(s) + 1e-6 * rng.standard_normal((96, 96)) * s[None, :])
    ctx.prof_enable(True)
    ctx.prof_read()
    _, S, _ = ctx.svd(torch.from_numpy(A[None]).cuda())
    st = ctx.prof_read()
    ctx.prof_enable(False)
    print("sweeps", st["jacobi_sweeps"])
    assert st["jacobi_sweeps"] <= 6


@pytest.mark.parametrize("k", [1, 7, 16, 33, 96, 128, 137, 160, 200])
def test_cholesky_inv_parity(ctx, k):
    """Blocked Cholesky and its inverse against LAPACK on SPD matrices, and a
    failing pivot reported on an indefinite one."""
    rng = np.random.default_rng(k)
    A = rng.standard_normal((2, k + 5, k))
    G = np.einsum("bik,bil->bkl", A, A)
    R, Ri, info = ctx.cholesky_inv(dev(G))
    assert info == [0, 0]
    for b in range(2):
        Rr = np.linalg.cholesky(G[b]).T
        np.testing.assert_allclose(np.triu(host(R)[b]), Rr, rtol=0, atol=1e-12 * np.abs(Rr).max())
        np.testing.assert_allclose(host(Ri)[b] @ Rr, np.eye(k), rtol=0,
                                   atol=1e-10 * np.linalg.cond(Rr))
    if k > 1:
        Gbad = G.copy()
        Gbad[1] = -Gbad[1]
        _, _, info = ctx.cholesky_inv(dev(Gbad))
        assert info[0] == 0 and info[1] == 1


@pytest.mark.parametrize("k,scale", [(96, 1e-12), (96, 3e-10), (40, 2e-8), (128, 1e-11)])
def test_cholesky_near_identity(ctx, k, scale):
    """Gram matrices I + E of almost orthonormal blocks (the second pass of
    Cholesky-QR): max|E| below 1e-9 takes the first-order closed form,
    above it the elimination; both match LAPACK to rounding."""
    rng = np.random.default_rng(k)
    E = scale * rng.standard_normal((2, k, k))
    G = np.eye(k)[None] + 0.5 * (E + E.transpose(0, 2, 1))
    R, Ri, info = ctx.cholesky_inv(dev(G))
    assert info == [0, 0]
    for b in range(2):
        Rr = np.linalg.cholesky(G[b]).T
        np.testing.assert_allclose(host(R)[b], Rr, rtol=0, atol=4e-16 * k)
        np.testing.assert_allclose(host(Ri)[b], np.linalg.inv(Rr), rtol=0, atol=4e-16 * k)


def test_cholesky_reports_nan(ctx):
    G = np.eye(16)[None].repeat(2, axis=0)
    G[1, 3, 5] = G[1, 5, 3] = np.nan
    _, _, info = ctx.cholesky_inv(dev(G))
    assert info[0] == 0 and info[1] > 0
