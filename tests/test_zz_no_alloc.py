"""The allocation-free transfer-matrix fixed point against tm_fixed_point,
through the C ABI: two calls in a row, the second on a smaller problem, cold
and warm-started, and the size limit of its fixed scratch."""
import numpy as np
import pytest

import tninputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1411_0391_amd as tn  # noqa: E402


def _chain_host(chi, seed):
    ga, _, gb, _ = tninputs.imps_two_site(seed, chi)
    return np.stack([ga / np.linalg.norm(ga), gb / np.linalg.norm(gb)])


def _chain(chi, seed, device="cuda"):
    return torch.from_numpy(_chain_host(chi, seed)).to(device)


def _nearby(chi, seed, device="cuda"):
    """The seed-th chain plus 1e-2 of another, each site at unit norm."""
    b = _chain_host(chi, seed) + 1e-2 * _chain_host(chi, seed + 7)
    b = b / np.sqrt((b.reshape(2, -1) ** 2).sum(axis=1)).reshape(2, 1, 1, 1)
    return torch.from_numpy(b).to(device)


def test_noalloc_fixed_point_matches_allocating_call():
    ctx = tn.Context()
    try:
        # chi = 48: the kernels' working set in the scratch array (beyond LDS);
        # then chi = 12, a smaller problem whose working set sits in LDS
        for chi, seed in ((48, 0), (12, 1)):
            A = _chain(chi, seed)
            vl, vr, eta, it, rc = ctx.tm_fixed_point(A, A, tol=1e-13)
            vl2, vr2 = torch.empty_like(vl), torch.empty_like(vr)
            eta2, it2, rc2 = ctx.tm_fixed_point_noalloc(A, A, vl2, vr2, tol=1e-13)
            assert (rc2, it2) == (rc, it)
            assert abs(eta2 - eta) <= 1e-14 * abs(eta)
            np.testing.assert_allclose(vl2.cpu().numpy(), vl.cpu().numpy(), rtol=0, atol=1e-14)
            np.testing.assert_allclose(vr2.cpu().numpy(), vr.cpu().numpy(), rtol=0,
                                       atol=1e-14 * float(vr.abs().max()))
            # warm start from the fixed points just found, on the mixed
            # transfer matrix of A and a nearby state B
            B = _nearby(chi, seed)
            wl, wr = vl.clone(), vr.clone()
            _, _, eta3, it3, rc3 = ctx.tm_fixed_point(A, B, tol=1e-13, vl=wl, vr=wr)
            ul, ur = vl.clone(), vr.clone()
            eta4, it4, rc4 = ctx.tm_fixed_point_noalloc(A, B, ul, ur, tol=1e-13, warm=True)
            assert (rc4, it4) == (rc3, it3)
            assert abs(eta4 - eta3) <= 1e-14 * abs(eta3)
            np.testing.assert_allclose(ul.cpu().numpy(), wl.cpu().numpy(), rtol=0, atol=1e-14)
            np.testing.assert_allclose(ur.cpu().numpy(), wr.cpu().numpy(), rtol=0,
                                       atol=1e-14 * float(wr.abs().max()))
        # beyond the fixed scratch (chi = 150 needs 26 chi^2 > 2^19 doubles)
        A = _chain(150, 2)
        v1, v2 = torch.empty((150, 150), dtype=torch.float64, device="cuda"), \
            torch.empty((150, 150), dtype=torch.float64, device="cuda")
        with pytest.raises(tn.TNError, match="scratch"):
            ctx.tm_fixed_point_noalloc(A, A, v1, v2)
    finally:
        ctx.close()
