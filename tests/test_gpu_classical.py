"""GPU parity of the classical-partition-function workload (Sec. I): the
power method on the row transfer matrix of the 2D Ising model with an iMPS,
plain, recycled and in the limit N_Re -> infinity, against the oracle and
Onsager's free energy."""
import numpy as np
import pytest

import tninputs
from oracle import classical as cl
from oracle import gates, imps
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


def _start(chi, seed=0):
    ga, _, gb, _ = tninputs.imps_two_site(seed, chi)
    return [ga / np.linalg.norm(ga), gb / np.linalg.norm(gb)]


def test_one_step_parity(ctx):
    # one plain step from a state 10 steps in: new spectra, truncation error,
    # ln Z of the new state against the oracle's step (the same iTEBD
    # arithmetic as the quantum step, with the transfer-matrix gate)
    beta, chi = 0.35, 8
    sites = cl.power_method(_start(chi), beta, chi, 10)
    J, h, dt = cl.row_gate(beta)
    new, _, _, spec, err = imps.itebd_plain_step(sites, gates.impo(J, h, dt), chi)
    A = dev(np.stack(sites))
    env = ctx.env1d(chi)
    lam = torch.empty((2, chi), dtype=torch.float64, device="cuda")
    gerr, lz, rc = ctx.ising2d_tm_step(A, beta, env, lnz=True, lam=lam)
    assert rc == tn.TN_OK
    np.testing.assert_allclose(host(lam), np.stack(spec), atol=1e-10)
    assert abs(gerr - err) < 1e-10 * max(err, 1e-30) + 1e-15
    assert abs(lz - cl.log_z(new, beta)) < 1e-12


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_power_method_reaches_onsager(ctx, beta):
    chi = 8
    A = dev(np.stack(_start(chi)))
    env = ctx.env1d(chi)
    for step in range(60):
        _, lz, rc = ctx.ising2d_tm_step(A, beta, env, lnz=(step == 59))
        assert rc == tn.TN_OK
    assert abs(lz - pins.onsager_free_energy(beta)) < 1e-12


def test_recycled_and_limit_power_method(ctx):
    # 20 plain steps, then the environment recycled (N_Re = 5) or its limit:
    # both reach the plain fixed point's ln Z (oracle) to 1e-10
    beta, chi = 0.4, 8
    ref = cl.log_z(cl.power_method(_start(chi, 1), beta, chi, 200), beta)
    for n_re in (5, None):
        A = dev(np.stack(_start(chi, 1)))
        env = ctx.env1d(chi)
        for _ in range(20):
            ctx.ising2d_tm_step(A, beta, env)
        if n_re:
            for step in range(180):
                mode = tn.TN_RECYCLE_BUILD if step % n_re == 0 else tn.TN_RECYCLE_APPLY
                _, lz, rc = ctx.ising2d_tm_step(A, beta, env, mode=mode, lnz=(step == 179))
                assert rc == tn.TN_OK
        else:
            for step in range(8):
                _, _, rc = ctx.ising2d_tm_step(A, beta, env, mode=tn.TN_RECYCLE_BUILD)
                assert rc >= 0
                _, lz, rc = ctx.ising2d_tm_step(A, beta, env, mode=tn.TN_RECYCLE_LIMIT, lnz=True)
                assert rc == tn.TN_OK
        assert abs(lz - ref) < 1e-10, n_re


def test_rejects_bad_beta(ctx):
    A = dev(np.stack(_start(4)))
    with pytest.raises(tn.TNError):
        ctx.ising2d_tm_step(A, 0.0, ctx.env1d(4))
