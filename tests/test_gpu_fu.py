"""GPU parity of the full-update rows against the CPU oracle, through the C ABI:
gate application, truncation, canonical form / pre-truncation, bond
environment, ALS, gauge fixing and the renormalized gate."""
import numpy as np
import pytest

import tninputs
from oracle import ctmrg as octm
from oracle import fu as ofu
from oracle import gates
from oracle import peps as opeps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1411_0391_amd as tn  # noqa: E402

LEGNUM = {"l": 1, "r": 2, "d": 3, "u": 4}


@pytest.fixture(scope="module")
def ctx():
    c = tn.Context()
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64))).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _cell(spec):
    Lx, Ly, cell = spec
    return Lx, Ly, list(cell), octm.Cell(Lx, Ly, list(cell)), max(cell) + 1


@pytest.mark.parametrize("D", [2, 3])
def test_gate_parity(ctx, D):
    A = tninputs.ipeps_sites(3, 2, D)
    ref = np.stack([gates.apply_ipepo(gates.ipepo(1.0, 3.0, 0.01), a) for a in A])
    got = host(ctx.ipeps_gate(dev(np.stack(A)), 1.0, 3.0, 0.01))
    assert got.shape == ref.shape
    assert rel(got, ref) < 1e-14


@pytest.mark.parametrize("spec,Din,Dout", [(tninputs.CHECKERBOARD, 4, 2),
                                           (tninputs.SINGLE_SITE, 6, 3),
                                           (tninputs.CHECKERBOARD, 7, 7)])
def test_truncate_parity(ctx, spec, Din, Dout):
    Lx, Ly, cell, oc, nsite = _cell(spec)
    links, _ = opeps.cell_links(oc)
    rng = np.random.default_rng(Din * 10 + Dout)
    th = [rng.standard_normal((2,) + (Din,) * 4) for _ in range(nsite)]
    P = [rng.standard_normal((Din, Dout)) for _ in links]
    Q = [rng.standard_normal((Dout, Din)) for _ in links]
    ref = np.stack(opeps.truncate(th, links, P, Q))
    got = host(ctx.ipeps_truncate(Lx, Ly, cell, dev(np.stack(th)), dev(np.stack(P)),
                                  dev(np.stack(Q))))
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("spec,D", [(tninputs.CHECKERBOARD, 3), (tninputs.SINGLE_SITE, 4),
                                    (tninputs.CHECKERBOARD, 5)])
def test_canonical_form_parity(ctx, spec, D):
    Lx, Ly, cell, oc, nsite = _cell(spec)
    A = tninputs.ipeps_sites(5, nsite, D)
    a1, lams, Pc, Qc, it = opeps.canonicalize_a_form(oc, A, tol=1e-13)
    g1, glam, gP, gQ, git, rc = ctx.ipeps_canonicalize(Lx, Ly, cell, dev(np.stack(A)), tol=1e-13)
    assert rc == 0
    assert abs(git - it) <= 1
    assert rel(host(glam), np.stack(lams)) < 1e-10
    assert rel(host(gP), np.stack(Pc)) < 1e-8
    assert rel(host(gQ), np.stack(Qc)) < 1e-8
    assert rel(host(g1), np.stack(a1)) < 1e-8
    # the GPU result is canonical on its own terms (Eqs. (17)-(20))
    links, leg_link = opeps.cell_links(oc)
    glams = list(host(glam))
    gam = []
    for s, t in enumerate(host(g1)):
        for leg, ax in opeps.LEGS.items():
            w = 1.0 / np.sqrt(glams[leg_link[s][leg]])
            shape = [1] * 5
            shape[ax] = D
            t = t * w.reshape(shape)
        gam.append(t)
    assert opeps.canonical_residual(oc, gam, glams) < 1e-9


def test_su_pretruncation_parity(ctx):
    Lx, Ly, cell, oc, nsite = _cell(tninputs.CHECKERBOARD)
    D = 3
    A = tninputs.ipeps_sites(7, nsite, D)
    th = [gates.apply_ipepo(gates.ipepo(1.0, 3.0, 0.01), a) for a in A]
    P, Q = ofu.su_truncation(oc, th, D, tol=1e-13)
    Thg = ctx.ipeps_gate(dev(np.stack(A)), 1.0, 3.0, 0.01)
    _, _, gP, gQ, _, rc = ctx.ipeps_canonicalize(Lx, Ly, cell, Thg, D_keep=D, tol=1e-13,
                                                 a_out=False)
    assert rc == 0
    # both sides stop the canonical-form iteration when the spectra move by
    # less than 1e-13; measured deviations 1e-13 to 4e-13 in P, Q and P Q
    for b in range(len(P)):
        assert rel(host(gP)[b] @ host(gQ)[b], P[b] @ Q[b]) < 1e-11
    assert rel(host(gP), np.stack(P)) < 1e-11
    assert rel(host(gQ), np.stack(Q)) < 1e-11


def _fu_state(spec, D, chi, converged, seed=0):
    """Theta of a gated random state, its simple-update (P, Q) and an
    environment of the pre-truncated state (converged by the oracle CTMRG, or
    the positive random start)."""
    Lx, Ly, cell, oc, nsite = _cell(spec)
    A = tninputs.ipeps_sites(seed, nsite, D)
    th = [gates.apply_ipepo(gates.ipepo(1.0, 3.0, 0.01), a) for a in A]
    P, Q = ofu.su_truncation(oc, th, D)
    links, _ = opeps.cell_links(oc)
    pre = opeps.truncate(th, links, P, Q)
    C, T = tninputs.ctm_env(seed + 1, Lx * Ly, chi, D, positive=True)
    if converged:
        C, T, _, _ = octm.ctmrg(oc, pre, C, T, chi, 100, 1e-10)
    return Lx, Ly, cell, oc, th, P, Q, C, T


@pytest.mark.parametrize("spec,D,chi,conv", [(tninputs.CHECKERBOARD, 2, 6, False),
                                             (tninputs.CHECKERBOARD, 3, 8, True),
                                             (tninputs.SINGLE_SITE, 2, 7, True)])
def test_bond_environment_parity(ctx, spec, D, chi, conv):
    """Both environments of every slot of the truncation block (Sec. VI B),
    entry by entry, with the internal links truncated by a zeta that differs
    from the pre-truncation on the environment legs."""
    Lx, Ly, cell, oc, th, P, Q, C, T = _fu_state(spec, D, chi, conv)
    rng = np.random.default_rng(D * 100 + chi)
    Pz = [p + 0.1 * rng.standard_normal(p.shape) for p in P]
    Qz = [q + 0.1 * rng.standard_normal(q.shape) for q in Q]
    slot_link = ofu.block_slot_links(oc)
    args = (dev(np.stack(th)), dev(C), dev(T), dev(np.stack(P)), dev(np.stack(Q)),
            dev(np.stack(Pz)), dev(np.stack(Qz)))
    for k in range(4):
        N, M = ofu.bond_environment(oc, th, P, Q, [Pz[b] for b in slot_link],
                                    [Qz[b] for b in slot_link], C, T, k)
        gN, gM = ctx.bond_environment(Lx, Ly, cell, *args, k)
        assert rel(host(gN), N) < 1e-11, k
        assert rel(host(gM), M) < 1e-11, k


def _truncate_problem(spec, D, chi, seed=0):
    Lx, Ly, cell, oc, th, P, Q, C, T = _fu_state(spec, D, chi, True, seed)
    return Lx, Ly, cell, oc, th, P, Q, C, T


@pytest.mark.parametrize("spec,D,chi", [(tninputs.CHECKERBOARD, 2, 6),
                                        (tninputs.CHECKERBOARD, 3, 8),
                                        (tninputs.SINGLE_SITE, 3, 9)])
def test_bond_env_truncate_parity(ctx, spec, D, chi):
    """A fixed number of cycles (the same arithmetic on both sides): the
    block cost, its scale and the truncations; then the converged call."""
    Lx, Ly, cell, oc, th, P, Q, C, T = _truncate_problem(spec, D, chi)
    for passes, tol in ((3, 0.0), (200, 1e-12)):
        Pr, Qr, fr, pr, swr, _ = ofu.fu_truncate(oc, th, P, Q, C, T, tol, passes, 1)
        tn = abs(ofu.block_norm(oc, th, P, Q, C, T))
        gP, gQ = dev(np.stack(P)), dev(np.stack(Q))
        f, t, gp, gsw = ctx.bond_env_truncate(Lx, Ly, cell, dev(np.stack(th)), dev(C), dev(T),
                                              dev(np.stack(P)), dev(np.stack(Q)), gP, gQ,
                                              passes, 1, tol)
        assert abs(t - tn) < 1e-12 * tn
        # f = T - 2c + q cancels down from T: its rounding is relative to T
        assert abs(f - fr) < 1e-11 * tn, (passes, f, fr)
        if tol == 0.0:
            # the same cycles on both sides: measured deviations 7e-14 to
            # 4e-13 in P Q and 1e-12 to 5e-12 in P, Q (these carry the
            # balancing SVD's basis, which near-degenerate singular values
            # of P Q fix less well than the product)
            assert gp == pr == passes and gsw == swr
            for b in range(len(P)):
                assert rel(host(gP)[b] @ host(gQ)[b], Pr[b] @ Qr[b]) < 1e-11, b
            assert rel(host(gP), np.stack(Pr)) < 1e-10
            assert rel(host(gQ), np.stack(Qr)) < 1e-10
        else:
            assert abs(gp - pr) <= 1


@pytest.fixture(scope="module")
def c2_state():
    """The full-update problem at the shape of the D = 4, chi = 32
    configuration: a gated seeded state, its pre-truncation and the oracle's
    environment of the pre-truncated state after 10 iterations (delta ~1e-5)
    from the positive seeded boundary."""
    Lx, Ly, cell, oc, th, P, Q, C, T = _fu_state(tninputs.CHECKERBOARD, 4, 32, False)
    links, _ = opeps.cell_links(oc)
    C, T, _, _ = octm.ctmrg(oc, opeps.truncate(th, links, P, Q), C, T, 32, 10, 0.0)
    return Lx, Ly, cell, oc, th, P, Q, C, T


def test_full_update_chain_d4_chi32(ctx, c2_state):
    """The full-update calls at the D = 4, chi = 32 shape: the pre-truncation
    (canonical form of Theta), two slots' environments, two cycles of the
    truncation, and the gauge fix of the truncated state's canonical form
    against a planted gauge."""
    Lx, Ly, cell, oc, th, P, Q, C, T = c2_state
    D = 4
    # pre-truncation
    Thg = dev(np.stack(th))
    _, _, gPs, gQs, _, rc = ctx.ipeps_canonicalize(Lx, Ly, cell, Thg, D_keep=D, tol=1e-13,
                                                   a_out=False)
    assert rc == 0
    Pt, Qt = ofu.su_truncation(oc, th, D, tol=1e-13)
    for b in range(len(P)):
        assert rel(host(gPs)[b] @ host(gQs)[b], Pt[b] @ Qt[b]) < 1e-11
    # environments of the top and bottom slots
    for k in (0, 2):
        N, M = ofu.bond_environment(oc, th, P, Q, P, Q, C, T, k)
        gN, gM = ctx.bond_environment(Lx, Ly, cell, Thg, dev(C), dev(T), dev(np.stack(P)),
                                      dev(np.stack(Q)), dev(np.stack(P)), dev(np.stack(Q)), k)
        assert rel(host(gN), N) < 1e-11
        assert rel(host(gM), M) < 1e-11
    # two cycles of the truncation
    Pr, Qr, fr, _, _, _ = ofu.fu_truncate(oc, th, P, Q, C, T, 0.0, 2, 1)
    tn = abs(ofu.block_norm(oc, th, P, Q, C, T))
    gP, gQ = dev(np.stack(P)), dev(np.stack(Q))
    f, t, _, _ = ctx.bond_env_truncate(Lx, Ly, cell, Thg, dev(C), dev(T), dev(np.stack(P)),
                                       dev(np.stack(Q)), gP, gQ, 2, 1, 0.0)
    assert abs(t - tn) < 1e-12 * tn
    assert abs(f - fr) < 1e-11 * tn
    for b in range(len(P)):
        assert rel(host(gP)[b] @ host(gQ)[b], Pr[b] @ Qr[b]) < 1e-8, b
    # gauge fix of the canonical truncated state against a planted gauge
    links, leg_link = opeps.cell_links(oc)
    a1, _, _, _, _ = opeps.canonicalize_a_form(oc, opeps.truncate(th, links, Pr, Qr), tol=1e-13)
    rng = np.random.default_rng(8)
    Ut = [_rot(rng, D, 0.3) for _ in links]
    a_new = [opeps._apply_all(a, s, leg_link, Ut) for s, a in enumerate(a1)]
    U0 = [np.eye(D) for _ in links]
    Ur, Fr, _ = opeps.gauge_fix(oc, a1, a_new, tol=1e-13, U0=U0)
    Ug = dev(np.stack(U0))
    Fg, _, rc = ctx.gauge_fix(Lx, Ly, cell, dev(np.stack(a1)), dev(np.stack(a_new)), Ug,
                              tol=1e-13)
    assert rc == 0
    assert abs(Fg - Fr) < 1e-12 and abs(Fr - 1) < 1e-10
    assert rel(host(Ug), np.stack(Ur)) < 1e-8
    # F is stationary at its maximum: the stop |dF| < 1e-13 fixes U to ~sqrt(1e-13)
    assert rel(host(Ug), np.stack(Ut)) < 1e-6


def _rot(rng, D, eps):
    a = rng.standard_normal((D, D))
    from scipy.linalg import expm
    return expm(eps * (a - a.T))


@pytest.mark.parametrize("spec,D", [(tninputs.CHECKERBOARD, 3), (tninputs.SINGLE_SITE, 4),
                                    (tninputs.CHECKERBOARD, 5)])
def test_gauge_fix_parity(ctx, spec, D):
    Lx, Ly, cell, oc, nsite = _cell(spec)
    links, leg_link = opeps.cell_links(oc)
    rng = np.random.default_rng(D)
    a_ref = tninputs.ipeps_sites(11, nsite, D)
    Ut = [_rot(rng, D, 0.3) for _ in links]
    a_new = []
    for s, a in enumerate(a_ref):
        t = opeps._apply_all(a, s, leg_link, Ut)
        a_new.append(t + 1e-3 * rng.standard_normal(t.shape))
    U0 = [np.eye(D) for _ in links]
    Ur, Fr, itr = opeps.gauge_fix(oc, a_ref, a_new, tol=1e-13, U0=U0)
    Ug = dev(np.stack(U0))
    Fg, itg, rc = ctx.gauge_fix(Lx, Ly, cell, dev(np.stack(a_ref)), dev(np.stack(a_new)), Ug,
                                tol=1e-13)
    assert rc == 0
    assert abs(Fg - Fr) < 1e-12
    assert abs(itg - itr) <= 1
    assert rel(host(Ug), np.stack(Ur)) < 1e-8
    # it found the planted gauge
    assert rel(host(Ug), np.stack(Ut)) < 1e-2


def test_recycling_factors_parity(ctx):
    rng = np.random.default_rng(4)
    nl, D, k = 4, 3, 2
    Dk = k * D
    P = [rng.standard_normal((Dk, D)) for _ in range(nl)]
    Q = [rng.standard_normal((D, Dk)) for _ in range(nl)]
    Pc = [rng.standard_normal((D, D)) for _ in range(nl)]
    Qc = [rng.standard_normal((D, D)) for _ in range(nl)]
    U = [_rot(rng, D, 1.0) for _ in range(nl)]
    Rf, Lf = ofu.renormalized_gate(P, Q, Pc, Qc, U)
    gRf, gLf = ctx.fu_renormalized_gate(dev(np.stack(P)), dev(np.stack(Q)), dev(np.stack(Pc)),
                                        dev(np.stack(Qc)), dev(np.stack(U)))
    assert rel(host(gRf), np.stack(Rf)) < 1e-13
    assert rel(host(gLf), np.stack(Lf)) < 1e-13
    U0 = ofu.gauge_start(P, Q, Pc, Qc, k)
    gU0 = ctx.fu_gauge_start(dev(np.stack(P)), dev(np.stack(Q)), dev(np.stack(Pc)),
                             dev(np.stack(Qc)), k)
    assert rel(host(gU0), np.stack(U0)) < 1e-10


def test_energy_parity(ctx):
    Lx, Ly, cell, oc, th, P, Q, C, T = _fu_state(tninputs.CHECKERBOARD, 2, 6, True)
    links, _ = opeps.cell_links(oc)
    pre = opeps.truncate(th, links, P, Q)
    ref = opeps.energy_per_site(oc, pre, C, T, 1.0, 3.0)
    got = ctx.ipeps_energy(Lx, Ly, dev(np.stack(pre)), cell, dev(C), dev(T), 1.0, 3.0)
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_full_update_rejects_bad_arguments(ctx):
    th = dev(np.zeros((2, 2, 4, 4, 4, 4)))
    P, Q = dev(np.zeros((4, 4, 2))), dev(np.zeros((4, 2, 4)))
    C, T = dev(np.zeros((4, 4, 3, 3))), dev(np.zeros((4, 4, 3, 2, 2, 3)))
    with pytest.raises(tn.TNError):
        ctx.ipeps_truncate(2, 2, [0, 1, 2, 0], th, P, Q)      # site index out of range
    with pytest.raises(tn.TNError):
        ctx.bond_env_truncate(2, 2, [0, 1, 1, 0], th, C, T, P, Q, P.clone(), Q.clone(),
                              max_sweeps=0)
    with pytest.raises(tn.TNError):
        ctx.bond_environment(2, 2, [0, 1, 1, 0], th, C, T, P, Q, P, Q, 7)   # no slot 7
    with pytest.raises(tn.TNError):
        # a cell with links outside the 2x2 block at the origin
        th3 = dev(np.zeros((3, 2, 4, 4, 4, 4)))
        P9, Q9 = dev(np.zeros((6, 4, 2))), dev(np.zeros((6, 2, 4)))
        C9, T9 = dev(np.zeros((3, 4, 3, 3))), dev(np.zeros((3, 4, 3, 2, 2, 3)))
        ctx.bond_env_truncate(3, 1, [0, 1, 2], th3, C9, T9, P9, Q9, P9.clone(), Q9.clone())
    with pytest.raises(tn.TNError):
        ctx.ipeps_gate(dev(np.zeros((1, 3, 2, 2, 2, 2))), 1.0, 3.0, 0.01)  # d must be 2


@pytest.mark.parametrize("n_re,n_warm,nsteps,force", [(1, 0, 3, False), (3, 1, 7, False),
                                                    (1, 0, 2, True)])
def test_full_update_driver_parity(ctx, n_re, n_warm, nsteps, force):
    """The GPU driver (library calls only) follows the oracle's full update
    with recycling step by step: energies at every environment step, which
    steps were recycled, the gauge-fix fidelities and the final tensors."""
    from paper_1411_0391_amd import driver
    Lx, Ly, cell, oc, nsite = _cell(tninputs.CHECKERBOARD)
    D, chi = 2, 8
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_sites(2, nsite, D)]
    C, T = tninputs.ctm_env(3, Lx * Ly, chi, D, positive=True)
    fids = []
    ref_sites, ref_log = ofu.run_fu(oc, A, 1.0, 3.0, 0.01, D, chi, nsteps, n_re=n_re,
                                    n_warm=n_warm, C=C, T=T, force_recycle=force,
                                    callback=lambda st, out: fids.append(out["fidelity"]))
    Cg, Tg = dev(C), dev(T)
    sites, log = driver.full_update(ctx, Lx, Ly, cell, dev(np.stack(A)), Cg, Tg, 1.0, 3.0, 0.01,
                                    nsteps, n_re=n_re, n_warm=n_warm, force_recycle=force)
    assert [s for s, *_ in log] == [s for s, *_ in ref_log]
    assert [r for _, _, _, r, _ in log] == [r for _, _, r in ref_log]
    for (_, e, _, _, F), (_, er, _), Fr in zip(log, ref_log, fids):
        assert abs(e - er) < 1e-9 * abs(er)
        if Fr is not None:
            assert abs(F - Fr) < 1e-9
    assert rel(host(sites), np.stack(ref_sites)) < 1e-6


def test_untruncated_environment_truncate_parity(ctx):
    """The form without pre-truncation (Sec. VI B, closing cost remark) on
    the one-site cell: the environment of Theta itself (bond kappa D) and
    identities on the block's outer legs (De = kappa D); a fixed number of
    cycles, then the links' (P, Q) means over their two slots each."""
    Lx, Ly, cell, oc, nsite = _cell(tninputs.SINGLE_SITE)
    D, chi = 2, 6
    a = tninputs.ipeps_sites(7, 1, D)[0]
    th = [gates.apply_ipepo(gates.ipepo(1.0, 3.0, 0.01), a / np.linalg.norm(a))]
    Dk = th[0].shape[1]
    links, _ = opeps.cell_links(oc)
    P, Q = ofu.su_truncation(oc, th, D)
    C, T = tninputs.ctm_env(1, 1, chi, Dk, positive=True)
    C, T, _, _ = octm.ctmrg(oc, th, C, T, chi, 200, 1e-12)
    eye = [np.eye(Dk) for _ in links]
    Pr, Qr, fr, _, _, _ = ofu.fu_truncate(oc, th, eye, eye, C, T, 0.0, 2, 1, P0=P, Q0=Q)
    tn_ = abs(ofu.block_norm(oc, th, eye, eye, C, T))
    gP, gQ = dev(np.stack(P)), dev(np.stack(Q))
    f, t, gp, _ = ctx.bond_env_truncate(Lx, Ly, cell, dev(np.stack(th)), dev(C), dev(T),
                                        dev(np.stack(eye)), dev(np.stack(eye)), gP, gQ, 2, 1, 0.0)
    assert gp == 2
    assert abs(t - tn_) < 1e-12 * tn_
    assert abs(f - fr) < 1e-11 * tn_
    for b in range(len(links)):
        assert rel(host(gP)[b] @ host(gQ)[b], Pr[b] @ Qr[b]) < 1e-9, b
    assert rel(host(gP), np.stack(Pr)) < 1e-8
    assert rel(host(gQ), np.stack(Qr)) < 1e-8


@pytest.fixture(scope="module")
def one_site_start():
    """A one-site D = 2 state 300 simple-update steps (oracle) from the
    seeded near-product state, E = -3.1931 at h = 3.0: entangled, smoothly
    evolving, and well conditioned (in the oracle a 1e-13 perturbation of it
    moves the sites after three full-update steps by 5e-10).  From a
    near-product state itself the block's environment has directions of
    weight ~1e-14 along which R^-1 S fixes (P, Q) only through the
    regularisation, and the sites move by 2e-7 under the same perturbation."""
    oc = octm.Cell(1, 1, [0])
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_near_product(0, 1, 2)]
    return ofu.run_su(oc, A, 1.0, 3.0, 0.01, 2, 300)


@pytest.mark.parametrize("n_re,nsteps,pretruncate", [(1, 3, True), (2, 5, True), (1, 3, False)])
def test_one_site_full_update_driver_parity(ctx, one_site_start, n_re, nsteps, pretruncate):
    """The paper's own scheme (Sec. VI B): one-site cell, the links' (P, Q)
    the means over their slots; plain and recycled, and the form without
    pre-truncation.  A fixed number of ALS cycles per step on both sides (20;
    3 without pre-truncation, its oracle block being slow)."""
    from paper_1411_0391_amd import driver
    Lx, Ly, cell, oc, nsite = _cell(tninputs.SINGLE_SITE)
    D, chi, kappa = 2, 8, 2
    A = one_site_start
    C, T = tninputs.ctm_env(3, 1, chi, D if pretruncate else kappa * D, positive=True)
    passes, tol = (20, 0.0) if pretruncate else (3, 0.0)
    fids = []
    ref_sites, ref_log = ofu.run_fu(oc, A, 1.0, 3.0, 0.01, D, chi, nsteps, n_re=n_re, C=C, T=T,
                                    als_tol=tol, als_passes=passes, pretruncate=pretruncate,
                                    callback=lambda st, out: fids.append(out["fidelity"]))
    sites, log = driver.full_update(ctx, Lx, Ly, cell, dev(np.stack(A)), dev(C), dev(T), 1.0,
                                    3.0, 0.01, nsteps, n_re=n_re, als_tol=tol, als_passes=passes,
                                    pretruncate=pretruncate)
    assert [s for s, *_ in log] == [s for s, *_ in ref_log]
    assert [r for _, _, _, r, _ in log] == [r for _, _, r in ref_log]
    for (_, e, _, _, F), (_, er, _), Fr in zip(log, ref_log, fids):
        assert abs(e - er) < 1e-9 * abs(er)
        if Fr is not None:
            assert abs(F - Fr) < 1e-9
    assert rel(host(sites), np.stack(ref_sites)) < 1e-6


def test_full_update_energy_within_the_ed_bracket(ctx):
    """The D = 2 full update from a near-product start at h = 3.0 (300 steps
    of dt = 0.01): its energy per site must lie below the mean-field value
    -2 - h^2/8 (the D = 2 state carries correlations a product state cannot)
    and above the 4x4 torus ED value less 1% (finite-size bias of the torus
    is downward and below 1% here)."""
    from paper_1411_0391_amd import driver
    from tests import pins
    Lx, Ly, cell, oc, nsite = _cell(tninputs.CHECKERBOARD)
    D, chi, h = 2, 16, 3.0
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_near_product(0, nsite, D)]
    C, T = tninputs.ctm_env(1, Lx * Ly, chi, D, positive=True)
    _, log = driver.full_update(ctx, Lx, Ly, cell, dev(np.stack(A)), dev(C), dev(T), 1.0, h, 0.01,
                                300)
    e = log[-1][1]
    e_ed = pins.tfim2d_torus_ed(4, 4, h)
    assert e < -2 - h * h / 8 - 0.05, e
    assert e > 1.01 * e_ed, e


@pytest.mark.parametrize("spec", [tninputs.SINGLE_SITE, tninputs.CHECKERBOARD])
def test_simple_update_parity(ctx, spec):
    """The simple update (Sec. VI A): 100 steps of gate and canonical-form
    truncation against the oracle's, the sites entry by entry and the energy
    and magnetisation of the result with its converged environment (chi = 4
    converges to 1e-12 here; a larger chi leaves noise directions on which
    delta stalls near 1e-9)."""
    from paper_1411_0391_amd import driver
    Lx, Ly, cell, oc, nsite = _cell(spec)
    D, chi, h = 2, 4, 3.0
    A = [a / np.linalg.norm(a) for a in tninputs.ipeps_near_product(0, nsite, D)]
    ref = ofu.run_su(oc, A, 1.0, h, 0.01, D, 100)
    got = driver.simple_update(ctx, Lx, Ly, cell, dev(np.stack(A)), 1.0, h, 0.01, 100)
    assert rel(host(got), np.stack(ref)) < 1e-8
    C, T = tninputs.ctm_env(1, Lx * Ly, chi, D, positive=True)
    Cr, Tr, _, dr = octm.ctmrg(oc, ref, C, T, chi, 100, 1e-11)
    er = opeps.energy_per_site(oc, ref, Cr, Tr, 1.0, h)
    mr = opeps.magnetization_z(oc, ref, Cr, Tr)
    Cg, Tg = dev(C), dev(T)
    _, _, dg = ctx.ctmrg_iterate(Lx, Ly, got, cell, Cg, Tg, 100, 1e-11)
    eg = ctx.ipeps_energy(Lx, Ly, got, cell, Cg, Tg, 1.0, h)
    r1 = host(ctx.ipeps_rdms(Lx, Ly, got, cell, Cg, Tg)[0])
    mg = float(np.mean([np.trace(r @ np.diag([1.0, -1.0])) for r in r1]))
    assert dr < 1e-10 and dg < 1e-10
    assert abs(eg - er) < 1e-9 * abs(er)
    assert abs(mg - mr) < 1e-8
