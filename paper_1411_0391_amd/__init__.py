"""Python binding of the MI355X environment-recycled iTEBD library.

Argument marshalling only: every call forwards device pointers of torch
tensors (PyTorch provides device memory and the stream) to the C ABI in
``include/itebd.h``; all arithmetic runs in the HIP kernels of
``libitebd.so``.  Importing this module on a machine without the built
library raises immediately -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libitebd.so")

TN_OK, TN_NOT_CONVERGED = 0, 1
TN_FP64, TN_FP32, TN_BF16 = 0, 1, 2
TN_PLAIN, TN_RECYCLE_BUILD, TN_RECYCLE_APPLY, TN_RECYCLE_LIMIT = 0, 1, 2, 3
TN_RECYCLE_BUILD_DIRECT = 4
TN_GAUGE_2D, TN_GAUGE_1D, TN_GAUGE_1D_DIRECT = 0, 1, 2
_PREC = {"fp64": TN_FP64, "fp32": TN_FP32, "bf16": TN_BF16}

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_double_p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); every symbol include/itebd.h declares
SIGNATURES = {
    "tn_create": (ctypes.c_int, [ctypes.POINTER(_vp), _vp]),
    "tn_destroy": (ctypes.c_int, [_vp]),
    "tn_last_error": (ctypes.c_char_p, [_vp]),
    "tn_version": (ctypes.c_char_p, []),
    "ctmrg_iterate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _vp, _c_int_p, ctypes.c_int, _vp, _vp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     _c_int_p, _c_double_p]),
    "ctmrg_moves": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _vp, _c_int_p, ctypes.c_int, _vp, _vp,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ipeps_rdms": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, _vp, _c_int_p, ctypes.c_int, _vp, _vp, _vp, _vp,
                                  _vp]),
    "tn_gemm": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                               ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    "tn_clear_cache": (ctypes.c_int, [_vp]),
    "tn_cholesky_inv": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_double, _vp,
                                       _vp, _c_int_p]),
    "tm_fixed_point_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                              _vp, _vp, _vp, _c_double_p, ctypes.c_double,
                                              ctypes.c_int, _c_int_p, ctypes.c_int]),
    "tn_env1d_size": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "tm_fixed_point": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                      _vp, _vp, _c_double_p, ctypes.c_double, ctypes.c_int,
                                      _c_int_p, ctypes.c_int]),
    "itebd_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _vp, _vp,
                                  ctypes.c_double, _c_double_p, _c_double_p]),
    "ising2d_tm_step": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_double, ctypes.c_int,
                                       _vp, _vp, ctypes.c_double, _c_double_p, _c_double_p]),
    "ipeps_cell_links": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                        _c_int_p, _c_int_p]),
    "ipeps_gate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _vp, _vp]),
    "ipeps_truncate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                      _vp]),
    "ipeps_canonicalize": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                          _vp, _vp, ctypes.c_double, ctypes.c_int, _c_int_p]),
    "gauge_fix": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 _c_int_p, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                 ctypes.c_double, ctypes.c_int, _c_double_p, _c_int_p]),
    "bond_env_truncate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _vp,
                                         ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         _c_double_p, _c_int_p, _c_int_p]),
    "bond_environment": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_int_p,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        _vp,
                                        ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_int, _vp, _vp]),
    "fu_gauge_start": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _vp, _vp, _vp, _vp, _vp]),
    "fu_renormalized_gate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                            _vp, _vp, _vp, _vp, _vp, _vp]),
    "ipeps_energy": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, _vp, _c_int_p, ctypes.c_int, _vp, _vp,
                                    ctypes.c_double, ctypes.c_double, _c_double_p]),
    "energy_grad": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, _c_double_p, _vp]),
    "tn_svd": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "tn_prof_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tn_prof_read": (ctypes.c_int, [_vp, _c_double_p, _c_double_p,
                                    ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_longlong)]),
}


class LibraryMissing(RuntimeError):
    pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libitebd.so and attach the C signatures; raise if it is absent."""
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run paper_1411_0391_amd/build.py")
    # torch first: it brings its own HIP runtime, and the library must bind
    # to that one (loaded first, the library would bind to the system copy,
    # and torch's streams would be foreign to it)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libitebd error {code}: {msg}")
        self.code = code


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a device (cuda/hip) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context bound to torch's current HIP stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        s = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = lib().tn_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            raise TNError(rc, "tn_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().tn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_nc=False):
        if rc < 0 or (rc == TN_NOT_CONVERGED and not allow_nc):
            raise TNError(rc, lib().tn_last_error(self._h).decode())
        return rc

    # -- 2D environment ----------------------------------------------------
    @staticmethod
    def _cell(cell):
        arr = (ctypes.c_int * len(cell))(*[int(c) for c in cell])
        return arr

    def ctmrg_iterate(self, Lx, Ly, sites, cell, C, T, max_iter, tol, precision="fp64",
                      n_polish=5):
        nsite, d, D = sites.shape[0], sites.shape[1], sites.shape[2]
        chi = C.shape[-1]
        it = ctypes.c_int(0)
        de = ctypes.c_double(0.0)
        rc = lib().ctmrg_iterate(self._h, Lx, Ly, D, d, nsite, _ptr(sites), self._cell(cell), chi,
                                 _ptr(C), _ptr(T), max_iter, tol, _PREC[precision], n_polish,
                                 ctypes.byref(it), ctypes.byref(de))
        self._check(rc, allow_nc=True)
        return rc, it.value, de.value

    def ctmrg_moves(self, Lx, Ly, sites, cell, C, T, n_moves, first_dir=0, precision="fp64"):
        nsite, d, D = sites.shape[0], sites.shape[1], sites.shape[2]
        chi = C.shape[-1]
        rc = lib().ctmrg_moves(self._h, Lx, Ly, D, d, nsite, _ptr(sites), self._cell(cell), chi,
                               _ptr(C), _ptr(T), n_moves, first_dir, _PREC[precision])
        self._check(rc)

    def ipeps_rdms(self, Lx, Ly, sites, cell, C, T):
        import torch
        nsite, d, D = sites.shape[0], sites.shape[1], sites.shape[2]
        chi = C.shape[-1]
        npos = Lx * Ly
        dev = sites.device
        r1 = torch.empty((npos, d, d), dtype=torch.float64, device=dev)
        rh = torch.empty((npos, d * d, d * d), dtype=torch.float64, device=dev)
        rv = torch.empty((npos, d * d, d * d), dtype=torch.float64, device=dev)
        rc = lib().ipeps_rdms(self._h, Lx, Ly, D, d, nsite, _ptr(sites), self._cell(cell), chi,
                              _ptr(C), _ptr(T), _ptr(r1), _ptr(rh), _ptr(rv))
        self._check(rc)
        return r1, rh, rv

    def ipeps_energy(self, Lx, Ly, sites, cell, C, T, J, h):
        nsite, d, D = sites.shape[0], sites.shape[1], sites.shape[2]
        chi = C.shape[-1]
        e = ctypes.c_double(0.0)
        rc = lib().ipeps_energy(self._h, Lx, Ly, D, d, nsite, _ptr(sites), self._cell(cell), chi,
                                _ptr(C), _ptr(T), J, h, ctypes.byref(e))
        self._check(rc)
        return e.value

    def energy_grad(self, A, C0, T0, J, h, n_iter=20, ckpt_every=5, precision="fp64",
                    broadening=1e-12):
        """E(A) after n_iter CTMRG iterations of the single-site cell from
        (C0, T0), and dE/dA (same shape as A, device)."""
        import torch
        d, D = A.shape[0], A.shape[1]
        chi = C0.shape[-1]
        g = torch.empty_like(A)
        e = ctypes.c_double(0.0)
        rc = lib().energy_grad(self._h, D, d, J, h, _ptr(A), chi, _ptr(C0), _ptr(T0), n_iter,
                               ckpt_every, _PREC[precision], broadening, ctypes.byref(e), _ptr(g))
        self._check(rc)
        return e.value, g

    # -- full update -----------------------------------------------------------
    def cell_links(self, Lx, Ly, nsite, cell):
        return cell_links(Lx, Ly, nsite, cell)

    def ipeps_gate(self, A, J, h, dt):
        import torch
        nsite, d, D = A.shape[0], A.shape[1], A.shape[2]
        Th = torch.empty((nsite, d) + (2 * D,) * 4, dtype=torch.float64, device=A.device)
        self._check(lib().ipeps_gate(self._h, nsite, D, d, J, h, dt, _ptr(A), _ptr(Th)))
        return Th

    def ipeps_truncate(self, Lx, Ly, cell, Theta, P, Q):
        import torch
        nsite, d, Din = Theta.shape[0], Theta.shape[1], Theta.shape[2]
        Dout = P.shape[2]
        out = torch.empty((nsite, d) + (Dout,) * 4, dtype=torch.float64, device=Theta.device)
        self._check(lib().ipeps_truncate(self._h, Lx, Ly, nsite, self._cell(cell), d, Din, Dout,
                                         _ptr(Theta), _ptr(P), _ptr(Q), _ptr(out)))
        return out

    def ipeps_canonicalize(self, Lx, Ly, cell, A, D_keep=None, tol=1e-14, max_iter=1000,
                           a_out=True):
        """Returns (A1 or None, lambdas, P, Q, iters, rc)."""
        import torch
        nsite, d, D = A.shape[0], A.shape[1], A.shape[2]
        Dk = D if D_keep is None else D_keep
        nl = len(self.cell_links(Lx, Ly, nsite, cell))
        dev = A.device
        A1 = torch.empty_like(A) if (a_out and Dk == D) else None
        lam = torch.empty((nl, D), dtype=torch.float64, device=dev)
        P = torch.empty((nl, D, Dk), dtype=torch.float64, device=dev)
        Q = torch.empty((nl, Dk, D), dtype=torch.float64, device=dev)
        it = ctypes.c_int(0)
        rc = lib().ipeps_canonicalize(self._h, Lx, Ly, nsite, self._cell(cell), d, D, Dk, _ptr(A),
                                      _ptr(A1) if A1 is not None else None, _ptr(lam), _ptr(P),
                                      _ptr(Q), tol, max_iter, ctypes.byref(it))
        self._check(rc, allow_nc=True)
        return A1, lam, P, Q, it.value, rc

    def gauge_fix(self, Lx, Ly, cell, a_ref, a_new, U, tol=1e-12, max_iter=1000):
        """U (device [nlink][D][D]) is updated in place; returns (F, iters, rc)."""
        nsite, d, D = a_ref.shape[0], a_ref.shape[1], a_ref.shape[2]
        F = ctypes.c_double(0)
        it = ctypes.c_int(0)
        rc = lib().gauge_fix(self._h, TN_GAUGE_2D, Lx, Ly, nsite, self._cell(cell), d, D,
                             _ptr(a_ref), _ptr(a_new), _ptr(U), tol, max_iter, ctypes.byref(F),
                             ctypes.byref(it))
        self._check(rc, allow_nc=True)
        return F.value, it.value, rc

    def gauge_fix_1d(self, a_ref, a_new, U, method="iterative", tol=1e-12, max_iter=1000):
        """Two-site iMPS gauge fix (device [2][chi][d][chi] A forms); U
        (device [2][chi][chi]) is the start (iterative) and the result;
        returns (F, iters, rc)."""
        chi, d = a_ref.shape[1], a_ref.shape[2]
        kind = {"iterative": TN_GAUGE_1D, "direct": TN_GAUGE_1D_DIRECT}[method]
        F = ctypes.c_double(0)
        it = ctypes.c_int(0)
        rc = lib().gauge_fix(self._h, kind, 0, 0, 0, None, d, chi, _ptr(a_ref), _ptr(a_new),
                             _ptr(U), tol, max_iter, ctypes.byref(F), ctypes.byref(it))
        self._check(rc, allow_nc=True)
        return F.value, it.value, rc

    def bond_env_truncate(self, Lx, Ly, cell, Theta, C, T, Psu, Qsu, P, Q, max_passes=50,
                          max_sweeps=1, tol=1e-12):
        """P, Q (device, per link) are updated in place from their start;
        the environment bond is the column count of Psu.  Returns
        (f, <Psi_g|Psi_g>, passes, sweeps)."""
        nsite, d, Dk = Theta.shape[0], Theta.shape[1], Theta.shape[2]
        D, De = P.shape[2], Psu.shape[2]
        chi = C.shape[-1]
        cost = (ctypes.c_double * 2)()
        npass, sw = ctypes.c_int(0), ctypes.c_int(0)
        rc = lib().bond_env_truncate(self._h, Lx, Ly, nsite, self._cell(cell), d, D, Dk, De,
                                     _ptr(Theta), chi, _ptr(C), _ptr(T), _ptr(Psu), _ptr(Qsu),
                                     _ptr(P), _ptr(Q), max_passes, max_sweeps, tol, cost,
                                     ctypes.byref(npass), ctypes.byref(sw))
        self._check(rc)
        return cost[0], cost[1], npass.value, sw.value

    def bond_environment(self, Lx, Ly, cell, Theta, C, T, Psu, Qsu, P, Q, slot):
        """(N, M) of one slot of the truncation block (device)."""
        import torch
        nsite, d, Dk = Theta.shape[0], Theta.shape[1], Theta.shape[2]
        D, De = P.shape[2], Psu.shape[2]
        chi = C.shape[-1]
        N = torch.empty((Dk,) * 4, dtype=torch.float64, device=Theta.device)
        M = torch.empty((Dk,) * 4, dtype=torch.float64, device=Theta.device)
        self._check(lib().bond_environment(self._h, Lx, Ly, nsite, self._cell(cell), d, D, Dk, De,
                                           _ptr(Theta), chi, _ptr(C), _ptr(T), _ptr(Psu),
                                           _ptr(Qsu), _ptr(P), _ptr(Q), slot, _ptr(N), _ptr(M)))
        return N, M

    def fu_gauge_start(self, P, Q, Pc, Qc, kappa=2):
        import torch
        nl, Dk, D = P.shape
        U0 = torch.empty((nl, D, D), dtype=torch.float64, device=P.device)
        self._check(lib().fu_gauge_start(self._h, nl, Dk, D, kappa, _ptr(P), _ptr(Q), _ptr(Pc),
                                         _ptr(Qc), _ptr(U0)))
        return U0

    def fu_renormalized_gate(self, P, Q, Pc, Qc, U):
        import torch
        nl, Dk, D = P.shape
        Rf = torch.empty_like(P)
        Lf = torch.empty_like(Q)
        self._check(lib().fu_renormalized_gate(self._h, nl, Dk, D, _ptr(P), _ptr(Q), _ptr(Pc),
                                               _ptr(Qc), _ptr(U), _ptr(Rf), _ptr(Lf)))
        return Rf, Lf

    # -- 1D ------------------------------------------------------------------
    def tm_fixed_point(self, kets, bras, tol=1e-14, max_iter=200000, vl=None, vr=None):
        import torch
        ns, chi, d, _ = kets.shape
        warm = vl is not None
        if vl is None:
            vl = torch.empty((chi, chi), dtype=torch.float64, device=kets.device)
            vr = torch.empty((chi, chi), dtype=torch.float64, device=kets.device)
        eta = ctypes.c_double(0)
        it = ctypes.c_int(0)
        rc = lib().tm_fixed_point(self._h, ns, chi, d, _ptr(kets), _ptr(bras), _ptr(vl), _ptr(vr),
                                  ctypes.byref(eta), tol, max_iter, ctypes.byref(it), int(warm))
        self._check(rc, allow_nc=True)
        return vl, vr, eta.value, it.value, rc

    def tm_fixed_point_noalloc(self, kets, bras, vl, vr, tol=1e-14, max_iter=200000,
                               warm=False):
        """tm_fixed_point on the library's fixed scratch: vl, vr (device,
        [chi][chi]) are outputs, and with ``warm`` also the start."""
        ns, chi, d, _ = kets.shape
        eta = ctypes.c_double(0)
        it = ctypes.c_int(0)
        rc = lib().tm_fixed_point_noalloc(self._h, ns, chi, d, _ptr(kets), _ptr(bras), _ptr(vl),
                                          _ptr(vr), ctypes.byref(eta), tol, max_iter,
                                          ctypes.byref(it), int(warm))
        self._check(rc, allow_nc=True)
        return eta.value, it.value, rc

    def env1d(self, chi, d=2):
        import torch
        n = lib().tn_env1d_size(chi, d)
        return torch.zeros(n, dtype=torch.float64, device="cuda")

    def itebd_step(self, A, J, h, dt, env, mode=0, tol=1e-13, energy=False, lam=None):
        chi, d = A.shape[1], A.shape[2]
        err = ctypes.c_double(0)
        e = ctypes.c_double(0)
        rc = lib().itebd_step(self._h, chi, d, _ptr(A), J, h, dt, mode, _ptr(env),
                              _ptr(lam) if lam is not None else None, tol, ctypes.byref(err),
                              ctypes.byref(e) if energy else None)
        self._check(rc, allow_nc=True)
        return err.value, (e.value if energy else None), rc

    def ising2d_tm_step(self, A, beta, env, mode=0, tol=1e-13, lnz=False, lam=None):
        """One power-method step on the row transfer matrix of the classical
        2D Ising model; returns (trunc_err, ln Z per site or None, rc)."""
        chi = A.shape[1]
        err = ctypes.c_double(0)
        z = ctypes.c_double(0)
        rc = lib().ising2d_tm_step(self._h, chi, _ptr(A), beta, mode, _ptr(env),
                                   _ptr(lam) if lam is not None else None, tol,
                                   ctypes.byref(err), ctypes.byref(z) if lnz else None)
        self._check(rc, allow_nc=True)
        return err.value, (z.value if lnz else None), rc

    def svd(self, A):
        """Batched small SVD of device matrices A [batch][m][n] -> U, S, V."""
        import torch
        b, m, n = A.shape
        U = torch.empty((b, m, n), dtype=torch.float64, device=A.device)
        S = torch.empty((b, n), dtype=torch.float64, device=A.device)
        V = torch.empty((b, n, n), dtype=torch.float64, device=A.device)
        self._check(lib().tn_svd(self._h, b, m, n, _ptr(A), _ptr(U), _ptr(S), _ptr(V)))
        return U, S, V

    def cholesky_inv(self, G, shift_rel=0.0):
        """Batched Cholesky of device G [batch][k][k] -> (R, Rinv, info)."""
        import torch
        b, k, _ = G.shape
        R = torch.empty_like(G)
        Ri = torch.empty_like(G)
        info = (ctypes.c_int * b)()
        self._check(lib().tn_cholesky_inv(self._h, b, k, _ptr(G), shift_rel, _ptr(R), _ptr(Ri),
                                          info))
        return R, Ri, list(info)

    def clear_cache(self):
        self._check(lib().tn_clear_cache(self._h))

    def prof_enable(self, on=True):
        self._check(lib().tn_prof_enable(self._h, int(on)))

    def prof_read(self):
        ms, fl = ctypes.c_double(0), ctypes.c_double(0)
        nl = ctypes.c_longlong(0)
        cnt = (ctypes.c_longlong * 7)()
        self._check(lib().tn_prof_read(self._h, ctypes.byref(ms), ctypes.byref(fl),
                                       ctypes.byref(nl), cnt))
        return dict(gemm_ms=ms.value, gemm_flops=fl.value, gemm_launches=nl.value,
                    moves=cnt[0], svd_calls=cnt[1], svd_iters=cnt[2], svd_unconverged=cnt[3],
                    svd_explicit=cnt[4], jacobi_sweeps=cnt[5], gemm_bytes=cnt[6])

    def gemm(self, A, B, C, ta=False, tb=False, alpha=1.0, beta=0.0, precision="fp64"):
        M = A.shape[1] if ta else A.shape[0]
        K = A.shape[0] if ta else A.shape[1]
        N = B.shape[0] if tb else B.shape[1]
        rc = lib().tn_gemm(self._h, M, N, K, _ptr(A), A.shape[1], int(ta), _ptr(B), B.shape[1],
                           int(tb), _ptr(C), C.shape[1], alpha, beta, _PREC[precision])
        self._check(rc)


def _energy_grad_function():
    import torch

    class EnergyGrad(torch.autograd.Function):
        """E(A) of ``Context.energy_grad`` as a differentiable function of
        the site tensor A (the environment (C0, T0) is a constant)."""

        @staticmethod
        def forward(fctx, A, C0, T0, ctx, J, h, n_iter, ckpt_every, precision, broadening):
            e, g = ctx.energy_grad(A.detach().contiguous(), C0, T0, J, h, n_iter, ckpt_every,
                                   precision, broadening)
            fctx.save_for_backward(g)
            return torch.tensor(e, dtype=A.dtype, device=A.device)

        @staticmethod
        def backward(fctx, grad_out):
            (g,) = fctx.saved_tensors
            return (grad_out * g,) + (None,) * 9

    return EnergyGrad


def energy(A, C0, T0, ctx, J=1.0, h=3.0, n_iter=20, ckpt_every=5, precision="fp64",
           broadening=1e-12):
    """Differentiable E(A) (torch.autograd): the forward call computes the
    gradient with the hand-written reverse pass and keeps it for backward."""
    global _EnergyGrad
    if _EnergyGrad is None:
        _EnergyGrad = _energy_grad_function()
    return _EnergyGrad.apply(A, C0, T0, ctx, J, h, n_iter, ckpt_every, precision, broadening)


_EnergyGrad = None


def cell_links(Lx, Ly, nsite, cell):
    """Link enumeration of a unit cell (host-only call into the library):
    list of (site1, leg1, site2, leg2), legs numbered 1 l, 2 r, 3 d, 4 u."""
    nl = ctypes.c_int(0)
    buf = (ctypes.c_int * 256)()
    arr = (ctypes.c_int * len(cell))(*[int(c) for c in cell])
    rc = lib().ipeps_cell_links(None, Lx, Ly, nsite, arr, ctypes.byref(nl), buf)
    if rc != 0:
        raise TNError(rc, "invalid unit cell")
    return [tuple(buf[4 * b:4 * b + 4]) for b in range(nl.value)]
