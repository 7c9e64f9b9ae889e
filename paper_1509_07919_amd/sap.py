"""Python binding of libsap (the C ABI in include/sap.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory and the current stream.  If libsap.so has not
been built, importing works but every call raises ``SapLibraryMissing``:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libsap.so")

SAP_OK = 0
SAP_NOT_CONVERGED = 1
SAP_ERR_INVALID = -1
SAP_ERR_NOSPACE = -2
SAP_ERR_HIP = -3
SAP_ERR_BREAKDOWN = -4
SAP_ERR_SINGULAR = -5
SAP_ERR_STATE = -6

SAP_DECOUPLED = 0
SAP_COUPLED = 1
SAP_PREC_FP64 = 0
SAP_PREC_FP32 = 1

EXPORTED = ("sap_workspace_bytes", "sap_create", "sap_factor", "sap_solve",
            "sap_solve_adjoint", "sap_band_grad", "sap_handle_status", "sap_spmv",
            "sap_precond_apply", "sap_get_tips", "sap_profile", "sap_kernel_time",
            "sap_destroy", "sap_last_error", "sap_solve_noalloc", "sap_solve_cg", "sap_solve_batch",
            "sap_get_factor_rows", "sap_tips_phase_times", "sap_sparse_create",
            "sap_sparse_info", "sap_sparse_times", "sap_sparse_assemble", "sap_solve_sparse",
            "sap_sparse_destroy")

KERNELS = ("norm", "lu", "tips", "sweep", "corr", "spmv", "krylov", "xfer")


class SapLibraryMissing(RuntimeError):
    pass


class SapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libsap error %d: %s" % (code, msg))
        self.code = code


class sap_options(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_int32), ("p", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("factor_prec", ctypes.c_int32),
                ("boost_eps", ctypes.c_double), ("adjoint", ctypes.c_int32),
                ("sweep_chunks", ctypes.c_int32), ("nrhs", ctypes.c_int32)]


class sap_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_double), ("rel_resid_true", ctypes.c_double),
                ("rel_resid_precond", ctypes.c_double), ("converged", ctypes.c_int32),
                ("n_boosted", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("n_apply", ctypes.c_int32), ("t_factor_ms", ctypes.c_float),
                ("t_lu_ms", ctypes.c_float), ("t_tips_ms", ctypes.c_float),
                ("t_solve_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsap.so (built in-tree by build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SapLibraryMissing("libsap.so not found at %s; run "
                                "`python paper_1509_07919_amd/build.py`" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.sap_workspace_bytes.argtypes = [P(sap_options), P(ctypes.c_size_t)]
    lib.sap_create.argtypes = [P(sap_options), vp, ctypes.c_size_t, P(vp)]
    lib.sap_factor.argtypes = [vp, vp, vp]
    lib.sap_solve.argtypes = [vp, vp, vp, dbl, i32, vp, P(sap_stats)]
    lib.sap_solve_adjoint.argtypes = [vp, vp, vp, dbl, i32, vp, P(sap_stats)]
    lib.sap_solve_cg.argtypes = [vp, vp, vp, dbl, i32, vp, P(sap_stats)]
    lib.sap_solve_batch.argtypes = [vp, vp, vp, i32, dbl, i32, vp, P(sap_stats)]
    lib.sap_band_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.sap_handle_status.argtypes = [vp, vp, P(i32)]
    lib.sap_spmv.argtypes = [vp, vp, vp, i32, vp]
    lib.sap_precond_apply.argtypes = [vp, vp, vp, i32, vp]
    lib.sap_get_tips.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.sap_get_factor_rows.argtypes = [vp, i32, i64, i64, vp, vp]
    lib.sap_tips_phase_times.argtypes = [vp, vp, vp]
    lib.sap_sparse_create.argtypes = [i64, vp, vp, vp, i32, i32, dbl, P(vp)]
    lib.sap_sparse_times.argtypes = [vp, P(dbl), P(dbl), P(dbl)]
    lib.sap_sparse_info.argtypes = [vp, P(i32), P(i32), vp, vp, vp, vp]
    lib.sap_sparse_assemble.argtypes = [vp, vp, vp, vp]
    lib.sap_solve_sparse.argtypes = [vp, vp, vp, vp, dbl, i32, vp, P(sap_stats)]
    lib.sap_sparse_destroy.argtypes = [vp]
    lib.sap_profile.argtypes = [vp, i32]
    lib.sap_kernel_time.argtypes = [vp, i32, P(dbl), P(i64)]
    lib.sap_destroy.argtypes = [vp]
    lib.sap_solve_noalloc.argtypes = [P(sap_options), vp, vp, vp, dbl, i32, vp, P(sap_stats)]
    lib.sap_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "sap_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, allow=(SAP_OK,)) -> int:
    if rc in allow:
        return rc
    raise SapError(rc, load_library().sap_last_error().decode())


def _dptr(t: torch.Tensor, n: int, name: str) -> ctypes.c_void_p:
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous float64 CUDA tensor of %d elements" % (name, n))
    return ctypes.c_void_p(t.data_ptr())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_options(n: int, k: int, p: int, mode: str = "coupled", factor_prec: str = "fp64",
                 boost_eps: float = 0.0, adjoint: bool = False,
                 sweep_chunks: int = 0, nrhs: int = 0) -> sap_options:
    m = {"decoupled": SAP_DECOUPLED, "coupled": SAP_COUPLED}[mode]
    f = {"fp64": SAP_PREC_FP64, "fp32": SAP_PREC_FP32}[factor_prec]
    return sap_options(n=n, k=k, p=p, mode=m, factor_prec=f, boost_eps=boost_eps,
                       adjoint=1 if adjoint else 0, sweep_chunks=sweep_chunks, nrhs=nrhs)


# ------------------------------------------------------------ thin wrappers

def sap_workspace_bytes(opt: sap_options) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().sap_workspace_bytes(ctypes.byref(opt), ctypes.byref(out)))
    return out.value


@dataclass
class SapStats:
    iters: float
    rel_resid_true: float
    rel_resid_precond: float
    converged: bool
    n_boosted: int
    restarts: int
    n_apply: int
    t_factor_ms: float
    t_lu_ms: float
    t_tips_ms: float
    t_solve_ms: float
    status: int = SAP_OK


class SapSolver:
    """One handle: workspace (a torch uint8 tensor), factorization, solves."""

    def __init__(self, n: int, k: int, p: int, mode: str = "coupled",
                 factor_prec: str = "fp64", boost_eps: float = 0.0, adjoint: bool = False,
                 device=None, sweep_chunks: int = 0, nrhs: int = 0):
        lib = load_library()
        self.opt = make_options(n, k, p, mode, factor_prec, boost_eps, adjoint, sweep_chunks,
                                nrhs)
        self.nrhs = max(1, nrhs)
        self.n, self.k, self.p = n, k, p
        nbytes = sap_workspace_bytes(self.opt)
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p(0)
        _check(lib.sap_create(ctypes.byref(self.opt), ctypes.c_void_p(self.workspace.data_ptr()),
                              nbytes, ctypes.byref(h)))
        self.handle = h
        self.a_band = None
        self.generation = 0          # bumped by every factor(): which A the factors belong to

    # -- life cycle --
    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().sap_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the three entry points of the method --
    def factor(self, a_band: torch.Tensor):
        """sap_factor: keeps a reference to a_band (the library borrows it)."""
        _check(load_library().sap_factor(self.handle,
                                         _dptr(a_band, (2 * self.k + 1) * self.n, "a_band"),
                                         _stream()))
        self.a_band = a_band
        self.generation += 1

    def _solve(self, fn, b, x, tol, maxit, raise_nc):
        st = sap_stats()
        rc = fn(self.handle, _dptr(b, self.n, "rhs"), _dptr(x, self.n, "x"), float(tol),
                int(maxit), _stream(), ctypes.byref(st))
        if rc not in (SAP_OK, SAP_NOT_CONVERGED) or (rc == SAP_NOT_CONVERGED and raise_nc):
            _check(rc)
        return SapStats(**st.as_dict(), status=rc)

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
              maxit: int = 200, raise_nc: bool = False):
        x = torch.empty_like(b) if x is None else x
        return x, self._solve(load_library().sap_solve, b, x, tol, maxit, raise_nc)

    def solve_batch(self, B: torch.Tensor, X: torch.Tensor | None = None, tol: float = 1e-10,
                    maxit: int = 200, raise_nc: bool = False):
        """sap_solve_batch: B is (m, N) (row c = right-hand side c, contiguous),
        i.e. the N x m column-major block of the C ABI.  Returns (X, [SapStats])."""
        if B.dim() != 2 or B.shape[1] != self.n:
            raise ValueError("B must be (m, N)")
        m = B.shape[0]
        X = torch.empty_like(B) if X is None else X
        sts = (sap_stats * m)()
        rc = load_library().sap_solve_batch(self.handle, _dptr(B, m * self.n, "B"),
                                            _dptr(X, m * self.n, "X"), m, float(tol), int(maxit),
                                            _stream(), sts)
        if rc not in (SAP_OK, SAP_NOT_CONVERGED) or (rc == SAP_NOT_CONVERGED and raise_nc):
            _check(rc)
        return X, [SapStats(**st.as_dict(), status=rc) for st in sts]

    def solve_sparse(self, sp: "SapSparse", b: torch.Tensor, x: torch.Tensor | None = None,
                     tol: float = 1e-10, maxit: int = 200, raise_nc: bool = False):
        """sap_solve_sparse: A x = b through the plan's reordering, with this
        handle's preconditioner (factored on sp.assemble's band)."""
        x = torch.empty_like(b) if x is None else x
        st = sap_stats()
        rc = load_library().sap_solve_sparse(self.handle, sp.plan, _dptr(b, self.n, "b"),
                                             _dptr(x, self.n, "x"), float(tol), int(maxit),
                                             _stream(), ctypes.byref(st))
        if rc not in (SAP_OK, SAP_NOT_CONVERGED) or (rc == SAP_NOT_CONVERGED and raise_nc):
            _check(rc)
        return x, SapStats(**st.as_dict(), status=rc)

    def solve_cg(self, b: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
                 maxit: int = 500, raise_nc: bool = False):
        """sap_solve_cg: preconditioned conjugate gradient for SPD A."""
        x = torch.empty_like(b) if x is None else x
        return x, self._solve(load_library().sap_solve_cg, b, x, tol, maxit, raise_nc)

    def solve_adjoint(self, g: torch.Tensor, lam: torch.Tensor | None = None,
                      tol: float = 1e-10, maxit: int = 200, raise_nc: bool = False):
        lam = torch.empty_like(g) if lam is None else lam
        return lam, self._solve(load_library().sap_solve_adjoint, g, lam, tol, maxit, raise_nc)

    # -- helpers --
    def band_grad(self, lam: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None):
        w = (2 * self.k + 1) * self.n
        out = torch.empty(w, dtype=torch.float64, device=lam.device) if out is None else out
        _check(load_library().sap_band_grad(self.handle, _dptr(lam, self.n, "lambda"),
                                            _dptr(x, self.n, "x"), _dptr(out, w, "g_band"),
                                            _stream()))
        return out

    def status(self):
        nb = ctypes.c_int32(0)
        rc = load_library().sap_handle_status(self.handle, _stream(), ctypes.byref(nb))
        return rc, nb.value

    def spmv(self, v: torch.Tensor, trans: bool = False, out: torch.Tensor | None = None):
        out = torch.empty_like(v) if out is None else out
        _check(load_library().sap_spmv(self.handle, _dptr(v, self.n, "v"),
                                       _dptr(out, self.n, "y"), int(trans), _stream()))
        return out

    def precond(self, r: torch.Tensor, trans: bool = False, out: torch.Tensor | None = None):
        out = torch.empty_like(r) if out is None else out
        _check(load_library().sap_precond_apply(self.handle, _dptr(r, self.n, "r"),
                                                _dptr(out, self.n, "z"), int(trans), _stream()))
        return out

    def profile(self, enable: bool):
        """Bracket every kernel launch with HIP events (resets the counters)."""
        _check(load_library().sap_profile(self.handle, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """{kernel class: (total device ms, launches)} since profile(True)."""
        out = {}
        for i, name in enumerate(KERNELS):
            ms, cnt = ctypes.c_double(0), ctypes.c_int64(0)
            _check(load_library().sap_kernel_time(self.handle, i, ctypes.byref(ms),
                                                  ctypes.byref(cnt)))
            out[name] = (ms.value, cnt.value)
        return out

    def tips_phase_times(self) -> dict:
        """T_BC, T_SPK, T_LUrdcd (ms) of the last factorization (Sec. 3.4)."""
        ms = (ctypes.c_double * 3)()
        _check(load_library().sap_tips_phase_times(self.handle, ms, _stream()))
        return {"t_bc_ms": ms[0], "t_spk_ms": ms[1], "t_lurdcd_ms": ms[2]}

    def factor_rows(self, which: str, j0: int = 0, count: int | None = None):
        """Rows of a factor coefficient array ("Lc", "Uc", "Lr", "Ur") as a
        (count, K+1) float64 array (sap_get_factor_rows)."""
        import numpy as np
        w = {"Lc": 0, "Uc": 1, "Lr": 2, "Ur": 3}[which]
        count = self.n - j0 if count is None else count
        out = np.zeros((count, self.k + 1))
        _check(load_library().sap_get_factor_rows(self.handle, w, j0, count,
                                                  out.ctypes.data_as(ctypes.c_void_p), _stream()))
        return out

    def tips(self, i: int):
        import numpy as np
        kk = self.k * self.k
        v, w, rb = (np.zeros(kk) for _ in range(3))
        _check(load_library().sap_get_tips(
            self.handle, i, v.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
            rb.ctypes.data_as(ctypes.c_void_p), _stream()))
        return v.reshape(self.k, self.k), w.reshape(self.k, self.k), rb.reshape(self.k, self.k)


class SapSparse:
    """Sparse front end (sap_sparse_*): host CSR in, reorderings on the host,
    the band and the reordered values built on the GPU."""

    def __init__(self, n: int, rowptr, colidx, vals, db: bool = True, cm: bool = True,
                 drop_frac: float = 0.0):
        import numpy as np
        lib = load_library()
        self.n = n
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._colidx = np.ascontiguousarray(colidx, dtype=np.int32)
        self._vals = np.ascontiguousarray(vals, dtype=np.float64)
        h = ctypes.c_void_p(0)
        _check(lib.sap_sparse_create(n, self._rowptr.ctypes.data_as(ctypes.c_void_p),
                                     self._colidx.ctypes.data_as(ctypes.c_void_p),
                                     self._vals.ctypes.data_as(ctypes.c_void_p), int(db), int(cm),
                                     float(drop_frac), ctypes.byref(h)))
        self.plan = h
        self.k = self.info()["k"]

    def info(self) -> dict:
        import numpy as np
        k, kf = ctypes.c_int32(0), ctypes.c_int32(0)
        nr, nc = np.zeros(self.n, dtype=np.int32), np.zeros(self.n, dtype=np.int32)
        rs, cs = np.zeros(self.n), np.zeros(self.n)
        vp = ctypes.c_void_p
        _check(load_library().sap_sparse_info(self.plan, ctypes.byref(k), ctypes.byref(kf),
                                              nr.ctypes.data_as(vp), nc.ctypes.data_as(vp),
                                              rs.ctypes.data_as(vp), cs.ctypes.data_as(vp)))
        return {"k": k.value, "k_full": kf.value, "new_row": nr, "new_col": nc,
                "row_scale": rs, "col_scale": cs}

    def times(self) -> dict:
        """Host ms of the analysis stages: matching and scaling, Cuthill-McKee,
        the reordered structure with the drop-off."""
        t = [ctypes.c_double(0) for _ in range(3)]
        _check(load_library().sap_sparse_times(self.plan, *[ctypes.byref(v) for v in t]))
        return {"t_db_ms": t[0].value, "t_cm_ms": t[1].value, "t_drop_ms": t[2].value}

    def assemble(self, vals: torch.Tensor, band: torch.Tensor | None = None) -> torch.Tensor:
        """The band of A_hat (device) from A's values (device, CSR order)."""
        w = (2 * self.k + 1) * self.n
        band = torch.empty(w, dtype=torch.float64, device=vals.device) if band is None else band
        _check(load_library().sap_sparse_assemble(self.plan, _dptr(vals, vals.numel(), "vals"),
                                                  _dptr(band, w, "band"), _stream()))
        return band

    def close(self):
        if getattr(self, "plan", None) and self.plan.value:
            load_library().sap_sparse_destroy(self.plan)
            self.plan = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NOALLOC_SCRATCH_BYTES = 64 << 20     # SAP_NOALLOC_SCRATCH_BYTES


def solve_noalloc(a_band: torch.Tensor, b: torch.Tensor, n: int, k: int, p: int,
                  mode: str = "coupled", factor_prec: str = "fp64", boost_eps: float = 0.0,
                  sweep_chunks: int = 0, x: torch.Tensor | None = None, tol: float = 1e-10,
                  maxit: int = 200):
    """sap_solve_noalloc: factor and solve in the library's static scratch
    (no workspace, handle or allocation on the library side).  Returns
    (x, SapStats); raises SapError on errors other than SAP_NOT_CONVERGED."""
    opt = make_options(n, k, p, mode, factor_prec, boost_eps, False, sweep_chunks)
    x = torch.empty_like(b) if x is None else x
    st = sap_stats()
    rc = load_library().sap_solve_noalloc(
        ctypes.byref(opt), _dptr(a_band, (2 * k + 1) * n, "a_band"), _dptr(b, n, "b"),
        _dptr(x, n, "x"), float(tol), int(maxit), _stream(), ctypes.byref(st))
    if rc not in (SAP_OK, SAP_NOT_CONVERGED):
        _check(rc)
    return x, SapStats(**st.as_dict(), status=rc)


class SapSolve(torch.autograd.Function):
    """x = A^{-1} b with A in band layout.  Backward: lambda = A^{-T} dL/dx by
    the adjoint solve on the same factors; dL/db = lambda and dL/dA_band =
    band(-lambda x^T).

    The band is saved for backward (autograd then rejects an in-place change
    to it).  If the solver has factored another matrix since this forward,
    backward factors the saved band again before the adjoint solve, so the
    gradient always belongs to the A of its own forward."""

    @staticmethod
    def forward(ctx, a_band, b, solver: SapSolver, tol: float = 1e-10, maxit: int = 200):
        solver.factor(a_band)
        x, st = solver.solve(b, tol=tol, maxit=maxit, raise_nc=True)
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        ctx.stats = st
        ctx.generation = solver.generation
        ctx.save_for_backward(a_band, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        a_band, x = ctx.saved_tensors
        if ctx.solver.generation != ctx.generation:
            ctx.solver.factor(a_band)
            ctx.generation = ctx.solver.generation
        lam, _ = ctx.solver.solve_adjoint(gx.contiguous(), tol=ctx.tol, maxit=ctx.maxit,
                                          raise_nc=True)
        ga = ctx.solver.band_grad(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return ga, gb, None, None, None


def sap_solve_autograd(a_band, b, solver: SapSolver, tol: float = 1e-10, maxit: int = 200):
    return SapSolve.apply(a_band, b, solver, tol, maxit)
