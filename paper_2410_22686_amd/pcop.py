"""Thin Python binding of the pcop C ABI (include/pcop.h).

Argument marshalling only: every numerical step runs in the HIP kernels of
libpcop.so.  PyTorch supplies device memory (the workspace and all vectors
are torch tensors on a ROCm device) and the stream.  Shapes and dtypes are
checked here before any pointer reaches the library, so that a kernel never
sees a buffer smaller than its grid assumes.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence, Union

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcop.so")

PCOP_OK, PCOP_ERR_INVALID_ARG, PCOP_ERR_UNSUPPORTED, PCOP_ERR_WORKSPACE, PCOP_ERR_DEVICE, PCOP_NOT_CONVERGED = range(6)
PCOP_FP64, PCOP_MIXED = 0, 1
PCOP_DST, PCOP_MG = 0, 1
PCOP_RIGHT, PCOP_LEFT, PCOP_FLEXIBLE = 0, 1, 2
PCOP_COEFF_ONE, PCOP_COEFF_HALFGRID = 0, 1
PCOP_PRECOND_EPS, PCOP_PRECOND_IDEAL = 0, 1
PCOP_MASS_IDENTITY, PCOP_MASS_Q1 = 0, 1

EXPORTED = [
    "pcop_validate", "pcop_default_options", "pcop_workspace_size", "pcop_setup", "pcop_rhs",
    "pcop_kkt_apply", "pcop_precond_apply", "pcop_solve", "pcop_unpack", "pcop_pack_cotangent",
    "pcop_data_grad", "pcop_get_params", "pcop_destroy", "pcop_status_string", "pcop_last_error",
    "pcop_timing_enable", "pcop_timing_read", "pcop_get_kernels", "pcop_post_solve", "pcop_error_eh",
    "pcop_precond_apply_noalloc",
]


class PcopError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pcop status {status}: {msg}")
        self.status = status


class NotConverged(PcopError):
    pass


class c_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("nt", ctypes.c_int), ("T", ctypes.c_double),
                ("batch", ctypes.c_int), ("gamma", ctypes.POINTER(ctypes.c_double)), ("eps", ctypes.c_double),
                ("coeff_kind", ctypes.c_int), ("coeff", ctypes.POINTER(ctypes.c_double)), ("mass", ctypes.c_int)]


class c_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("spatial", ctypes.c_int), ("side", ctypes.c_int),
                ("restart", ctypes.c_int), ("maxit", ctypes.c_int), ("rtol", ctypes.c_double),
                ("graph", ctypes.c_int), ("graph_chunk", ctypes.c_int), ("reorth_tol", ctypes.c_double),
                ("time_cols", ctypes.c_int), ("dst_kernel", ctypes.c_int), ("tune", ctypes.c_int),
                ("precond", ctypes.c_int), ("kkt_jchunk", ctypes.c_int), ("krylov_blocks", ctypes.c_int),
                ("gs_update", ctypes.c_int), ("stream", ctypes.c_void_p), ("mg_smoother", ctypes.c_int)]


class c_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class c_kernel_choice(ctypes.Structure):
    _fields_ = [("time_cols", ctypes.c_int), ("dst_kernel", ctypes.c_int), ("kkt_jchunk", ctypes.c_int),
                ("krylov_blocks", ctypes.c_int), ("gs_update", ctypes.c_int), ("tuned_precond_ms", ctypes.c_double)]


class c_member_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("relres_est", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libpcop.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run paper_2410_22686_amd.build.build() first")
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    P, O = ctypes.POINTER(c_problem), ctypes.POINTER(c_options)
    sig = {
        "pcop_validate": (ip, [P, O]),
        "pcop_default_options": (None, [O]),
        "pcop_workspace_size": (ip, [P, O, ctypes.POINTER(ctypes.c_size_t)]),
        "pcop_setup": (ip, [ctypes.POINTER(vp), P, O, vp, ctypes.c_size_t]),
        "pcop_rhs": (ip, [vp, vp, vp, vp, vp]),
        "pcop_kkt_apply": (ip, [vp, vp, vp, ip]),
        "pcop_precond_apply": (ip, [vp, vp, vp]),
        "pcop_precond_apply_noalloc": (ip, [vp, vp, vp]),
        "pcop_solve": (ip, [vp, vp, vp, ip, ctypes.POINTER(c_member_info), dp]),
        "pcop_unpack": (ip, [vp, vp, vp, vp]),
        "pcop_pack_cotangent": (ip, [vp, vp, vp, vp]),
        "pcop_data_grad": (ip, [vp, vp, vp, vp, vp]),
        "pcop_get_params": (ip, [vp, dp, dp, dp]),
        "pcop_get_kernels": (ip, [vp, ctypes.POINTER(c_kernel_choice)]),
        "pcop_post_solve": (ip, [vp, vp, vp, vp, vp, vp, vp, dp]),
        "pcop_error_eh": (ip, [vp, vp, vp, vp, vp, vp, dp]),
        "pcop_destroy": (None, [vp]),
        "pcop_status_string": (ctypes.c_char_p, [ip]),
        "pcop_last_error": (ctypes.c_char_p, []),
        "pcop_timing_enable": (ip, [vp, ip]),
        "pcop_timing_read": (ip, [vp, ctypes.POINTER(c_kernel_stat), ip, ctypes.POINTER(ctypes.c_int), ip]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status == PCOP_OK:
        return
    lib = load_library()
    msg = lib.pcop_last_error().decode()
    if status == PCOP_NOT_CONVERGED:
        raise NotConverged(status, msg)
    raise PcopError(status, msg)


def halfgrid_samples(coeff: Callable, dim: int, nx: int):
    """a(x) sampled at x = k h/2, k = 1..2nx+1 per dimension (x1 fastest),
    the layout PCOP_COEFF_HALFGRID expects."""
    import numpy as np
    h = 1.0 / (nx + 1)
    x = np.arange(1, 2 * nx + 2) * (h / 2.0)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    coords = [np.ascontiguousarray(grids[dim - 1 - d]).reshape(-1) for d in range(dim)]
    return np.ascontiguousarray(coeff(*coords), dtype=np.float64)


_PREC = {"fp64": PCOP_FP64, "mixed": PCOP_MIXED}
_SPAT = {"dst": PCOP_DST, "mg": PCOP_MG}
_SIDE = {"right": PCOP_RIGHT, "left": PCOP_LEFT, "flexible": PCOP_FLEXIBLE}
_PRECOND = {"eps": PCOP_PRECOND_EPS, "ideal": PCOP_PRECOND_IDEAL}
_MASS = {"identity": PCOP_MASS_IDENTITY, "q1": PCOP_MASS_Q1}
_MG_SMOOTHER = {"rb": 0, "lex": 1, "sym": 2}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    relres_est: float
    relres_true: float


class Solver:
    """One pcop context: a batch of KKT systems sharing (dim, nx, nt, T, eps, a).

    Methods mirror the C entry points: ``rhs`` (pcop_rhs), ``kkt_apply``
    (pcop_kkt_apply), ``precond_apply`` (pcop_precond_apply), ``solve``
    (pcop_solve), ``unpack``, ``pack_cotangent``, ``data_grad``."""

    def __init__(self, dim: int, nx: int, nt: int, gamma: Union[float, Sequence[float]], T: float = 1.0,
                 eps: Optional[float] = None, coeff: Optional[Callable] = None, precision: str = "fp64",
                 spatial: str = "dst", side: str = "right", restart: int = 30, maxit: int = 300,
                 rtol: float = 1e-8, graph: bool = False, graph_chunk: int = 4, reorth_tol: float = 1e-8,
                 time_cols: int = 0, dst_kernel: int = 0, tune: bool = False, precond: str = "eps",
                 kkt_jchunk: int = 0, krylov_blocks: int = 0, gs_update: int = 0, mass: str = "identity",
                 device: Union[str, torch.device] = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 mg_smoother: str = "rb"):
        import numpy as np
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("pcop needs a ROCm GPU (torch.cuda.is_available() is False)")
        gam = [float(gamma)] if isinstance(gamma, (int, float)) else [float(v) for v in gamma]
        self.dim, self.nx, self.nt, self.T = int(dim), int(nx), int(nt), float(T)
        self.batch = len(gam)
        self.n, self.m = self.nt - 1, self.nx ** self.dim
        self.device = torch.device(device)
        self._gamma = (ctypes.c_double * self.batch)(*gam)
        self._coeff_np = None
        prob = c_problem()
        prob.dim, prob.nx, prob.nt, prob.T, prob.batch = self.dim, self.nx, self.nt, self.T, self.batch
        prob.gamma = ctypes.cast(self._gamma, ctypes.POINTER(ctypes.c_double))
        prob.eps = -1.0 if eps is None else float(eps)
        prob.mass = _MASS[mass]
        self.mass = mass
        if coeff is None:
            prob.coeff_kind, prob.coeff = PCOP_COEFF_ONE, None
        else:
            self._coeff_np = halfgrid_samples(coeff, self.dim, self.nx)
            prob.coeff_kind = PCOP_COEFF_HALFGRID
            prob.coeff = self._coeff_np.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        opts = c_options()
        self.lib.pcop_default_options(ctypes.byref(opts))
        opts.precision, opts.spatial, opts.side = _PREC[precision], _SPAT[spatial], _SIDE[side]
        opts.restart, opts.maxit, opts.rtol = int(restart), int(maxit), float(rtol)
        opts.graph, opts.graph_chunk, opts.reorth_tol = int(bool(graph)), int(graph_chunk), float(reorth_tol)
        opts.time_cols, opts.dst_kernel, opts.tune = int(time_cols), int(dst_kernel), int(bool(tune))
        opts.precond = _PRECOND[precond]
        opts.kkt_jchunk, opts.krylov_blocks, opts.gs_update = int(kkt_jchunk), int(krylov_blocks), int(gs_update)
        opts.mg_smoother = _MG_SMOOTHER[mg_smoother]
        self.stream = stream
        with torch.cuda.device(self.device):
            st = stream if stream is not None else torch.cuda.current_stream(self.device)
        opts.stream = ctypes.c_void_p(st.cuda_stream)
        self._torch_stream = st
        self.prob, self.opts = prob, opts
        self.maxit = int(maxit)
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.pcop_workspace_size(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        ctx = ctypes.c_void_p()
        _check(self._call(self.lib.pcop_setup, ctypes.byref(ctx), ctypes.byref(prob), ctypes.byref(opts),
                                   ctypes.c_void_p(aligned), ctypes.c_size_t(self.workspace_bytes)))
        self.ctx = ctx
        tau, eps_out = ctypes.c_double(), ctypes.c_double()
        alpha = (ctypes.c_double * self.batch)()
        _check(self.lib.pcop_get_params(ctx, ctypes.byref(tau), alpha, ctypes.byref(eps_out)))
        self.tau, self.eps, self.alpha = tau.value, eps_out.value, list(alpha)
        self.gamma = gam
        kc = c_kernel_choice()
        _check(self.lib.pcop_get_kernels(ctx, ctypes.byref(kc)))
        # kernel choices in effect: time_cols -P two-buffer / +P in place (Stockham),
        # +P 256 threads / -P 512 threads (chirp-z), 0 ideal preconditioner;
        # dst_kernel 1 register / 2 LDS-staged / 3 wide columns / 4 half-length strided / 5 half-length on
        # every axis / 0 multigrid
        self.kernels = {"time_cols": kc.time_cols, "dst_kernel": kc.dst_kernel, "kkt_jchunk": kc.kkt_jchunk,
                        "krylov_blocks": kc.krylov_blocks, "gs_update": kc.gs_update, "tuned_ms": kc.tuned_precond_ms}

    # ------------------------------------------------------------------
    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.pcop_destroy(ctx)
            self.ctx = None

    @property
    def vec_shape(self):
        return (self.batch, 2, self.n, self.m)

    @property
    def field_shape(self):
        return (self.batch, self.n, self.m)

    def _vec(self, t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
        shape = self.vec_shape if shape is None else shape
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if t.device != self.device and not (t.device.type == "cuda" and self.device.type == "cuda"
                                             and (self.device.index is None or t.device.index == self.device.index)):
            raise ValueError(f"{name} must live on {self.device}")
        if t.numel() != math.prod(shape):
            raise ValueError(f"{name} must have {math.prod(shape)} elements (shape {shape}), got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.data_ptr() % 16:
            raise ValueError(f"{name} must be 16-byte aligned")
        return t

    def new_vector(self) -> torch.Tensor:
        return torch.zeros(self.vec_shape, dtype=torch.float64, device=self.device)

    def _call(self, fn, *args):
        """Run one enqueuing library call on the solver's stream in order with
        the caller's current stream.  Tensors are allocated (and zero-filled)
        on the current stream, so the solver's stream first waits for it; the
        current stream then waits for the solver's stream, so results are
        visible there and torch's allocator never recycles memory the library
        still uses."""
        cur = torch.cuda.current_stream(self.device)
        st = self._torch_stream
        if st != cur:
            st.wait_stream(cur)
        try:
            return fn(*args)
        finally:
            if st != cur:
                cur.wait_stream(st)

    # ------------------------------------------------------------------
    def rhs(self, g: torch.Tensor, f: torch.Tensor, y0: torch.Tensor, out: Optional[torch.Tensor] = None):
        self._vec(g, "g", self.field_shape)
        self._vec(f, "f", self.field_shape)
        self._vec(y0, "y0", (self.batch, self.m))
        b = self.new_vector() if out is None else self._vec(out, "out")
        _check(self._call(self.lib.pcop_rhs, self.ctx, _ptr(g), _ptr(f), _ptr(y0), _ptr(b)))
        return b

    def kkt_apply(self, x: torch.Tensor, transpose: bool = False, out: Optional[torch.Tensor] = None):
        self._vec(x, "x")
        y = self.new_vector() if out is None else self._vec(out, "out")
        _check(self._call(self.lib.pcop_kkt_apply, self.ctx, _ptr(x), _ptr(y), int(bool(transpose))))
        return y

    def post_solve(self, x: torch.Tensor, fN: torch.Tensor, g0: torch.Tensor, y0: torch.Tensor):
        """End levels (y^N, p^0), each [batch][m], of the discrete solution x
        (pcop_post_solve); also returns the final relative residuals."""
        self._vec(x, "x")
        for t, name in ((fN, "fN"), (g0, "g0"), (y0, "y0")):
            self._vec(t, name, (self.batch, self.m))
        yN = torch.empty((self.batch, self.m), dtype=torch.float64, device=self.device)
        p0 = torch.empty_like(yN)
        rel = (ctypes.c_double * self.batch)()
        _check(self._call(self.lib.pcop_post_solve, self.ctx, _ptr(x), _ptr(fN), _ptr(g0), _ptr(y0), _ptr(yN), _ptr(p0), rel))
        return yN, p0, list(rel)

    def error_eh(self, x: torch.Tensor, yN: torch.Tensor, p0: torch.Tensor, y_exact: torch.Tensor,
                 p_exact: torch.Tensor):
        """e_h of Section 3 per member (pcop_error_eh); y_exact, p_exact are
        [batch][nt+1][m] values of the exact solution at t_j = j tau."""
        self._vec(x, "x")
        self._vec(yN, "yN", (self.batch, self.m))
        self._vec(p0, "p0", (self.batch, self.m))
        self._vec(y_exact, "y_exact", (self.batch, self.nt + 1, self.m))
        self._vec(p_exact, "p_exact", (self.batch, self.nt + 1, self.m))
        eh = (ctypes.c_double * self.batch)()
        _check(self._call(self.lib.pcop_error_eh, self.ctx, _ptr(x), _ptr(yN), _ptr(p0), _ptr(y_exact), _ptr(p_exact), eh))
        return list(eh)

    def precond_apply(self, v: torch.Tensor, out: Optional[torch.Tensor] = None):
        self._vec(v, "v")
        w = self.new_vector() if out is None else self._vec(out, "out")
        _check(self._call(self.lib.pcop_precond_apply, self.ctx, _ptr(v), _ptr(w)))
        return w

    def precond_apply_noalloc(self, v: torch.Tensor, out: torch.Tensor):
        """pcop_precond_apply_noalloc: the same apply with the library's static
        spectrum scratch; the output tensor is the caller's."""
        self._vec(v, "v")
        self._vec(out, "out")
        _check(self._call(self.lib.pcop_precond_apply_noalloc, self.ctx, _ptr(v), _ptr(out)))
        return out

    def solve(self, b: torch.Tensor, x0: Optional[torch.Tensor] = None, transpose: bool = False,
              history: bool = False, raise_on_fail: bool = False):
        """Returns (x, [SolveInfo per member], history or None)."""
        self._vec(b, "b")
        x = self.new_vector() if x0 is None else self._vec(x0, "x0").clone()
        info = (c_member_info * self.batch)()
        hist = None
        hist_ptr = None
        if history:
            import numpy as np
            hist = np.full((self.batch, self.maxit + 1), np.nan)
            hist_ptr = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        st = self._call(self.lib.pcop_solve, self.ctx, _ptr(b), _ptr(x), int(bool(transpose)), info, hist_ptr)
        if st not in (PCOP_OK, PCOP_NOT_CONVERGED) or (raise_on_fail and st != PCOP_OK):
            _check(st)
        infos = [SolveInfo(i.iters, bool(i.converged), i.relres_est, i.relres_true) for i in info]
        return x, infos, hist

    def unpack(self, x: torch.Tensor):
        self._vec(x, "x")
        y = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        p = torch.empty_like(y)
        _check(self._call(self.lib.pcop_unpack, self.ctx, _ptr(x), _ptr(y), _ptr(p)))
        return y, p

    def pack_cotangent(self, ybar: Optional[torch.Tensor], pbar: Optional[torch.Tensor]):
        if ybar is not None:
            self._vec(ybar, "ybar", self.field_shape)
        if pbar is not None:
            self._vec(pbar, "pbar", self.field_shape)
        r = self.new_vector()
        _check(self._call(self.lib.pcop_pack_cotangent, self.ctx, _ptr(ybar), _ptr(pbar), _ptr(r)))
        return r

    def timing_enable(self, enable: bool = True):
        """Start (and reset) or stop per-kernel HIP-event timing."""
        _check(self.lib.pcop_timing_enable(self.ctx, int(bool(enable))))

    def timing_read(self, reset: bool = False):
        """{family: {"launches", "ms", "bytes"}} accumulated since timing_enable."""
        cap = 32
        arr = (c_kernel_stat * cap)()
        cnt = ctypes.c_int(0)
        _check(self.lib.pcop_timing_read(self.ctx, arr, cap, ctypes.byref(cnt), int(bool(reset))))
        return {arr[i].name.decode(): {"launches": int(arr[i].launches), "ms": float(arr[i].ms),
                                       "bytes": float(arr[i].bytes)} for i in range(min(cnt.value, cap))}

    def data_grad(self, lam: torch.Tensor):
        self._vec(lam, "lam")
        dg = torch.empty(self.field_shape, dtype=torch.float64, device=self.device)
        df = torch.empty_like(dg)
        dy0 = torch.empty((self.batch, self.m), dtype=torch.float64, device=self.device)
        _check(self._call(self.lib.pcop_data_grad, self.ctx, _ptr(lam), _ptr(dg), _ptr(df), _ptr(dy0)))
        return dg, df, dy0


class KKTSolve(torch.autograd.Function):
    """(g, f, y0) -> (y, p) through one preconditioned KKT solve.

    The backward pass solves the adjoint system A^T lam = dL/dx with the same
    solver (A^T = J A J with J = diag(I, -I), so the same preconditioner
    serves) and maps lam to dL/dg, dL/df, dL/dy0 with pcop_data_grad."""

    @staticmethod
    def forward(ctx, solver: Solver, g, f, y0):
        b = solver.rhs(g.contiguous(), f.contiguous(), y0.contiguous())
        x, infos, _ = solver.solve(b)
        if not all(i.converged for i in infos):
            raise NotConverged(PCOP_NOT_CONVERGED, "forward KKT solve did not converge")
        y, p = solver.unpack(x)
        ctx.solver = solver
        ctx.infos = infos
        return y, p

    @staticmethod
    def backward(ctx, ybar, pbar):
        solver = ctx.solver
        yb = None if ybar is None else ybar.contiguous()
        pb = None if pbar is None else pbar.contiguous()
        r = solver.pack_cotangent(yb, pb)
        lam, infos, _ = solver.solve(r, transpose=True)
        if not all(i.converged for i in infos):
            raise NotConverged(PCOP_NOT_CONVERGED, "adjoint KKT solve did not converge")
        dg, df, dy0 = solver.data_grad(lam)
        return None, dg, df, dy0


def kkt_solve(solver: Solver, g, f, y0):
    """Differentiable solve: returns (y, p) with gradients to g, f, y0."""
    return KKTSolve.apply(solver, g, f, y0)
