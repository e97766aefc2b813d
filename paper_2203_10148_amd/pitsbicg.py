"""ctypes binding of libpitsbicg (include/pitsbicg.h).

Argument marshalling only: torch tensors become raw device pointers, the
current torch stream becomes the hipStream_t, and the workspace is a torch
uint8 tensor the context binds.  Every step of the method runs in the HIP
kernels of libpitsbicg.so; there is no fallback path.  If the library is
missing this module raises on first use.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpitsbicg.so")
CHECK_LIB_PATH = os.path.join(_PKG, "libpitsbicg_check.so")

# status codes
OK, EINVAL, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, EAGAIN = 0, -1, -2, -3, -4, -5, 1
DIRICHLET0, PERIODIC = 0, 1
IE, CN, ADI_PR = 0, 1, 2
F64, F32 = 0, 1
ABS, REL = 0, 1
X0_ZERO, X0_GIVEN, X0_COARSE = 0, 1, 2
APPLY_RAW, APPLY_LAST = 1, 2
NOALLOC_SCRATCH_BYTES = 32 << 20  # PIT_NOALLOC_SCRATCH_BYTES


class PitError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} (code {code}, hip error {last_hip_error()})")


class pit_problem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("M", ct.c_int32 * 2), ("bc", ct.c_int32),
                ("length", ct.c_double * 2), ("nu", ct.c_double), ("adv", ct.c_double * 2),
                ("react", ct.c_double), ("T", ct.c_double), ("rot", ct.c_double)]


class pit_stepper(ct.Structure):
    _fields_ = [("scheme", ct.c_int32), ("substeps", ct.c_int32), ("prec", ct.c_int32),
                ("reserved", ct.c_int32)]


class pit_solve_opts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("restart_tol", ct.c_double), ("max_iter", ct.c_int32),
                ("norm_mode", ct.c_int32), ("x0_mode", ct.c_int32),
                ("half_step_check", ct.c_int32), ("stall_window", ct.c_int32),
                ("timing", ct.c_int32)]


class pit_solve_info(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iters", ct.c_int32), ("matvecs", ct.c_int32),
                ("restarts", ct.c_int32), ("res_norm", ct.c_double),
                ("history", ct.POINTER(ct.c_double)), ("history_cap", ct.c_int32),
                ("history_len", ct.c_int32), ("ms_total", ct.c_float),
                ("ms_fine", ct.c_float), ("ms_coarse", ct.c_float), ("n_fine", ct.c_int32),
                ("n_coarse", ct.c_int32), ("n_fine_timed", ct.c_int32), ("n_coarse_timed", ct.c_int32),
                ("ms_krylov", ct.c_float), ("n_krylov_timed", ct.c_int32)]


class pit_server_cfg(ct.Structure):
    _fields_ = [("arena", ct.c_void_p), ("arena_bytes", ct.c_uint64), ("device", ct.c_int32),
                ("max_slots", ct.c_int32), ("reserved", ct.c_int32 * 2)]


class pit_request(ct.Structure):
    _fields_ = [("problem", pit_problem), ("N", ct.c_int32), ("m", ct.c_int32), ("fine", pit_stepper),
                ("coarse", pit_stepper), ("u0", ct.c_void_p), ("X", ct.c_void_p), ("opts", pit_solve_opts)]


class pit_result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("iters", ct.c_int32), ("matvecs", ct.c_int32),
                ("restarts", ct.c_int32), ("res_norm", ct.c_double), ("t_submit_ms", ct.c_double),
                ("t_admit_ms", ct.c_double), ("t_done_ms", ct.c_double), ("workspace_bytes", ct.c_uint64),
                ("hip_error", ct.c_int32), ("reserved", ct.c_int32)]


EXPORTS = (
    "pit_create", "pit_destroy", "pit_workspace_bytes", "pit_bind_workspace", "pit_apply_F",
    "pit_coarse_sweep", "pit_solve", "pit_strerror", "pit_last_hip_error", "pit_kernel_shape",
    "pit_batch_create", "pit_batch_workspace_bytes", "pit_batch_bind_workspace", "pit_batch_destroy",
    "pit_batch_solve", "pit_server_create", "pit_submit", "pit_poll", "pit_server_load",
    "pit_server_destroy", "pit_autotune_scratch_bytes", "pit_autotune", "pit_autotune_reset", "pit_autotune_adi", "pit_stream_copy", "pit_set_nu_t",
    "pit_parareal", "pit_set_source", "pit_set_source_t", "pit_coarse_sweep_noalloc",
)

_lib = None


def load(path: str | None = None):
    """Load libpitsbicg.so (raises if it has not been built).  The
    environment variable PIT_LIBRARY=check loads the checking build
    libpitsbicg_check.so instead (LDS poisoned with NaN before first use)."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = CHECK_LIB_PATH if os.environ.get("PIT_LIBRARY") == "check" else LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2203_10148_amd.build`")
    lib = ct.CDLL(path)
    vp, i32, sz = ct.c_void_p, ct.c_int32, ct.c_size_t
    lib.pit_create.argtypes = [ct.POINTER(pit_problem), i32, i32, pit_stepper, pit_stepper,
                               ct.POINTER(vp)]
    lib.pit_create.restype = ct.c_int
    lib.pit_destroy.argtypes = [vp]
    lib.pit_workspace_bytes.argtypes = [vp]
    lib.pit_workspace_bytes.restype = sz
    lib.pit_bind_workspace.argtypes = [vp, vp, sz]
    lib.pit_set_source.argtypes = [vp, ct.POINTER(ct.c_double)]
    lib.pit_set_source_t.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    lib.pit_apply_F.argtypes = [vp, vp, vp, i32, vp]
    lib.pit_coarse_sweep.argtypes = [vp, vp, vp, vp]
    lib.pit_coarse_sweep_noalloc.argtypes = [vp, vp, vp, vp]
    lib.pit_solve.argtypes = [vp, vp, vp, ct.POINTER(pit_solve_opts), ct.POINTER(pit_solve_info), vp]
    lib.pit_parareal.argtypes = [vp, vp, vp, ct.POINTER(pit_solve_opts), ct.POINTER(pit_solve_info), vp]
    lib.pit_strerror.argtypes = [ct.c_int]
    lib.pit_strerror.restype = ct.c_char_p
    lib.pit_last_hip_error.restype = ct.c_int
    lib.pit_kernel_shape.argtypes = [vp, ct.POINTER(i32)]
    lib.pit_batch_create.argtypes = [i32, ct.POINTER(vp)]
    lib.pit_batch_workspace_bytes.argtypes = [vp]
    lib.pit_batch_workspace_bytes.restype = sz
    lib.pit_batch_bind_workspace.argtypes = [vp, vp, sz]
    lib.pit_batch_destroy.argtypes = [vp]
    lib.pit_batch_solve.argtypes = [vp, ct.POINTER(vp), i32, ct.POINTER(vp), ct.POINTER(vp),
                                    ct.POINTER(pit_solve_opts), ct.POINTER(pit_solve_info), vp]
    lib.pit_server_create.argtypes = [ct.POINTER(pit_server_cfg), ct.POINTER(vp)]
    lib.pit_submit.argtypes = [vp, ct.POINTER(pit_request), ct.POINTER(ct.c_uint64)]
    lib.pit_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(pit_result)]
    lib.pit_server_load.argtypes = [vp, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(ct.c_uint64)]
    lib.pit_server_destroy.argtypes = [vp]
    lib.pit_autotune_scratch_bytes.argtypes = [ct.POINTER(pit_problem), i32, i32, pit_stepper, pit_stepper]
    lib.pit_autotune_scratch_bytes.restype = sz
    lib.pit_stream_copy.argtypes = [vp, vp, sz, vp]
    lib.pit_set_nu_t.argtypes = [vp, ct.POINTER(ct.c_double)]
    lib.pit_autotune_adi.argtypes = [ct.POINTER(pit_problem), i32, i32, pit_stepper, pit_stepper, vp, sz,
                                     ct.POINTER(i32), ct.POINTER(ct.c_float), vp]
    lib.pit_autotune.argtypes = [ct.POINTER(pit_problem), i32, i32, pit_stepper, pit_stepper, vp, sz,
                                 ct.POINTER(i32), ct.POINTER(ct.c_float), vp]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().pit_strerror(int(code)).decode()


def last_hip_error() -> int:
    return int(load().pit_last_hip_error())


def _check(rc: int, what: str):
    if rc < 0:
        raise PitError(rc, what)
    return rc


def make_problem(p) -> pit_problem:
    """pit_problem from a workloads.Problem (or anything with the same fields)."""
    pb = pit_problem()
    pb.dim = p.dim
    pb.M[0], pb.M[1] = int(p.M[0]), int(p.M[1]) if p.dim == 2 else 1
    pb.bc = p.bc
    pb.length[0], pb.length[1] = float(p.length[0]), float(p.length[1])
    pb.nu = float(p.nu)
    pb.adv[0], pb.adv[1] = float(p.adv[0]), float(p.adv[1])
    pb.react = float(p.react)
    pb.T = float(p.T)
    pb.rot = float(getattr(p, "rot", 0.0))
    return pb


def _ptr(t, numel=None) -> int:
    """Device pointer of a contiguous FP64 CUDA tensor, checked against the expected size."""
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"expected float64, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


@dataclass
class SolveInfo:
    status: int
    iters: int
    matvecs: int
    restarts: int
    res_norm: float
    history: np.ndarray
    ms_total: float
    ms_fine: float = 0.0
    ms_coarse: float = 0.0
    n_fine: int = 0
    n_coarse: int = 0
    n_fine_timed: int = 0
    n_coarse_timed: int = 0
    ms_krylov: float = 0.0
    n_krylov_timed: int = 0


class Context:
    """A pit_ctx plus its torch-allocated workspace."""

    def __init__(self, p, *, fine_prec=None, device=None, bind=True):
        lib = load()
        self.p = p
        self._pb = make_problem(p)
        fine = pit_stepper(p.fine, p.m, p.prec if fine_prec is None else fine_prec, 0)
        coarse = pit_stepper(p.coarse, p.c, F64, 0)
        h = ct.c_void_p()
        _check(lib.pit_create(ct.byref(self._pb), p.N, p.m, fine, coarse, ct.byref(h)), "pit_create")
        self._h = h
        self.ws = None
        if bind:
            self.bind(device)

    @property
    def workspace_bytes(self) -> int:
        return int(load().pit_workspace_bytes(self._h))

    def set_source(self, f, g=None):
        """Source constant in time (one slice of values, host), or None to
        remove it; with g (N m + 1 values at the fine step times) the source
        g(t) f(x).  A bound workspace that is too small for g is replaced by
        one of the new size."""
        if f is None:
            _check(load().pit_set_source(self._h, None), "pit_set_source")
            return
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        if f.size != self.p.npts:
            raise ValueError("set_source: one slice of npts values expected")
        fp = f.ctypes.data_as(ct.POINTER(ct.c_double))
        if g is None:
            _check(load().pit_set_source(self._h, fp), "pit_set_source")
            return
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        if g.size != self.p.N * self.p.m + 1:
            raise ValueError("set_source: N m + 1 profile values expected")
        rc = load().pit_set_source_t(self._h, fp, g.ctypes.data_as(ct.POINTER(ct.c_double)))
        if rc == ENOMEM and self.ws is not None:  # unbound: bind one of the new size
            self.bind(self.ws.device)
            return
        _check(rc, "pit_set_source_t")

    def set_nu_t(self, s):
        """A time-dependent operator constant on each slice (1D): the
        diffusion coefficient on slice n is nu * s[n] (N positive values), or
        constant again with None.  A bound workspace that is too small for the
        per-slice tables is replaced by one of the new size."""
        if s is None:
            _check(load().pit_set_nu_t(self._h, None), "pit_set_nu_t")
            return
        s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(-1))
        if s.size != self.p.N:
            raise ValueError("set_nu_t: N factors expected")
        rc = load().pit_set_nu_t(self._h, s.ctypes.data_as(ct.POINTER(ct.c_double)))
        if rc == ENOMEM and self.ws is not None:  # unbound: bind one of the new size
            self.bind(self.ws.device)
            return
        _check(rc, "pit_set_nu_t")

    def kernel_shape(self):
        out = (ct.c_int32 * 4)()
        _check(load().pit_kernel_shape(self._h, out), "pit_kernel_shape")
        return tuple(out)

    def bind(self, device=None):
        import torch

        n = self.workspace_bytes
        self.ws = torch.empty(n + 256, dtype=torch.uint8, device=device or "cuda")
        base = self.ws.data_ptr()
        off = (-base) % 256
        _check(load().pit_bind_workspace(self._h, base + off, n), "pit_bind_workspace")

    def close(self):
        if getattr(self, "_h", None):
            load().pit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- operators -------------------------------------------------------
    def apply_F(self, lam, y=None, raw=False, last=False, stream=None):
        import torch

        if y is None:
            y = torch.empty_like(lam)
        nt = self.p.N * self.p.npts
        flags = (APPLY_RAW if raw else 0) | (APPLY_LAST if last else 0)
        _check(load().pit_apply_F(self._h, _ptr(lam, nt), _ptr(y, nt), flags, _stream(stream)),
               "pit_apply_F")
        return y

    def coarse_sweep(self, v, z=None, stream=None):
        import torch

        if z is None:
            z = torch.empty_like(v)
        nt = self.p.N * self.p.npts
        _check(load().pit_coarse_sweep(self._h, _ptr(v, nt), _ptr(z, nt), _stream(stream)),
               "pit_coarse_sweep")
        return z

    def coarse_sweep_noalloc(self, v, z=None, stream=None):
        """pit_coarse_sweep_noalloc: the sweep with the library's fixed
        scratch array (z must be given for a call that allocates nothing)."""
        import torch

        if z is None:
            z = torch.empty_like(v)
        nt = self.p.N * self.p.npts
        _check(load().pit_coarse_sweep_noalloc(self._h, _ptr(v, nt), _ptr(z, nt), _stream(stream)),
               "pit_coarse_sweep_noalloc")
        return z

    def solve(self, u0, X=None, *, tol=None, restart_tol=1e-30, max_iter=0, norm_mode=ABS,
              x0_mode=X0_ZERO, half_step_check=0, stall_window=0, hist_cap=4096, stream=None,
              timing=0, raise_on_error=False):
        # timing: 0 off; k > 0 times the first fine apply and coarse sweep and every k-th
        # after them with HIP events (1: every launch), see pit_solve_opts.timing
        import torch

        if X is None:
            X = torch.empty(self.p.N * self.p.npts, dtype=torch.float64, device=u0.device)
        o = pit_solve_opts(self.p.tol if tol is None else tol, restart_tol, max_iter, norm_mode,
                           x0_mode, half_step_check, stall_window, int(timing))
        hist = np.zeros(hist_cap, dtype=np.float64)
        info = pit_solve_info()
        info.history = hist.ctypes.data_as(ct.POINTER(ct.c_double))
        info.history_cap = hist_cap
        rc = load().pit_solve(self._h, _ptr(u0, self.p.npts), _ptr(X, self.p.N * self.p.npts),
                              ct.byref(o), ct.byref(info),
                              _stream(stream))
        if rc in (EINVAL, EHIP) or (raise_on_error and rc < 0):
            raise PitError(rc, "pit_solve")
        return X, SolveInfo(info.status, info.iters, info.matvecs, info.restarts, info.res_norm,
                            hist[: info.history_len].copy(), info.ms_total, info.ms_fine,
                            info.ms_coarse, info.n_fine, info.n_coarse, info.n_fine_timed,
                            info.n_coarse_timed, info.ms_krylov, info.n_krylov_timed)

    def parareal(self, u0, X=None, *, tol=0.0, max_iter=0, norm_mode=ABS, x0_mode=X0_ZERO, hist_cap=4096,
                 stream=None, timing=0):
        """Parareal (Richardson form) with the library's apply and sweep; returns (X, SolveInfo)."""
        import torch

        if X is None:
            X = torch.empty(self.p.N * self.p.npts, dtype=torch.float64, device=u0.device)
        o = pit_solve_opts(tol, 0.0, max_iter, norm_mode, x0_mode, 0, 0, int(timing))
        hist = np.zeros(hist_cap, dtype=np.float64)
        info = pit_solve_info()
        info.history = hist.ctypes.data_as(ct.POINTER(ct.c_double))
        info.history_cap = hist_cap
        rc = load().pit_parareal(self._h, _ptr(u0, self.p.npts), _ptr(X, self.p.N * self.p.npts), ct.byref(o),
                                 ct.byref(info), _stream(stream))
        if rc in (EINVAL, EHIP):
            raise PitError(rc, "pit_parareal")
        return X, SolveInfo(info.status, info.iters, info.matvecs, info.restarts, info.res_norm,
                            hist[: info.history_len].copy(), info.ms_total, info.ms_fine,
                            info.ms_coarse, info.n_fine, info.n_coarse, info.n_fine_timed,
                            info.n_coarse_timed, info.ms_krylov, info.n_krylov_timed)


def autotune(p, device=None, stream=None):
    """Time every line shape for workloads.Problem p (1D) and record the fastest for
    later contexts of the same class; returns ((NT, C), ms)."""
    lib = load()
    pb = make_problem(p)
    fine = pit_stepper(p.fine, p.m, p.prec, 0)
    coarse = pit_stepper(p.coarse, p.c, F64, 0)
    n = int(lib.pit_autotune_scratch_bytes(ct.byref(pb), p.N, p.m, fine, coarse))
    if n == 0:
        raise PitError(EINVAL, "pit_autotune_scratch_bytes")
    buf, base = _aligned(n, device)
    out = (ct.c_int32 * 2)()
    ms = ct.c_float()
    _check(lib.pit_autotune(ct.byref(pb), p.N, p.m, fine, coarse, base, n, out, ct.byref(ms), _stream(stream)),
           "pit_autotune")
    del buf
    return (int(out[0]), int(out[1])), float(ms.value)


def autotune_adi(p, device=None, stream=None):
    """Time the 2D half-step launch shapes for workloads.Problem p (2D, no
    velocity field) and record the fastest for later contexts of the same
    class; returns ((R, wy, cy, seg, columns), (apply ms, sweep ms))."""
    lib = load()
    pb = make_problem(p)
    fine = pit_stepper(p.fine, p.m, p.prec, 0)
    coarse = pit_stepper(p.coarse, p.c, F64, 0)
    n = int(lib.pit_autotune_scratch_bytes(ct.byref(pb), p.N, p.m, fine, coarse))
    if n == 0:
        raise PitError(EINVAL, "pit_autotune_scratch_bytes")
    buf, base = _aligned(n, device)
    out = (ct.c_int32 * 5)()
    ms = (ct.c_float * 2)()
    _check(lib.pit_autotune_adi(ct.byref(pb), p.N, p.m, fine, coarse, base, n, out, ms, _stream(stream)),
           "pit_autotune_adi")
    del buf
    return tuple(int(v) for v in out), (float(ms[0]), float(ms[1]))


def stream_copy(dst, src, stream=None):
    """pit_stream_copy of the tensor src into dst (same byte size)."""
    n = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == n
    _check(load().pit_stream_copy(dst.data_ptr(), src.data_ptr(), n, _stream(stream)), "pit_stream_copy")
    return dst


def autotune_reset():
    load().pit_autotune_reset()


def _opts(p, tol=None, restart_tol=1e-30, max_iter=0, norm_mode=ABS, stall_window=0):
    return pit_solve_opts(p.tol if tol is None else tol, restart_tol, max_iter, norm_mode, X0_ZERO, 0,
                          stall_window, 0)


def _aligned(nbytes, device):
    import torch

    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    return buf, buf.data_ptr() + (-buf.data_ptr()) % 256


class Batch:
    """pit_batch: many independent solves advanced together (see pitsbicg.h)."""

    def __init__(self, max_count, device=None):
        lib = load()
        h = ct.c_void_p()
        _check(lib.pit_batch_create(int(max_count), ct.byref(h)), "pit_batch_create")
        self._h = h
        self.max_count = int(max_count)
        n = int(lib.pit_batch_workspace_bytes(h))
        self.ws, base = _aligned(n, device)
        _check(lib.pit_batch_bind_workspace(h, base, n), "pit_batch_bind_workspace")

    def solve(self, ctxs, u0s, Xs=None, *, tol=None, restart_tol=1e-30, max_iter=0, norm_mode=ABS,
              stall_window=0, hist_cap=4096, stream=None):
        """Solve every context's problem; returns (Xs, [SolveInfo])."""
        import torch

        n = len(ctxs)
        if Xs is None:
            Xs = [torch.empty(c.p.N * c.p.npts, dtype=torch.float64, device=u.device) for c, u in zip(ctxs, u0s)]
        hs = (ct.c_void_p * n)(*[c._h.value for c in ctxs])
        u = (ct.c_void_p * n)(*[_ptr(x, c.p.npts) for c, x in zip(ctxs, u0s)])
        x = (ct.c_void_p * n)(*[_ptr(X, c.p.N * c.p.npts) for c, X in zip(ctxs, Xs)])
        tols = tol if isinstance(tol, (list, tuple)) else [tol] * n
        opts = (pit_solve_opts * n)(*[_opts(c.p, t, restart_tol, max_iter, norm_mode, stall_window)
                                      for c, t in zip(ctxs, tols)])
        hists = [np.zeros(hist_cap, dtype=np.float64) for _ in range(n)]
        infos = (pit_solve_info * n)()
        for i in range(n):
            infos[i].history = hists[i].ctypes.data_as(ct.POINTER(ct.c_double))
            infos[i].history_cap = hist_cap
        rc = load().pit_batch_solve(self._h, hs, n, u, x, opts, infos, _stream(stream))
        if rc in (EINVAL, EHIP, ENOMEM):
            raise PitError(rc, "pit_batch_solve")
        out = [SolveInfo(f.status, f.iters, f.matvecs, f.restarts, f.res_norm, hists[i][: f.history_len].copy(),
                         f.ms_total, 0.0, 0.0, f.n_fine, f.n_coarse) for i, f in enumerate(infos)]
        return Xs, out

    def close(self):
        if getattr(self, "_h", None):
            load().pit_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    status: int
    iters: int
    matvecs: int
    restarts: int
    res_norm: float
    t_submit_ms: float
    t_admit_ms: float
    t_done_ms: float
    workspace_bytes: int
    hip_error: int

    @property
    def latency_ms(self):
        return self.t_done_ms - self.t_submit_ms


class Server:
    """pit_server: request loop with HBM-budget admission and continuous batching.

    The arena (the HBM budget) is a torch uint8 tensor owned here."""

    def __init__(self, arena_bytes, max_slots=256, device=None):
        import torch

        dev = torch.device(device or "cuda")
        self.arena, base = _aligned(int(arena_bytes), dev)
        cfg = pit_server_cfg(base, int(arena_bytes), dev.index or 0, int(max_slots))
        h = ct.c_void_p()
        _check(load().pit_server_create(ct.byref(cfg), ct.byref(h)), "pit_server_create")
        self._h = h

    def submit(self, p, u0, X, *, tol=None, restart_tol=1e-30, max_iter=0, norm_mode=ABS, stall_window=0):
        """Queue a solve of workloads.Problem p; u0 and X are device tensors the caller keeps alive
        (their pending writes must be complete: synchronize first)."""
        r = pit_request()
        r.problem = make_problem(p)
        r.N, r.m = p.N, p.m
        r.fine = pit_stepper(p.fine, p.m, p.prec, 0)
        r.coarse = pit_stepper(p.coarse, p.c, F64, 0)
        r.u0 = _ptr(u0, p.npts)
        r.X = _ptr(X, p.N * p.npts)
        r.opts = _opts(p, tol, restart_tol, max_iter, norm_mode, stall_window)
        t = ct.c_uint64()
        _check(load().pit_submit(self._h, ct.byref(r), ct.byref(t)), "pit_submit")
        return int(t.value)

    def poll(self, ticket):
        """None while pending, else the Result."""
        r = pit_result()
        rc = load().pit_poll(self._h, ct.c_uint64(ticket), ct.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc, "pit_poll")
        return Result(r.status, r.iters, r.matvecs, r.restarts, r.res_norm, r.t_submit_ms, r.t_admit_ms,
                      r.t_done_ms, int(r.workspace_bytes), r.hip_error)

    def load(self):
        q, r, u = ct.c_int32(), ct.c_int32(), ct.c_uint64()
        _check(load().pit_server_load(self._h, ct.byref(q), ct.byref(r), ct.byref(u)), "pit_server_load")
        return int(q.value), int(r.value), int(u.value)

    def close(self):
        if getattr(self, "_h", None):
            load().pit_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
