"""CPU oracle for PiTSBiCG (test infrastructure only).

A thin ctypes wrapper around ``pit_oracle.c``: plain FP64 C, no code shared
with the HIP library.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product path never does.

Every function follows the paper (Riahi, "PiTSBiCG: Parallel in Time Stable
Bi-Conjugate Gradient Algorithm"):
  * ``F`` / ``G``       -- fine / coarse slice propagators (Sec. 2, eq. (continuity));
  * ``apply``           -- all-at-once operator (Sec. 2, eq. (algebraiclinearsystem));
  * ``sweep``           -- coarse preconditioner solve by forward substitution
                           (Sec. 3, eq. (eqinverse));
  * ``dot`` / ``norm``  -- block inner product and the N,inf stopping norm (Sec. 3);
  * ``pitsbicg``        -- Algorithm 1 (Sec. 3);
  * ``parareal_*``      -- Sec. 2, eqs. (pararealAlgebraic) and (pararealscheme);
  * ``serial``          -- the serial fine trajectory, the exact solution;
  * ``set_nu_t``        -- a time-dependent operator, constant on each slice
                           (nu s_n on slice n): per-slice F_n and G_n;
  * ``set_fine_f32``    -- the FP32-fine form of F, emulated (1D: FP32 increment
                           steps with a compensated float state; 2D: FP32 field
                           storage between half steps), to predict its accuracy;
  * ``source``/``forced`` -- an optional source (Sec. 2, eq. (Cauchy)), constant
                           in time or separable, f(t, x) = g(t) h(x): the
                           propagator of slice n becomes affine, F_n(u) =
                           F0(u) + b_n, and B = (u0, b_0, .., b_{N-2}) with
                           b_n = F_n(0) the forced response of slice n.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DIRICHLET, PERIODIC = 0, 1
IE, CN, ADI, ADI_IE = 0, 1, 2, 3  # ADI_IE: the 2D backward-Euler splitting
ABS, REL = 0, 1
X0_ZERO, X0_GIVEN, X0_COARSE = 0, 1, 2
OK, EINVAL, ENOCONV, EBREAKDOWN = 0, -1, -4, -5


def build(force: bool = True) -> str:
    """Compile pit_oracle.c into liboracle.so (plain IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = ct.POINTER(ct.c_double)


class _Info(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters", ct.c_int), ("matvecs", ct.c_int),
                ("restarts", ct.c_int), ("res_norm", ct.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ct.CDLL(_LIB)
    lib.orc_create.restype = ct.c_void_p
    lib.orc_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double,
                               ct.c_double, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                               ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_double]
    lib.orc_destroy.argtypes = [ct.c_void_p]
    lib.orc_set_source.argtypes = [ct.c_void_p, _D]
    lib.orc_set_source_t.argtypes = [ct.c_void_p, _D, _D]
    lib.orc_set_fine_f32.argtypes = [ct.c_void_p, ct.c_int]
    lib.orc_set_nu_t.argtypes = [ct.c_void_p, _D]
    lib.orc_set_nu_t.restype = ct.c_int
    lib.orc_G_slice.argtypes = [ct.c_void_p, ct.c_int, _D, _D]
    lib.orc_set_fine_f32.restype = ct.c_int
    lib.orc_forced.argtypes = [ct.c_void_p, _D]
    lib.orc_forced_slice.argtypes = [ct.c_void_p, ct.c_int, _D]
    lib.orc_F_slice.argtypes = [ct.c_void_p, ct.c_int, _D, _D]
    lib.orc_npts.argtypes = [ct.c_void_p]
    lib.orc_npts.restype = ct.c_int
    lib.orc_weight.argtypes = [ct.c_void_p]
    lib.orc_weight.restype = ct.c_double
    for name in ("orc_F", "orc_G", "orc_apply", "orc_apply_raw", "orc_sweep"):
        getattr(lib, name).argtypes = [ct.c_void_p, _D, _D]
    lib.orc_step.argtypes = [ct.c_void_p, ct.c_int, ct.c_double, _D, _D]
    lib.orc_serial.argtypes = [ct.c_void_p, _D, _D, _D]
    lib.orc_dot.argtypes = [ct.c_void_p, _D, _D]
    lib.orc_dot.restype = ct.c_double
    lib.orc_norm.argtypes = [ct.c_void_p, _D]
    lib.orc_norm.restype = ct.c_double
    lib.orc_pitsbicg.argtypes = [ct.c_void_p, _D, _D, ct.c_double, ct.c_double, ct.c_int,
                                 ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Info), _D,
                                 ct.c_int, ct.POINTER(ct.c_int)]
    lib.orc_pitsbicg.restype = ct.c_int
    lib.orc_parareal_richardson.argtypes = [ct.c_void_p, _D, _D, ct.c_int, _D]
    lib.orc_parareal_pc.argtypes = [ct.c_void_p, _D, _D, ct.c_int]
    lib.orc_tridiag_solve.argtypes = [ct.c_int, _D, _D, _D, _D, _D]
    lib.orc_cyclic_solve.argtypes = [ct.c_int, _D, _D, _D, _D, _D]
    lib.orc_set_threads.argtypes = [ct.c_int]
    lib.orc_get_threads.restype = ct.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def tridiag_solve(a, b, c, d):
    """Thomas solve; a = sub-diagonal (a[0] unused), c = super (c[-1] unused)."""
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.empty_like(d)
    _load().orc_tridiag_solve(len(d), _p(a), _p(b), _p(c), _p(d), _p(x))
    return x


def cyclic_solve(a, b, c, d):
    """Cyclic tridiagonal solve; a[0] couples row 0 to column n-1, c[-1] row n-1 to column 0."""
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.empty_like(d)
    _load().orc_cyclic_solve(len(d), _p(a), _p(b), _p(c), _p(d), _p(x))
    return x


@dataclass
class SolveInfo:
    status: int
    iters: int
    matvecs: int
    restarts: int
    res_norm: float
    history: np.ndarray


class Oracle:
    """One PiT problem: a grid, an operator, N slices, fine and coarse steppers."""

    def __init__(self, *, dim=1, M=(64, 1), bc=DIRICHLET, length=(1.0, 1.0), nu=1.0,
                 adv=(0.0, 0.0), react=0.0, T=1.0, N=4, m=4, fine=IE, c=1, coarse=IE, source=None, rot=0.0,
                 fine_f32=False, nu_t=None):
        lib = _load()
        Mx, My = (M, 1) if isinstance(M, int) else (int(M[0]), int(M[1]))
        self.dim, self.Mx, self.My, self.N, self.m = dim, Mx, (My if dim == 2 else 1), N, m
        h = lib.orc_create(dim, Mx, My, bc, float(length[0]), float(length[1]), float(nu),
                           float(adv[0]), float(adv[1]), float(react), float(T), N, m, fine, c,
                           coarse, float(rot))
        if not h:
            raise ValueError("oracle: invalid problem description")
        self._h = h
        self.npts = lib.orc_npts(h)
        self.weight = lib.orc_weight(h)
        if source is not None:
            self.set_source(source)
        if fine_f32:
            self.set_fine_f32(True)
        if nu_t is not None:
            self.set_nu_t(nu_t)

    def set_nu_t(self, s):
        """A time-dependent operator constant on each slice: the diffusion
        coefficient on slice n is nu * s[n] (N positive values), or constant
        again with None.  F, G, the apply, the sweep and Algorithm 1 all use
        the slice's operator."""
        if s is None:
            _lib.orc_set_nu_t(self._h, None)
            return
        s = self._c(s)
        if s.size != self.N or _lib.orc_set_nu_t(self._h, _p(s)) != OK:
            raise ValueError("oracle: nu_t needs N finite positive factors")

    def set_fine_f32(self, on=True):
        """The fine propagator F as the emulated FP32-fine form (1D: FP32
        increment-form steps with a compensated float state; 2D: FP32 storage
        of the fields between half steps), or FP64 again.  Everything else
        (the coarse propagator, the block products, Algorithm 1) stays FP64.
        Not with a source."""
        if _lib.orc_set_fine_f32(self._h, 1 if on else 0) != OK:
            raise ValueError("oracle: the FP32-fine form takes no source")

    def set_source(self, f, g=None):
        """Set the source f (one slice of values), or remove it with None.
        With g (N m + 1 values, g(t_j) at the fine step times t_j = j dt) the
        source is f(t, x) = g(t) f(x)."""
        if f is None:
            _lib.orc_set_source(self._h, None)
            return
        f = self._c(f)
        if f.size != self.npts:
            raise ValueError("oracle: source size")
        if g is None:
            _lib.orc_set_source(self._h, _p(f))
            return
        g = self._c(g)
        if g.size != self.N * self.m + 1:
            raise ValueError("oracle: time profile size")
        _lib.orc_set_source_t(self._h, _p(f), _p(g))

    def forced(self, n=0):
        """b_n = F_n(0): the forced response of slice n."""
        b = self._slice()
        _lib.orc_forced_slice(self._h, int(n), _p(b))
        return b

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    def _slice(self):
        return np.empty(self.npts, dtype=np.float64)

    def _block(self):
        return np.empty(self.N * self.npts, dtype=np.float64)

    @staticmethod
    def _c(a):
        return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))

    def F(self, u, n=0):
        """The fine propagator of slice n (the source's slice n with a
        time-dependent source)."""
        u = self._c(u); out = self._slice()
        _lib.orc_F_slice(self._h, int(n), _p(u), _p(out)); return out

    def G(self, u, n=0):
        """The coarse propagator of slice n."""
        u = self._c(u); out = self._slice()
        _lib.orc_G_slice(self._h, int(n), _p(u), _p(out)); return out

    def step(self, scheme, dt, u):
        u = self._c(u); out = self._slice()
        _lib.orc_step(self._h, scheme, float(dt), _p(u), _p(out)); return out

    def apply(self, lam):
        lam = self._c(lam); y = self._block()
        _lib.orc_apply(self._h, _p(lam), _p(y)); return y

    def apply_raw(self, lam):
        lam = self._c(lam); y = self._block()
        _lib.orc_apply_raw(self._h, _p(lam), _p(y)); return y

    def sweep(self, v):
        v = self._c(v); z = self._block()
        _lib.orc_sweep(self._h, _p(v), _p(z)); return z

    def serial(self, u0, want_uT=False):
        u0 = self._c(u0); lam = self._block(); uT = self._slice()
        _lib.orc_serial(self._h, _p(u0), _p(lam), _p(uT) if want_uT else None)
        return (lam, uT) if want_uT else lam

    def dot(self, U, V):
        return float(_lib.orc_dot(self._h, _p(self._c(U)), _p(self._c(V))))

    def norm(self, U):
        return float(_lib.orc_norm(self._h, _p(self._c(U))))

    def pitsbicg(self, u0, *, tol=1e-10, eps0=1e-30, max_iter=None, norm_mode=ABS,
                 x0_mode=X0_ZERO, X0=None, half_step_check=0, stall_window=0, hist_cap=4096):
        u0 = self._c(u0)
        X = self._block() if X0 is None else self._c(X0).copy()
        if max_iter is None:
            max_iter = 2 * self.N
        info = _Info()
        hist = np.zeros(hist_cap, dtype=np.float64)
        hl = ct.c_int(0)
        _lib.orc_pitsbicg(self._h, _p(u0), _p(X), float(tol), float(eps0), int(max_iter),
                          int(norm_mode), int(x0_mode), int(half_step_check), int(stall_window),
                          ct.byref(info), _p(hist), hist_cap, ct.byref(hl))
        return X, SolveInfo(info.status, info.iters, info.matvecs, info.restarts, info.res_norm,
                            hist[: hl.value].copy())

    def parareal_richardson(self, u0, iters, X0=None):
        u0 = self._c(u0)
        X = np.zeros(self.N * self.npts) if X0 is None else self._c(X0).copy()
        hist = np.zeros(max(iters, 1))
        _lib.orc_parareal_richardson(self._h, _p(u0), _p(X), int(iters), _p(hist))
        return X, hist[:iters]

    def parareal_pc(self, u0, Lam0, iters):
        u0 = self._c(u0); Lam = self._c(Lam0).copy()
        _lib.orc_parareal_pc(self._h, _p(u0), _p(Lam), int(iters))
        return Lam
