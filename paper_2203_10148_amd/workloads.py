"""Seeded synthetic inputs for the PiT workloads.

This module holds no arithmetic of the method: it describes problems (grid,
coefficients, slicing, steppers) and draws initial conditions.  Both the HIP
path and the CPU oracle take their inputs from here.

The paper's experiments (Sec. 4) use FreeFem++ finite elements with a Gaussian
initial condition; those meshes and that software are not available, so the
synthetic finite-difference problems below stand in for them:

* ``c1_heat1d``      1D heat, nu = 0.1, Dirichlet-0, M = 64, T = 1, N = 16, fine 64 IE
                     steps per slice, coarse 1 IE step, u0 = sin(pi x) + 0.5 sin(3 pi x).
* ``c2_advdiff1d``   1D periodic advection-diffusion, a = 1, nu = 1e-3, M = 4096, T = 2,
                     N = 256, fine 200 CN steps per slice, coarse 2 IE steps,
                     random-Fourier u0 (k <= 64, amplitude k^-2, seed 2).
* ``c3_heat2d``      2D heat, nu = 0.05, 512 x 512 interior points of the unit square,
                     T = 0.5, N = 128, fine 64 PR-ADI steps, coarse 1 PR-ADI step,
                     u0 = 8 Gaussian bumps (seed 3).
* ``c4_batch``       64 random 1D advection-diffusion instances (seed 4).
* ``c5_requests``    a Poisson stream of 1D/2D requests (seed 5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

DIRICHLET, PERIODIC = 0, 1
IE, CN, ADI, ADI_IE = 0, 1, 2, 3  # ADI_IE: the 2D backward-Euler splitting
F64, F32 = 0, 1


@dataclass(frozen=True)
class Problem:
    """A PiT problem description (plain data)."""
    dim: int = 1
    M: tuple = (64, 1)          # points per axis (interior for Dirichlet)
    bc: int = DIRICHLET
    length: tuple = (1.0, 1.0)
    nu: float = 0.1
    adv: tuple = (0.0, 0.0)
    react: float = 0.0
    T: float = 1.0
    N: int = 16                 # time slices
    m: int = 64                 # fine steps per slice
    fine: int = IE
    c: int = 1                  # coarse steps per slice
    coarse: int = IE
    prec: int = F64             # fine-propagator precision
    tol: float = 1e-10
    name: str = "custom"
    rot: float = 0.0            # 2D: rate of a rigid rotation about the domain centre

    @property
    def npts(self) -> int:
        return self.M[0] * (self.M[1] if self.dim == 2 else 1)

    @property
    def cells_per_apply(self) -> int:
        """Fine cell-updates in one all-at-once apply: (N-1) slices x m steps x npts."""
        return (self.N - 1) * self.m * self.npts

    def oracle_kwargs(self) -> dict:
        return dict(dim=self.dim, M=self.M, bc=self.bc, length=self.length, nu=self.nu,
                    adv=self.adv, react=self.react, T=self.T, N=self.N, m=self.m,
                    fine=self.fine, c=self.c, coarse=self.coarse, rot=self.rot)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# grids
# ---------------------------------------------------------------------------

def grid_1d(p: Problem) -> np.ndarray:
    """Grid points: Dirichlet x_j = (j+1) h, h = L/(M+1); periodic x_j = j h, h = L/M."""
    M, L = p.M[0], p.length[0]
    if p.bc == PERIODIC:
        return np.arange(M) * (L / M)
    return np.arange(1, M + 1) * (L / (M + 1))


def grid_2d(p: Problem):
    """(X, Y) arrays of shape (My, Mx), x fastest; Dirichlet interior points."""
    Mx, My = p.M
    x = np.arange(1, Mx + 1) * (p.length[0] / (Mx + 1))
    y = np.arange(1, My + 1) * (p.length[1] / (My + 1))
    return np.meshgrid(x, y, indexing="xy")


# ---------------------------------------------------------------------------
# initial conditions
# ---------------------------------------------------------------------------

def u0_sines(p: Problem, modes=((1, 1.0), (3, 0.5))) -> np.ndarray:
    """sum of amp * sin(k pi x / L) on the Dirichlet grid."""
    x = grid_1d(p)
    return sum(a * np.sin(k * math.pi * x / p.length[0]) for k, a in modes)


@dataclass
class Fourier:
    """u0(x) = sum_k k^-2 (a_k cos(2 pi k x/L) + b_k sin(2 pi k x/L)), k = 1..K."""
    k: np.ndarray
    a: np.ndarray
    b: np.ndarray


def fourier_coeffs(seed: int, kmax: int = 64) -> Fourier:
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(kmax)
    b = rng.standard_normal(kmax)
    k = np.arange(1, kmax + 1)
    return Fourier(k=k, a=a, b=b)


def u0_fourier(p: Problem, seed: int, kmax: int = 64) -> np.ndarray:
    f = fourier_coeffs(seed, kmax)
    x = grid_1d(p)
    ph = 2.0 * math.pi * np.outer(f.k, x) / p.length[0]
    amp = f.k.astype(np.float64) ** -2
    return (amp[:, None] * (f.a[:, None] * np.cos(ph) + f.b[:, None] * np.sin(ph))).sum(0)


def u0_bumps(p: Problem, seed: int, nbumps: int = 8) -> np.ndarray:
    """Sum of Gaussian bumps: A ~ U[0.5,1], centres ~ U[0.15,0.85]^2, sigma ~ U[0.02,0.1]."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.5, 1.0, nbumps)
    cx = rng.uniform(0.15, 0.85, nbumps) * p.length[0]
    cy = rng.uniform(0.15, 0.85, nbumps) * p.length[1]
    sg = rng.uniform(0.02, 0.1, nbumps)
    X, Y = grid_2d(p)
    u = np.zeros_like(X)
    for i in range(nbumps):
        u += A[i] * np.exp(-((X - cx[i]) ** 2 + (Y - cy[i]) ** 2) / (2.0 * sg[i] ** 2))
    return u.reshape(-1)


def source_bumps(p: Problem, seed: int, nbumps: int = 4) -> np.ndarray:
    """A seeded source field (constant in time): Gaussian bumps, A ~ U[-1,1],
    centres ~ U[0,1) of each axis, sigma ~ U[0.03,0.1]; the distance wraps on
    a periodic axis."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, nbumps)
    cx = rng.uniform(0.0, 1.0, nbumps) * p.length[0]
    cy = rng.uniform(0.0, 1.0, nbumps) * p.length[1]
    sg = rng.uniform(0.03, 0.1, nbumps)
    if p.dim == 1:
        x = grid_1d(p)
        f = np.zeros_like(x)
        for i in range(nbumps):
            d = x - cx[i]
            if p.bc == PERIODIC:
                d = (d + 0.5 * p.length[0]) % p.length[0] - 0.5 * p.length[0]
            f += A[i] * np.exp(-d ** 2 / (2.0 * sg[i] ** 2))
        return f
    X, Y = grid_2d(p)
    f = np.zeros_like(X)
    for i in range(nbumps):
        f += A[i] * np.exp(-((X - cx[i]) ** 2 + (Y - cy[i]) ** 2) / (2.0 * sg[i] ** 2))
    return f.reshape(-1)


def source_profile(p: Problem, seed: int, nwaves: int = 3) -> np.ndarray:
    """A seeded time profile g(t_j) at the fine step times t_j = j T/(N m),
    j = 0..N m, for a separable source g(t) h(x): 1 plus a few sine waves,
    amplitudes ~ U[-0.5,0.5], angular frequencies ~ U[0,4 pi/T] (up to two
    periods over the horizon), phases ~ U[0,2 pi)."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-0.5, 0.5, nwaves)
    om = rng.uniform(0.0, 4.0 * np.pi / p.T, nwaves)
    ph = rng.uniform(0.0, 2.0 * np.pi, nwaves)
    t = (p.T / (p.N * p.m)) * np.arange(p.N * p.m + 1)
    g = np.ones_like(t)
    for i in range(nwaves):
        g += amp[i] * np.sin(om[i] * t + ph[i])
    return g


def nu_factors(p: Problem, seed: int) -> np.ndarray:
    """Seeded per-slice diffusion factors s_n for a time-dependent operator
    constant on each slice (nu s_n on slice n): a slow oscillation between
    1/2 and 2 over the horizon, s_n = 2^sin(2 pi (n + 1/2)/N * f + phase),
    with f ~ U[0.5, 2] periods and phase ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.5, 2.0)
    ph = rng.uniform(0.0, 2.0 * np.pi)
    n = np.arange(p.N) + 0.5
    return 2.0 ** np.sin(2.0 * np.pi * f * n / p.N + ph)


def random_block(p: Problem, seed: int) -> np.ndarray:
    """A seeded N x npts block vector of standard normals (operator parity inputs)."""
    return np.random.default_rng(seed).standard_normal(p.N * p.npts)


# ---------------------------------------------------------------------------
# named configurations
# ---------------------------------------------------------------------------

C1 = Problem(dim=1, M=(64, 1), bc=DIRICHLET, nu=0.1, T=1.0, N=16, m=64, fine=IE, c=1, coarse=IE,
             prec=F64, tol=1e-10, name="c1_heat1d")
C2 = Problem(dim=1, M=(4096, 1), bc=PERIODIC, nu=1e-3, adv=(1.0, 0.0), T=2.0, N=256, m=200,
             fine=CN, c=2, coarse=IE, prec=F64, tol=1e-8, name="c2_advdiff1d")
C3 = Problem(dim=2, M=(512, 512), bc=DIRICHLET, nu=0.05, T=0.5, N=128, m=64, fine=ADI, c=1,
             coarse=ADI, prec=F32, tol=1e-8, name="c3_heat2d")


# The advection-diffusion-reaction test of Sec. 4 (rotating velocity
# u = [-y, x] about the centre of the unit square, mu = 0.1, r = 0.5, h = 0.02
# (49 interior points per axis), dt = 1e-3, T = 6.4) as a PR-ADI problem:
# 64 slices of 100 fine steps, coarse one PR-ADI step per slice.
F2 = Problem(dim=2, M=(49, 49), bc=DIRICHLET, nu=0.1, react=0.5, rot=1.0, T=6.4, N=64, m=100, fine=ADI, c=1,
             coarse=ADI, prec=F64, tol=1e-8, name="f2_rotating_adr")

# The other two cases of Sec. 4 on the same grid and time line: diffusion
# (mu = 1) and diffusion-reaction (mu = 1, r = 1.5); Gaussian u0 at the centre.
F3_DIFF = Problem(dim=2, M=(49, 49), bc=DIRICHLET, nu=1.0, T=6.4, N=64, m=100, fine=ADI, c=1, coarse=ADI,
                  prec=F64, tol=1e-8, name="f3_diffusion")
F3_DR = F3_DIFF.with_(react=1.5, name="f3_diffusion_reaction")

# Sec. 4 runs each case on 2^n slices, n = 2..6, with the fine step fixed.
PAPER_CASES = (F3_DIFF, F3_DR, F2)
PAPER_SLICES = (4, 8, 16, 32, 64)


def paper_case(p: Problem, N: int) -> Problem:
    """Case p on N slices with the same fine step (N m = 6400 steps over T)."""
    steps = p.N * p.m
    return p.with_(N=N, m=steps // N)


def u0_gaussian(p: Problem, centre=(0.75, 0.5), sigma=0.1) -> np.ndarray:
    """A Gaussian (2D) at `centre` (fractions of the side lengths)."""
    X, Y = grid_2d(p)
    cx, cy = centre[0] * p.length[0], centre[1] * p.length[1]
    return np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sigma ** 2)).reshape(-1)


def u0_for(p: Problem, seed: int | None = None) -> np.ndarray:
    """The initial condition a named configuration uses."""
    if p.name.startswith("c1"):
        return u0_sines(p)
    if p.name.startswith("f2"):
        return u0_gaussian(p)
    if p.name.startswith("f3"):
        return u0_gaussian(p, centre=(0.5, 0.5))
    if p.dim == 2:
        return u0_bumps(p, 3 if seed is None else seed)
    return u0_fourier(p, 2 if seed is None else seed)


def c4_batch(seed: int = 4, count: int = 64) -> list:
    """Batched workload: `count` 1D periodic CN instances, M ~ U{256..8192},
    N ~ U{32..512}, m ~ U{16..256}, nu log-uniform in [1e-4, 1e-1], a ~ U[0, 2],
    T = 2, coarse 2 IE steps, FP32 fine, tol 1e-8.  Returns (Problem, u0 seed) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        M = int(rng.integers(256, 8193))
        N = int(rng.integers(32, 513))
        m = int(rng.integers(16, 257))
        nu = float(10.0 ** rng.uniform(-4.0, -1.0))
        a = float(rng.uniform(0.0, 2.0))
        p = Problem(dim=1, M=(M, 1), bc=PERIODIC, nu=nu, adv=(a, 0.0), T=2.0, N=N, m=m,
                    fine=CN, c=2, coarse=IE, prec=F32, tol=1e-8, name=f"c4_inst{i}")
        out.append((p, 1000 + i))
    return out


def c5_requests(seed: int = 5, count: int = 2000, rate: float = 200.0) -> list:
    """Serving workload: Poisson arrivals at `rate`/s; 70% 1D periodic CN
    (M ~ U{512..16384}, N ~ U{64..512}, m ~ U{16..256}, T = 2), 30% 2D heat
    (side ~ U{128..1024}, N ~ U{32..256}, m = 64, nu = 0.05, T = 0.5).
    FP32 fine, tol 1e-8.  Returns (arrival_s, Problem, u0 seed) triples."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < 0.7:
            M = int(rng.integers(512, 16385))
            N = int(rng.integers(64, 513))
            m = int(rng.integers(16, 257))
            nu = float(10.0 ** rng.uniform(-4.0, -1.0))
            a = float(rng.uniform(0.0, 2.0))
            p = Problem(dim=1, M=(M, 1), bc=PERIODIC, nu=nu, adv=(a, 0.0), T=2.0, N=N, m=m,
                        fine=CN, c=2, coarse=IE, prec=F32, tol=1e-8, name=f"c5_req{i}")
        else:
            s = int(rng.integers(128, 1025))
            N = int(rng.integers(32, 257))
            p = Problem(dim=2, M=(s, s), bc=DIRICHLET, nu=0.05, T=0.5, N=N, m=64, fine=ADI, c=1,
                        coarse=ADI, prec=F32, tol=1e-8, name=f"c5_req{i}")
        out.append((t, p, 5000 + i))
    return out
