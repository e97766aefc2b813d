"""Closed forms of the discrete schemes on their exact eigenvectors (test helpers).

On the periodic grid x_j = j h, h = L/M, every Fourier mode e^{2 pi i k x/L} is
an exact eigenvector of the central-difference operator
L = nu D2 - a D1c - r, with symbol

    mu_k = -(4 nu / h^2) sin^2(pi k h / L) - i a sin(2 pi k h / L) / h - r,

so one Crank-Nicolson step of dt multiplies the mode by
rho_k = (1 + dt mu_k / 2) / (1 - dt mu_k / 2).  The random-Fourier initial
condition u0 = sum_{k<=K} k^-2 (a_k cos + b_k sin) = Re sum_k k^-2 (a_k - i b_k)
e^{2 pi i k x/L} holds K modes only (K < M/2: no aliasing), so the serial fine
trajectory lambda_n = F^n(u0) of the all-at-once system (Sec. 2) is a direct
sum over those modes, with no time stepping at all.
"""
import math

import numpy as np

from paper_2203_10148_amd import workloads as wl


def periodic_cn_factor(p, k):
    """rho_k of one CN fine step (dt = T/(N m)) of the periodic 1D problem p."""
    M, L = p.M[0], p.length[0]
    h = L / M
    dt = p.T / (p.N * p.m)
    th = 2.0 * math.pi * k * h / L
    mu = -(4.0 * p.nu / h ** 2) * np.sin(0.5 * th) ** 2 - 1j * p.adv[0] * np.sin(th) / h - p.react
    return (1.0 + 0.5 * dt * mu) / (1.0 - 0.5 * dt * mu)


def fourier_serial(p, seed, kmax=64):
    """The serial fine trajectory [N][M] of the CN periodic problem p from
    wl.u0_fourier(p, seed), by the modal closed form."""
    assert p.dim == 1 and p.bc == wl.PERIODIC and p.fine == wl.CN and 2 * kmax < p.M[0]
    f = wl.fourier_coeffs(seed, kmax)
    x = wl.grid_1d(p)
    k = f.k.astype(np.float64)
    c = k ** -2 * (f.a - 1j * f.b)                           # complex mode amplitudes
    rho_m = periodic_cn_factor(p, k) ** p.m                  # one slice (m steps)
    n = np.arange(p.N)
    amp = c[None, :] * rho_m[None, :] ** n[:, None]          # [N][K]
    modes = np.exp(2j * math.pi * np.outer(k, x) / p.length[0])  # [K][M]
    return (amp @ modes).real
