"""Problems on which Algorithm 1 reaches its special branches in exact arithmetic.

With nu = 0 and no advection every grid point evolves on its own: one implicit
step multiplies it by a scalar factor.  The factors below are powers of two,
the grid spacing is 1/4 (three Dirichlet points), and the data are small
integers, so every value Algorithm 1 forms up to the branch (the block inner
products with their weight h, alpha, omega, beta, the vectors S, K, D) is a
short dyadic number: IEEE FP64 computes it exactly in any summation order.
That makes an exact zero of <D, R~> or <K, S> reachable, which rounding
otherwise never produces.

Per point the preconditioned operator G^{-1} F (Sec. 3) is the N x N unit
lower-triangular matrix with entries g^{i-j-1}(g - f) below the diagonal
(f, g: the fine and coarse factors over one slice).  The data below were found
by an exact search over small integer vectors (Python fractions).

* ``OMEGA_ZERO``: IE fine steps with dt r = -1/2 (factor 2 per step, f = 8 over
  m = 3 steps), one IE coarse step with DT r = -3/2 (g = -2).  R^0 holds
  (-4, 0) at the first point and (-1, 1) at the other two: alpha = 1/2 and
  <K, S> = 0 exactly, so omega = 0 in the first iteration.  The restart that
  follows makes R~ = R = S, so the next <D, R~> = <K, S> = 0 again: the
  shadow-product restart cannot change it, and the solve ends in a breakdown
  after one iteration with X = X^0 + alpha R^0.
* ``SHADOW_ZERO``: CN fine steps with dt r = 2 (factor 0: F = 0), one CN coarse
  step with DT r = 6 (g = -1/2), N = 3, R^0 = (u, 0, 0).  The first iteration
  gives alpha = 1, omega = 3/4, R^1 = (0, u/8, u/8), <R^1, R^0> = 0 (so
  beta = 0, P^1 = R^1) and then <G^{-1}F P^1, R^0> = 0: the second iteration
  meets <D, R~> = 0 with R~ != R, restarts with R~ = P = R^1 and continues as a
  fresh BiCGStab from X^1.  The restart test with epsilon_0 is switched off
  (epsilon_0 < 0), since |<R^1, R~>| = 0 would otherwise trigger it first.
"""
import numpy as np

from paper_2203_10148_amd import workloads as wl

# (problem, fine factor f over a slice, coarse factor g over a slice)
OMEGA_ZERO = wl.Problem(dim=1, M=(3, 1), bc=wl.DIRICHLET, nu=0.0, react=-1.0, T=3.0, N=2, m=3,
                        fine=wl.IE, c=1, coarse=wl.IE, prec=wl.F64, name="omega_zero")
OMEGA_ZERO_FG = (8.0, -2.0)
SHADOW_ZERO = wl.Problem(dim=1, M=(3, 1), bc=wl.DIRICHLET, nu=0.0, react=1.0, T=18.0, N=3, m=3,
                         fine=wl.CN, c=1, coarse=wl.CN, prec=wl.F64, name="shadow_zero")
SHADOW_ZERO_FG = (0.0, -0.5)


def point_operator(N, f, g):
    """Per-point G^{-1} F: unit lower triangular, g^{i-j-1} (g - f) below the diagonal."""
    A = np.eye(N)
    for i in range(N):
        for j in range(i):
            A[i, j] = g ** (i - j - 1) * (g - f)
    return A


def block_operator(p, f, g):
    """G^{-1} F on block vectors [N][npts]: the point operator on every point."""
    return np.kron(point_operator(p.N, f, g), np.eye(p.npts))


def x0_for(p, f, g, u0, R0):
    """The initial guess whose residual G^{-1}(B - F X^0) is R0 (B = (u0, 0, ..)),
    from the scalar forms (F X)_n = X_n - f X_{n-1}, (G Z)_n = Z_n - g Z_{n-1}."""
    R = R0.reshape(p.N, -1)
    B = np.zeros_like(R)
    B[0] = u0
    GR = R.copy()
    GR[1:] -= g * R[:-1]
    W = B - GR  # = F X^0
    X = W.copy()
    for n in range(1, p.N):
        X[n] = W[n] + f * X[n - 1]
    return X.reshape(-1)


def omega_zero_data():
    """(u0, X0, R0) of the omega = 0 case."""
    p = OMEGA_ZERO
    R0 = np.array([[-4.0, -1.0, -1.0], [0.0, 1.0, 1.0]])
    u0 = R0[0].copy()
    X0 = x0_for(p, *OMEGA_ZERO_FG, u0, R0.reshape(-1))
    return u0, X0, R0.reshape(-1)


def shadow_zero_data():
    """(u0, X0, R0) of the <D, R~> = 0 case."""
    p = SHADOW_ZERO
    u = np.array([1.0, -2.0, 3.0])
    R0 = np.zeros((p.N, p.npts))
    R0[0] = u
    X0 = x0_for(p, *SHADOW_ZERO_FG, u, R0.reshape(-1))
    return u, X0, R0.reshape(-1)
