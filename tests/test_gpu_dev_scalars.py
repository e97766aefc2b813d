"""GPU: pit_solve's one-sync iteration (alpha, omega, beta formed on the device
from the reductions' outputs, one host read-back per iteration) against the
iteration that reads every reduction back before going on (PIT_DEV_SCALARS=0).
Both evaluate the same FP64 operations in the same order, so the iterates,
the residual history and the counters must agree bit for bit.  The cases
cover the regular path, the half step that solves the system (one slice:
S = 0 exactly, kk = 0), the restart test of Algorithm 1 firing at the end of
every iteration (rho then comes from the second inner product), an FP32 fine
propagator, 2D problems (one of odd vector length) and a source term, and
one oracle check of the solution.
"""
import os
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2203_10148_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_10148_amd import pitsbicg as P

    P.load()  # fail loudly if the HIP library is missing
    orc.set_threads(min(16, os.cpu_count() or 1))
    yield


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


HEAT1D = wl.Problem(dim=1, M=(300, 1), bc=wl.DIRICHLET, nu=0.05, T=0.5, N=12, m=20, fine=wl.CN, c=2,
                    coarse=wl.IE, prec=wl.F64, tol=1e-10, name="heat1d_300")
CASES = {
    "c2": (wl.C2, {}),
    "c2_f32": (wl.C2.with_(prec=wl.F32), {"stall_window": 10}),
    "heat1d": (HEAT1D, {}),
    "one_slice": (HEAT1D.with_(N=1, m=30), {}),
    "restart_every_iteration": (HEAT1D, {"restart_tol": 1e300}),
    "heat2d": (wl.Problem(dim=2, M=(40, 30), bc=wl.DIRICHLET, nu=0.05, T=0.3, N=8, m=6, fine=wl.ADI, c=1,
                          coarse=wl.ADI, prec=wl.F64, tol=1e-10, name="heat2d_40x30"), {}),
    "f2_short": (wl.F2.with_(T=0.4, N=4, m=25), {}),
    # 7 slices of 41 x 31 points: an odd vector length, so the paired updates
    # take their last element on its own
    "heat2d_odd": (wl.Problem(dim=2, M=(41, 31), bc=wl.DIRICHLET, nu=0.05, T=0.3, N=7, m=6, fine=wl.ADI, c=1,
                              coarse=wl.ADI, prec=wl.F64, tol=1e-10, name="heat2d_41x31"), {}),
}


def solve(p, u0, monkeypatch, flag, source=None, **kw):
    from paper_2203_10148_amd import pitsbicg as P

    monkeypatch.setenv("PIT_DEV_SCALARS", flag)
    c = P.Context(p)
    if source is not None:
        c.set_source(source)
    kw.setdefault("tol", p.tol)
    X, info = c.solve(dev(u0), **kw)
    return host(X), info


def u0_of(p):
    return wl.u0_gaussian(p) if p.dim == 2 else wl.u0_for(p)


@pytest.mark.parametrize("case", list(CASES))
def test_one_sync_iteration_equals_read_back_iteration(case, monkeypatch):
    p, kw = CASES[case]
    say(f"one-sync vs read-back {case}")
    u0 = u0_of(p)
    Xa, ia = solve(p, u0, monkeypatch, "1", **kw)
    Xb, ib = solve(p, u0, monkeypatch, "0", **kw)
    print(f"status {ia.status}/{ib.status} iters {ia.iters}/{ib.iters} restarts {ia.restarts}/{ib.restarts}",
          flush=True)
    assert (ia.status, ia.iters, ia.matvecs, ia.restarts) == (ib.status, ib.iters, ib.matvecs, ib.restarts)
    assert np.array_equal(ia.history, ib.history)
    assert ia.res_norm == ib.res_norm or (np.isnan(ia.res_norm) and np.isnan(ib.res_norm))
    assert np.array_equal(Xa, Xb)
    if case == "restart_every_iteration":
        assert ia.restarts >= ia.iters - 1 > 0
    if case == "one_slice":
        assert ia.status == orc.OK and ia.iters == 1


def test_one_sync_iteration_with_a_source_matches_the_oracle(monkeypatch):
    p = HEAT1D
    say("one-sync with a source vs oracle")
    x = wl.grid_1d(p)
    f = np.sin(np.pi * x) * (1.0 + x)
    u0 = u0_of(p)
    Xa, ia = solve(p, u0, monkeypatch, "1", source=f, tol=1e-12)
    Xb, ib = solve(p, u0, monkeypatch, "0", source=f, tol=1e-12)
    assert ia.iters == ib.iters and np.array_equal(Xa, Xb)
    serial = orc.Oracle(**p.oracle_kwargs(), source=f).serial(u0)
    err = float(np.linalg.norm(Xa - serial) / np.linalg.norm(serial))
    assert ia.status == orc.OK and err < 1e-10


@pytest.mark.parametrize("stride", [0, 1, 3, 7])
def test_timing_stride_counts_and_averages(stride):
    """pit_solve_opts.timing = k times the first fine apply and coarse sweep
    and every k-th after them: the info counts the timed launches, and the
    timing leaves the iterates alone."""
    from paper_2203_10148_amd import pitsbicg as P

    p = HEAT1D
    say(f"timing stride {stride}")
    c = P.Context(p)
    u0 = dev(u0_of(p))
    X0, i0 = c.solve(u0, tol=p.tol)
    X, info = c.solve(u0, tol=p.tol, timing=stride)
    assert np.array_equal(host(X), host(X0)) and info.iters == i0.iters
    if stride == 0:
        assert info.n_fine_timed == info.n_coarse_timed == info.n_krylov_timed == 0
        assert info.ms_fine == info.ms_coarse == info.ms_krylov == 0.0
        return
    assert info.n_fine_timed == -(-info.n_fine // stride)
    assert info.n_coarse_timed == -(-info.n_coarse // stride)
    assert info.ms_fine > 0.0 and info.ms_coarse > 0.0
    # the vector updates and inner products of iterations 0, stride, 2 stride, ..
    assert info.n_krylov_timed == -(-info.iters // stride) and info.ms_krylov > 0.0


def test_negative_timing_stride_is_rejected():
    from paper_2203_10148_amd import pitsbicg as P

    c = P.Context(HEAT1D)
    with pytest.raises(P.PitError):
        c.solve(dev(u0_of(HEAT1D)), timing=-1)


@pytest.mark.parametrize("case", ["omega_zero", "shadow_zero"])
@pytest.mark.parametrize("flag", ["1", "0"])
def test_breakdown_branches_on_exact_cases(case, flag, monkeypatch):
    """Algorithm 1's omega = 0 and <D, R~> = 0 branches, reached in exact
    arithmetic (dyadic data, factors that are powers of two; the CPU pins of
    these cases fix the oracle's behaviour).  Both iteration forms follow the
    oracle's status, iterations, restarts and residual history, and give its
    iterate.  The one-sync iteration learns <D, R~> = 0 only after it has
    queued the product of K, so each such breakdown costs it one product more
    than the oracle and the read-back form."""
    import exact_cases as ec
    from paper_2203_10148_amd import pitsbicg as P

    say(f"exact breakdown case {case}, one-sync={flag}")
    if case == "omega_zero":
        p = ec.OMEGA_ZERO
        u0, X0, _ = ec.omega_zero_data()
        kw = dict(tol=1e-12)
        okw = dict(tol=1e-12)
    else:
        p = ec.SHADOW_ZERO
        u0, X0, _ = ec.shadow_zero_data()
        kw = dict(tol=1e-13, restart_tol=-1.0, max_iter=20)
        okw = dict(tol=1e-13, eps0=-1.0, max_iter=20)
    o = orc.Oracle(**p.oracle_kwargs())
    Xo, io = o.pitsbicg(u0, x0_mode=orc.X0_GIVEN, X0=X0, **okw)
    monkeypatch.setenv("PIT_DEV_SCALARS", flag)
    c = P.Context(p)
    Xd = dev(X0)
    Xd, ig = c.solve(dev(u0), Xd, x0_mode=P.X0_GIVEN, **kw)
    Xg = host(Xd)
    print(f"gpu status {ig.status} iters {ig.iters} restarts {ig.restarts} matvecs {ig.matvecs}; oracle "
          f"{io.status} {io.iters} {io.restarts} {io.matvecs}", flush=True)
    assert (ig.status, ig.iters, ig.restarts) == (io.status, io.iters, io.restarts)
    extra = 1 if flag == "1" else 0  # one <D, R~> = 0 breakdown in either case
    assert ig.matvecs == io.matvecs + extra
    if case == "omega_zero":
        assert ig.status == orc.EBREAKDOWN
        assert np.array_equal(Xg, Xo)
        assert np.array_equal(ig.history[:2], io.history[:2])
    else:
        assert ig.status == orc.OK
        assert np.array_equal(ig.history[:3], io.history[:3])  # exact through the restart
        assert float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)) < 1e-12
