"""GPU: the separable time-dependent source f(t, x) = g(t) h(x)
(pit_set_source_t), through the C ABI.

Slice n carries f on [T_n, T_{n+1}] (Sec. 2, eq. (Cauchyn)): its propagator is
affine, F_n(u) = F0(u) + b_n, and B = (u0, b_0, .., b_{N-2}).  Checked against
the oracle, whose handling of the profile is pinned by modal recursions and a
closed form in test_oracle_pins.py:
  * every slice's forced response b_n (apply_F RAW on zeros), 1e-12;
  * apply_F RAW / LAST (affine) and plain (linear), FP64 1e-12;
  * pit_solve against the serial trajectory (FP64 1e-10 at tol 1e-12; FP32
    fine 1e-5), pit_parareal, and batched against alone (bitwise);
  * the source set before binding and after (the binding grows the
    workspace), and a constant profile against the constant source.
"""
import math
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


def P_():
    from paper_2203_10148_amd import pitsbicg as P

    return P


def say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def problem(case):
    if case == "d_ie":
        return wl.C1.with_(N=8, m=16, name="c1_src_t")
    if case in ("p_cn", "p_cn_f32"):
        return wl.Problem(dim=1, M=(1000, 1), bc=wl.PERIODIC, nu=2e-3, adv=(0.7, 0.0), react=0.1, T=0.5, N=8,
                          m=20, fine=wl.CN, c=2, coarse=wl.IE, prec=wl.F32 if case.endswith("f32") else wl.F64)
    if case == "p_long":  # compact FP64 line tables (above 8192 points)
        return wl.Problem(dim=1, M=(9001, 1), bc=wl.PERIODIC, nu=2e-3, adv=(0.5, 0.0), T=0.5, N=3, m=4,
                          fine=wl.IE, c=2, coarse=wl.IE)
    if case in ("adi", "adi_f32"):
        return wl.Problem(dim=2, M=(40, 30), bc=wl.DIRICHLET, nu=0.05, react=0.2, T=0.2, N=4, m=5,
                          fine=wl.ADI, c=1, coarse=wl.ADI, prec=wl.F32 if case.endswith("f32") else wl.F64)
    if case == "vel":  # slices in LDS
        return wl.F2.with_(T=0.4, N=5, m=10, name="f2_src_t")
    if case == "vel_big":  # per-half-step kernels
        return wl.Problem(dim=2, M=(150, 100), bc=wl.DIRICHLET, nu=0.02, adv=(0.2, 0.1), react=0.5, rot=1.0,
                          T=0.3, N=3, m=3, fine=wl.ADI, c=2, coarse=wl.ADI, name="vel_big")
    raise KeyError(case)


def inputs(p, seed=17):
    f = wl.source_bumps(p, seed)
    g = wl.source_profile(p, seed + 1)
    if p.dim == 1:
        u0 = wl.u0_sines(p) if p.bc == wl.DIRICHLET else wl.u0_fourier(p, 11)
    else:
        u0 = wl.u0_bumps(p, 5)
    return f, g, u0


CASES = ["d_ie", "p_cn", "p_cn_f32", "p_long", "adi", "adi_f32", "vel", "vel_big"]


@pytest.mark.parametrize("case", CASES)
def test_source_t_operators_and_solve_match_oracle(case):
    P = P_()
    p = problem(case)
    say(f"time-dependent source {case}")
    f, g, u0 = inputs(p)
    o = orc.Oracle(**p.oracle_kwargs())
    o.set_source(f, g)
    f64 = p.prec == wl.F64
    # one context gets the source after binding (the binding grows), one before
    c = P.Context(p)
    base = c.workspace_bytes
    c.set_source(f, g)
    assert c.workspace_bytes > base and c.ws.numel() >= c.workspace_bytes
    cb = P.Context(p, bind=False)
    cb.set_source(f, g)
    cb.bind()
    zeros = dev(np.zeros(p.N * p.npts))
    bs = [o.forced(n) for n in range(p.N)]
    for ctx in (c, cb):
        yb = host(ctx.apply_F(zeros, raw=True)).reshape(p.N, -1)
        assert max(relerr(yb[n], bs[n]) for n in range(p.N)) < 1e-12
    lam = wl.random_block(p, 93)
    if f64:
        assert relerr(host(c.apply_F(dev(lam), raw=True)), o.apply_raw(lam)) < 1e-12
        assert relerr(host(c.apply_F(dev(lam))), o.apply(lam)) < 1e-12  # the system operator stays linear
        yl = host(c.apply_F(dev(lam), last=True)).reshape(p.N, -1)
        assert relerr(yl[-1], o.apply_raw(lam).reshape(p.N, -1)[-1]) < 1e-12
    serial, uT = o.serial(u0, want_uT=True)
    if f64:
        Xg, ig = c.solve(dev(u0), tol=1e-12)
        err = relerr(host(Xg), serial)
        assert ig.status == orc.OK and err < 1e-10
    else:
        Xg, ig = c.solve(dev(u0), tol=1e-8, stall_window=10)
        err = relerr(host(Xg), serial)
        assert ig.status in (orc.OK, orc.ENOCONV) and err < 1e-5
    print(f"{case}: status {ig.status} iters {ig.iters} vs serial {err:.2e}", flush=True)
    yT = host(c.apply_F(Xg, last=True)).reshape(p.N, -1)[-1]
    assert relerr(yT, uT) < (1e-10 if f64 else 1e-5)


@pytest.mark.parametrize("case", ["p_cn", "vel"])
def test_source_t_parareal_reaches_the_serial_trajectory(case):
    P = P_()
    p = problem(case)
    say(f"time-dependent source parareal {case}")
    f, g, u0 = inputs(p, 23)
    o = orc.Oracle(**p.oracle_kwargs())
    o.set_source(f, g)
    serial = o.serial(u0)
    c = P.Context(p, bind=False)
    c.set_source(f, g)
    c.bind()
    X, info = c.parareal(dev(u0), tol=1e-12)
    assert info.status == orc.OK and relerr(host(X), serial) < 1e-10


def test_source_t_constant_profile_matches_the_constant_source():
    P = P_()
    p = problem("p_cn")
    say("constant profile vs constant source")
    f, _, u0 = inputs(p, 29)
    a = P.Context(p)
    a.set_source(f)
    b = P.Context(p)
    b.set_source(f, np.ones(p.N * p.m + 1))
    zeros = dev(np.zeros(p.N * p.npts))
    assert relerr(host(b.apply_F(zeros, raw=True)), host(a.apply_F(zeros, raw=True))) < 1e-13
    Xa, _ = a.solve(dev(u0), tol=1e-12)
    Xb, _ = b.solve(dev(u0), tol=1e-12)
    assert relerr(host(Xb), host(Xa)) < 1e-11
    # and back to the constant source: the workspace need shrinks again
    need = b.workspace_bytes
    b.set_source(f)
    assert b.workspace_bytes < need


def test_source_t_batched_equals_alone_and_oracle():
    """A batch of three instances against batches of one (bitwise) and the
    oracle's serial trajectory."""
    P = P_()
    say("time-dependent source batched")
    probs = [problem("d_ie"), problem("adi"), problem("vel")]
    data = [inputs(p, 31 + i) for i, p in enumerate(probs)]

    def run(idx):
        ctxs, u0s = [], []
        for i in idx:
            f, g, u0 = data[i]
            cx = P.Context(probs[i], bind=False)
            cx.set_source(f, g)
            cx.bind()
            ctxs.append(cx)
            u0s.append(dev(u0))
        Xs, infos = P.Batch(len(idx)).solve(ctxs, u0s, tol=1e-10)
        return [host(X) for X in Xs], infos

    Xs, infos = run([0, 1, 2])
    for i, (X, inf) in enumerate(zip(Xs, infos)):
        Xa, ia = run([i])
        assert ia[0].iters == inf.iters and np.array_equal(Xa[0], X), i
        f, g, u0 = data[i]
        o = orc.Oracle(**probs[i].oracle_kwargs())
        o.set_source(f, g)
        assert inf.status == orc.OK and relerr(X, o.serial(u0)) < 1e-8, i
