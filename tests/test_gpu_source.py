"""GPU: the source term constant in time (pit_set_source), through the C ABI.

With a source f the slice propagator is affine, F(u) = F0(u) + b with
b = F(0), and the all-at-once system keeps its linear operator with
B = (u0, b, .., b) (Sec. 2, eqs. (Cauchy) and (algebraiclinearsystem)).
Checked against the oracle, whose source handling is pinned by modal closed
forms in test_oracle_pins.py:
  * the forced response b (apply_F RAW on zeros), FP64 1e-12;
  * apply_F RAW / LAST (affine) and plain (linear), FP64 1e-12;
  * pit_solve: the iterations of the oracle's Algorithm 1 (within 1) and the
    serial trajectory (FP64 1e-10 at tol 1e-12; FP32 fine 1e-5);
  * pit_parareal and batched solves; alone vs batched bitwise.
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
        return wl.C1.with_(name="c1_src")
    if case in ("p_cn", "p_cn_f32"):
        return wl.Problem(dim=1, M=(1000, 1), bc=wl.PERIODIC, nu=2e-3, adv=(0.7, 0.0), react=0.1, T=0.5, N=8,
                          m=20, fine=wl.CN, c=2, coarse=wl.IE, prec=wl.F32 if case.endswith("f32") else wl.F64)
    if case == "p_long":  # compact FP64 line tables (above 8192 points)
        return wl.Problem(dim=1, M=(9001, 1), bc=wl.PERIODIC, nu=2e-3, adv=(0.5, 0.0), T=0.5, N=3, m=4,
                          fine=wl.IE, c=2, coarse=wl.IE)
    if case in ("adi", "adi_f32"):
        return wl.Problem(dim=2, M=(40, 30), bc=wl.DIRICHLET, nu=0.05, react=0.2, T=0.2, N=4, m=5,
                          fine=wl.ADI, c=1, coarse=wl.ADI, prec=wl.F32 if case.endswith("f32") else wl.F64)
    raise KeyError(case)


def source_and_u0(p):
    if p.dim == 1:
        x = wl.grid_1d(p)
        f = 2.0 * np.exp(-((x - 0.35) ** 2) / 0.004) - 0.5 * np.cos(2 * math.pi * x) + 0.3
        u0 = wl.u0_sines(p) if p.bc == wl.DIRICHLET else wl.u0_fourier(p, 11)
    else:
        X, Y = wl.grid_2d(p)
        f = (np.sin(math.pi * X) * (1 + Y) + 0.2 * np.cos(3 * math.pi * Y)).reshape(-1)
        u0 = wl.u0_bumps(p, 5)
    return f, u0


CASES = ["d_ie", "p_cn", "p_cn_f32", "p_long", "adi", "adi_f32"]


@pytest.mark.parametrize("case", CASES)
def test_source_operators_and_solve_match_oracle(case):
    P = P_()
    p = problem(case)
    say(f"source {case}")
    f, u0 = source_and_u0(p)
    o = orc.Oracle(**p.oracle_kwargs(), source=f)
    f64 = p.prec == wl.F64
    # one context gets the source after binding, one before
    c = P.Context(p)
    c.set_source(f)
    cb = P.Context(p, bind=False)
    cb.set_source(f)
    cb.bind()
    zeros = dev(np.zeros(p.N * p.npts))
    b = o.forced()
    for ctx in (c, cb):
        yb = host(ctx.apply_F(zeros, raw=True)).reshape(p.N, -1)
        assert max(relerr(yb[n], b) for n in range(p.N)) < 1e-12
    lam = wl.random_block(p, 91)
    if f64:
        assert relerr(host(c.apply_F(dev(lam), raw=True)), o.apply_raw(lam)) < 1e-12
        assert relerr(host(c.apply_F(dev(lam))), o.apply(lam)) < 1e-12  # the system operator stays linear
        yl = host(c.apply_F(dev(lam), last=True)).reshape(p.N, -1)
        assert relerr(yl[-1], o.apply_raw(lam).reshape(p.N, -1)[-1]) < 1e-12
    serial, uT = o.serial(u0, want_uT=True)
    if f64:
        _, io = o.pitsbicg(u0, tol=1e-10)
        Xg, ig = c.solve(dev(u0), tol=1e-10)
        print(f"iters gpu {ig.iters} oracle {io.iters}", flush=True)
        assert ig.status == io.status == orc.OK and abs(ig.iters - io.iters) <= 1
        Xg, ig = c.solve(dev(u0), tol=1e-12)
        err = relerr(host(Xg), serial)
        assert ig.status == orc.OK and err < 1e-10
    else:
        Xg, ig = c.solve(dev(u0), tol=1e-8, stall_window=10)
        err = relerr(host(Xg), serial)
        assert ig.status in (orc.OK, orc.ENOCONV) and err < 1e-5
    print(f"{case}: status {ig.status} iters {ig.iters} vs serial {err:.2e}", flush=True)
    # u(T) = F(lambda_{N-1}), the source included
    yT = host(c.apply_F(Xg, last=True)).reshape(p.N, -1)[-1]
    assert relerr(yT, uT) < (1e-10 if f64 else 1e-5)


def test_source_removed_gives_the_linear_problem_back():
    P = P_()
    p = problem("p_cn")
    say("source removed")
    f, u0 = source_and_u0(p)
    c = P.Context(p)
    c.set_source(f)
    c.set_source(None)
    ref = P.Context(p)
    lam = dev(wl.random_block(p, 3))
    assert np.array_equal(host(c.apply_F(lam, raw=True)), host(ref.apply_F(lam, raw=True)))
    X1, _ = c.solve(dev(u0), tol=1e-10)
    X2, _ = ref.solve(dev(u0), tol=1e-10)
    assert np.array_equal(host(X1), host(X2))


@pytest.mark.parametrize("case", ["p_cn", "adi"])
def test_source_parareal_reaches_the_serial_trajectory(case):
    P = P_()
    p = problem(case)
    say(f"source parareal {case}")
    f, u0 = source_and_u0(p)
    o = orc.Oracle(**p.oracle_kwargs(), source=f)
    c = P.Context(p)
    c.set_source(f)
    X, info = c.parareal(dev(u0))
    assert relerr(host(X), o.serial(u0)) < 1e-10


def test_source_batched_equals_alone_and_oracle():
    P = P_()
    say("source batch")
    probs = [problem("p_cn"), problem("d_ie"), problem("adi")]
    srcs = [source_and_u0(p)[0] for p in probs]
    srcs[1] = None  # one instance without a source

    def run(idx):
        ctxs, u0s = [], []
        for i in idx:
            cx = P.Context(probs[i])
            if srcs[i] is not None:
                cx.set_source(srcs[i])
            ctxs.append(cx)
            u0s.append(dev(source_and_u0(probs[i])[1]))
        Xs, infos = P.Batch(len(idx)).solve(ctxs, u0s, tol=1e-10)
        return [host(X) for X in Xs], infos

    Xs, infos = run([0, 1, 2])
    for i, (X, inf) in enumerate(zip(Xs, infos)):
        Xa, ia = run([i])
        assert ia[0].iters == inf.iters and np.array_equal(Xa[0], X)
        p = probs[i]
        o = orc.Oracle(**p.oracle_kwargs(), source=srcs[i])
        assert inf.status == orc.OK and relerr(X, o.serial(source_and_u0(p)[1])) < 1e-8
