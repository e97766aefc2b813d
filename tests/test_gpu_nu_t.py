"""GPU: a time-dependent operator, constant on each slice (pit_set_nu_t), in
1D: the diffusion coefficient of slice n is nu * s_n, so row n of the
all-at-once operator carries F_{n-1} and the sweep G_{n-1} (Sec. 2, eqs.
(Cauchy) and (Cauchyn)).  Checked through the C ABI against the oracle
with the same per-slice factors: the operators to 1e-12 relative (FP64),
Algorithm 1 with the same iteration count and 1e-10, the FP32-fine form
within 1e-5 of the FP64 serial trajectory, parareal exact at k = N, and an
instance alone and in a batch with identical bits.  With every s_n = 1 the
results are bit for bit those of the constant operator.
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


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def factors(N, seed=1):
    """Seeded per-slice factors in [0.3, 3]."""
    return np.exp(np.random.default_rng(seed).uniform(np.log(0.3), np.log(3.0), N))


def both(p, s):
    from paper_2203_10148_amd import pitsbicg as P

    c = P.Context(p)
    c.set_nu_t(s)
    o = orc.Oracle(**p.oracle_kwargs())
    o.set_nu_t(s)
    return c, o


def p1d(M, bc, N, m, fine=wl.CN, c=2, coarse=wl.IE, nu=1e-3, a=1.0, prec=wl.F64, T=1.0, name=""):
    return wl.Problem(dim=1, M=(M, 1), bc=bc, nu=nu, adv=(a if bc == wl.PERIODIC else 0.0, 0.0), T=T, N=N, m=m,
                      fine=fine, c=c, coarse=coarse, prec=prec, tol=1e-10, name=name)


OPS = [
    wl.C1.with_(name="heat64"),                                      # IE Dirichlet, one wave
    p1d(1000, wl.PERIODIC, 6, 9, name="p1000"),                       # CN periodic, ragged, 2 waves
    p1d(777, wl.DIRICHLET, 5, 7, fine=wl.CN, coarse=wl.CN, c=3, nu=2e-3, name="d777"),
    wl.C2.with_(N=12, m=20, T=wl.C2.T * 12 / 256, prec=wl.F64, name="c2_12"),  # the 4096-point line
    p1d(12000, wl.PERIODIC, 4, 3, name="p12000"),                     # compact tables, 16 waves
]


@pytest.mark.parametrize("p", OPS, ids=lambda p: p.name)
def test_operators_match_the_oracle(p):
    say(f"nu_t operators {p.name}")
    s = factors(p.N)
    c, o = both(p, s)
    lam = wl.random_block(p, 4)
    d = dev(lam)
    e1 = relerr(host(c.apply_F(d)), o.apply(lam))
    e2 = relerr(host(c.apply_F(d, raw=True)), o.apply_raw(lam))
    yl = host(c.apply_F(d, last=True)).reshape(p.N, -1)[-1]
    e3 = relerr(yl, o.F(lam.reshape(p.N, -1)[-1], p.N - 1))
    e4 = relerr(host(c.coarse_sweep(d)), o.sweep(lam))
    print(f"apply {e1:.2e} raw {e2:.2e} last {e3:.2e} sweep {e4:.2e}", flush=True)
    assert e1 < 1e-12 and e2 < 1e-12 and e3 < 1e-12 and e4 < 1e-12


def test_unit_factors_are_the_constant_operator_bit_for_bit():
    from paper_2203_10148_amd import pitsbicg as P

    say("nu_t with s = 1")
    p = OPS[1]
    c0 = P.Context(p)
    c1 = P.Context(p)
    c1.set_nu_t(np.ones(p.N))
    d = dev(wl.random_block(p, 6))
    assert torch.equal(c0.apply_F(d), c1.apply_F(d))
    assert torch.equal(c0.coarse_sweep(d), c1.coarse_sweep(d))
    u0 = dev(wl.u0_fourier(p, 3))
    X0, i0 = c0.solve(u0, tol=1e-10)
    X1, i1 = c1.solve(u0, tol=1e-10)
    assert i0.iters == i1.iters and torch.equal(X0, X1)
    c1.set_nu_t(None)
    assert torch.equal(c0.apply_F(d), c1.apply_F(d))


@pytest.mark.parametrize("p", OPS[:4], ids=lambda p: p.name)
def test_solve_matches_the_oracle(p):
    say(f"nu_t solve {p.name}")
    s = factors(p.N, 2)
    c, o = both(p, s)
    u0 = wl.u0_for(p) if p.name == "heat64" else wl.u0_fourier(p, 5)
    X, ig = c.solve(dev(u0), tol=1e-10)
    Xo, io = o.pitsbicg(u0, tol=1e-10)
    serial = o.serial(u0)
    print(f"iters gpu {ig.iters} oracle {io.iters}; vs oracle {relerr(host(X), Xo):.2e}, "
          f"vs serial {relerr(host(X), serial):.2e}", flush=True)
    assert ig.status == io.status == orc.OK
    assert ig.iters == io.iters and ig.matvecs == io.matvecs
    assert relerr(host(X), Xo) < 1e-10
    assert relerr(Xo, serial) < 1e-8


def test_fp32_fine_solve_within_1e_5_of_the_fp64_trajectory():
    """The 4096-point workload's first 32 slices with per-slice factors,
    FP32 fine: every slice within 1e-5 of the FP64 serial trajectory, and no
    further from it than three times the oracle's FP32 emulation plus 1e-7."""
    say("nu_t fp32 solve")
    p = wl.C2.with_(N=32, T=wl.C2.T * 32 / 256, prec=wl.F32)
    s = factors(p.N, 3)
    c, o = both(p, s)
    u0 = wl.u0_for(p)
    X, ig = c.solve(dev(u0), tol=1e-8, stall_window=10)
    serial = o.serial(u0)
    o32 = orc.Oracle(**p.oracle_kwargs())
    o32.set_nu_t(s)
    o32.set_fine_f32(True)
    emul = relerr(o32.serial(u0), serial)
    Xg = host(X).reshape(p.N, -1)
    S = serial.reshape(p.N, -1)
    worst = max(relerr(Xg[n], S[n]) for n in range(p.N))
    e = relerr(Xg, S)
    print(f"status {ig.status} iters {ig.iters}: block {e:.2e}, worst slice {worst:.2e}, "
          f"oracle FP32 emulation {emul:.2e}", flush=True)
    from paper_2203_10148_amd import pitsbicg as P

    assert ig.status in (P.OK, P.ENOCONV) and ig.res_norm <= 1e-6
    assert e < 1e-5 and worst < 1e-5
    assert e < 3 * emul + 1e-7


def test_parareal_is_exact_at_k_equals_n():
    from paper_2203_10148_amd import pitsbicg as P

    say("nu_t parareal")
    p = OPS[1]
    s = factors(p.N, 4)
    c, o = both(p, s)
    u0 = wl.u0_fourier(p, 8)
    X, info = c.parareal(dev(u0), max_iter=p.N)
    serial = o.serial(u0)
    assert info.status in (P.OK, P.ENOCONV)
    assert relerr(host(X), serial) < 1e-12


def test_alone_equals_batched_bitwise():
    """Instances with per-slice operators (and one without) in one batch: the
    same bits as each alone, and as pit_solve's iteration count."""
    from paper_2203_10148_amd import pitsbicg as P

    say("nu_t batch")
    probs = [OPS[1], OPS[2], OPS[3], wl.C1]
    ctxs, u0s = [], []
    for i, p in enumerate(probs):
        c = P.Context(p)
        if i < 3:
            c.set_nu_t(factors(p.N, 10 + i))
        ctxs.append(c)
        u0s.append(dev(wl.u0_for(p) if p.name.startswith("c1_") or p.name == "heat64" else wl.u0_fourier(p, 9)))
    Xs, infos = P.Batch(len(probs)).solve(ctxs, u0s, tol=1e-10)
    for i, (c, u0) in enumerate(zip(ctxs, u0s)):
        Xa, ia = P.Batch(1).solve([c], [u0], tol=1e-10)
        _, isolve = c.solve(u0, tol=1e-10)
        assert ia[0].iters == infos[i].iters == isolve.iters
        assert torch.equal(Xa[0], Xs[i]), i
