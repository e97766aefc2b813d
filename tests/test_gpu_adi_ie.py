"""GPU: the 2D backward-Euler splitting (PIT_ADI_IE, the paper's time
marching in 2D) through the C ABI against the oracle, whose scheme is pinned
by the dense product of the two factors and modal closed forms: the
shared-table kernels (FP64 and FP32 fields), the whole-slice LDS kernels
with and without the rotating velocity, the per-half-step kernels, PR-ADI
and backward Euler mixed as fine and coarse, and a source (constant and
separable in time)."""
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


IE = wl.ADI_IE
CASES = {
    # (problem, PIT_VEL_LDS): the path each takes is asserted from the kernel shape
    "shared_f64": (wl.Problem(dim=2, M=(100, 70), length=(1.0, 0.7), nu=0.05, react=1.5, T=0.3, N=4, m=4,
                              fine=IE, c=1, coarse=IE), "1"),
    "shared_f32": (wl.Problem(dim=2, M=(100, 70), length=(1.0, 0.7), nu=0.05, react=1.5, T=0.3, N=4, m=4,
                              fine=IE, c=1, coarse=IE, prec=wl.F32), "1"),
    "shared_small": (wl.F3_DR.with_(fine=IE, coarse=IE, N=5, m=20, T=0.1, name="dr_shared"), "0"),
    "lds": (wl.F3_DR.with_(fine=IE, coarse=IE, N=5, m=20, T=0.1, name="dr_lds"), "1"),
    "lds_rot": (wl.F2.with_(fine=IE, coarse=IE, N=5, m=20, T=0.4, name="f2_ie"), "1"),
    "halfsteps_rot": (wl.F2.with_(fine=IE, coarse=IE, N=5, m=20, T=0.4, name="f2_ie_hs"), "0"),
    "mixed_pr_fine": (wl.F2.with_(fine=wl.ADI, coarse=IE, c=2, N=5, m=20, T=0.4, name="f2_mixed"), "1"),
}
PATH = {"shared_f64": "shared", "shared_f32": "shared", "shared_small": "shared", "lds": "lds",
        "lds_rot": "lds", "halfsteps_rot": "lines", "mixed_pr_fine": "lds"}


def check_path(ctx, want):
    sh = ctx.kernel_shape()
    got = "lines" if sh[0] == 1 and sh[2] == 0 else ("lds" if sh[0] == 1 else "shared")
    assert got == want, sh


@pytest.mark.parametrize("case", list(CASES))
def test_adi_ie_operators_and_solve_match_oracle(case, monkeypatch):
    from paper_2203_10148_amd import pitsbicg as P

    p, lds = CASES[case]
    monkeypatch.setenv("PIT_VEL_LDS", lds)
    say(f"backward-Euler splitting {case}")
    o = orc.Oracle(**p.oracle_kwargs())
    c = P.Context(p)
    check_path(c, PATH[case])
    f64 = p.prec == wl.F64
    tol = 1e-12 if f64 else 1e-5
    lam = wl.random_block(p, 41)
    d = dev(lam)
    assert relerr(host(c.apply_F(d)), o.apply(lam)) < tol
    assert relerr(host(c.apply_F(d, raw=True)), o.apply_raw(lam)) < tol
    assert relerr(host(c.coarse_sweep(d)), o.sweep(lam)) < 1e-12
    u0 = wl.u0_gaussian(p)
    serial = o.serial(u0)
    if f64:
        _, io = o.pitsbicg(u0, tol=1e-10)
        _, ig = c.solve(dev(u0), tol=1e-10)
        print(f"iters gpu {ig.iters} oracle {io.iters}", flush=True)
        assert ig.status == io.status == orc.OK and abs(ig.iters - io.iters) <= 1
        X, ig = c.solve(dev(u0), tol=1e-12)
        assert ig.status == orc.OK and relerr(host(X), serial) < 1e-10
    else:
        X, ig = c.solve(dev(u0), tol=1e-8, stall_window=10)
        assert relerr(host(X), serial) < 1e-5


@pytest.mark.parametrize("case", ["shared_f64", "lds_rot"])
@pytest.mark.parametrize("timed", [False, True], ids=["constant", "separable"])
def test_adi_ie_source_matches_oracle(case, timed, monkeypatch):
    from paper_2203_10148_amd import pitsbicg as P

    p, lds = CASES[case]
    monkeypatch.setenv("PIT_VEL_LDS", lds)
    say(f"backward-Euler splitting with a source {case} timed={timed}")
    f = wl.source_bumps(p, 43)
    g = wl.source_profile(p, 44) if timed else None
    o = orc.Oracle(**p.oracle_kwargs())
    o.set_source(f, g)
    c = P.Context(p, bind=False)
    c.set_source(f, g)
    c.bind()
    zeros = dev(np.zeros(p.N * p.npts))
    yb = host(c.apply_F(zeros, raw=True)).reshape(p.N, -1)
    assert max(relerr(yb[n], o.forced(n)) for n in range(p.N)) < 1e-12
    u0 = wl.u0_gaussian(p)
    X, ig = c.solve(dev(u0), tol=1e-12)
    assert ig.status == orc.OK and relerr(host(X), o.serial(u0)) < 1e-10
