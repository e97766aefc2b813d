"""GPU: 2D PR-ADI with a velocity field, constant plus a rigid rotation about
the domain centre (the advection-diffusion-reaction test of Sec. 4,
u = [-y, x]), through the C ABI, against the oracle (whose per-line operators
are pinned by dense matrices and by the direction of the rotation in
test_oracle_pins.py):
  * apply_F (plain, RAW, LAST) and the coarse sweep, FP64 1e-12;
  * pit_solve: Algorithm 1's iterations (within 1) and the serial trajectory
    (1e-10 at tol 1e-12), also with a source term;
  * parareal; graph replay vs eager launches; batched equals alone bitwise.
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


CASES = {
    # the paper's grid and coefficients, shortened in time
    "f2_short": wl.F2.with_(T=0.4, N=4, m=25),
    # rectangle, constant velocity plus rotation, two coarse steps
    "rect": wl.Problem(dim=2, M=(24, 20), length=(1.0, 1.3), bc=wl.DIRICHLET, nu=0.03, adv=(0.3, -0.2),
                       react=0.2, rot=0.7, T=0.5, N=5, m=6, fine=wl.ADI, c=2, coarse=wl.ADI, name="rect"),
    # more lines than one 64-thread block along both axes, ragged
    "wide": wl.Problem(dim=2, M=(130, 70), bc=wl.DIRICHLET, nu=0.02, react=0.5, rot=1.0, T=0.3, N=3, m=4,
                       fine=wl.ADI, c=1, coarse=wl.ADI, name="wide"),
    # degenerate sizes: the smallest grid, one slice (the apply has no
    # slice to propagate, the sweep copies)
    "tiny": wl.Problem(dim=2, M=(3, 3), bc=wl.DIRICHLET, nu=0.05, adv=(0.3, -0.1), react=0.5, rot=1.0, T=0.2,
                       N=3, m=2, fine=wl.ADI, c=1, coarse=wl.ADI, name="tiny"),
    "one_slice": wl.F2.with_(T=0.1, N=1, m=10, name="one_slice"),
    # column walks over two wavefronts, fields and tables in LDS
    "cols70": wl.Problem(dim=2, M=(70, 20), bc=wl.DIRICHLET, nu=0.02, adv=(0.1, 0.2), react=0.3, rot=1.5, T=0.3,
                         N=4, m=3, fine=wl.ADI, c=2, coarse=wl.ADI, name="cols70"),
    # fields in LDS, tables read from global memory
    "mid": wl.Problem(dim=2, M=(80, 66), bc=wl.DIRICHLET, nu=0.02, adv=(-0.1, 0.2), react=0.5, rot=1.0, T=0.3,
                      N=3, m=3, fine=wl.ADI, c=2, coarse=wl.ADI, name="mid"),
    # too large for a slice in LDS: the half-step kernels
    "big": wl.Problem(dim=2, M=(150, 100), bc=wl.DIRICHLET, nu=0.02, adv=(0.2, 0.1), react=0.5, rot=1.0, T=0.3,
                      N=3, m=3, fine=wl.ADI, c=2, coarse=wl.ADI, name="big"),
}


@pytest.mark.parametrize("lds", ["1", "0"], ids=["lds", "halfsteps"])
@pytest.mark.parametrize("case", list(CASES))
def test_velocity_operators_match_oracle(case, lds, monkeypatch):
    """Whole slices in LDS (when they fit) and the half-step kernels."""
    P = P_()
    p = CASES[case]
    monkeypatch.setenv("PIT_VEL_LDS", lds)
    say(f"velocity operators {case} lds={lds}")
    o = orc.Oracle(**p.oracle_kwargs())
    c = P.Context(p)
    lam = wl.random_block(p, 17)
    d = dev(lam)
    assert relerr(host(c.apply_F(d)), o.apply(lam)) < 1e-12
    assert relerr(host(c.apply_F(d, raw=True)), o.apply_raw(lam)) < 1e-12
    yl = host(c.apply_F(d, last=True)).reshape(p.N, -1)
    assert relerr(yl[-1], o.apply_raw(lam).reshape(p.N, -1)[-1]) < 1e-12
    assert relerr(host(c.coarse_sweep(d)), o.sweep(lam)) < 1e-12
    d2 = dev(lam)
    c.coarse_sweep(d2, d2)  # in place
    assert relerr(host(d2), o.sweep(lam)) < 1e-12


@pytest.mark.parametrize("case", list(CASES))
def test_velocity_solve_matches_oracle(case):
    P = P_()
    p = CASES[case]
    say(f"velocity solve {case}")
    o = orc.Oracle(**p.oracle_kwargs())
    u0 = wl.u0_gaussian(p)
    _, io = o.pitsbicg(u0, tol=1e-10)
    c = P.Context(p)
    _, ig = c.solve(dev(u0), tol=1e-10)
    print(f"iters gpu {ig.iters} oracle {io.iters}", flush=True)
    assert ig.status == io.status == orc.OK and abs(ig.iters - io.iters) <= 1
    Xg, ig = c.solve(dev(u0), tol=1e-12)
    assert ig.status == orc.OK and relerr(host(Xg), o.serial(u0)) < 1e-10


def test_velocity_with_source_and_parareal():
    P = P_()
    p = CASES["rect"]
    say("velocity + source, parareal")
    X, Y = wl.grid_2d(p)
    f = (np.sin(math.pi * X) * (1.0 + Y)).reshape(-1)
    o = orc.Oracle(**p.oracle_kwargs(), source=f)
    u0 = wl.u0_gaussian(p)
    serial = o.serial(u0)
    c = P.Context(p)
    c.set_source(f)
    assert relerr(host(c.apply_F(dev(np.zeros(p.N * p.npts)), raw=True)).reshape(p.N, -1)[0], o.forced()) < 1e-12
    Xg, ig = c.solve(dev(u0), tol=1e-12)
    assert ig.status == orc.OK and relerr(host(Xg), serial) < 1e-10
    Xp, ip = c.parareal(dev(u0))
    assert relerr(host(Xp), serial) < 1e-10


def test_velocity_graphs_equal_eager_launches(monkeypatch):
    """The per-half-step kernels run as captured HIP graphs (the whole-slice
    LDS kernels launch directly): replays give the bits of eager launches."""
    P = P_()
    p = CASES["rect"]
    say("velocity graphs vs eager")
    monkeypatch.setenv("PIT_VEL_LDS", "0")
    lam = dev(wl.random_block(p, 5))
    c = P.Context(p)
    ys = [host(c.apply_F(lam)) for _ in range(3)]
    zs = [host(c.coarse_sweep(lam)) for _ in range(3)]
    monkeypatch.setenv("PIT_GRAPHS", "0")
    ye, ze = host(c.apply_F(lam)), host(c.coarse_sweep(lam))
    for y, z in zip(ys, zs):
        assert np.array_equal(y, ye) and np.array_equal(z, ze)


def test_velocity_batched_equals_alone():
    P = P_()
    say("velocity batch")
    probs = [CASES["rect"], CASES["f2_short"], wl.C1]

    def run(idx):
        ctxs = [P.Context(probs[i]) for i in idx]
        u0s = [dev(wl.u0_gaussian(probs[i]) if probs[i].dim == 2 else wl.u0_for(probs[i])) for i in idx]
        Xs, infos = P.Batch(len(idx)).solve(ctxs, u0s, tol=1e-10)
        return [host(X) for X in Xs], infos

    Xs, infos = run([0, 1, 2])
    for i, (X, inf) in enumerate(zip(Xs, infos)):
        Xa, ia = run([i])
        assert ia[0].iters == inf.iters and np.array_equal(Xa[0], X)
