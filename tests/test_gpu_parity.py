"""GPU parity: libpitsbicg (through its C ABI) against the CPU oracle.

Operators (all-at-once apply, coarse sweep) are compared element by element
on seeded inputs at sizes that span several per-thread chunks, several
wavefronts and a ragged tail; the full 4096 x 256 workload is compared on
sampled slices the oracle computes one by one.  The FP64 bar is 1e-12
relative for one operator application and 1e-10 relative (same iteration
count) for a whole solve.
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


def ctx(p, **kw):
    from paper_2203_10148_amd import pitsbicg as P

    return P.Context(p, **kw)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def make_oracle(p):
    return orc.Oracle(**p.oracle_kwargs())


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

OP_CASES = [
    # (M, bc, fine, coarse, c, N, m)
    (64, wl.DIRICHLET, wl.IE, wl.IE, 1, 16, 64),      # the 64-point heat workload
    (3, wl.DIRICHLET, wl.IE, wl.IE, 1, 3, 2),         # smallest line
    (5, wl.PERIODIC, wl.CN, wl.IE, 2, 4, 3),
    (63, wl.PERIODIC, wl.CN, wl.IE, 2, 5, 4),
    (65, wl.DIRICHLET, wl.CN, wl.CN, 2, 4, 5),
    (200, wl.PERIODIC, wl.IE, wl.IE, 1, 3, 7),
    (1000, wl.PERIODIC, wl.CN, wl.IE, 2, 4, 6),       # ragged: 1000 on 128 x 8
    (1023, wl.DIRICHLET, wl.CN, wl.IE, 2, 3, 4),
    (4096, wl.PERIODIC, wl.CN, wl.IE, 2, 4, 5),
    (5000, wl.PERIODIC, wl.CN, wl.IE, 2, 3, 3),       # 1024 threads, ragged
    (16384, wl.DIRICHLET, wl.IE, wl.IE, 1, 3, 2),     # largest line
    # lines above 8192 points: compact solver tables, 16 waves combined by a lane scan
    (12345, wl.PERIODIC, wl.CN, wl.IE, 2, 3, 3),
    (9001, wl.PERIODIC, wl.IE, wl.IE, 2, 3, 4),
    (16384, wl.PERIODIC, wl.IE, wl.CN, 1, 3, 2),
    (8193, wl.DIRICHLET, wl.CN, wl.IE, 2, 3, 3),      # one point past the register form
]


def op_problem(M, bc, fine, coarse, c, N, m):
    adv = 0.7 if bc == wl.PERIODIC else 0.3
    return wl.Problem(dim=1, M=(M, 1), bc=bc, nu=2e-3, adv=(adv, 0.0), react=0.1, T=0.5, N=N,
                      m=m, fine=fine, c=c, coarse=coarse, prec=wl.F64)


@pytest.mark.parametrize("case", OP_CASES, ids=lambda c: f"M{c[0]}_bc{c[1]}_f{c[2]}_N{c[5]}_m{c[6]}")
def test_apply_and_sweep_match_oracle(case):
    p = op_problem(*case)
    say(f"apply/sweep {case}")
    o = make_oracle(p)
    c = ctx(p)
    lam = wl.random_block(p, 1234 + case[0])
    d = dev(lam)
    y = host(c.apply_F(d))
    assert relerr(y, o.apply(lam)) < 1e-12
    yr = host(c.apply_F(d, raw=True))
    assert relerr(yr, o.apply_raw(lam)) < 1e-12
    # PIT_APPLY_LAST: only slice N-1 is written, F(lam_{N-1})
    mark = dev(np.full(p.N * p.npts, 7.0))
    yl = host(c.apply_F(d, mark, last=True)).reshape(p.N, -1)
    yo = o.apply_raw(lam).reshape(p.N, -1)
    assert relerr(yl[-1], yo[-1]) < 1e-12
    assert np.all(yl[:-1] == 7.0)
    z = host(c.coarse_sweep(d))
    assert relerr(z, o.sweep(lam)) < 1e-12
    # in place
    d2 = dev(lam)
    c.coarse_sweep(d2, d2)
    assert relerr(host(d2), o.sweep(lam)) < 1e-12


SHAPES = [(64, 1), (64, 2), (64, 4), (64, 8), (128, 8), (256, 4), (256, 8), (256, 16), (512, 4),
          (512, 8), (512, 16), (1024, 4), (1024, 8), (1024, 16)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"NT{s[0]}_C{s[1]}")
def test_every_line_shape(shape, monkeypatch):
    NT, C = shape
    M = NT * C - 3 if NT * C > 8 else NT * C
    monkeypatch.setenv("PIT_LINE_SHAPE", f"{NT},{C}")
    p = op_problem(M, wl.PERIODIC, wl.CN, wl.IE, 2, 3, 3)
    say(f"shape NT={NT} C={C} M={M}")
    c = ctx(p)
    assert c.kernel_shape() == (NT, C, NT, C)
    o = make_oracle(p)
    lam = wl.random_block(p, 77)
    d = dev(lam)
    assert relerr(host(c.apply_F(d)), o.apply(lam)) < 1e-12
    assert relerr(host(c.coarse_sweep(d)), o.sweep(lam)) < 1e-12


@pytest.mark.parametrize("shape", [(64, 1), (64, 2), (128, 8), (256, 4), (256, 16), (512, 8), (512, 16), (1024, 4),
                                   (1024, 8), (1024, 16)],
                         ids=lambda s: f"NT{s[0]}_C{s[1]}")
def test_solve_every_layout(shape, monkeypatch):
    """pit_solve keeps its vectors in the chunked layout of the line shape
    (pairs of points per lane, single points at C = 1, padded to NT*C
    points); a ragged line exercises the padding.  The shapes cover the
    sweep's two-buffer prefetch (C <= 8, NT*C <= 4096), its one-buffer
    prefetch with an L2 touch (C = 16, or 1024 threads) and the compact
    solver tables (1024 x 16)."""
    NT, C = shape
    M = NT * C - 5
    monkeypatch.setenv("PIT_LINE_SHAPE", f"{NT},{C}")
    p = wl.Problem(dim=1, M=(M, 1), bc=wl.PERIODIC, nu=2e-3, adv=(0.8, 0.0), T=0.6, N=6, m=4,
                   fine=wl.CN, c=2, coarse=wl.IE, prec=wl.F64)
    say(f"solve layout NT={NT} C={C} M={M}")
    o = make_oracle(p)
    u0 = wl.u0_fourier(p, 5)
    Xo, io = o.pitsbicg(u0, tol=1e-10)
    c = ctx(p)
    assert c.kernel_shape() == (NT, C, NT, C)
    Xg, ig = c.solve(dev(u0), tol=1e-10)
    Xg = host(Xg)
    assert ig.status == io.status == orc.OK
    assert abs(ig.iters - io.iters) <= 1
    assert relerr(Xg, Xo) < 1e-9
    assert relerr(Xg, o.serial(u0)) < 1e-9


IE_SPREAD = [
    # (NT, C, c, bc, M, N): the implicit-Euler sweep with interleaved traffic
    # (8 or 16 points per lane, two or more waves), one solve per slice and more
    (256, 16, 1, wl.PERIODIC, 4096, 6),
    (256, 16, 1, wl.DIRICHLET, 4001, 5),
    (256, 16, 2, wl.DIRICHLET, 4096, 6),
    (256, 16, 3, wl.PERIODIC, 3001, 5),
    (256, 16, 4, wl.DIRICHLET, 2049, 4),
    (256, 16, 2, wl.PERIODIC, 4090, 2),   # one slice step
    (256, 16, 1, wl.PERIODIC, 4096, 1),   # no slice step: z_0 = v_0 only
    (128, 8, 1, wl.PERIODIC, 1000, 5),
    (128, 8, 2, wl.DIRICHLET, 1024, 4),
    (256, 8, 3, wl.PERIODIC, 2047, 4),
    (512, 8, 1, wl.DIRICHLET, 4000, 4),
    (512, 16, 2, wl.PERIODIC, 8000, 4),
    (512, 16, 1, wl.DIRICHLET, 7001, 4),
    (1024, 8, 2, wl.PERIODIC, 8192, 4),
    (1024, 8, 1, wl.PERIODIC, 5003, 4),
]


@pytest.mark.parametrize("case", IE_SPREAD, ids=lambda c: f"NT{c[0]}_C{c[1]}_c{c[2]}_bc{c[3]}_M{c[4]}_N{c[5]}")
def test_ie_sweep_with_interleaved_traffic(case, monkeypatch):
    """The implicit-Euler sweep at 8 or 16 points per lane and two or more
    waves stores z_{n-1} and loads v_n between the phases of slice n's solves
    (out of place first solve; the loads in the second solve, or after the
    stores in the one solve when c = 1).  Against the oracle's sweep, out of
    place and in place, ragged lines and both boundary conditions; then
    Algorithm 1 through pit_solve and through the batch engine's
    multi-instance kernel."""
    from paper_2203_10148_amd import pitsbicg as P

    NT, C, cc, bc, M, N = case
    monkeypatch.setenv("PIT_LINE_SHAPE", f"{NT},{C}")
    p = op_problem(M, bc, wl.CN, wl.IE, cc, N, 2)
    say(f"ie interleaved sweep {case}")
    c = ctx(p)
    assert c.kernel_shape() == (NT, C, NT, C)
    o = make_oracle(p)
    lam = wl.random_block(p, 99 + cc)
    ref = o.sweep(lam)
    assert relerr(host(c.coarse_sweep(dev(lam))), ref) < 1e-12
    d2 = dev(lam)
    c.coarse_sweep(d2, d2)
    assert relerr(host(d2), ref) < 1e-12
    if N < 4:
        return
    u0 = wl.u0_fourier(p, 3)
    Xo, io = o.pitsbicg(u0, tol=1e-10)
    X, ig = c.solve(dev(u0), tol=1e-10)
    assert ig.status == io.status == orc.OK and ig.iters == io.iters
    assert relerr(host(X), Xo) < 1e-10
    Xb, ib = P.Batch(1).solve([c], [dev(u0)], tol=1e-10)
    assert ib[0].iters == ig.iters
    assert relerr(host(Xb[0]), Xo) < 1e-10


def test_serial_trajectory_is_annihilated():
    """F applied to the serial fine trajectory gives (u0, 0, .., 0)."""
    p = wl.C1
    say("serial trajectory residual")
    o = make_oracle(p)
    u0 = wl.u0_for(p)
    lam = o.serial(u0)
    c = ctx(p)
    y = host(c.apply_F(dev(lam))).reshape(p.N, -1)
    assert relerr(y[0], u0) < 1e-15
    assert np.abs(y[1:]).max() < 1e-13 * np.abs(u0).max()


def test_c2_full_size_apply_all_slices():
    """The 4096-point, 256-slice advection-diffusion apply (200 CN steps),
    every slice against the oracle's apply."""
    p = wl.C2.with_(prec=wl.F64)
    say("c2 full apply")
    c = ctx(p)
    o = make_oracle(p)
    lam = wl.random_block(p, 2)
    y = host(c.apply_F(dev(lam)))
    ref = o.apply(lam)
    Y, R = y.reshape(p.N, -1), ref.reshape(p.N, -1)
    assert np.array_equal(Y[0], R[0])
    worst = max(relerr(Y[n], R[n]) for n in range(1, p.N))
    print(f"c2 apply: whole block {relerr(y, ref):.2e}, worst slice {worst:.2e}", flush=True)
    assert relerr(y, ref) < 1e-12 and worst < 1e-12


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

def u0_of(p):
    if p.name.startswith(("c1_", "c2_", "c3_")):
        return wl.u0_for(p)
    return wl.u0_fourier(p, 3) if p.bc == wl.PERIODIC else wl.u0_sines(p)


def compare_solve(p, tol, eps0=1e-30, max_iter=None, norm_mode=orc.ABS, x0_mode=orc.X0_ZERO,
                  X0=None, half_step_check=0):
    o = make_oracle(p)
    u0 = u0_of(p)
    Xo, io = o.pitsbicg(u0, tol=tol, eps0=eps0, max_iter=max_iter, norm_mode=norm_mode,
                        x0_mode=x0_mode, X0=X0, half_step_check=half_step_check)
    c = ctx(p)
    Xg, ig = c.solve(dev(u0), None if X0 is None else dev(X0), tol=tol, restart_tol=eps0,
                     max_iter=max_iter or 0, norm_mode=norm_mode, x0_mode=x0_mode,
                     half_step_check=half_step_check)
    return Xo, io, host(Xg), ig, o, u0


def test_c1_solve_matches_oracle():
    p = wl.C1
    say("c1 solve")
    Xo, io, Xg, ig, o, u0 = compare_solve(p, p.tol)
    assert ig.status == io.status == orc.OK
    assert ig.iters == io.iters and ig.matvecs == io.matvecs
    assert relerr(Xg, Xo) < 1e-10
    assert relerr(Xg, o.serial(u0)) < 1e-9
    h = min(len(ig.history), len(io.history))
    assert np.allclose(ig.history[:h], io.history[:h], rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("opt", ["restart_every", "max_iter1", "x0_coarse", "x0_given", "rel",
                                 "half_step", "tol12"])
def test_solve_options_match_oracle(opt):
    p = wl.C1.with_(N=8)
    say(f"solve option {opt}")
    o = make_oracle(p)
    kw = {"restart_every": dict(eps0=1e30, max_iter=100), "max_iter1": dict(max_iter=1),
          "x0_coarse": dict(x0_mode=orc.X0_COARSE), "rel": dict(norm_mode=orc.REL),
          "half_step": dict(half_step_check=1), "tol12": dict(),
          "x0_given": dict(x0_mode=orc.X0_GIVEN, X0=o.serial(wl.u0_for(p)) * (1 + 1e-3))}[opt]
    tol = 1e-12 if opt == "tol12" else 1e-10
    Xo, io, Xg, ig, o, u0 = compare_solve(p, tol, **kw)
    assert ig.status == io.status
    assert ig.iters == io.iters and ig.matvecs == io.matvecs and ig.restarts == io.restarts
    assert relerr(Xg, Xo) < 1e-10


def test_g_equals_f_and_single_slice():
    say("special cases")
    p = wl.C1.with_(N=8, c=64)
    Xo, io, Xg, ig, o, u0 = compare_solve(p, 1e-12)
    assert ig.iters == 1 and ig.matvecs == 2
    assert relerr(Xg, o.serial(u0)) < 1e-13
    p1 = wl.C1.with_(N=1)
    Xo, io, Xg, ig, o, u0 = compare_solve(p1, 1e-14)
    assert ig.status == orc.OK and ig.iters == 1
    assert relerr(Xg, u0) < 1e-15


PARAREAL_CASES = {
    "heat64": wl.C1,
    "periodic1000": wl.Problem(dim=1, M=(1000, 1), bc=wl.PERIODIC, nu=1e-3, adv=(1.0, 0.0), T=1.0, N=12, m=20,
                               fine=wl.CN, c=2, coarse=wl.IE, prec=wl.F64),
    "adi40x33": wl.Problem(dim=2, M=(40, 33), length=(1.0, 1.0), nu=0.05, T=0.5, N=8, m=8, fine=wl.ADI, c=1,
                           coarse=wl.ADI, prec=wl.F64),
}


@pytest.mark.parametrize("name", sorted(PARAREAL_CASES))
def test_parareal_matches_oracle_and_is_exact_at_n(name):
    """Parareal as preconditioned Richardson (Sec. 2, eq. (pararealAlgebraic)):
    k iterations against the oracle's (iterate and update norms), and N
    iterations against the serial fine trajectory (nilpotency)."""
    p = PARAREAL_CASES[name]
    say(f"parareal {name}")
    o = make_oracle(p)
    u0 = wl.u0_bumps(p, 3) if p.dim == 2 else u0_of(p)
    c = ctx(p)
    k = 3
    Xo, ho = o.parareal_richardson(u0, k)
    Xg, ig = c.parareal(dev(u0), max_iter=k)
    assert ig.status == orc.OK and ig.iters == k and ig.matvecs == k
    assert relerr(host(Xg), Xo) < 1e-12
    assert np.allclose(ig.history, ho, rtol=1e-10, atol=1e-300)
    Xn, inn = c.parareal(dev(u0), max_iter=p.N)
    e = relerr(host(Xn), o.serial(u0))
    print(f"{name}: {k} iterations vs oracle {relerr(host(Xg), Xo):.2e}; N={p.N} iterations vs serial {e:.2e}",
          flush=True)
    assert e < 1e-12
    # with a tolerance: stops after the first update below it
    Xt, it = c.parareal(dev(u0), tol=1e-6)
    assert it.status == orc.OK and it.history[-1] <= 1e-6 and (len(it.history) == 1 or it.history[-2] > 1e-6)
    # from a given iterate (the oracle's X^1) and from the coarse trajectory (= X^1 from zero)
    X1, _ = o.parareal_richardson(u0, 1)
    Xo2, _ = o.parareal_richardson(u0, 2, X0=X1)
    Xg2, _ = c.parareal(dev(u0), dev(X1.copy()), max_iter=2, x0_mode=orc.X0_GIVEN)
    assert relerr(host(Xg2), Xo2) < 1e-12
    Xc2, _ = c.parareal(dev(u0), max_iter=2, x0_mode=orc.X0_COARSE)
    assert relerr(host(Xc2), Xo2) < 1e-12


def test_nan_input_is_a_breakdown():
    from paper_2203_10148_amd import pitsbicg as P

    p = wl.C1
    say("nan input")
    c = ctx(p)
    u0 = wl.u0_for(p)
    u0[5] = np.nan
    _, info = c.solve(dev(u0))
    assert info.status == P.EBREAKDOWN


@pytest.mark.parametrize("M,bc,N", [(1000, wl.PERIODIC, 12), (777, wl.DIRICHLET, 9)])
def test_ragged_solve_matches_oracle(M, bc, N):
    p = wl.Problem(dim=1, M=(M, 1), bc=bc, nu=1e-3, adv=(1.0, 0.0), T=1.0, N=N, m=20, fine=wl.CN,
                   c=2, coarse=wl.IE, prec=wl.F64)
    say(f"ragged solve M={M} bc={bc}")
    Xo, io, Xg, ig, o, u0 = compare_solve(p, 1e-10)
    assert ig.status == io.status == orc.OK
    assert abs(ig.iters - io.iters) <= 1
    assert relerr(Xg, Xo) < 1e-9
    assert relerr(Xg, o.serial(u0)) < 1e-8


def test_c2_full_size_fp64_solve():
    """The 4096 x 256 advection-diffusion workload, FP64, against the oracle's
    Algorithm 1 on the same input.

    At the workload tolerance (1e-8, absolute) two correct runs of Algorithm 1
    that round differently agree only to the level of their remaining error
    (about 1e-9 relative here), so there the checks are the iteration count,
    the stopping residual and agreement to 1e-8.  At tol 1e-12 both runs are
    within 1e-10 of the serial fine trajectory (the exact solution) and of each
    other.
    """
    p = wl.C2.with_(prec=wl.F64)
    say("c2 fp64 full solve")
    o = make_oracle(p)
    u0 = wl.u0_for(p)
    serial = o.serial(u0)
    c = ctx(p)
    Xg, ig = c.solve(dev(u0), tol=p.tol)
    Xg = host(Xg)
    Xo, io = o.pitsbicg(u0, tol=p.tol)
    print(f"tol {p.tol}: gpu iters={ig.iters} ms={ig.ms_total:.1f}  oracle iters={io.iters} "
          f"gpu-vs-oracle {relerr(Xg, Xo):.2e} gpu-vs-serial {relerr(Xg, serial):.2e} "
          f"oracle-vs-serial {relerr(Xo, serial):.2e}", flush=True)
    assert ig.status == io.status == orc.OK
    assert ig.iters == io.iters and ig.matvecs == io.matvecs
    assert ig.res_norm <= p.tol and io.res_norm <= p.tol
    assert relerr(Xg, Xo) < 1e-8 and relerr(Xg, serial) < 1e-7
    Xg, ig = c.solve(dev(u0), tol=1e-12)
    Xg = host(Xg)
    Xo, io = o.pitsbicg(u0, tol=1e-12)
    print(f"tol 1e-12: gpu iters={ig.iters} oracle iters={io.iters} gpu-vs-serial {relerr(Xg, serial):.2e} "
          f"oracle-vs-serial {relerr(Xo, serial):.2e} gpu-vs-oracle {relerr(Xg, Xo):.2e}", flush=True)
    assert ig.status == io.status == orc.OK
    assert relerr(Xg, serial) < 1e-10 and relerr(Xo, serial) < 1e-10
    assert relerr(Xg, Xo) < 1e-10


# ---------------------------------------------------------------------------
# FP32 fine propagator (increment form); coarse sweep and Krylov stay FP64
# ---------------------------------------------------------------------------

F32_CASES = [
    # (M, bc, fine, shape)  -- shapes cover one wave, several waves and padding
    (64, wl.DIRICHLET, wl.IE, (64, 1)),
    (500, wl.PERIODIC, wl.CN, (64, 8)),
    (1000, wl.PERIODIC, wl.CN, (128, 8)),
    (4096, wl.PERIODIC, wl.CN, (256, 16)),
    (4000, wl.DIRICHLET, wl.CN, (512, 8)),
    (3000, wl.PERIODIC, wl.IE, (1024, 4)),
    (16384, wl.PERIODIC, wl.CN, (1024, 16)),
    (10000, wl.PERIODIC, wl.IE, (1024, 16)),
    (9000, wl.DIRICHLET, wl.CN, (1024, 16)),
    # padding that starts at a wave's first lane (its first point gets no
    # right-hand side from the left neighbour): 2 and 16 waves
    (512, wl.PERIODIC, wl.CN, (128, 8)),
    (8192, wl.PERIODIC, wl.IE, (1024, 16)),
]


@pytest.mark.parametrize("case", F32_CASES, ids=lambda c: f"M{c[0]}_bc{c[1]}_f{c[2]}_NT{c[3][0]}_C{c[3][1]}")
def test_fp32_apply_matches_oracle(case, monkeypatch):
    M, bc, fine, (NT, C) = case
    monkeypatch.setenv("PIT_LINE_SHAPE", f"{NT},{C}")
    p = wl.Problem(dim=1, M=(M, 1), bc=bc, nu=2e-3, adv=(0.7, 0.0), react=0.05, T=0.5, N=4, m=50,
                   fine=fine, c=2, coarse=wl.IE, prec=wl.F32)
    say(f"fp32 apply {case}")
    o = make_oracle(p)
    c = ctx(p)
    assert c.kernel_shape()[:2] == (NT, C)
    # A smooth block (the regime of the method) must meet 1e-5.  For a rough
    # block the FP32 rounding of a right-hand side of size ~s*|u| (s = nu dt/h^2,
    # the diffusion number) reaches the smooth modes, which A^{-1} does not
    # damp, so the attainable accuracy scales with s: bound 1e-5 * max(1, s/64).
    x = wl.grid_1d(p)
    h = x[1] - x[0]
    s_diff = p.nu * (p.T / p.N / p.m) / h ** 2
    smooth = np.concatenate([np.sin(2 * np.pi * (n + 1) * x) + 0.3 * np.cos(6 * np.pi * x) for n in range(p.N)])
    for lam, bound in ((smooth, 1e-5), (wl.random_block(p, 31), 1e-5 * max(1.0, s_diff / 64))):
        y = host(c.apply_F(dev(lam)))
        e1 = relerr(y, o.apply(lam))
        yr = host(c.apply_F(dev(lam), raw=True))
        e2 = relerr(yr, o.apply_raw(lam))
        print(f"s={s_diff:.3g} bound={bound:.2e} apply {e1:.2e} raw {e2:.2e}", flush=True)
        assert e1 < bound and e2 < bound


def test_fp32_c2_full_size_solve():
    """The 4096 x 256 advection-diffusion workload with an FP32 fine
    propagator: within 1e-5 (relative, all slices) of the FP64 serial fine
    trajectory, with FP64 dots, scalars and coarse sweep."""
    p = wl.C2.with_(prec=wl.F32)
    say("c2 fp32 full solve")
    o = make_oracle(p)
    u0 = wl.u0_for(p)
    serial = o.serial(u0)
    c = ctx(p)
    Xg, ig = c.solve(dev(u0), tol=p.tol, stall_window=10)
    Xg = host(Xg)
    err = relerr(Xg, serial)
    print(f"fp32: status={ig.status} iters={ig.iters} ms={ig.ms_total:.1f} rel.err vs fp64 serial={err:.2e}",
          flush=True)
    assert ig.status in (orc.OK, orc.ENOCONV)
    assert err < 1e-5


def test_fp32_small_solve_and_final_state():
    p = wl.C1.with_(prec=wl.F32)
    say("c1 fp32 solve")
    o = make_oracle(p)
    u0 = wl.u0_for(p)
    serial, uT = o.serial(u0, want_uT=True)
    c = ctx(p)
    Xg, ig = c.solve(dev(u0), tol=1e-8, stall_window=10)
    assert relerr(host(Xg), serial) < 1e-5
    yl = host(c.apply_F(Xg, last=True)).reshape(p.N, -1)
    assert relerr(yl[-1], uT) < 1e-5


# ---------------------------------------------------------------------------
# 2D Peaceman-Rachford ADI
# ---------------------------------------------------------------------------

ADI_CASES = [
    # (Mx, My, Lx, Ly, N, m, c, prec)
    (24, 20, 1.0, 1.3, 4, 3, 1, wl.F64),
    (100, 70, 1.0, 0.7, 3, 4, 2, wl.F64),
    (64, 128, 1.0, 1.0, 3, 2, 1, wl.F64),
    (130, 257, 1.0, 1.0, 2, 2, 1, wl.F64),
    (512, 512, 1.0, 1.0, 3, 3, 1, wl.F64),
    (100, 70, 1.0, 0.7, 3, 4, 2, wl.F32),
    (512, 512, 1.0, 1.0, 3, 3, 1, wl.F32),
    (300, 600, 1.0, 1.2, 2, 2, 1, wl.F64),     # 600 rows: two row segments per wavefront
    (700, 130, 1.0, 0.8, 2, 3, 2, wl.F64),     # 700-point rows on two wavefronts, ragged
    (1024, 1024, 1.0, 1.0, 2, 4, 1, wl.F32, 1.8e-3),   # largest side; time step of the served 2D requests
]


def adi_problem(Mx, My, Lx, Ly, N, m, c, prec, T=None):
    return wl.Problem(dim=2, M=(Mx, My), length=(Lx, Ly), bc=wl.DIRICHLET, nu=0.05, react=0.2,
                      T=0.05 * N if T is None else T, N=N, m=m, fine=wl.ADI, c=c, coarse=wl.ADI, prec=prec)


@pytest.mark.parametrize("case", ADI_CASES, ids=lambda c: f"{c[0]}x{c[1]}_N{c[4]}_m{c[5]}_c{c[6]}_p{c[7]}"
                         + (f"_T{c[8]}" if len(c) > 8 else ""))
def test_adi_apply_and_sweep_match_oracle(case):
    p = adi_problem(*case)
    say(f"adi apply/sweep {case}")
    o = make_oracle(p)
    c = ctx(p)
    # FP32 storage of the fields between half steps: a smooth block must meet
    # 1e-5.  For a rough block the explicit half of a PR-ADI step amplifies
    # modes rough along one axis by up to 1 + 4*rho (rho = theta nu / h^2) in the
    # intermediate field, whose FP32 rounding then reaches the smooth modes:
    # bound 1e-5 * max(1, rho/16).
    hx, hy = p.length[0] / (p.M[0] + 1), p.length[1] / (p.M[1] + 1)
    rho = 0.5 * (p.T / p.N / p.m) * p.nu / min(hx, hy) ** 2
    rough_tol = 1e-12 if p.prec == wl.F64 else 1e-5 * max(1.0, rho / 16)
    X, Y = wl.grid_2d(p)
    smooth = np.concatenate([(np.sin(np.pi * X / p.length[0]) * np.sin((n + 1) * np.pi * Y / p.length[1])).reshape(-1)
                             for n in range(p.N)])
    for lam, tol in ((smooth, 1e-12 if p.prec == wl.F64 else 1e-5), (wl.random_block(p, 17), rough_tol)):
        d = dev(lam)
        e1 = relerr(host(c.apply_F(d)), o.apply(lam))
        e2 = relerr(host(c.apply_F(d, raw=True)), o.apply_raw(lam))
        yl = host(c.apply_F(d, last=True)).reshape(p.N, -1)
        e3 = relerr(yl[-1], o.F(lam.reshape(p.N, -1)[-1]))
        print(f"rho={rho:.3g} tol={tol:.2e} apply {e1:.2e} raw {e2:.2e} last {e3:.2e}", flush=True)
        assert e1 < tol and e2 < tol and e3 < tol
        assert relerr(host(c.coarse_sweep(d)), o.sweep(lam)) < 1e-12
        d2 = dev(lam)
        c.coarse_sweep(d2, d2)
        assert relerr(host(d2), o.sweep(lam)) < 1e-12


@pytest.mark.parametrize("yshape,reported", [("16,32,1", (1024, 32)), ("16,16,2", (1024, 32)),
                                             ("8,16,2", (512, 32))])
def test_adi_other_y_shapes_on_a_short_column(yshape, reported, monkeypatch):
    """The y shapes the default menu does not pick, forced on a short column
    (rows past the last one inside the last segment), against the oracle."""
    monkeypatch.setenv("PIT_ADI_YSHAPE", yshape)
    rows = 250 if yshape == "8,16,2" else 500
    p = adi_problem(200, rows, 1.0, 1.0, 3, 2, 1, wl.F64)
    say(f"adi y shape {yshape} on 200x{rows}")
    c = ctx(p)
    assert c.kernel_shape()[2:] == reported
    o = make_oracle(p)
    lam = wl.random_block(p, 5)
    assert relerr(host(c.apply_F(dev(lam))), o.apply(lam)) < 1e-12
    assert relerr(host(c.coarse_sweep(dev(lam))), o.sweep(lam)) < 1e-12


@pytest.mark.parametrize("yc", ["", "1", "4", "0"])
@pytest.mark.parametrize("Mx,My,c", [(130, 257, 2), (512, 512, 1), (150, 90, 3), (151, 90, 2)])
def test_adi_sweep_y_kernels(Mx, My, c, yc, monkeypatch):
    """The coarse sweep's single-slice y half step, one column per wavefront
    (the default for columns up to 512 rows, 2 columns per workgroup; 1 and 4
    by PIT_ADI_YC) and the column-strip kernel (PIT_ADI_YC=0), in and out of
    place, against the oracle's forward substitution; c coarse steps per
    slice."""
    if yc:
        monkeypatch.setenv("PIT_ADI_YC", yc)
    else:
        monkeypatch.delenv("PIT_ADI_YC", raising=False)
    p = adi_problem(Mx, My, 1.0, 1.1, 5, 2, c, wl.F64)
    say(f"adi sweep y kernel yc={yc} {Mx}x{My} c={c}")
    cx = ctx(p)
    o = make_oracle(p)
    lam = wl.random_block(p, 23)
    ref = o.sweep(lam)
    e1 = relerr(host(cx.coarse_sweep(dev(lam))), ref)
    d = dev(lam)
    cx.coarse_sweep(d, d)
    e2 = relerr(host(d), ref)
    print(f"sweep vs oracle {e1:.2e}, in place {e2:.2e}", flush=True)
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("Mx,My,c", [(130, 257, 2), (512, 512, 1), (150, 90, 3), (64, 512, 1), (151, 90, 2),
                                    (130, 40, 2)])
def test_adi_sweep_preformed_rhs_is_bitwise(Mx, My, c, monkeypatch):
    """With the one-column y kernel the coarse sweep's x half step stores the
    y half step's right-hand side (I + theta Lx) u* itself: the same bits as
    the y kernel forming it from u* and its neighbour columns
    (PIT_ADI_PRE=0), in and out of place, one and several coarse steps per
    slice, and the same solve.  Even widths move the two columns of a
    workgroup with one 16-byte access per row, odd widths (151) one value at
    a time; 40 rows take one point per lane."""
    monkeypatch.delenv("PIT_ADI_YC", raising=False)
    p = adi_problem(Mx, My, 1.0, 1.1, 5, 2, c, wl.F64)
    say(f"adi sweep pre-formed rhs {Mx}x{My} c={c}")
    monkeypatch.delenv("PIT_ADI_PRE", raising=False)
    c1 = ctx(p)
    monkeypatch.setenv("PIT_ADI_PRE", "0")
    c0 = ctx(p)
    lam = dev(wl.random_block(p, 29))
    z1 = c1.coarse_sweep(lam)
    z0 = c0.coarse_sweep(lam)
    torch.cuda.synchronize()
    assert torch.equal(z0, z1)
    d = lam.clone()
    c1.coarse_sweep(d, d)
    torch.cuda.synchronize()
    assert torch.equal(d, z1)
    u0 = dev(wl.u0_for(p))
    X1, i1 = c1.solve(u0, tol=1e-10)
    X0, i0 = c0.solve(u0, tol=1e-10)
    assert i1.iters == i0.iters and torch.equal(X0, X1)


@pytest.mark.parametrize("Mx,My,prec", [(130, 257, wl.F64), (512, 512, wl.F64), (150, 90, wl.F64),
                                         (700, 130, wl.F64), (777, 65, wl.F64), (100, 70, wl.F32),
                                         (512, 512, wl.F32), (700, 130, wl.F32), (520, 33, wl.F32)])
def test_adi_apply_preformed_rhs(Mx, My, prec, monkeypatch):
    """The fine apply's x half step stores the y half step's right-hand side
    (I + theta Lx) u* itself (PIT_ADI_FPRE=0: it stores u* and the y kernel
    forms the right-hand side from u* and two halo columns); rows of 700
    points run on two wavefronts, whose edge points cross through LDS.  FP64
    fields: the same bits in every apply form and the same solve.  FP32
    fields: the right-hand side is rounded to FP32 where u* was, so the bits
    differ; both forms hold the FP32 bound against the oracle."""
    p = adi_problem(Mx, My, 1.0, 1.1, 4, 3, 1, prec)
    say(f"adi apply pre-formed rhs {Mx}x{My} prec={prec}")
    monkeypatch.delenv("PIT_ADI_FPRE", raising=False)
    c1 = ctx(p)
    monkeypatch.setenv("PIT_ADI_FPRE", "0")
    c0 = ctx(p)
    lam = wl.random_block(p, 31)
    d = dev(lam)
    forms = [dict(), dict(raw=True), dict(last=True)]
    ys = [(host(c1.apply_F(d, **kw)), host(c0.apply_F(d, **kw))) for kw in forms]
    if prec == wl.F64:
        for y1, y0 in ys:
            assert np.array_equal(y1, y0)
        u0 = dev(wl.u0_for(p))
        X1, i1 = c1.solve(u0, tol=1e-10)
        X0, i0 = c0.solve(u0, tol=1e-10)
        assert i1.iters == i0.iters and torch.equal(X0, X1)
        return
    assert not np.array_equal(ys[0][0], ys[0][1])  # the pre-formed path ran
    o = make_oracle(p)
    X, Y = wl.grid_2d(p)
    smooth = np.concatenate([(np.sin(np.pi * X / p.length[0]) * np.sin((n + 1) * np.pi * Y / p.length[1])).reshape(-1)
                             for n in range(p.N)])
    ref = o.apply(smooth)
    for cc in (c1, c0):
        e = relerr(host(cc.apply_F(dev(smooth))), ref)
        print(f"FP32 apply vs oracle {e:.2e}", flush=True)
        assert e < 1e-5


def test_adi_shared_tables_on_a_small_fp64_slice(monkeypatch):
    """The shared-table kernels on a slice that would otherwise take the LDS
    path (PIT_VEL_LDS=0 at creation), against the oracle."""
    monkeypatch.setenv("PIT_VEL_LDS", "0")
    p = adi_problem(24, 20, 1.0, 1.3, 4, 3, 1, wl.F64)
    say("adi shared tables 24x20")
    c = ctx(p)
    assert c.kernel_shape()[0] >= 64
    o = make_oracle(p)
    lam = wl.random_block(p, 19)
    d = dev(lam)
    assert relerr(host(c.apply_F(d)), o.apply(lam)) < 1e-12
    assert relerr(host(c.apply_F(d, raw=True)), o.apply_raw(lam)) < 1e-12
    assert relerr(host(c.coarse_sweep(d)), o.sweep(lam)) < 1e-12


def test_adi_graph_replays_equal_eager_launches(monkeypatch):
    """The 2D apply and sweep run as captured HIP graphs; every replay, with
    other work and synchronisations in between, gives the bits of the eager
    launch sequence (PIT_GRAPHS=0)."""
    p = adi_problem(100, 70, 1.0, 0.7, 4, 3, 2, wl.F32)
    say("adi graph replays")
    lam1, lam2 = dev(wl.random_block(p, 21)), dev(wl.random_block(p, 22))
    monkeypatch.setenv("PIT_GRAPHS", "0")
    ce = ctx(p)
    ref = [host(ce.apply_F(lam1)), host(ce.coarse_sweep(lam1)), host(ce.apply_F(lam2)), host(ce.coarse_sweep(lam2))]
    monkeypatch.delenv("PIT_GRAPHS")
    cg = ctx(p)
    y1, z1 = torch.empty_like(lam1), torch.empty_like(lam1)
    y2, z2 = torch.empty_like(lam2), torch.empty_like(lam2)
    for rep in range(3):
        cg.apply_F(lam1, y1)
        scratch = lam2 * 2.0 + 1.0  # other work on the stream between replays
        cg.coarse_sweep(lam1, z1)
        torch.cuda.synchronize()
        cg.apply_F(lam2, y2)
        cg.coarse_sweep(lam2, z2)
        got = [host(y1), host(z1), host(y2), host(z2)]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
        del scratch


@pytest.mark.parametrize("prec,lds", [(wl.F64, "1"), (wl.F64, "0"), (wl.F32, "1")],
                         ids=["f64_lds", "f64_shared_tables", "f32"])
def test_adi_small_solve_matches_oracle(prec, lds, monkeypatch):
    """FP64 slices that fit in LDS take the per-line whole-slice kernels;
    PIT_VEL_LDS=0 at creation keeps the shared-table kernels."""
    monkeypatch.setenv("PIT_VEL_LDS", lds)
    p = wl.Problem(dim=2, M=(40, 33), length=(1.0, 1.0), nu=0.05, T=0.5, N=8, m=8, fine=wl.ADI, c=1,
                   coarse=wl.ADI, prec=prec)
    say(f"adi small solve prec={prec} lds={lds}")
    o = make_oracle(p)
    u0 = wl.u0_bumps(p, 3)
    Xo, io = o.pitsbicg(u0, tol=1e-10)
    c = ctx(p)
    Xg, ig = c.solve(dev(u0), tol=1e-10 if prec == wl.F64 else 1e-8, stall_window=0 if prec == wl.F64 else 10)
    Xg = host(Xg)
    serial = o.serial(u0)
    if prec == wl.F64:
        assert ig.status == io.status == orc.OK
        assert abs(ig.iters - io.iters) <= 1
        assert relerr(Xg, Xo) < 1e-9
        assert relerr(Xg, serial) < 1e-9
    else:
        assert relerr(Xg, serial) < 1e-5


def test_c3_full_size_fp32():
    """The 512 x 512, 128-slice heat workload (64 PR-ADI steps, FP32 fine):
    the apply of a random block on every slice against the oracle's apply,
    and the solve on every slice against the FP64 serial fine trajectory, with
    the final state u(T) = F(lambda_{N-1}) (PIT_APPLY_LAST) against the
    oracle's.  The bar is the FP32-fine one: 1e-5 relative."""
    from paper_2203_10148_amd import pitsbicg as P

    p = wl.C3
    say("c3 full size")
    c = ctx(p)
    o = make_oracle(p)
    lam = wl.random_block(p, 3)
    y = host(c.apply_F(dev(lam)))
    ref = o.apply(lam)
    worst = max(relerr(y.reshape(p.N, -1)[n], ref.reshape(p.N, -1)[n]) for n in range(1, p.N))
    print(f"c3 apply: block {relerr(y, ref):.2e}, worst slice {worst:.2e}", flush=True)
    assert relerr(y, ref) < 1e-5 and worst < 1e-5
    u0 = wl.u0_for(p)
    Xd, ig = c.solve(dev(u0), tol=p.tol, stall_window=10)
    Xg = host(Xd).reshape(p.N, -1)
    uT_g = host(c.apply_F(Xd, last=True)).reshape(p.N, -1)[-1]
    serial, uT = o.serial(u0, want_uT=True)
    S = serial.reshape(p.N, -1)
    errs = np.array([relerr(Xg[n], S[n]) for n in range(p.N)])
    e_all = relerr(Xg, S)
    print(f"c3 fp32 solve: status={ig.status} iters={ig.iters} ms={ig.ms_total:.1f} res={ig.res_norm:.2e} "
          f"block err {e_all:.2e}, worst slice {errs.max():.2e} (slice {errs.argmax()}), "
          f"u(T) err {relerr(uT_g, uT):.2e}", flush=True)
    assert ig.status in (P.OK, P.ENOCONV)
    assert ig.res_norm <= 1e-6  # converged to tol or stopped at the FP32 floor, well below the data
    assert e_all < 1e-5 and errs.max() < 1e-5
    assert relerr(uT_g, uT) < 1e-5


@pytest.mark.parametrize("nbytes", [16, 16 * 1023, 16 * 4096 * 4 + 48, 64 << 20])
def test_stream_copy_copies_exactly(nbytes):
    """pit_stream_copy (the bandwidth reference) copies every byte, also a
    ragged tail of the grid-stride loop; misaligned sizes are refused."""
    from paper_2203_10148_amd import pitsbicg as P

    say(f"stream copy {nbytes} B")
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    P.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    with pytest.raises(P.PitError):
        P.stream_copy(dst[:8], src[:8])
