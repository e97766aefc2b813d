"""Parity cases run against the checking build (PIT_LIBRARY=check: every
kernel's LDS is filled with NaN before first use).  Run as a script in its
own process by tests/test_gpu_check_build.py; prints one line per case and
exits 0 when every result is finite and within its bound of the oracle."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle as orc  # noqa: E402
from paper_2203_10148_amd import pitsbicg as P  # noqa: E402
from paper_2203_10148_amd import workloads as wl  # noqa: E402


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def p1d(M, bc, N, m, prec=wl.F64, fine=wl.CN):
    return wl.Problem(dim=1, M=(M, 1), bc=bc, nu=2e-3, adv=(0.7 if bc == wl.PERIODIC else 0.0, 0.0), T=0.5, N=N,
                      m=m, fine=fine, c=2, coarse=wl.IE, prec=prec, tol=1e-10)


def p2d(Mx, My, prec, rot=0.0, c=2):
    return wl.Problem(dim=2, M=(Mx, My), bc=wl.DIRICHLET, nu=0.05, react=0.2, rot=rot, T=0.15, N=3, m=3, fine=wl.ADI,
                      c=c, coarse=wl.ADI, prec=prec, tol=1e-10)


CASES = [
    ("64 IE", wl.C1.with_(N=6)),
    ("1000 periodic CN, 2 waves", p1d(1000, wl.PERIODIC, 4, 5)),
    ("4096 periodic CN, 4 waves", p1d(4096, wl.PERIODIC, 4, 3)),
    ("12000 periodic CN, compact tables", p1d(12000, wl.PERIODIC, 3, 2)),
    ("1000 periodic CN FP32", p1d(1000, wl.PERIODIC, 4, 5, prec=wl.F32)),
    ("100x70 FP64 (whole slices in LDS)", p2d(100, 70, wl.F64)),
    ("300x200 FP32 (strip kernels, one-column sweep)", p2d(300, 200, wl.F32)),
    ("700x130 FP64 (two-wave rows)", p2d(700, 130, wl.F64)),
    ("160x150 rotating velocity (per-line kernels)", p2d(160, 150, wl.F64, rot=1.0)),
]


def main():
    assert os.environ.get("PIT_LIBRARY") == "check"
    torch.cuda.set_device(0)
    P.load()
    ok = True
    for name, p in CASES:
        c = P.Context(p)
        o = orc.Oracle(**p.oracle_kwargs())
        if p.dim == 2:
            X, Y = wl.grid_2d(p)
            lam = np.concatenate([(np.sin(np.pi * X) * np.sin((n + 1) * np.pi * Y)).reshape(-1) for n in range(p.N)])
        else:
            lam = wl.random_block(p, 3)
        d = torch.as_tensor(lam, device="cuda")
        ya = c.apply_F(d).cpu().numpy()
        za = c.coarse_sweep(d).cpu().numpy()
        ea, es = relerr(ya, o.apply(lam)), relerr(za, o.sweep(lam))
        bound = 1e-12 if p.prec == wl.F64 else 1e-5
        good = np.isfinite(ya).all() and np.isfinite(za).all() and ea < bound and es < 1e-12
        print(f"{name}: apply {ea:.2e} sweep {es:.2e} {'ok' if good else 'FAILED'}", flush=True)
        ok &= bool(good)
    # reductions and the iteration: one solve each, single and batched
    p = wl.C1.with_(N=8)
    u0 = wl.u0_for(p)
    c = P.Context(p)
    X, info = c.solve(torch.as_tensor(u0, device="cuda"), tol=1e-10)
    Xo, io = orc.Oracle(**p.oracle_kwargs()).pitsbicg(u0, tol=1e-10)
    e = relerr(X.cpu().numpy(), Xo)
    Xs, infos = P.Batch(1).solve([c], [torch.as_tensor(u0, device="cuda")], tol=1e-10)
    eb = relerr(Xs[0].cpu().numpy(), Xo)
    good = info.iters == io.iters == infos[0].iters and e < 1e-10 and eb < 1e-10
    print(f"solve: iters {info.iters}/{io.iters}/{infos[0].iters} err {e:.2e} batched {eb:.2e} "
          f"{'ok' if good else 'FAILED'}", flush=True)
    ok &= bool(good)
    print("check build: " + ("ok" if ok else "FAILED"), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
