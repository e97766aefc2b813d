#!/usr/bin/env python3
"""Benchmark of the PiTSBiCG hot path on one MI355X.

A step is one whole PiTSBiCG solve of the workload to its tolerance (every
all-at-once fine apply, coarse sweep and BiCGStab vector/reduction kernel of
Algorithm 1) plus the final state u(T) = F(lambda_{N-1}), with every input
already resident in HBM.  `value` is fine cell-updates per second over the
timed steps: (fine applies x (N-1) x m x npts + the final m x npts) / time.

The dominant kernel's roofline is measured live: the solves in the timed
region record HIP events around every fine apply and coarse sweep on the
solve's stream.  The CPU baseline is the oracle (plain C, FP64) running the
same solve truncated to a bounded number of iterations on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3] [--prec f32]

The default line is the 512 x 512 heat workload (128 slices, 64 PR-ADI fine steps
per slice, FP32 fine fields, FP64 Krylov), whose fine apply is bound by HBM
bandwidth.  It also carries the same fine apply on a 1024 x 1024 grid (a working
set beyond the 256 MiB Infinity Cache) and the 4096-point advection-diffusion
workload (FP64 and FP32 fine) as extra keys.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp64_vec_TFs": 78.6, "fp32_vec_TFs": 157.3, "cus": 256}

# Algorithmic FLOPs per fine cell-update of one implicit step with
# precomputed LU factors: forward substitution 2, back substitution 3,
# Sherman-Morrison correction 2 (periodic), CN combination 2u - A^{-1}... 2.
FLOPS_PER_CU = {("ie", 0): 5, ("ie", 1): 7, ("cn", 0): 7, ("cn", 1): 9}

# Algorithmic FLOPs per point of one 2D step on per-line tables, per
# half-step: explicit part u + lo u_m + di u + up u_q (6, PR-ADI only; the
# backward-Euler splitting has none), forward elimination (r - a d) w (3),
# back substitution d - c x (2).
VEL_FLOPS_PER_POINT_STEP = {"adi": 2 * (6 + 3 + 2), "adi_ie": 2 * (3 + 2)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources that the fine apply and coarse sweep kernels are compiled from; a
# stored counter summary is only used while these files are unchanged.
KERNEL_SOURCES = {1: ["fine1d.hip", "line1d.hpp", "pit_internal.hpp"],
                  2: ["adi2d.hip", "line1d.hpp", "pit_internal.hpp"]}
CSRC = os.path.join(ROOT, "paper_2203_10148_amd", "csrc")
CAL_BYTES = 1 << 30  # the probe's device copy (read 1 GiB, write 1 GiB)
# The timed solves time one fine apply and one coarse sweep in KERNEL_SAMPLE
# of each with HIP events (the first of a solve and every KERNEL_SAMPLE-th
# after it): an event pair around every launch put a 10 us gap between each
# apply and its sweep, 0.5 ms of a 4096-point solve.  Launches of one kernel
# in a solve do the same work (rocprofv3 min/max within 3%).
KERNEL_SAMPLE = 7


def sources_sha(dim):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[dim]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    return re.sub(r"\(.*", "", name).replace("pit::", "")


def summarize_stats(stats_csv, out, title, command):
    """Markdown table of a rocprofv3 --stats kernel summary."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def pmc_dispatches(path, counter):
    """{dispatch id: (kernel name, KiB)} from a rocprofv3 --pmc counter_collection.csv."""
    d = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        name, v = d.get(k, (r["Kernel_Name"], 0.0))
        d[k] = (name, v + float(r["Counter_Value"]))
    return d


def summarize_pmc(fetch_csv, write_csv, out, p, prec, unit, kernels, units, commands):
    """HBM-side traffic per fine apply / coarse sweep from two counter runs of --probe.

    FETCH_SIZE and WRITE_SIZE are each scaled by what they read for the
    probe's 1 GiB device copy, then summed over the dispatches whose kernel
    name matches `kernels` and divided by the number of probed units."""
    res = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        d = pmc_dispatches(path, counter)
        cal = max(v for n, v in d.values() if "copyBuffer" in n)
        factor = CAL_BYTES / (cal * 1024.0)
        per_kernel = {}
        for n, v in d.values():
            if "pit::" not in n or not re.search(kernels, n):
                continue
            c, t = per_kernel.get(short_name(n), (0, 0.0))
            per_kernel[short_name(n)] = (c + 1, t + v * 1024.0 * factor)
        n_units = sum(c for c, _ in per_kernel.values()) if units == 0 else units
        res[key] = {"factor": factor, "cal_kib": cal, "kernels": per_kernel,
                    "bytes": sum(t for _, t in per_kernel.values()) / n_units}
    units = n_units
    alg = algorithmic_bytes(p, prec, unit)
    rec = {"workload": p.name, "prec": prec, "unit": unit, "fetch_bytes": res["fetch"]["bytes"],
           "write_bytes": res["write"]["bytes"], "traffic_bytes": res["fetch"]["bytes"] + res["write"]["bytes"],
           "algorithmic_bytes": alg, "fetch_factor": res["fetch"]["factor"], "write_factor": res["write"]["factor"],
           "sources_sha256": sources_sha(p.dim)}
    lines = [f"# HBM traffic: {unit} on {p.name} ({prec} fine)", "",
             "Counter runs (from the repository root on one MI355X), one counter per run:", "", "```"]
    lines += commands + ["```", "",
                         f"Calibration: the probe's 1 GiB device copy reads FETCH_SIZE = {res['fetch']['cal_kib']:.0f} KiB "
                         f"and WRITE_SIZE = {res['write']['cal_kib']:.0f} KiB, so the counters are scaled by "
                         f"{res['fetch']['factor']:.4f} (fetch) and {res['write']['factor']:.4f} (write).", "",
                         "| kernel | dispatches | fetch MiB/dispatch | write MiB/dispatch |", "|---|---:|---:|---:|"]
    for n in res["fetch"]["kernels"]:
        cf, tf = res["fetch"]["kernels"][n]
        cw, tw = res["write"]["kernels"].get(n, (1, 0.0))
        lines.append(f"| `{n}` | {cf} | {tf / cf / 2**20:.2f} | {tw / cw / 2**20:.2f} |")
    lines += ["", f"Per {unit} ({units} probed): fetch {rec['fetch_bytes'] / 2**20:.1f} MiB, write "
                  f"{rec['write_bytes'] / 2**20:.1f} MiB, total {rec['traffic_bytes'] / 2**20:.1f} MiB against "
                  f"{alg / 2**20:.1f} MiB algorithmic ({rec['traffic_bytes'] / alg:.3f}x).", "",
              f"<!-- traffic-json: {json.dumps(rec)} -->"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return rec


def stored_traffic(p, prec, unit):
    """Traffic per unit from a committed counter summary, if the kernel sources still match."""
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md"))):
        m = re.search(r"<!-- traffic-json: (\{.*\}) -->", open(path).read())
        if not m:
            continue
        rec = json.loads(m.group(1))
        if (rec["workload"], rec["prec"], rec["unit"]) == (p.name, prec, unit):
            if rec["sources_sha256"] == sources_sha(p.dim):
                return rec, os.path.relpath(path, ROOT)
            return None, os.path.relpath(path, ROOT) + " (stale: kernel sources changed since)"
    return None, None


def algorithmic_bytes(p, prec, unit):
    """Algorithmic HBM bytes of one fine apply or coarse sweep (block vectors FP64).

    1D fine apply: each of the N-1 slices reads lam_{n-1} and lam_n (the
    epilogue's subtraction) and writes y_n; the state stays on chip across the
    m steps.  1D coarse sweep: v_n in, z_n out.  2D fine apply: each PR-ADI
    half step reads and writes the field once in the fine precision, except
    that the first reads lam_{n-1} (FP64) and the last reads lam_n and writes
    y_n (FP64).  2D coarse sweep per slice and step: x half (read 8 + write 8),
    y half (read 8 + base 8 + write 8).
    """
    ns = p.N - 1
    if p.dim == 1:
        if unit == "fine_apply":
            return ns * p.npts * 24
        return 2 * p.N * p.npts * 8
    if unit == "fine_apply":
        f = 4 if prec == "f32" else 8
        per_point = 2 * p.m * 2 * f + 2 * (8 - f) + 8  # 4m field passes; FP64 first read and last write; lam_n
        return ns * p.npts * per_point
    return ns * p.c * p.npts * 40


def workload(name, prec, side=None, time_scheme="pr"):
    from paper_2203_10148_amd import workloads as wl

    p = {"c1": wl.C1, "c2": wl.C2, "c3": wl.C3, "f2": wl.F2, "f3d": wl.F3_DIFF, "f3r": wl.F3_DR}[name]
    if side and p.dim == 2 and side != p.M[0]:
        # the same 2D recipe on a larger square (its working set beyond the 256 MiB MALL)
        p = p.with_(M=(side, side), name=f"{p.name}_{side}")
    if time_scheme == "ie" and p.dim == 2:
        p = p.with_(fine=wl.ADI_IE, coarse=wl.ADI_IE, name=f"{p.name}_ie")
    if prec is None:
        return p
    return p.with_(prec=wl.F64 if prec == "f64" else wl.F32)


def gpu_serial(p, u0, dev):
    """The sequential method on the same GPU kernels: one slice of all N m fine
    steps (same fine step), u(T) = F^{N m}(u0) by one RAW apply; the 2D
    half-step launches go eagerly (no graph of that many nodes).  Second of
    two runs."""
    import torch

    from paper_2203_10148_amd import pitsbicg as P

    q = p.with_(N=1, m=p.N * p.m)
    ctx = P.Context(q, device=dev)
    u = torch.as_tensor(u0, dtype=torch.float64, device=dev)
    y = torch.empty_like(u)
    old = os.environ.get("PIT_GRAPHS")
    os.environ["PIT_GRAPHS"] = "0"
    try:
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.apply_F(u, y, raw=True)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
    finally:
        if old is None:
            del os.environ["PIT_GRAPHS"]
        else:
            os.environ["PIT_GRAPHS"] = old
    return {"ms": ms, "steps": p.N * p.m, "kind": "the fine propagator over all N m steps of one slice, "
            "the sequential method on the same kernels (u(T) only)"}


def cpu_serial(p, u0, seconds=1.0):
    """The oracle's serial fine solve (the sequential time stepping that the
    parallel-in-time method replaces) on one core: the first k slices of the
    same workload (same fine step), k doubled until about `seconds` of work,
    and the full serial time to solution estimated from that rate."""
    import oracle as orc

    orc.set_threads(1)
    k = 1
    while True:
        q = p.with_(N=k, T=p.T * k / p.N)
        o = orc.Oracle(**q.oracle_kwargs())
        t0 = time.perf_counter()
        o.serial(u0, want_uT=True)  # lambda_1 .. lambda_{k-1} and u(T_k): k slices of m steps
        dt = time.perf_counter() - t0
        if dt >= seconds or k >= p.N:
            break
        k = min(p.N, 2 * k)
    cells = k * p.m * p.npts
    rate = cells / dt
    return {"value": rate, "unit": "cell-updates/s", "cores": 1, "kind": "oracle serial fine solve",
            "sample": f"first {k} of {p.N} slices ({cells} cell-updates, {dt:.2f} s)",
            "time_to_solution_s_est": p.N * p.m * p.npts / rate}


def host_cores():
    """Threads for the oracle: the cores this process may run on, at most 16
    (the host share of a one-GPU job; the machine may show more cores than
    the job is given)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(p, u0, seconds, source=None, profile=None):
    """Oracle PiTSBiCG on the host cores, truncated to a few iterations."""
    import oracle as orc

    threads = host_cores()
    orc.set_threads(threads)
    o = orc.Oracle(**p.oracle_kwargs())
    if source is not None:
        o.set_source(source, profile)
    iters = 1
    while True:
        t0 = time.perf_counter()
        _, info = o.pitsbicg(u0, tol=p.tol, max_iter=iters)
        dt = time.perf_counter() - t0
        if dt >= seconds or info.iters < iters or iters >= 24:
            break
        iters = max(iters + 1, int(iters * seconds / max(dt, 1e-3)))
        iters = min(iters, 24)
    cells = info.matvecs * p.cells_per_apply
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Algorithm 1 on the same {p.name} input truncated to "
                      f"{info.iters} iteration(s) ({info.matvecs} preconditioned products), "
                      f"{dt:.1f} s, {threads} OpenMP threads over slices (over the lines of a 2D step where one slice "
                      f"runs alone): the host cores this process may use, at most the 16 a one-GPU job is given"}


def solve_summary(infos, P):
    """Status, iterations and time of the timed solves; the time to tol only
    when every timed solve reached it."""
    import numpy as np

    status = sorted({i.status for i in infos})
    ms = float(np.median([i.ms_total for i in infos]))
    d = {"status": status, "iters": infos[-1].iters, "matvecs": infos[-1].matvecs, "restarts": infos[-1].restarts,
         "res_norm": infos[-1].res_norm, "reached_tol": status == [P.OK]}
    if status == [P.OK]:
        d["time_to_tol_ms"] = ms
    else:
        d["time_to_stop_ms"] = ms
    return d


def compare_form(p, other, u0, X, source_f, source_g, dev, reps):
    """The same solve with the other fine precision (FP32 fine with FP64
    reductions, or plain FP64): time, outcome and distance from the timed
    form's solution."""
    import numpy as np
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    po = p.with_(prec=other)
    co = P.Context(po, device=dev)
    if source_f is not None:
        co.set_source(source_f, source_g)
    Xo = torch.empty_like(X)
    so = 10 if other == wl.F32 else 0
    co.solve(u0, Xo, tol=p.tol, stall_window=so)
    torch.cuda.synchronize()
    infos = []
    for _ in range(reps):
        _, io = co.solve(u0, Xo, tol=p.tol, stall_window=so)
        infos.append(io)
    diff = float(torch.linalg.vector_norm(Xo - X) / torch.linalg.vector_norm(X))
    d = {"form": "f32" if other == wl.F32 else "f64", "ms": float(np.median([i.ms_total for i in infos])),
         **solve_summary(infos, P), "rel_diff_from_timed_form": diff}
    if not d["reached_tol"]:
        d["note"] = ("an FP32 fine propagator stops at its residual floor (stall rule, status -4) when tol is "
                     "below it")
    return d


def fine_apply_rate(p, prec, dev, reps=5):
    """Average duration (HIP events on the launching stream) and algorithmic
    HBM rate of the fine apply of a random block on problem p."""
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    ctx = P.Context(p, device=dev)
    g = torch.Generator(device=dev).manual_seed(1)
    lam = torch.randn(p.N * p.npts, dtype=torch.float64, device=dev, generator=g)
    y = torch.empty_like(lam)
    st = torch.cuda.current_stream(dev)
    ctx.apply_F(lam, y, stream=st)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(st)
        ctx.apply_F(lam, y, stream=st)
        b.record(st)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps
    by = algorithmic_bytes(p, prec, "fine_apply")
    gbs = by / (ms * 1e-3) / 1e9
    del ctx
    return {"workload": p.name, "M": list(p.M), "N": p.N, "m": p.m, "fine_prec": prec, "avg_ms": ms,
            "launches": reps, "algorithmic_bytes": by, "achieved": gbs, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": gbs / PEAK["hbm_GBs"], "cell_updates_per_s": p.cells_per_apply / (ms * 1e-3)}


def c2_summary(dev, reps=5):
    """The 4096-point advection-diffusion workload (N 256, m 200): time to
    tol 1e-8 with a plain FP64 and with an FP32 fine propagator (FP64
    reductions), whole-solve fine cell-updates/s, and the average fine apply
    and coarse sweep (HIP events, every 7th launch)."""
    import numpy as np
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    res = {}
    X64 = None
    for prec in ("f64", "f32"):
        p = wl.C2.with_(prec=wl.F64 if prec == "f64" else wl.F32)
        ctx = P.Context(p, device=dev)
        u0 = torch.as_tensor(wl.u0_for(p), dtype=torch.float64, device=dev)
        X = torch.empty(p.N * p.npts, dtype=torch.float64, device=dev)
        stall = 10 if prec == "f32" else 0
        ctx.solve(u0, X, tol=p.tol, stall_window=stall)
        torch.cuda.synchronize()
        infos = [ctx.solve(u0, X, tol=p.tol, stall_window=stall, timing=KERNEL_SAMPLE)[1] for _ in range(reps)]
        ms = float(np.median([i.ms_total for i in infos]))
        fine = sum(i.ms_fine for i in infos) / max(sum(i.n_fine_timed for i in infos), 1)
        sweep = sum(i.ms_coarse for i in infos) / max(sum(i.n_coarse_timed for i in infos), 1)
        kry = sum(i.ms_krylov for i in infos) / max(sum(i.n_krylov_timed for i in infos), 1)
        last = infos[-1]
        d = {"ms": ms, **solve_summary(infos, P),
             "cell_updates_per_s": last.n_fine * p.cells_per_apply / (ms * 1e-3),
             "fine_apply_avg_ms": fine, "coarse_sweep_avg_ms": sweep, "krylov_per_iter_ms": kry,
             # per-phase split of one solve from the sampled averages (the
             # rest of the wall time is launch gaps and host round trips)
             "phase_ms": {"fine": fine * last.n_fine, "sweep": sweep * last.n_coarse,
                          "krylov": kry * last.iters}}
        if X64 is None:
            X64 = X.clone()
        else:
            d["rel_diff_from_f64"] = float(torch.linalg.vector_norm(X - X64) / torch.linalg.vector_norm(X64))
        res[prec] = d
    res["workload"] = wl.C2.name
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "f2", "f3d", "f3r"],
                    help="c1-c3, f2, f3d (diffusion), f3r (diffusion-reaction): one solve per step; c4: the "
                         "64-instance batch per step; c5: a served Poisson stream (one pass of --requests "
                         "requests)")
    ap.add_argument("--time-scheme", choices=["pr", "ie"], default="pr",
                    help="2D workloads: Peaceman-Rachford ADI (pr) or the backward-Euler splitting (ie, the "
                         "paper's time marching) as fine and coarse stepper")
    ap.add_argument("--restart-study", action="store_true",
                    help="Algorithm 1's restart threshold epsilon_0 (|<R, R~>| <= epsilon_0 restarts the shadow "
                         "residual) swept over C1, C2 and the cases of Sec. 4 at N = 64: iterations, products, "
                         "restarts and time per value (one JSON line)")
    ap.add_argument("--paper-cases", action="store_true",
                    help="the experiment of Sec. 4: the diffusion, diffusion-reaction and rotating "
                         "advection-diffusion-reaction cases on 4..64 slices, PiTSBiCG against parareal by "
                         "preconditioned products to tol (one JSON line)")
    ap.add_argument("--requests", type=int, default=120, help="c5: how many requests of the stream to serve")
    ap.add_argument("--rate", type=float, default=200.0, help="c5: arrival rate (requests/s)")
    ap.add_argument("--arena-gib", type=float, default=160.0, help="c5: HBM budget of the server (GiB)")
    ap.add_argument("--no-autotune", action="store_true", help="c4: keep the default line shapes")
    ap.add_argument("--no-compare", action="store_true", help="skip the solve in the other fine precision, parareal and (c3) the extra keys")
    ap.add_argument("--side", type=int, default=None, help="c3: grid side (default 512)")
    ap.add_argument("--no-singles", action="store_true", help="c4: skip the single-instance baseline solves")
    ap.add_argument("--prec", default=None, choices=["f64", "f32"],
                    help="fine-propagator precision (default: the workload's)")
    ap.add_argument("--nu-t", type=int, default=None, metavar="SEED",
                    help="c1, c2: a time-dependent operator constant on each slice, nu s_n with seeded factors "
                         "(pit_set_nu_t)")
    ap.add_argument("--source", type=int, default=None, metavar="SEED",
                    help="c1-c3, f2: add a seeded source term constant in time (pit_set_source)")
    ap.add_argument("--source-profile", action="store_true",
                    help="with --source: make it g(t) h(x), g a seeded time profile (pit_set_source_t)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", choices=["apply", "sweep", "solve"], default=None,
                    help="counter-collection mode: run two fine applies (or two coarse sweeps, or a one-iteration "
                         "solve) of the workload and a 1 GiB device copy (the byte-count calibration)")
    ap.add_argument("--stats-summary", nargs=4, metavar=("CSV", "OUT", "TITLE", "COMMAND"),
                    help="write a markdown summary of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--pmc-summary", nargs=8,
                    metavar=("FETCH_CSV", "WRITE_CSV", "OUT", "UNIT", "KERNEL_REGEX", "UNITS", "FETCH_CMD", "WRITE_CMD"),
                    help="write the traffic summary of two --probe counter runs (FETCH_SIZE, WRITE_SIZE) and exit: "
                         "UNIT is fine_apply or coarse_sweep, made of the dispatches matching KERNEL_REGEX, UNITS of "
                         "them were probed (0: one unit per matching dispatch); --workload/--prec name the probed workload")
    args = ap.parse_args()
    if args.stats_summary:
        summarize_stats(*args.stats_summary)
        return
    if args.pmc_summary:
        p = workload(args.workload, args.prec, args.side, args.time_scheme)
        from paper_2203_10148_amd import workloads as wl
        prec = "f32" if p.prec == wl.F32 else "f64"
        fc, wc, out, unit, rx, units, cf, cw = args.pmc_summary
        print(json.dumps(summarize_pmc(fc, wc, out, p, prec, unit, rx, int(units), [cf, cw])))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.paper_cases:
        return bench_paper_cases(args, dev)
    if args.restart_study:
        return bench_restart_study(args, dev)
    if args.workload == "c4":
        return bench_batch(args, dev)
    if args.workload == "c5":
        return bench_serve(args, dev)
    p = workload(args.workload, args.prec, args.side, args.time_scheme)
    args.prec = "f32" if p.prec == wl.F32 else "f64"
    u0h = wl.u0_for(p)
    log(f"[bench] workload {p.name} M={p.M} N={p.N} m={p.m} prec={args.prec}")
    ctx = P.Context(p, device=dev)
    source_f, source_g, src_ms = None, None, None
    if args.nu_t is not None:
        # the per-slice step tables are built and uploaded here (setup, not timed)
        ctx.set_nu_t(wl.nu_factors(p, args.nu_t))
        log(f"[bench] time-dependent operator: nu s_n per slice (seed {args.nu_t})")
    if args.source is not None:
        # the forced responses are computed at pit_set_source(_t) (setup, not timed)
        source_f = wl.source_bumps(p, args.source)
        if args.source_profile:
            source_g = wl.source_profile(p, args.source + 1)
        t0 = time.perf_counter()
        ctx.set_source(source_f, source_g)
        torch.cuda.synchronize()
        src_ms = 1e3 * (time.perf_counter() - t0)
        what = "all N slices' forced responses" if source_g is not None else "forced response"
        log(f"[bench] source (seed {args.source}): {what} set up in {src_ms:.2f} ms")
    if args.probe:
        lam = torch.as_tensor(wl.random_block(p, 1), dtype=torch.float64, device=dev)
        out = torch.empty_like(lam)
        if args.probe == "solve":
            ctx.solve(torch.as_tensor(u0h, dtype=torch.float64, device=dev), out, tol=p.tol, max_iter=1,
                      raise_on_error=False)
        for _ in range(2 if args.probe != "solve" else 0):
            if args.probe == "apply":
                ctx.apply_F(lam, out)
            else:
                ctx.coarse_sweep(lam, out)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        # the library's own streaming copy: the achievable-bandwidth reference
        P.stream_copy(b, a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            P.stream_copy(b, a)
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / 5
        log(f"[bench] probe {args.probe} done; pit_stream_copy of 1 GiB: {cms:.3f} ms = "
            f"{2 * CAL_BYTES / cms / 1e6:.0f} GB/s read + write")
        return
    u0 = torch.as_tensor(u0h, dtype=torch.float64, device=dev)
    X = torch.empty(p.N * p.npts, dtype=torch.float64, device=dev)
    uT = torch.empty_like(X)
    stall = 10 if args.prec == "f32" else 0

    def step(timing):
        _, info = ctx.solve(u0, X, tol=p.tol, stall_window=stall, timing=KERNEL_SAMPLE if timing else 0)
        ctx.apply_F(X, uT, last=True)
        return info

    for i in range(args.warmup):
        info = step(False)
        log(f"[bench] warmup {i}: status={info.status} iters={info.iters} ms={info.ms_total:.2f}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step(True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    status = {i.status for i in infos}
    iters = infos[-1].iters
    matvecs = infos[-1].matvecs
    n_apply = sum(i.n_fine for i in infos)
    cells = sum(i.n_fine for i in infos) * p.cells_per_apply + args.steps * p.m * p.npts
    value = cells / elapsed
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, iters={iters}, status={status}")

    # live per-kernel durations (HIP events on the solve stream)
    ms_fine = sum(i.ms_fine for i in infos)
    ms_coarse = sum(i.ms_coarse for i in infos)
    n_coarse = sum(i.n_coarse for i in infos)
    n_fine_timed = sum(i.n_fine_timed for i in infos)
    n_coarse_timed = sum(i.n_coarse_timed for i in infos)
    avg_fine = ms_fine / max(n_fine_timed, 1)
    avg_coarse = ms_coarse / max(n_coarse_timed, 1)
    periodic = 1 if p.bc == wl.PERIODIC else 0
    if p.dim == 1:
        scheme = "cn" if p.fine == wl.CN else "ie"
        cscheme = "cn" if p.coarse == wl.CN else "ie"
        fl_fine = p.cells_per_apply * FLOPS_PER_CU[(scheme, periodic)]
        fl_coarse = (p.N - 1) * p.c * p.npts * FLOPS_PER_CU[(cscheme, periodic)] + (p.N - 1) * p.npts
        peak = PEAK["fp64_vec_TFs"] if args.prec == "f64" else PEAK["fp32_vec_TFs"]
        kern = {
            "fine_apply": {"avg_ms": avg_fine, "total_ms": avg_fine * n_apply, "launches": n_apply,
                           "timed_ms": ms_fine, "timed_launches": n_fine_timed, "bound": "alu",
                           "work_per_launch": fl_fine, "unit": "TFLOP/s", "peak": peak},
            "coarse_sweep": {"avg_ms": avg_coarse, "total_ms": avg_coarse * n_coarse, "launches": n_coarse,
                             "timed_ms": ms_coarse, "timed_launches": n_coarse_timed, "bound": "alu",
                             "work_per_launch": fl_coarse, "unit": "TFLOP/s", "peak": PEAK["fp64_vec_TFs"]},
        }
    elif ctx.kernel_shape()[0] == 1 and ctx.kernel_shape()[2] > 0:
        # 2D on per-line tables with the slices held in LDS for all their steps:
        # HBM sees each slice once per launch, the steps are FP64 arithmetic.
        scheme = "adi_ie" if p.fine == wl.ADI_IE else "adi"
        cscheme = "adi_ie" if p.coarse == wl.ADI_IE else "adi"
        fl_fine = p.cells_per_apply * VEL_FLOPS_PER_POINT_STEP[scheme]
        fl_coarse = (p.N - 1) * p.c * p.npts * VEL_FLOPS_PER_POINT_STEP[cscheme] + (p.N - 1) * p.npts
        kern = {
            "fine_apply": {"avg_ms": avg_fine, "total_ms": avg_fine * n_apply, "launches": n_apply,
                           "timed_ms": ms_fine, "timed_launches": n_fine_timed, "bound": "alu",
                           "work_per_launch": fl_fine, "unit": "TFLOP/s", "peak": PEAK["fp64_vec_TFs"]},
            "coarse_sweep": {"avg_ms": avg_coarse, "total_ms": avg_coarse * n_coarse, "launches": n_coarse,
                             "timed_ms": ms_coarse, "timed_launches": n_coarse_timed, "bound": "alu",
                             "work_per_launch": fl_coarse, "unit": "TFLOP/s", "peak": PEAK["fp64_vec_TFs"]},
        }
    else:
        # 2D: the fine apply streams the field through HBM twice per PR-ADI step
        # (x half step: read + write, y half step: read + write).
        scheme = "adi_ie" if p.fine == wl.ADI_IE else "adi"
        cscheme = "adi_ie" if p.coarse == wl.ADI_IE else "adi"
        by_fine = algorithmic_bytes(p, args.prec, "fine_apply")
        by_coarse = algorithmic_bytes(p, args.prec, "coarse_sweep")
        kern = {
            "fine_apply": {"avg_ms": avg_fine, "total_ms": avg_fine * n_apply, "launches": n_apply,
                           "timed_ms": ms_fine, "timed_launches": n_fine_timed, "bound": "hbm",
                           "work_per_launch": by_fine, "unit": "GB/s", "peak": PEAK["hbm_GBs"]},
            "coarse_sweep": {"avg_ms": avg_coarse, "total_ms": avg_coarse * n_coarse, "launches": n_coarse,
                             "timed_ms": ms_coarse, "timed_launches": n_coarse_timed, "bound": "hbm",
                             "work_per_launch": by_coarse, "unit": "GB/s", "peak": PEAK["hbm_GBs"]},
        }
    # Algorithm 1's vector updates and inner products, sampled per iteration
    n_kry_timed = sum(i.n_krylov_timed for i in infos)
    kry_iter = sum(i.ms_krylov for i in infos) / max(n_kry_timed, 1)
    phase_ms = {"fine": avg_fine * n_apply / args.steps, "sweep": avg_coarse * n_coarse / args.steps,
                "krylov": kry_iter * sum(i.iters for i in infos) / args.steps}
    scale = {"TFLOP/s": 1e12, "GB/s": 1e9}

    def rate(v):
        return v["work_per_launch"] / (v["avg_ms"] * 1e-3) / scale[v["unit"]] if v["avg_ms"] > 0 else 0.0

    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    k = kern[dom]
    achieved = rate(k)
    roofline = {"bound": k["bound"], "kernel": dom, "achieved": achieved, "peak": k["peak"], "unit": k["unit"],
                "frac": achieved / k["peak"], "traffic": None}
    if k["bound"] == "alu" and dom == "coarse_sweep":
        # The sweep is sequential by construction and runs on one CU: its
        # ceiling is one CU's share of the FP64 vector peak (context only; the
        # fields above keep the chip's peak).
        roofline["peak_one_cu"] = k["peak"] / PEAK["cus"]
        roofline["frac_one_cu"] = achieved / roofline["peak_one_cu"]
    rec, src = stored_traffic(p, args.prec, dom)
    if rec is not None:
        roofline["traffic"] = rec["traffic_bytes"]
        roofline["traffic_unit"] = f"bytes per {dom}"
        roofline["traffic_vs_algorithmic"] = rec["traffic_bytes"] / algorithmic_bytes(p, args.prec, dom)
    if src is not None:
        roofline["traffic_source"] = src
    fine_cu_s = p.cells_per_apply / (avg_fine * 1e-3) if avg_fine > 0 else 0.0
    out = {
        "metric": "fine cell-updates/s and % HBM peak; PiT time-to-1e-8 vs plain FP64, 1 GPU",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": p.name, "M": list(p.M[: p.dim]), "N": p.N, "m": p.m,
                   "fine": scheme, "coarse": f"{p.c}x{cscheme}", "bc": "periodic" if periodic else "dirichlet0",
                   "tol": p.tol, "fine_prec": args.prec,
                   **({"nu_t_seed": args.nu_t} if args.nu_t is not None else {})},
        "roofline": roofline,
        "solve": solve_summary(infos, P),
        "kernels": {name: {**v, "achieved": rate(v)} for name, v in kern.items()},
        "krylov_per_iter_ms": kry_iter, "phase_ms_per_solve": phase_ms,
        "fine_kernel_cell_updates_per_s": fine_cu_s,
        "kernel_shape": ctx.kernel_shape(),
    }
    if source_f is not None:
        out["config"]["source_seed"] = args.source
        if source_g is not None:
            out["config"]["source_profile"] = True
            note = ("forced responses b_n = F_n(0) of all N slices for g(t) h(x), computed on the device at "
                    "pit_set_source_t; B = (u0, b_0, .., b_{N-2})")
        else:
            note = "forced response b = F(0) of one slice, computed on the device at pit_set_source; B = (u0, b, .., b)"
        out["source"] = {"setup_ms": src_ms, "note": note}
    # the other fine-propagator form on the same input (FP32 fine with FP64
    # reductions vs plain FP64), outside the timed region
    if not args.no_compare and p.dim in (1, 2) and not (p.dim == 2 and p.rot != 0.0):
        other = wl.F64 if p.prec == wl.F32 else wl.F32
        out["compare"] = compare_form(p, other, u0, X, source_f, source_g, dev, reps=3 if p.dim == 1 else 2)
        log(f"[bench] compare {out['compare']['form']}: {out['compare']['ms']:.2f} ms, "
            f"status {out['compare']['status']}, iters {out['compare']['iters']}, "
            f"rel. diff {out['compare']['rel_diff_from_timed_form']:.2e}")
    # parareal (Sec. 2, eq. (pararealAlgebraic)) on the same input and kernels,
    # to the same tolerance on its update norm: the paper's comparison
    if not args.no_compare:
        Xp = torch.empty_like(X)
        ctx.parareal(u0, Xp, tol=p.tol)
        torch.cuda.synchronize()
        times = []
        for _ in range(2):
            _, ip = ctx.parareal(u0, Xp, tol=p.tol)
            times.append(ip.ms_total)
        out["compare_parareal"] = {"time_to_tol_ms": float(np.median(times)), "status": ip.status,
                                   "iters": ip.iters, "matvecs": ip.matvecs, "final_update_norm": ip.res_norm,
                                   "pitsbicg_matvecs": matvecs}
        log(f"[bench] parareal: {float(np.median(times)):.2f} ms, {ip.iters} iterations ({ip.matvecs} products) "
            f"vs PiTSBiCG {matvecs} products")
    # the sequential method on the same GPU (context, not the timed region)
    if args.workload in ("c1", "c2", "c3", "f2", "f3d", "f3r") and source_f is None:
        gs = gpu_serial(p, u0h, dev)
        gs["pit_speedup"] = gs["ms"] / ms_per_step
        out["gpu_serial"] = gs
        log(f"[bench] gpu serial fine solve: {gs['ms']:.2f} ms for {gs['steps']} steps; PiTSBiCG {ms_per_step:.2f} ms "
            f"({gs['pit_speedup']:.2f}x)")
    if args.workload == "c3" and not args.no_compare and source_f is None and args.time_scheme == "pr":
        if p.M[0] == 512:
            out["c3_1024_fine_apply"] = fine_apply_rate(p.with_(M=(1024, 1024), name=f"{p.name}_1024"),
                                                        args.prec, dev)
            log(f"[bench] 1024^2 fine apply: {out['c3_1024_fine_apply']['avg_ms']:.2f} ms, "
                f"frac {out['c3_1024_fine_apply']['frac']:.3f}")
        out["c2"] = c2_summary(dev)
        log(f"[bench] c2 fp64: {out['c2']['f64']['ms']:.2f} ms, fp32: {out['c2']['f32']['ms']:.2f} ms")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, u0h, args.cpu_seconds, source_f, source_g)
        if source_f is None:
            out["cpu_serial"] = cpu_serial(p, u0h)
            log(f"[bench] cpu serial fine solve: {out['cpu_serial']['value']:.3g} cell-updates/s on one core, "
                f"{out['cpu_serial']['time_to_solution_s_est']:.2f} s to solution (estimated)")
    print(json.dumps(out), flush=True)


def bench_paper_cases(args, dev):
    """Sec. 4's experiment on the synthetic stand-ins: each case on N = 4..64
    slices with the fine step fixed (N m = 6400), PiTSBiCG and parareal to the
    same tolerance on the preconditioned residual (parareal's update is that
    residual), compared by preconditioned products and by time (second of two
    runs of each)."""
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    rows = []
    for case in wl.PAPER_CASES:
        if args.time_scheme == "ie":
            case = case.with_(fine=wl.ADI_IE, coarse=wl.ADI_IE)
        for N in wl.PAPER_SLICES:
            p = wl.paper_case(case, N)
            ctx = P.Context(p, device=dev)
            u0 = torch.as_tensor(wl.u0_for(p), dtype=torch.float64, device=dev)
            X = torch.empty(p.N * p.npts, dtype=torch.float64, device=dev)
            for _ in range(2):
                _, si = ctx.solve(u0, X, tol=p.tol)
            for _ in range(2):
                _, pi = ctx.parareal(u0, X, tol=p.tol)
            row = {"case": case.name, "N": N, "m": p.m,
                   "pitsbicg": {"status": si.status, "iters": si.iters, "products": si.matvecs,
                                "ms": si.ms_total, "res_norm": si.res_norm},
                   "parareal": {"status": pi.status, "iters": pi.iters, "products": pi.matvecs,
                                "ms": pi.ms_total, "res_norm": pi.res_norm}}
            rows.append(row)
            log(f"[bench] {case.name} N={N} m={p.m}: PiTSBiCG {si.matvecs} products {si.ms_total:.1f} ms "
                f"(status {si.status}); parareal {pi.matvecs} products {pi.ms_total:.1f} ms (status {pi.status})")
            del ctx
    print(json.dumps({"metric": "preconditioned products to tol, PiTSBiCG vs parareal (Sec. 4)",
                      "unit": "products", "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
                      "data": "synthetic", "tol": wl.F2.tol,
                      "time_scheme": "backward-Euler splitting" if args.time_scheme == "ie" else "PR-ADI",
                      "rows": rows}), flush=True)


def bench_restart_study(args, dev):
    """Algorithm 1 with the restart threshold epsilon_0 swept (the paper fixes
    no value): each workload solved to its tolerance from X0 = 0, second of
    two runs timed."""
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    cases = [wl.C1, wl.C2.with_(prec=wl.F64)]
    for case in wl.PAPER_CASES:
        cases.append(case)
        cases.append(case.with_(fine=wl.ADI_IE, coarse=wl.ADI_IE, name=case.name + "_ie"))
    eps0 = [1e-30, 1e-14, 1e-12, 1e-10, 1e-8, 1e-6]
    rows = []
    for p in cases:
        ctx = P.Context(p, device=dev)
        u0 = torch.as_tensor(wl.u0_for(p), dtype=torch.float64, device=dev)
        X = torch.empty(p.N * p.npts, dtype=torch.float64, device=dev)
        for e0 in eps0:
            for _ in range(2):
                _, si = ctx.solve(u0, X, tol=p.tol, restart_tol=e0)
            rows.append({"case": p.name, "tol": p.tol, "eps0": e0, "status": si.status, "iters": si.iters,
                         "products": si.matvecs, "restarts": si.restarts, "ms": si.ms_total,
                         "res_norm": si.res_norm})
            log(f"[bench] {p.name} eps0={e0:g}: status {si.status}, {si.iters} iterations, {si.matvecs} "
                f"products, {si.restarts} restarts, {si.ms_total:.1f} ms")
        del ctx
    print(json.dumps({"metric": "Algorithm 1 against its restart threshold epsilon_0", "n_gpus": 1,
                      "dtype": "f64", "data": "synthetic", "rows": rows}), flush=True)


def bench_batch(args, dev):
    """The 64-instance batch (FP32 fine, tol 1e-8): a step is one batched solve
    of all instances; also the single-instance solves, plain FP64 and FP32, one
    after the other (the batch's baseline)."""
    import numpy as np
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    insts = wl.c4_batch()
    probs = [p for p, _ in insts]
    u0h = [wl.u0_fourier(p, s) for p, s in insts]
    log(f"[bench] c4: {len(probs)} instances, {sum(p.cells_per_apply for p in probs):.3e} cell-updates per apply round")
    # line shapes: autotune one instance per line-length class, the one with
    # the longest chain of line solves per product (it sets the makespan)
    tuned = {}
    if not args.no_autotune:
        reps = {}
        for p in probs:
            k = 1 << max(6, (p.M[0] - 1).bit_length())
            chain = (p.m + (p.N - 1) * p.c) * p.M[0]
            if k not in reps or chain > reps[k][0]:
                reps[k] = (chain, p)
        for k, (_, p) in sorted(reps.items()):
            tuned[k] = P.autotune(p, device=dev)
            log(f"[bench] autotune class {k}: shape {tuned[k][0]}, {tuned[k][1]:.3f} ms per product")
    ctxs = [P.Context(p, device=dev) for p in probs]
    u0s = [torch.as_tensor(u, dtype=torch.float64, device=dev) for u in u0h]
    Xs = [torch.empty(p.N * p.npts, dtype=torch.float64, device=dev) for p in probs]
    b = P.Batch(len(probs), device=dev)

    def step():
        return b.solve(ctxs, u0s, Xs, tol=1e-8, stall_window=10)[1]

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    cells = sum(i.n_fine * p.cells_per_apply for i, p in zip(infos, probs))
    st = [i.status for i in infos]
    log(f"[bench] batch: {ms:.1f} ms per batched solve, {st.count(0)} of {len(st)} reached tol")

    # accuracy against the exact (serial fine FP64) trajectory of each
    # instance, by the modal closed form of periodic CN (every Fourier mode of
    # u0 is an exact grid eigenvector), for instances that reached tol
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from closed_forms import fourier_serial

    exact = [fourier_serial(p, sd).reshape(-1) for p, sd in insts]

    def err_of(i, X):
        x = X.detach().cpu().numpy()
        return float(np.linalg.norm(x - exact[i]) / np.linalg.norm(exact[i]))

    batch_err = {i: err_of(i, Xs[i]) for i, inf in enumerate(infos) if inf.status == 0}

    def singles(prec, tol=1e-8):
        tot, its, mx, errs = 0.0, 0, 0.0, {}
        for i, (p, u) in enumerate(zip(probs, u0s)):
            c = P.Context(p.with_(prec=prec), device=dev)
            torch.cuda.synchronize()
            t = time.perf_counter()
            X, inf = c.solve(u, tol=tol, stall_window=10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            tot += dt
            mx = max(mx, dt)
            its += inf.iters
            if inf.status == 0:
                errs[i] = err_of(i, X)
            c.close()
        return tot, its, mx, errs

    def err_stats(errs, among):
        v = np.array([errs[i] for i in among if i in errs])
        return {"n": int(v.size), "median": float(np.median(v)) if v.size else None,
                "max": float(v.max()) if v.size else None}

    if args.no_singles:
        out = {"metric": "c4 batch only", "makespan_ms": ms, "value": cells * args.steps / elapsed,
               "reached_tol": st.count(0)}
        print(json.dumps(out), flush=True)
        return
    s64, it64, m64, e64 = singles(wl.F64)
    log(f"[bench] single-instance plain FP64: {s64 * 1e3:.1f} ms summed, slowest {m64 * 1e3:.1f} ms")
    s64b, it64b, m64b, e64b = singles(wl.F64, tol=1e-6)
    log(f"[bench] single-instance plain FP64 at tol 1e-6: {s64b * 1e3:.1f} ms summed")
    s32, it32, m32, _ = singles(wl.F32)
    log(f"[bench] single-instance FP32: {s32 * 1e3:.1f} ms summed, slowest {m32 * 1e3:.1f} ms")
    both = sorted(set(batch_err) & set(e64) & set(e64b))
    accuracy = {"against": "exact FP64 serial fine trajectory (modal closed form), every slice",
                "instances": "those that reached tol in every form compared",
                "batch_fp32_tol1e-8": err_stats(batch_err, both),
                "single_fp64_tol1e-8": err_stats(e64, both),
                "single_fp64_tol1e-6": err_stats(e64b, both)}
    log(f"[bench] accuracy over {len(both)} instances: {json.dumps(accuracy)}")
    out = {
        "metric": "fine cell-updates/s, 64-instance batched PiTSBiCG (FP32 fine, tol 1e-8), 1 GPU",
        "value": cells * args.steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batch64", "instances": len(probs), "seed": 4, "tol": 1e-8, "fine_prec": "f32",
                   "stall_window": 10, "autotuned_shapes": {str(k): list(v[0]) for k, v in tuned.items()}},
        "roofline": None,
        "batch": {"makespan_ms": ms, "reached_tol": st.count(0), "stalled": st.count(-4),
                  "iters": [i.iters for i in infos],
                  "sum_single_fp64_ms": s64 * 1e3, "sum_single_fp64_iters": it64,
                  "sum_single_fp32_ms": s32 * 1e3, "sum_single_fp32_iters": it32,
                  "slowest_single_fp64_ms": m64 * 1e3, "slowest_single_fp32_ms": m32 * 1e3,
                  "sum_single_fp64_tol1e-6_ms": s64b * 1e3, "sum_single_fp64_tol1e-6_iters": it64b,
                  "speedup_vs_single_fp64": s64 * 1e3 / ms, "speedup_vs_single_fp32": s32 * 1e3 / ms,
                  "speedup_vs_single_fp64_tol1e-6": s64b * 1e3 / ms,
                  "accuracy": accuracy},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, dev):
    """A served stream: the first --requests requests of the Poisson stream
    (70% 1D advection-diffusion, 30% 2D heat, FP32 fine, tol 1e-8), submitted
    at their arrival times; latency is arrival to completion."""
    import numpy as np
    import torch

    from paper_2203_10148_amd import pitsbicg as P
    from paper_2203_10148_amd import workloads as wl

    reqs = wl.c5_requests(rate=args.rate)[: args.requests]
    fprec = wl.F64 if args.prec == "f64" else wl.F32  # --prec f64: the same stream with plain FP64 fine
    reqs = [(t, p.with_(prec=fprec), sd) for t, p, sd in reqs]
    log(f"[bench] c5: {len(reqs)} requests at {args.rate}/s, arena {args.arena_gib} GiB, "
        f"fine {'FP64' if fprec == wl.F64 else 'FP32'}")
    u0s, Xs = [], []
    for _, p, seed in reqs:
        u = wl.u0_bumps(p, seed) if p.dim == 2 else wl.u0_fourier(p, seed)
        u0s.append(torch.as_tensor(u, dtype=torch.float64, device=dev))
        Xs.append(torch.empty(p.N * p.npts, dtype=torch.float64, device=dev))
    srv = P.Server(int(args.arena_gib * 2**30), max_slots=256, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets, results = [], [None] * len(reqs)
    nxt, last_log = 0, t0
    while True:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt][0] <= now:
            _, p, _ = reqs[nxt]
            tickets.append(srv.submit(p, u0s[nxt], Xs[nxt], tol=1e-8, stall_window=10))
            nxt += 1
        for i, t in enumerate(tickets):
            if results[i] is None:
                results[i] = srv.poll(t)
        done = sum(r is not None for r in results)
        if time.perf_counter() - last_log > 5.0:
            q, r, used = srv.load()
            log(f"[bench] t={now:.1f}s submitted {nxt} done {done} queued {q} running {r} arena {used / 2**30:.1f} GiB")
            last_log = time.perf_counter()
        if done == len(reqs):
            break
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array([r.latency_ms for r in results])
    wait = np.array([r.t_admit_ms - r.t_submit_ms for r in results])
    dims = np.array([p.dim for _, p, _ in reqs])
    st = [r.status for r in results]
    cells = sum(r.matvecs * p.cells_per_apply for r, (_, p, _) in zip(results, reqs))
    # the server clock starts at creation; first arrival to last completion
    span = (max(r.t_done_ms for r in results) - min(r.t_submit_ms for r in results)) / 1e3

    def pct(a, q):
        return float(np.percentile(a, q)) if len(a) else None

    out = {
        "metric": f"served PiTSBiCG solves/s with p50/p99 latency ({'FP64' if fprec == wl.F64 else 'FP32'} fine, "
                  "tol 1e-8), 1 GPU",
        "value": len(reqs) / span, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if fprec == wl.F64 else "f32", "data": "synthetic",
        "config": {"workload": "c5_serving", "requests": len(reqs), "rate_per_s": args.rate, "seed": 5,
                   "fine_prec": "f64" if fprec == wl.F64 else "f32",
                   "arena_gib": args.arena_gib, "max_slots": 256, "tol": 1e-8},
        "roofline": None,
        "serving": {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": float(lat.max()),
                    "p50_1d_ms": pct(lat[dims == 1], 50), "p99_1d_ms": pct(lat[dims == 1], 99),
                    "p50_2d_ms": pct(lat[dims == 2], 50), "p99_2d_ms": pct(lat[dims == 2], 99),
                    "p50_admission_wait_ms": pct(wait, 50), "p99_admission_wait_ms": pct(wait, 99),
                    "span_s": span, "fine_cell_updates_per_s": cells / span,
                    "reached_tol": st.count(0), "stalled": st.count(-4), "other_status": len(st) - st.count(0) - st.count(-4)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
