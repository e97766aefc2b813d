"""C-ABI checks that need no GPU: the library loads, exports every entry point
the public header declares, and validates its arguments on the host."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2203_10148_amd import pitsbicg as P
from paper_2203_10148_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pitsbicg.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pit_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.load()
    names = declared_symbols()
    assert "pit_apply_F" in names and "pit_solve" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    # sizes fixed by the header's field list (int32 / double / pointer, natural alignment)
    assert ct.sizeof(P.pit_problem) == 4 * 4 + 8 * 8
    assert ct.sizeof(P.pit_stepper) == 16
    assert ct.sizeof(P.pit_solve_opts) == 8 * 2 + 4 * 6
    assert ct.sizeof(P.pit_solve_info) == 4 * 4 + 8 + 8 + 4 * 2 + 4 * 3 + 4 * 4 + 4 * 2 + 4  # + tail padding to 8
    assert ct.sizeof(P.pit_server_cfg) == 8 + 8 + 4 * 4
    assert ct.sizeof(P.pit_request) == ct.sizeof(P.pit_problem) + 4 * 2 + 16 * 2 + 8 * 2 + ct.sizeof(P.pit_solve_opts)
    assert ct.sizeof(P.pit_result) == 4 * 4 + 8 * 4 + 8 + 4 * 2



def test_struct_sizes_and_offsets_match_the_c_header(tmp_path):
    """The ctypes mirrors against the header itself: a C program built with
    gcc prints sizeof and every field's offsetof."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = [P.pit_problem, P.pit_stepper, P.pit_solve_opts, P.pit_solve_info, P.pit_server_cfg,
               P.pit_request, P.pit_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pitsbicg.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for f in st._fields_:
            lines.append(f'printf("{st.__name__}.{f[0]} %zu\\n", offsetof({st.__name__}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for st in structs:
        assert int(got[st.__name__]) == ct.sizeof(st), st.__name__
        for f in st._fields_:
            assert int(got[f"{st.__name__}.{f[0]}"]) == getattr(st, f[0]).offset, (st.__name__, f[0])

def create(p, fine=None, coarse=None, N=None, m=None):
    lib = P.load()
    pb = P.make_problem(p)
    f = fine or P.pit_stepper(p.fine, p.m, p.prec, 0)
    g = coarse or P.pit_stepper(p.coarse, p.c, P.F64, 0)
    h = ct.c_void_p()
    rc = lib.pit_create(ct.byref(pb), p.N if N is None else N, p.m if m is None else m, f, g,
                        ct.byref(h))
    return rc, h


def test_create_accepts_the_1d_workloads():
    for p in (wl.C1, wl.C2.with_(prec=wl.F64)):
        rc, h = create(p)
        assert rc == P.OK and h.value
        assert P.load().pit_workspace_bytes(h) > 0
        P.load().pit_destroy(h)


@pytest.mark.parametrize("bad", [
    dict(N=0), dict(m=0), dict(M=(2, 1)), dict(M=(20000, 1)), dict(dim=3), dict(T=0.0),
    dict(nu=-1.0), dict(fine=7), dict(coarse=7), dict(fine=wl.ADI), dict(bc=5),
])
def test_create_rejects_bad_arguments(bad):
    kw = dict(bad)
    N = kw.pop("N", None)
    m = kw.pop("m", None)
    p = wl.C1.with_(**kw)
    rc, h = create(p, N=N, m=m)
    assert rc == P.EINVAL and not h.value


def test_create_rejects_mismatched_fine_substeps():
    p = wl.C1
    rc, _ = create(p, fine=P.pit_stepper(p.fine, p.m + 1, P.F64, 0))
    assert rc == P.EINVAL
    rc, _ = create(p, coarse=P.pit_stepper(p.coarse, 0, P.F64, 0))
    assert rc == P.EINVAL


def test_workspace_scales_with_problem():
    lib = P.load()
    _, h1 = create(wl.C1)
    _, h2 = create(wl.C1.with_(N=32))
    b1, b2 = lib.pit_workspace_bytes(h1), lib.pit_workspace_bytes(h2)
    assert b2 > b1 >= 7 * wl.C1.N * wl.C1.npts * 8
    lib.pit_destroy(h1)
    lib.pit_destroy(h2)


def test_unbound_context_and_null_pointers_are_rejected():
    lib = P.load()
    _, h = create(wl.C1)
    assert lib.pit_apply_F(h, None, None, 0, None) == P.EINVAL
    assert lib.pit_coarse_sweep(h, None, None, None) == P.EINVAL
    assert lib.pit_coarse_sweep_noalloc(h, None, None, None) == P.EINVAL
    assert lib.pit_coarse_sweep_noalloc(None, None, None, None) == P.EINVAL
    assert lib.pit_solve(h, None, None, None, None, None) == P.EINVAL
    assert lib.pit_bind_workspace(h, None, 0) == P.EINVAL
    assert lib.pit_bind_workspace(h, ct.c_void_p(256 * 1000 + 8), 1 << 30) == P.EINVAL  # misaligned
    assert lib.pit_bind_workspace(h, ct.c_void_p(256 * 1000), 16) == P.ENOMEM
    lib.pit_destroy(h)


def test_velocity_fields_validate_on_the_host():
    """2D velocity (constant and rotation): FP64 fine only; 1D takes no rotation."""
    lib = P.load()
    p2 = wl.F2.with_(N=4, m=5)
    rc, h = create(p2)
    assert rc == P.OK
    lib.pit_destroy(h)
    rc, h = create(p2.with_(rot=0.0, adv=(0.3, -0.2)))
    assert rc == P.OK
    lib.pit_destroy(h)
    rc, _ = create(p2.with_(prec=wl.F32))
    assert rc == P.EINVAL
    rc, _ = create(wl.C1.with_(rot=1.0))
    assert rc == P.EINVAL
    rc, _ = create(p2.with_(rot=float("nan")))
    assert rc == P.EINVAL


def test_set_source_validates_on_the_host():
    """pit_set_source on an unbound context only keeps a host copy."""
    import numpy as np
    lib = P.load()
    _, h = create(wl.C1)
    dp = ct.POINTER(ct.c_double)
    f = np.linspace(0.0, 1.0, wl.C1.npts)
    assert lib.pit_set_source(None, f.ctypes.data_as(dp)) == P.EINVAL
    bad = f.copy()
    bad[3] = np.nan
    assert lib.pit_set_source(h, bad.ctypes.data_as(dp)) == P.EINVAL
    assert lib.pit_set_source(h, f.ctypes.data_as(dp)) == P.OK
    assert lib.pit_set_source(h, None) == P.OK
    lib.pit_destroy(h)


def test_strerror_covers_codes():
    for code in (P.OK, P.EINVAL, P.ENOMEM, P.EHIP, P.ENOCONV, P.EBREAKDOWN, P.EAGAIN):
        assert P.strerror(code) and P.strerror(code) != "unknown status"


def test_kernel_shapes_cover_the_line():
    lib = P.load()
    for M in (3, 64, 65, 1000, 4096, 8192, 16384):
        rc, h = create(wl.C2.with_(M=(M, 1), prec=wl.F64, N=4, m=2))
        assert rc == P.OK
        out = (ct.c_int32 * 4)()
        lib.pit_kernel_shape(h, out)
        assert out[0] * out[1] >= M and out[2] * out[3] >= M
        assert out[0] % 64 == 0 and out[0] <= 1024
        lib.pit_destroy(h)


def test_velocity_kernel_shape_reports_where_a_slice_lives(monkeypatch):
    """One thread per line; 2 = fields and tables in LDS (the 49x49 case),
    1 = fields only, 0 = per-half-step kernels (too large, or switched off)."""
    lib = P.load()
    for M, want in (((49, 49), 2), ((80, 66), 1), ((130, 70), 0)):
        rc, h = create(wl.F2.with_(M=M, N=4, m=2))
        assert rc == P.OK
        out = (ct.c_int32 * 4)()
        assert lib.pit_kernel_shape(h, out) == P.OK
        assert list(out) == [1, 0, want, 0], (M, list(out))
        monkeypatch.setenv("PIT_VEL_LDS", "0")
        lib.pit_kernel_shape(h, out)
        assert out[2] == 0
        monkeypatch.delenv("PIT_VEL_LDS")
        lib.pit_destroy(h)


def test_time_dependent_source_sizes_the_workspace_on_the_host():
    """pit_set_source_t on an unbound context: validation, and the workspace
    grows by the N forced responses and N m weights (256-byte aligned), and
    shrinks back when the source becomes constant or goes."""
    lib = P.load()
    p = wl.C1.with_(N=8, m=16)
    rc, h = create(p)
    assert rc == P.OK
    dp = ct.POINTER(ct.c_double)
    base = lib.pit_workspace_bytes(h)
    f = np.linspace(0.0, 1.0, p.npts)
    g = np.ones(p.N * p.m + 1)
    assert lib.pit_set_source_t(h, f.ctypes.data_as(dp), g.ctypes.data_as(dp)) == P.OK
    up = lambda n: (n + 255) // 256 * 256
    assert lib.pit_workspace_bytes(h) == up(up(base + p.N * p.npts * 8) + p.N * p.m * 8)
    bad = g.copy()
    bad[5] = np.nan
    assert lib.pit_set_source_t(h, f.ctypes.data_as(dp), bad.ctypes.data_as(dp)) == P.EINVAL
    assert lib.pit_set_source_t(None, f.ctypes.data_as(dp), g.ctypes.data_as(dp)) == P.EINVAL
    assert lib.pit_set_source_t(h, f.ctypes.data_as(dp), None) == P.OK  # constant source
    assert lib.pit_workspace_bytes(h) == base
    assert lib.pit_set_source_t(h, f.ctypes.data_as(dp), g.ctypes.data_as(dp)) == P.OK
    assert lib.pit_set_source(h, None) == P.OK  # removed
    assert lib.pit_workspace_bytes(h) == base
    lib.pit_destroy(h)


def test_small_fp64_2d_problems_take_the_lds_kernels(monkeypatch):
    """Without a velocity, an FP64 2D slice that fits in LDS takes the
    per-line path as well; FP32 fields, larger slices or PIT_VEL_LDS=0 at
    creation keep the shared-table kernels (64-lane strips)."""
    lib = P.load()
    out = (ct.c_int32 * 4)()

    def shape(p):
        rc, h = create(p)
        assert rc == P.OK
        lib.pit_kernel_shape(h, out)
        lib.pit_destroy(h)
        return list(out)

    small = wl.F3_DIFF.with_(N=4, m=2)
    assert shape(small) == [1, 0, 2, 0]
    assert shape(small.with_(prec=wl.F32))[0] >= 64
    assert shape(small.with_(M=(300, 200)))[0] >= 64
    monkeypatch.setenv("PIT_VEL_LDS", "0")
    assert shape(small)[0] >= 64


def test_backward_euler_splitting_is_2d_only():
    """PIT_ADI_IE (3) is a 2D scheme, as fine or coarse; 1D takes IE/CN."""
    for p in (wl.F2.with_(fine=wl.ADI_IE, coarse=wl.ADI_IE, N=4, m=2), wl.F2.with_(coarse=wl.ADI_IE, N=4, m=2)):
        rc, h = create(p)
        assert rc == P.OK
        P.load().pit_destroy(h)
    assert create(wl.C1.with_(fine=wl.ADI_IE, N=4, m=2))[0] == P.EINVAL
    assert create(wl.C1.with_(coarse=wl.ADI_IE, N=4, m=2))[0] == P.EINVAL
    assert create(wl.F2.with_(fine=wl.IE, N=4, m=2))[0] == P.EINVAL


def test_batch_and_server_validate_on_the_host():
    lib = P.load()
    h = ct.c_void_p()
    assert lib.pit_batch_create(0, ct.byref(h)) == P.EINVAL
    assert lib.pit_batch_create(4, ct.byref(h)) == P.OK
    need = lib.pit_batch_workspace_bytes(h)
    assert need > 0
    assert lib.pit_batch_bind_workspace(h, None, need) == P.EINVAL
    assert lib.pit_batch_bind_workspace(h, ct.c_void_p(256 * 1000 + 8), need) == P.EINVAL  # misaligned
    assert lib.pit_batch_bind_workspace(h, ct.c_void_p(256 * 1000), 16) == P.ENOMEM
    # unbound engine: rejected before any device work
    assert lib.pit_batch_solve(h, None, 0, None, None, None, None, None) == P.EINVAL
    lib.pit_batch_destroy(h)
    cfg = P.pit_server_cfg(None, 1 << 20, 0, 4)
    s = ct.c_void_p()
    assert lib.pit_server_create(ct.byref(cfg), ct.byref(s)) == P.EINVAL  # no arena
    cfg = P.pit_server_cfg(256 * 1000, 1 << 20, 0, 0)
    assert lib.pit_server_create(ct.byref(cfg), ct.byref(s)) == P.EINVAL  # no slots
    cfg = P.pit_server_cfg(256 * 1000, 1024, 0, 4)
    assert lib.pit_server_create(ct.byref(cfg), ct.byref(s)) == P.ENOMEM  # arena below its own buffers
    assert lib.pit_submit(None, None, None) == P.EINVAL
    assert lib.pit_poll(None, 1, None) == P.EINVAL


def test_autotune_scratch_covers_every_candidate_shape():
    lib = P.load()
    p = wl.C2.with_(N=4, m=2)
    pb = P.make_problem(p)
    f, g = P.pit_stepper(p.fine, p.m, p.prec, 0), P.pit_stepper(p.coarse, p.c, P.F64, 0)
    n = lib.pit_autotune_scratch_bytes(ct.byref(pb), p.N, p.m, f, g)
    _, h = create(p)
    assert n >= lib.pit_workspace_bytes(h) > 0
    lib.pit_destroy(h)
    out = (ct.c_int32 * 2)()
    assert lib.pit_autotune(ct.byref(pb), p.N, p.m, f, g, None, n, out, None, None) == P.EINVAL
    p2 = wl.C3.with_(N=2, m=2)
    pb2 = P.make_problem(p2)
    f2, g2 = P.pit_stepper(p2.fine, p2.m, p2.prec, 0), P.pit_stepper(p2.coarse, p2.c, P.F64, 0)
    n2 = lib.pit_autotune_scratch_bytes(ct.byref(pb2), p2.N, p2.m, f2, g2)  # 2D: every launch-shape candidate
    _, h2 = create(p2)
    assert n2 >= lib.pit_workspace_bytes(h2) > 0
    lib.pit_destroy(h2)
    out5 = (ct.c_int32 * 5)()
    fake = ct.c_void_p(256 * 4096)  # never touched: the arguments are refused first
    assert lib.pit_autotune_adi(ct.byref(pb), p.N, p.m, f, g, fake, n, out5, None, None) == P.EINVAL  # 1D
    assert lib.pit_autotune_adi(ct.byref(pb2), p2.N, p2.m, f2, g2, None, n2, out5, None, None) == P.EINVAL
    assert lib.pit_autotune_adi(ct.byref(pb2), p2.N, p2.m, f2, g2, fake, n2, None, None, None) == P.EINVAL


def test_stream_copy_refuses_bad_arguments():
    lib = P.load()
    a = ct.c_void_p(256 * 4096)  # never touched: the arguments are refused first
    assert lib.pit_stream_copy(None, a, 16, None) == P.EINVAL
    assert lib.pit_stream_copy(a, None, 16, None) == P.EINVAL
    assert lib.pit_stream_copy(a, a, 24, None) == P.EINVAL
    assert lib.pit_stream_copy(ct.c_void_p(256 * 4096 + 8), a, 16, None) == P.EINVAL


def test_time_dependent_operator_validates_and_sizes_on_the_host():
    """pit_set_nu_t: N positive finite factors on a 1D context; the per-slice
    tables enlarge the workspace; 2D, bad values and a source are refused;
    NULL restores the constant operator's size."""
    lib = P.load()
    p = wl.C2.with_(N=6, m=4)
    _, h = create(p)
    base = lib.pit_workspace_bytes(h)
    s = (ct.c_double * p.N)(*[1.0, 2.0, 0.5, 1.5, 3.0, 0.7])
    assert lib.pit_set_nu_t(h, s) == P.OK
    assert lib.pit_workspace_bytes(h) > base
    bad = (ct.c_double * p.N)(*[1.0, 2.0, 0.0, 1.5, 3.0, 0.7])
    assert lib.pit_set_nu_t(h, bad) == P.EINVAL
    f = (ct.c_double * p.npts)(*([0.1] * p.npts))
    assert lib.pit_set_source(h, f) == P.EINVAL  # not with a time-dependent operator
    assert lib.pit_set_nu_t(h, None) == P.OK
    assert lib.pit_workspace_bytes(h) == base
    assert lib.pit_set_source(h, f) == P.OK
    assert lib.pit_set_nu_t(h, s) == P.EINVAL  # not with a source
    lib.pit_destroy(h)
    _, h2 = create(wl.C3.with_(N=2, m=2))
    assert lib.pit_set_nu_t(h2, (ct.c_double * 2)(1.0, 2.0)) == P.EINVAL  # 1D only
    lib.pit_destroy(h2)
    assert lib.pit_set_nu_t(None, s) == P.EINVAL
