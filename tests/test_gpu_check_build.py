"""GPU: the checking build (libpitsbicg_check.so, -DPIT_CHECK: every
kernel's LDS filled with NaN before first use) gives the oracle's results on
every kernel family, so no kernel reads LDS that its workgroup did not
write.  Runs tests/check_build_cases.py in a process of its own (the library
choice is made at load)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_checking_build_matches_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = os.path.join(ROOT, "paper_2203_10148_amd", "libpitsbicg_check.so")
    assert os.path.exists(lib), "build it with `python -m paper_2203_10148_amd.build`"
    print("\n[case] checking build", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "check_build_cases.py")],
                       env=dict(os.environ, PIT_LIBRARY="check"), capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "check build: ok" in r.stdout
