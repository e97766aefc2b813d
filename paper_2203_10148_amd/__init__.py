"""libpitsbicg: an MI355X-native (gfx950, HIP) PiTSBiCG hot path.

The compute lives in ``libpitsbicg.so`` (HIP kernels behind a C ABI declared in
``include/pitsbicg.h``).  ``paper_2203_10148_amd.pitsbicg`` is the thin ctypes
binding; ``paper_2203_10148_amd.workloads`` holds the seeded synthetic inputs.
Importing the package itself loads nothing.
"""

__all__ = ["pitsbicg", "workloads"]
__version__ = "0.1.0"


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
