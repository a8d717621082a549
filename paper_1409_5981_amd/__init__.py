"""PMMM far field on MI355X (gfx950): HIP kernels behind a C ABI.

``paper_1409_5981_amd.Plan`` (from ``_lib``) is the Python entry point; it
loads ``libpmmm.so`` on first use and raises if the library is missing.
``paper_1409_5981_amd.inputs`` holds the seeded synthetic workloads.
"""
from __future__ import annotations

__all__ = ["Plan", "load"]


def __getattr__(name):
    if name in ("Plan", "load", "PMMMError"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
