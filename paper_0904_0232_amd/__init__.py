"""MI355X-native GRPIC hot path (Watson & Nishikawa, arXiv:0904.0232).

The compute lives in ``libgrpic.so`` (hand-written HIP for gfx950) behind the
C ABI of ``include/grpic.h``; ``capi`` is its ctypes binding and ``run`` a
small convenience layer that fills a ``grpic_config`` from a workload
description.  ``inputs`` holds the seeded synthetic workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "capi", "run"]


def __getattr__(name):
    if name in ("capi", "run"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
