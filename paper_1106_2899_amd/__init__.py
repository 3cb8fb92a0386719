"""MI355X-native single-chain slip-spring ensembles (HIP, gfx950).

The step of the method runs in libssp.so (built from csrc/ by
``python -m paper_1106_2899_amd.build``); this package is its Python binding.
"""
from ._lib import SspError  # noqa: F401

__all__ = ["Ensemble", "SspError", "workloads"]


def __getattr__(name):
    if name == "Ensemble":
        from .ensemble import Ensemble

        return Ensemble
    raise AttributeError(name)
