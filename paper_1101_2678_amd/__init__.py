"""Ant System for the symmetric Euclidean TSP on AMD Instinct MI355X (gfx950).

The hot path of Cecilia et al. (arXiv:1101.2678) -- tour construction by the
random proportional rule (Eq. 1) and the pheromone update (Eqs. 2-4) -- runs
as hand-written HIP kernels in ``libaco.so`` behind the C ABI of
``include/aco.h``.  ``paper_1101_2678_amd.aco`` is the ctypes binding.

The binding is imported lazily so that ``import paper_1101_2678_amd`` works
on a machine without the built library (for example to run the build).
"""
from __future__ import annotations

__all__ = ["aco", "Colony"]


def __getattr__(name):
    import importlib

    if name == "aco":
        return importlib.import_module(".aco", __name__)
    if name == "Colony":
        return importlib.import_module(".aco", __name__).Colony
    raise AttributeError(name)
