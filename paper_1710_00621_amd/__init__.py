"""MI355X (gfx950) solver for the multi-resolution Wiener-filter /
constrained-realization system of Seljebotn et al. (arXiv:1710.00621).

The compute path is the HIP library ``libcrsolve.so`` (C ABI in
``include/crsolve.h``); ``crsolve`` binds it on torch tensors.  ``inputs``
draws seeded synthetic workloads.  Submodules are imported lazily so that
``inputs`` can be used without a built library.
"""
__all__ = ["crsolve", "inputs"]
