"""MI355X-native dense-INLA Laplace evaluation (arXiv 2311.08050 hot path).

The compute path is the HIP library ``libinla_dense.so`` (C-ABI declared in
``include/inla_dense.h``); ``binding`` marshals arguments to it.  ``synth`` draws
seeded synthetic inputs.  Importing this package loads nothing; the library is
loaded on first use of ``binding.Library``.
"""
__all__ = ["binding", "synth"]
