"""Plain FP64 CPU oracle for the dense-INLA per-theta Laplace evaluation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library under ``paper_2311_08050_amd/``; the two meet only at the seeded
input generators of ``paper_2311_08050_amd.synth``, which hold none of the
method's arithmetic.

Modules
-------
``inla_oracle``  the method, step by step, in float64 numpy/scipy.
``brute``        an independent exact-rational twin for tiny problems
                 (Gaussian elimination over ``fractions.Fraction``), used to pin
                 ``inla_oracle``.
"""
from . import inla_oracle, brute  # noqa: F401
