"""FP64 CPU oracle of the differentiable Poisson solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It shares no code with the HIP library
(``paper_2106_03452_amd``) and neither side imports the other; both consume the
float32 inputs produced by ``psr_synth``.

Every function is pinned by ``tests/test_oracle_*.py`` against values fixed by
the paper and by mathematics (worked splat example, brute-force trilinear
weights, naive DFT, single-Fourier-mode closed forms, a dense FFT-free spectral
solve, adjoint dot products, finite differences, invariants).
"""
from .dpsr import *  # noqa: F401,F403
from . import dpsr  # noqa: F401
