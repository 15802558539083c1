"""FP64 CPU oracle of the differentiable Poisson solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It shares no code with the HIP library
(``paper_2106_03452_amd``) and neither side imports the other; both consume the
float32 inputs produced by ``psr_synth``.

Every function is pinned by ``tests/test_oracle_*.py`` against values fixed by
the paper and by mathematics (worked splat example, brute-force trilinear
weights, naive DFT, single-Fourier-mode closed forms, a dense FFT-free spectral
solve, adjoint dot products, finite differences, invariants).
The Marching Cubes layer and its inverse-normal gradient (main Sec. 3.2,
Eq. 6) are in ``oracle.mc``, pinned by ``tests/test_mc_oracle.py``; the
pieces of the optimisation loop (mesh sampling, Chamfer loss, connected
components for the resampling) in ``oracle.opt``, pinned by
``tests/test_opt_oracle.py``.
"""
from .dpsr import *  # noqa: F401,F403
from . import dpsr  # noqa: F401
from . import mc  # noqa: F401
from . import opt  # noqa: F401
