"""CPU FP64 oracle for FGFRFT -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The GPU library never
calls it and shares no code with it: both sides receive the same inputs
from :mod:`synth` and nothing else.

Every routine is a plain, slow, direct statement of a definition or
algorithm from the paper (arXiv 2602.20870), in float64 / complex128,
with NumPy/SciPy primitives (matmul, Schur, eigh) as the only library
steps.  See :mod:`oracle.fgfrft` for the citations; each function is
pinned by a test under ``tests/test_oracle_*.py`` against values fixed by
the paper or by the mathematics (closed forms, printed tables, exact
identities, brute force), not by re-typing its own formula.

Parity status: every public routine is pinned except where its docstring
says "parity unpinned".
"""
from .fgfrft import *  # noqa: F401,F403
from .fgfrft import __all__  # noqa: F401
