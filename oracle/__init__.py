"""FP64 CPU oracle for the ERBF-fit hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 numpy
restatement of what the method computes, written from the paper's equations.
It exists to check the HIP path; nothing in the product may import, call or
link it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

It shares no code with the HIP path.  Inputs (grid axes, raw signed
distances, float32 parameters) come from the ``synth`` package, which holds
none of the method's arithmetic; the oracle upcasts them to float64.

Every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants, brute force and
finite differences.  Functions without such a pin say "parity unpinned" in
their docstring.
"""

from .erbf import *  # noqa: F401,F403
from . import schedule  # noqa: F401,E402
from . import metrics  # noqa: F401,E402
