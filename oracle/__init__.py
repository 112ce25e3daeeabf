"""FP64 CPU oracle for mixTS-PIMD.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The product library never imports it.
"""
from .oracle import (  # noqa: F401
    OracleSystem, build, slice_bead, nm_basis, nm_lambda, constants,
    set_threads, num_threads, E_NAMES, E_N, N_POT,
)
