"""Oracle: plain arbitrary-precision CPU MPS simulator (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
import this package.  The device library never does, and this package never
imports the device library.  See ``mps_oracle.cpp`` for what each routine follows
in the paper (Section 3.1, Eqs. (1) and (2)).
"""
from .oracle import OracleMPS, OracleSV, osvd, oracle_threads, set_max_sweeps, lib_path  # noqa: F401
