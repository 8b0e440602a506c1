"""FP64 CPU oracle for the FWI hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
bench.py's CPU-baseline leg, never by the product path. It shares no code with
the HIP library. Each function cites the passage of the paper it follows;
pins live in tests/test_oracle_*.py.
"""
from . import fwi_oracle, series  # noqa: F401
