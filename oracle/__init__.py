"""Oracle package: double-precision CPU reference of the t-SVDM path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py, never by the product path.
"""
from .oracle import *  # noqa: F401,F403
from . import oracle  # noqa: F401
