"""Oracle package: the CPU reference of the rounded-KLT codec.

TEST INFRASTRUCTURE ONLY.  Imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py; never by the product library or its binding.
It shares no code with the HIP path.
"""
from .rklt_oracle import *  # noqa: F401,F403
from . import metrics  # noqa: F401
