"""FP64 CPU oracle for the ESDG shallow-water right-hand side (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline legs (the cpu_baseline
of the RHS benchmark and the CPU side of the volume-kernel ratio, both skipped by
--no-cpu-baseline) may import this package.  The HIP library never imports it and shares no code with it.
"""
from .esdg_oracle import *  # noqa: F401,F403
