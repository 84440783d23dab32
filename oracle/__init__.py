"""FP64 CPU oracle for the LB-SMRT collide-and-stream step.

Test infrastructure only: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only code allowed to import it.
It shares no code with the HIP library in ``paper_2401_11086_amd``.
"""
from .lbsmrt_oracle import *  # noqa: F401,F403
