"""FP64 CPU oracle for random-projection classical MDS.

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``.  The GPU library neither imports nor
links anything here; the two share no code.  See ``mds_oracle`` for what each
function computes and which passage of the paper it follows.
"""
from .mds_oracle import *  # noqa: F401,F403
from .mds_oracle import __all__  # noqa: F401
from . import mds_oracle_large  # noqa: F401  (row-blocked variant for large n)
from . import distances  # noqa: F401  (pairwise distances, the input step)
from . import components  # noqa: F401  (threshold-graph connected components)
