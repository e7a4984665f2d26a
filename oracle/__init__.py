"""FP64 CPU oracle for the compress-and-eliminate factorization.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything
in this package.  The product path (``paper_1603_09133_amd``) never does,
and the two share no code: the only module both use is ``problems`` (seeded
matrix and right-hand-side generators, none of the method's arithmetic).
"""
from .symbolic import (morton_key, grid_order, level1_pattern, coarsen, coarse_pattern,
                       colour_order, element_order, simulate_level, adjacency, live_pairs)
from .ce import (NotSPD, CEOptions, CEFactor, LevelFactor, ce_factor, ce_solve,
                 ce_multiply, ce_dense, pcg, minres)
