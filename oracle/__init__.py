"""Plain FP64 CPU oracle for the FAST-HALS sweep of PL-NMF (arXiv 1904.07935).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path.

Modules
-------
hals        FAST-HALS (Alg. 1) step by step, the tiled W/H update of Alg. 2
            (Eq. 4-6), the objective (Eq. 2) and the relative objective of
            Sec. 6.2, and H-only fold-in with W fixed.
mlp         FP64 forward/backward/Adam for the fold-in warm-start network.
mu          The multiplicative-update baseline (Sec. 2.1; Lee-Seung rules).
tile_model  The data-movement model of Sec. 5 (Eq. 9-11), model only.
"""
from . import hals, mlp, mu, tile_model  # noqa: F401
