"""Plain FP64 CPU oracle of the correction-function KFBI method (Zhou & Ying,
arXiv 2309.05965).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test-suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path never does, and it shares no code with the HIP
library.

Modules
  levelset     level-set functions H and their gradients (Sec. 5.1)
  geometry     node regions, surface points, collocation stencils,
               irregular nodes, closest-centre map, interpolation blocks
               (Secs. 5.1, 5.2, 5.3, 5.5)
  collocation  local Cauchy problem by square collocation (Secs. 5.3.1, 5.4)
  fd           compact finite-difference operators and the DST box solve
               (Sec. 5.2, eqs. 9p-cds / 27p-cds; FFT solver of Alg. 1 Step 3.3)
  kfbi         simple interface solve, BIE operator, GMRES, full solve
               (Secs. 3.2, 4, 5.5, Alg. 1)

Every readings of the paper that the oracle takes where the paper is silent
is listed in the repository design notes; each function cites the passage it
follows.  Parity status: every function is pinned by a ``-m "not gpu"`` test
(see tests/test_oracle_*.py); none is "parity unpinned".
"""
