"""Plain FP64 CPU oracle for the curvilinear steepest-descent minimizer.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test suite,
the package smoke check and the benchmark's CPU-baseline leg may import it;
the library never does, and it shares no code with the library (the two only
consume the same seeded inputs from ``paper_1309_5796_amd.meshgen``).

Method: Exl et al., "LaBonte's method revisited" (arXiv:1309.5796).
* ``fem``       -- P1 tetrahedral discretization of the four energy terms and
                   the scalar-potential stray field with the open-boundary
                   space transformation (Method section, eq. (1); Results,
                   "Comparison with LLG solver").
* ``minimize``  -- the Cayley curvilinear step (eq. (8)), BB step lengths
                   (eq. (10)) with the adaptive switching rule, the 20-energy
                   nonmonotone globalization, the stopping test, and the
                   hysteresis continuation (Introduction, Hysteresis).

Where the paper is silent the oracle follows the readings listed in the
design notes (variational lumped field, Rodrigues form of the Cayley step,
adaptive BB constants, Armijo parameters, shell map).  Every function that
has no independent pin says "parity unpinned" in its docstring.
"""
from .fem import MU0, System, shell_metric, tet_geometry  # noqa: F401
from .minimize import (cayley, hysteresis, minimize, Options, Result,  # noqa: F401
                       switching_fields)
