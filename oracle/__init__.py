"""FP64 CPU oracle for the multi-rhs x multi-shift twisted-mass multigrid path.

TEST INFRASTRUCTURE ONLY.  This package may be imported by the tests, by the
package's smoke check and by the benchmark's CPU-baseline leg, and by nothing
else: the GPU library never routes any computation through it.  It shares no
code with the GPU path (the seeded input generators live in ``synthetic``,
which holds none of the method's arithmetic).

Plain, slow, obviously-correct numpy in complex128:

* ``dirac``     - the twisted-mass Wilson operator (Fig. 6 caption of the paper)
* ``multigrid`` - SAP, aggregation, R/P, Galerkin coarse operators (section 2)
* ``krylov``    - GMRES / FGMRES / block GMRES (section 4)
* ``solver``    - the MG-preconditioned simultaneous multi-rhs multi-shift solve
* ``ptc``       - gauge-covariant parallel-transport convolution smoother
* ``nondegenerate`` - the non-degenerate twisted-mass doublet operator
"""
from .dirac import WilsonTM, gammas, gamma5
from .multigrid import (Blocking, FineLevel, CoarseOp, build_prolongator, restrict, prolong,
                        galerkin, sap, mr_smoother, block_mr, block_mr_oddeven)
from .krylov import gmres, fgmres, block_gmres, gmres_dr, harmonic_ritz, col_norm, col_dot
from .solver import MGParams, OracleMG
from . import ptc
from .nondegenerate import nd_apply, nd_mus
