"""Plain FP64 CPU oracle for the parallel-in-time multigrid FGMRES solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP path is checked against.  Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it;
the product path never does, and it shares no code with the HIP library.

What it computes (arXiv 2405.04808):
  * system.py   -- the lifted augmented matrix in type-major order (Fig. 4),
                   its time-major permutation (Fig. 5, eq. (augsysp)) and the
                   block split L + D + L^T (Sec. 5.3.2);
  * transfer.py -- injection / linear interpolation in time, averaging /
                   piecewise-constant for the control (Sec. 5.3.1);
  * krylov.py   -- right-preconditioned GMRES and flexible GMRES (Saad 1993),
                   written out with modified Gram-Schmidt and a dense
                   least-squares solve of the Hessenberg problem;
  * multigrid.py-- block Jacobi (eq. (jacobi)), forward / backward /
                   symmetric block Gauss-Seidel (Sec. 5.3.4), the recursive
                   V-cycle (Alg. 1) with its W and F variants, and the
                   preconditioned outer solve (Sec. 6);
  * unlifted.py -- the system without virtual variables (Fig. 2) and the
                   lift / project maps that carry the lifted cycle to it;
  * dogleg.py   -- the discrete Burgers equation F(u, z~) = 0, its Jacobian
                   B = dF, minimum-norm Gauss-Newton steps from the augmented
                   system (Sec. 3) and Powell's dogleg with viscosity
                   continuation (Sec. 6, Sec. 6.2, Table 6).

Everything is assembled scipy.sparse matrices and SuperLU factorisations of
the block parts; no Schur complement or other derived block algebra is used,
so the oracle also checks the HIP path's derived formulas.
"""
from .system import (type_offsets, assemble_B, assemble_A, time_major_perm,
                     block_bounds, split_blocks)
from .transfer import restriction, interpolation
from .krylov import gmres_right, fgmres
from .multigrid import OracleLevel, Hierarchy, direct_solve

__all__ = ["type_offsets", "assemble_B", "assemble_A", "time_major_perm",
           "block_bounds", "split_blocks", "restriction", "interpolation",
           "gmres_right", "fgmres", "OracleLevel", "Hierarchy", "direct_solve"]
