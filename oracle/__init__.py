"""Plain CPU oracle for GMRES(m), GMRES-IR, GMRES-FD and the polynomial and block Jacobi preconditioners.

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports this
package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may call it.  It is written straight from the paper (Alg. 1,
Alg. 2, §III-A, §III-B, §III-C, §III-D, §V-D) in numpy, slow and unblocked, so that
each step can be checked against the text by eye.  It shares no code with the
GPU path; the two only meet through the seeded inputs of ``workloads``.
"""
from .krylov import (spmv, cgs2, apply_givens_column, back_substitute, gmres,  # noqa: F401
                     gmres_ir, gmres_fd, cast_wrapped, half_sigma, half_store, GmresOutcome, arnoldi)
from .poly import harmonic_ritz_values, leja_order, poly_roots, poly_apply  # noqa: F401
from .precond import bjac_apply, diagonal_block  # noqa: F401
from .block import block_arnoldi, block_gmres_ir, cholqr2, dependent_columns, spmm, start_block  # noqa: F401,E402
