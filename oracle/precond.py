"""Oracle: the block Jacobi right preconditioner (§III-D; "J k" in Table III, §V-G).

TEST INFRASTRUCTURE ONLY (see the package docstring).

M = blockdiag(A)^-1 with diagonal blocks of ``block`` consecutive rows (the
last block takes the remaining rows).  z = M v solves A_bb z_b = v_b for every
block b with a dense LU solve in the working precision ``dt`` (numpy's LAPACK
gesv; float32 data gives a float32 factorisation).
"""
from __future__ import annotations

import numpy as np


def diagonal_block(A, r0: int, r1: int) -> np.ndarray:
    """Dense A[r0:r1, r0:r1] from the CSR rows (duplicate entries summed)."""
    B = np.zeros((r1 - r0, r1 - r0))
    for r in range(r0, r1):
        for k in range(A.row_ptr[r], A.row_ptr[r + 1]):
            c = A.col_idx[k]
            if r0 <= c < r1:
                B[r - r0, c - r0] += A.val[k]
    return B


def bjac_apply(A, block: int, v: np.ndarray, dt=np.float64) -> np.ndarray:
    dt = np.dtype(dt)
    v = np.asarray(v).astype(dt)
    z = np.zeros(A.n, dtype=dt)
    for r0 in range(0, A.n, block):
        r1 = min(r0 + block, A.n)
        B = diagonal_block(A, r0, r1).astype(dt)
        z[r0:r1] = np.linalg.solve(B, v[r0:r1])
    return z
