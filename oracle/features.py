"""Oracle: the 16 matrix features of the parameter predictor, from their definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper guides the choice of restart length, polynomial degree and inner
precision by properties of the matrix: how hard it is to converge (§V-E),
how the polynomial behaves for non-normal or indefinite spectra (§V-C, §V-F)
and whether float32 suffices (§V-B).  The features are cheap estimates of
those properties; their list is this project's reading (the paper names
none).  Every value is computed here from a dense copy of A in float64, row by
row, and the spectral ones from the Ritz values of a float64 Arnoldi run
(Alg. 1 with CGS2) of min(5, n) steps from the caller's start vector.
"""
from __future__ import annotations

import math

import numpy as np

from .krylov import arnoldi

ARNOLDI_STEPS = 5


def row_stats(A) -> dict:
    """Per-row quantities of A: diagonal a_ii, off-diagonal absolute sum
    r_i = sum_{j != i} |a_ij| (added in ascending j, so that the decision
    ratio >= 1 is taken on one well-defined floating-point value), nonzeros per
    row, ||A||_F^2 and ||A - A^T||_F^2, from the dense matrix."""
    D = A.to_dense()
    n = A.n
    d = np.diag(D).copy()
    r = np.zeros(n)
    for i in range(n):
        for j in range(n):
            if j != i and D[i, j] != 0.0:
                r[i] += abs(D[i, j])
    return dict(d=d, r=r, nnz_row=np.diff(A.row_ptr), fro2=float((D * D).sum()),
                skew2=float(((D - D.T) ** 2).sum()))


def features(A, v0: np.ndarray) -> np.ndarray:
    """The 16 features in the library's order (see matrix_features)."""
    n = A.n
    s = row_stats(A)
    d, r = s["d"], s["r"]
    maxd = max(float(np.abs(d).max()), 1e-300)
    off = r > 0
    dom = np.abs(d[off]) / r[off]
    mean_d = float(d.mean())
    std_d = float(np.sqrt(max((d * d).mean() - mean_d * mean_d, 0.0)))
    # at most n steps: the Krylov space of an n x n matrix has dimension <= n
    _, H, k = arnoldi(A, v0, min(ARNOLDI_STEPS, n), np.float64)
    theta = np.linalg.eigvals(H[:k, :k])
    mod = np.abs(theta)
    amax, amin = float(mod.max()), float(mod.min())
    f = [
        math.log10(n),
        A.nnz / n,
        float(s["nnz_row"].max()),
        float(dom.min()) if off.any() else 10.0,
        float(dom.sum()) / max(int(off.sum()), 1),
        float((dom >= 1).sum()) / n,
        float((d - r).min()) / maxd,
        float((d + r).max()) / maxd,
        float(r.max()) / maxd,
        math.sqrt(s["skew2"] / max(s["fro2"], 1e-300)),
        std_d / max(abs(mean_d), 1e-300),
        amax / maxd,
        amin / maxd,
        math.log10(amax / max(amin, 1e-300)),
        float(np.abs(theta.imag).max()) / amax,
        float(H[k, k - 1]) / amax,
    ]
    return np.nan_to_num(np.array(f), nan=0.0, posinf=1e6, neginf=-1e6)
