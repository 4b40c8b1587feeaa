"""Finite-difference test matrices in CSR form (int32 indices, float64 values).

The paper generates its model problems with finite-difference stencils
(§V, opening paragraph) but does not print the stencils, so the definitions
below are this project's reading:

* domain (0,1)^D with N interior points per side and mesh width h = 1/(N+1);
* unknown (i, j[, k]) (1-based) sits in row (k-1)N^2 + (j-1)N + (i-1), x fastest;
* Dirichlet neighbours are dropped (eliminated boundary), columns ascend in a row;
* Laplacians use the unscaled stencils 4/-1 (2D) and 6/-1 (3D);
* convection-diffusion -eps*Lap(u) + w.grad(u) is discretised with
  first-order upwinding and every row is multiplied by h^2, the wind being
  sampled at the node.

This module only builds inputs; it holds none of the solver's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col_idx] = self.val
        return d


def _assemble(n: int, offsets, masks, values) -> CSR:
    """Build CSR from per-row stencil entries given in ascending column order.

    ``offsets[k]`` is the column offset of entry k, ``masks[k]`` a bool array
    (length n) saying which rows have it, ``values[k]`` its value per row
    (scalar or length-n array).
    """
    counts = np.zeros(n, dtype=np.int64)
    for m in masks:
        counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz does not fit int32")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = row_ptr[:-1].copy()
    rows = np.arange(n, dtype=np.int64)
    for off, m, v in zip(offsets, masks, values):
        r = rows[m]
        p = pos[r]
        col[p] = (r + off).astype(np.int32)
        val[p] = v[m] if isinstance(v, np.ndarray) else v
        pos[r] += 1
    return CSR(n, row_ptr.astype(np.int32), col, val)


def _grid2(N: int):
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N + 1          # x index, 1..N
    j = r // N + 1         # y index, 1..N
    return n, i, j


def laplace2d(N: int) -> CSR:
    """5-point Laplacian 4/-1 on an N x N interior grid."""
    n, i, j = _grid2(N)
    return _assemble(
        n,
        [-N, -1, 0, 1, N],
        [j > 1, i > 1, np.ones(n, bool), i < N, j < N],
        [-1.0, -1.0, 4.0, -1.0, -1.0],
    )


def laplace3d(N: int) -> CSR:
    """7-point Laplacian 6/-1 on an N x N x N interior grid."""
    n = N * N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N + 1
    j = (r // N) % N + 1
    k = r // (N * N) + 1
    NN = N * N
    return _assemble(
        n,
        [-NN, -N, -1, 0, 1, N, NN],
        [k > 1, j > 1, i > 1, np.ones(n, bool), i < N, j < N, k < N],
        [-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0],
    )


def convdiff2d(N: int, eps: float, wind) -> CSR:
    """Upwind 5-point convection-diffusion, rows scaled by h^2.

    ``wind(x, y) -> (wx, wy)`` takes node coordinates (arrays) and returns the
    velocity there.  Entries: diagonal 4 eps + h(|wx| + |wy|); west
    -eps - h max(wx, 0); east -eps - h max(-wx, 0); south -eps - h max(wy, 0);
    north -eps - h max(-wy, 0).
    """
    n, i, j = _grid2(N)
    h = 1.0 / (N + 1)
    wx, wy = wind(i * h, j * h)
    wx = np.broadcast_to(np.asarray(wx, dtype=np.float64), (n,))
    wy = np.broadcast_to(np.asarray(wy, dtype=np.float64), (n,))
    diag = 4.0 * eps + h * (np.abs(wx) + np.abs(wy))
    west = -eps - h * np.maximum(wx, 0.0)
    east = -eps - h * np.maximum(-wx, 0.0)
    south = -eps - h * np.maximum(wy, 0.0)
    north = -eps - h * np.maximum(-wy, 0.0)
    return _assemble(
        n,
        [-N, -1, 0, 1, N],
        [j > 1, i > 1, np.ones(n, bool), i < N, j < N],
        [south, west, diag, east, north],
    )


def nnz_closed_form_2d(N: int) -> int:
    return 5 * N * N - 4 * N


def nnz_closed_form_3d(N: int) -> int:
    return 7 * N ** 3 - 6 * N ** 2


def laplacian_eigs_closed_form(N: int, dim: int) -> np.ndarray:
    """All eigenvalues of the dim-D Dirichlet Laplacian (2*dim/-1 stencil)."""
    k = np.arange(1, N + 1)
    lam1 = 4.0 * np.sin(np.pi * k / (2.0 * (N + 1))) ** 2
    if dim == 1:
        return lam1
    if dim == 2:
        return (lam1[:, None] + lam1[None, :]).ravel()
    return (lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]).ravel()
