"""The benchmark workloads as seeded synthetic problems.

The paper's problems come from a finite-difference generator and from a
public sparse-matrix collection (§V, §V-G); neither is available here, so the
stencil matrices of :mod:`workloads.stencils` stand in for them.  Sizes follow
the paper where it prints them (Table III: Laplace3D150 has n = 3,375,000 and
nnz = 23,490,000; UniFlow2D2500 has n = 6,250,000 and nnz = 31,240,000).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .prng import uniform01, uniform_pm1, uniform_int
from .stencils import CSR, laplace2d, laplace3d, convdiff2d

__all__ = ["Problem", "host_matvec", "config1_laplace2d", "config2_laplace3d", "fd_laplace3d",
           "config3_convdiff", "config4_batch", "random_rhs", "poly_start_vector", "block_diag",
           "stack_rows", "config5_systems"]


def host_matvec(A: CSR, x: np.ndarray) -> np.ndarray:
    """Right-hand side construction b = A x in float64 (scipy, input prep only)."""
    import scipy.sparse as sp
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return M @ np.asarray(x, dtype=np.float64)


@dataclass
class Problem:
    name: str
    A: CSR
    b: np.ndarray
    x_true: Optional[np.ndarray]
    restart: int
    poly_degree: int
    inner: str            # "f32" (GMRES-IR) or "f64" (plain GMRES)
    tol: float = 1e-10
    poly_seed: int = 0
    meta: dict = field(default_factory=dict)


def poly_start_vector(n: int, seed: int) -> np.ndarray:
    """Start vector of the polynomial's Arnoldi run: U(-1,1) from stream seed+1."""
    return uniform_pm1(seed + 1, n)


def config1_laplace2d(N: int = 64, restart: int = 50) -> Problem:
    """2D Laplacian 4/-1, b = A * ones, x0 = 0, plain FP64 GMRES(50)."""
    A = laplace2d(N)
    b = host_matvec(A, np.ones(A.n))
    return Problem(f"laplace2d_N{N}", A, b, np.ones(A.n), restart, 0, "f64")


def config2_laplace3d(N: int = 150, seed: int = 2, restart: int = 50) -> Problem:
    """3D Laplacian 6/-1, b = A x_true with x_true ~ U(-1,1), GMRES(50)-IR."""
    A = laplace3d(N)
    x_true = uniform_pm1(seed, A.n)
    return Problem(f"laplace3d_N{N}", A, host_matvec(A, x_true), x_true, restart, 0, "f32")


def fd_laplace3d(N: int = 200, restart: int = 50) -> Problem:
    """The GMRES-FD switch-point problem of §V-A: 3D Laplacian 6/-1 on N^3, b = ones
    and x0 = 0 (the right-hand side and start vector of every experiment, §V)."""
    A = laplace3d(N)
    return Problem(f"laplace3d_N{N}_ones", A, np.ones(A.n), None, restart, 0, "f32")


def uniflow_wind(x, y):
    return np.cos(np.pi * x), np.sin(np.pi * y)


def config3_convdiff(N: int = 2500, seed: int = 3, restart: int = 100, degree: int = 25,
                     eps: float = 1e-3) -> Problem:
    """Upwind conv-diff, eps = 1e-3, wind (cos pi x, sin pi y), GMRES(100)-IR + poly(25)."""
    A = convdiff2d(N, eps, uniflow_wind)
    x_true = uniform_pm1(seed, A.n)
    return Problem(f"convdiff2d_N{N}", A, host_matvec(A, x_true), x_true, restart, degree,
                   "f32", poly_seed=seed)


def random_rhs(seed: int, n: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` right-hand sides of length n (column-major, shape n x count), U(-1,1)."""
    return uniform_pm1(seed, n * count, offset).reshape(count, n).T.copy()


def config4_batch(count: int = 256, seed: int = 4, nrhs: int = 16, side_lo: int = 32,
                  side_hi: int = 256):
    """Independent conv-diff systems with several right-hand sides each.

    System i draws from stream ``seed ^ i``: draw 1 the grid side U{lo..hi},
    draw 2 the diffusion 10^U(-3,0), draw 3 the wind angle U[0, 2 pi), then
    ``nrhs * n`` entries U(-1,1) for the right-hand sides (column by column).
    """
    systems = []
    for i in range(count):
        s = seed ^ i
        N = int(uniform_int(s, side_lo, side_hi, 1)[0])
        eps = float(10.0 ** (-3.0 + 3.0 * uniform01(s, 1, 1)[0]))
        phi = float(2.0 * np.pi * uniform01(s, 1, 2)[0])
        A = convdiff2d(N, eps, lambda x, y, p=phi: (np.cos(p), np.sin(p)))
        B = random_rhs(s, A.n, nrhs, offset=3)
        systems.append(dict(A=A, B=B, N=N, eps=eps, phi=phi))
    return systems


def block_diag(mats) -> CSR:
    """One CSR matrix with the given matrices as diagonal blocks (global columns)."""
    n = sum(A.n for A in mats)
    nnz = sum(A.nnz for A in mats)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    r = c = 0
    for A in mats:
        row_ptr[r + 1:r + A.n + 1] = A.row_ptr[1:].astype(np.int64) + c
        col[c:c + A.nnz] = A.col_idx + r
        val[c:c + A.nnz] = A.val
        r += A.n
        c += A.nnz
    return CSR(n, row_ptr.astype(np.int32), col, val)


def stack_rows(blocks) -> np.ndarray:
    """Row-major (rows x p) array from per-system (n_s x p) blocks."""
    return np.ascontiguousarray(np.concatenate(blocks, axis=0))


def config5_systems(count: int, seed: int = 5, side2d=(64, 1024), side3d=(16, 101), start: int = 0):
    """Systems start .. start+count-1 for the parameter predictor: half upwind
    convection-diffusion (diffusion 10^U(-3,0), random wind angle), a quarter
    2D and a quarter 3D Laplacians; 2D grid side U{64..1024}, 3D side
    U{16..101} (n of the same range).  System i draws from stream
    seed ^ (i + 1): draw 1 the kind, draw 2 the grid side, draws 3-4 diffusion
    and wind angle, then x_true."""
    out = []
    for i in range(start, start + count):
        s = seed ^ (i + 1)
        u = uniform01(s, 4)
        kind = "convdiff" if u[0] < 0.5 else ("laplace2d" if u[0] < 0.75 else "laplace3d")
        if kind == "laplace3d":
            N = side3d[0] + min(int(u[1] * (side3d[1] - side3d[0] + 1)), side3d[1] - side3d[0])
            A = laplace3d(N)
            meta = dict(kind=kind, N=N)
        else:
            N = side2d[0] + min(int(u[1] * (side2d[1] - side2d[0] + 1)), side2d[1] - side2d[0])
            if kind == "laplace2d":
                A = laplace2d(N)
                meta = dict(kind=kind, N=N)
            else:
                eps = float(10.0 ** (-3.0 + 3.0 * u[2]))
                phi = float(2.0 * np.pi * u[3])
                A = convdiff2d(N, eps, lambda x, y, p=phi: (np.cos(p), np.sin(p)))
                meta = dict(kind=kind, N=N, eps=eps, phi=phi)
        x_true = uniform_pm1(s, A.n, 4)
        out.append(dict(A=A, b=host_matvec(A, x_true), x_true=x_true, seed=s, index=i, **meta))
    return out
