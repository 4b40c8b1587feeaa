"""Oracle: CSR SpMV, CGS2 Arnoldi, Givens least squares, GMRES(m), GMRES-IR, GMRES-FD.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Precision model.  ``dt`` is the working precision of vector arithmetic
(numpy float64 or float32).  The Hessenberg matrix, the Givens rotations, the
right-hand side g of the small least-squares problem and its solution y are
always float64, which is this project's reading for the inner solve of
GMRES-IR (the paper's solver kept them in the working precision on the host).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

FLT_MIN = float(np.finfo(np.float32).tiny)


# ---------------------------------------------------------------------------
# O1: CSR SpMV, the dot product of one matrix row with x (§V-D):
#     y_i = sum_{k = rowptr[i]}^{rowptr[i+1]-1} val[k] * x[col[k]],
# summed in ascending k, in the working precision of ``x``.
# ---------------------------------------------------------------------------
def spmv(A, x: np.ndarray, dt=None) -> np.ndarray:
    dt = np.dtype(dt or x.dtype)
    val = A.val.astype(dt, copy=False)
    x = np.asarray(x).astype(dt, copy=False)
    start = A.row_ptr[:-1].astype(np.int64)
    lens = np.diff(A.row_ptr).astype(np.int64)
    y = np.zeros(A.n, dtype=dt)
    for s in range(int(lens.max()) if A.n else 0):
        rows = np.nonzero(lens > s)[0]
        k = start[rows] + s
        y[rows] = y[rows] + val[k] * x[A.col_idx[k]]
    return y


# ---------------------------------------------------------------------------
# O2: one CGS2 step (Alg. 1 with the two Gram-Schmidt passes of §III-A):
#     h1 = V_j^T w ; w = w - V_j h1 ; h2 = V_j^T w ; w = w - V_j h2 ;
#     H[:j, j] = h1 + h2 ; beta = ||w||.
# ---------------------------------------------------------------------------
def cgs2(V: np.ndarray, j: int, w: np.ndarray):
    Vj = V[:, :j]
    h1 = Vj.T @ w
    w = w - Vj @ h1
    h2 = Vj.T @ w
    w = w - Vj @ h2
    beta = np.sqrt(w @ w)
    return w, h1, h2, beta


def arnoldi(A, v0: np.ndarray, k: int, dt=np.float64, prec: Optional[Callable] = None):
    """k Arnoldi steps with CGS2 from v0; returns V (n x k+1), Hbar (k+1 x k, float64), steps."""
    n = A.n
    V = np.zeros((n, k + 1), dtype=dt)
    H = np.zeros((k + 1, k))
    v = np.asarray(v0).astype(dt)
    V[:, 0] = v / np.sqrt(v @ v)
    steps = 0
    for j in range(k):
        z = prec(V[:, j]) if prec else V[:, j]
        w = spmv(A, z, dt)
        w, h1, h2, beta = cgs2(V, j + 1, w)
        H[: j + 1, j] = h1.astype(np.float64) + h2.astype(np.float64)
        H[j + 1, j] = float(beta)
        steps = j + 1
        if _is_breakdown(beta, dt):
            break
        V[:, j + 1] = w / beta
    return V, H, steps


def _is_breakdown(beta, dt) -> bool:
    """Lucky breakdown (Alg. 1): h_{j+1,j} = 0.  In float32 a value below
    1e3 * FLT_MIN, and any non-finite value, is taken as zero."""
    b = float(beta)
    if not np.isfinite(b):
        return True
    if np.dtype(dt) == np.float32:
        return b <= 1e3 * FLT_MIN
    return b == 0.0


# ---------------------------------------------------------------------------
# O3: least squares on Hbar by Givens rotations (Saad, Iterative Methods,
# §6.5.3, the reference the paper gives for Alg. 1).
# ---------------------------------------------------------------------------
def apply_givens_column(h: np.ndarray, cs: np.ndarray, sn: np.ndarray, g: np.ndarray, j: int):
    """Rotate column j (entries h[0..j+1]) by the j earlier rotations, build
    rotation j, and update g.  Modifies h, cs, sn, g in place; returns |g[j+1]|."""
    for i in range(j):
        hi, hi1 = h[i], h[i + 1]
        h[i] = cs[i] * hi + sn[i] * hi1
        h[i + 1] = -sn[i] * hi + cs[i] * hi1
    a, b = h[j], h[j + 1]
    rho = float(np.hypot(a, b))
    if rho == 0.0:
        cs[j], sn[j] = 1.0, 0.0
    else:
        cs[j], sn[j] = a / rho, b / rho
    h[j] = cs[j] * a + sn[j] * b
    h[j + 1] = 0.0
    g[j + 1] = -sn[j] * g[j]
    g[j] = cs[j] * g[j]
    return abs(g[j + 1])


def back_substitute(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve the upper-triangular system R y = g (k x k) from the bottom up."""
    k = R.shape[0]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        s = g[i]
        for c in range(i + 1, k):
            s -= R[i, c] * y[c]
        y[i] = s / R[i, i]
    return y


@dataclass
class GmresOutcome:
    x: np.ndarray
    converged: bool
    iters: int
    cycles: int
    rel_res: float                    # explicit ||b - A x|| / ||b|| in float64
    implicit_rel_res: float = float("nan")
    history: List[float] = field(default_factory=list)   # explicit rel. residual per restart
    implicit_history: List[float] = field(default_factory=list)  # |g_{j+1}|/||b|| per iteration
    loss_of_accuracy: int = 0         # restarts whose cycle met tol implicitly but not explicitly
    stopped_on_loss: bool = False


def _explicit_rel_res(A, b, x):
    r = b.astype(np.float64) - spmv(A, x.astype(np.float64), np.float64)
    return float(np.linalg.norm(r) / np.linalg.norm(b.astype(np.float64)))


# ---------------------------------------------------------------------------
# O4: restarted GMRES(m) in one working precision (Alg. 1, §III-A).
# The implicit residual |g_{j+1}| is tested after every iteration so that a
# cycle may stop early (§III-B contrasts this with GMRES-IR); convergence is
# then confirmed with the explicit residual, and a false signal (the loss of
# accuracy of §V-F) is counted and simply leads to another restart, or ends
# the solve when ``stop_on_loss`` is set.
# Right preconditioning (§III-D): w = A M v_j and the correction is M V y.
# ---------------------------------------------------------------------------
def gmres(A, b, x0, m: int, tol: float, max_iters: int, dt=np.float64,
          prec: Optional[Callable] = None, max_cycles: Optional[int] = None,
          stop_on_loss: bool = False) -> GmresOutcome:
    n = A.n
    b_w = np.asarray(b).astype(dt)
    bnorm = float(np.linalg.norm(np.asarray(b, dtype=np.float64)))
    x = np.asarray(x0).astype(dt).copy()
    r = b_w - spmv(A, x, dt)
    gamma = np.sqrt(r @ r)
    out = GmresOutcome(x, False, 0, 0, float("nan"))
    out.history.append(_explicit_rel_res(A, b, x))
    if out.history[-1] <= tol:
        out.converged, out.rel_res = True, out.history[-1]
        return out
    it = 0
    cycles = 0
    while it < max_iters and (max_cycles is None or cycles < max_cycles):
        V = np.zeros((n, m + 1), dtype=dt)
        H = np.zeros((m + 1, m))
        cs, sn, g = np.zeros(m), np.zeros(m), np.zeros(m + 1)
        V[:, 0] = r / gamma
        g[0] = float(gamma)
        k = 0
        signalled = False
        for j in range(m):
            z = prec(V[:, j]) if prec else V[:, j]
            w = spmv(A, z, dt)
            w, h1, h2, beta = cgs2(V, j + 1, w)
            H[: j + 1, j] = h1.astype(np.float64) + h2.astype(np.float64)
            H[j + 1, j] = float(beta)
            res = apply_givens_column(H[:, j], cs, sn, g, j)
            it += 1
            k = j + 1
            out.implicit_history.append(res / bnorm)
            brk = _is_breakdown(beta, dt)
            if not brk:
                V[:, j + 1] = w / beta
            signalled = res / bnorm <= tol or brk
            if signalled or it >= max_iters:
                break
        y = back_substitute(H[:k, :k], g[:k])
        u = V[:, :k] @ y.astype(dt)
        if prec:
            u = prec(u)
        x = x + u
        cycles += 1
        r = b_w - spmv(A, x, dt)
        gamma = np.sqrt(r @ r)
        out.implicit_rel_res = float(abs(g[k]) / bnorm)
        rel = _explicit_rel_res(A, b, x)
        out.history.append(rel)
        if rel <= tol:
            out.converged = True
            break
        if not np.isfinite(rel):
            break
        if signalled:   # implicit convergence that the explicit residual does not confirm
            out.loss_of_accuracy += 1
            if stop_on_loss:
                out.stopped_on_loss = True
                break
    out.x, out.iters, out.cycles = x, it, cycles
    out.rel_res = out.history[-1]
    return out


# ---------------------------------------------------------------------------
# O5: GMRES-IR (Alg. 2, §III-B).  The residual and the solution update are in
# float64; the correction equation A u = r is solved by exactly m iterations
# of GMRES in float32 with the float32 copy of A (no inner convergence test,
# only breakdown ends a cycle early).  The residual is scaled by its float64
# norm gamma before the cast so it cannot underflow, renormalised in float32,
# and gamma scales the correction back.
# ---------------------------------------------------------------------------
def gmres_ir(A, b, x0, m: int, tol: float, max_iters: int,
             prec32: Optional[Callable] = None, max_cycles: Optional[int] = None,
             half_basis: bool = False) -> GmresOutcome:
    n = A.n
    # third precision (§VI): the basis used by Gram-Schmidt and the update is
    # stored in float16; the preconditioner and the SpMV take the float32
    # vector before rounding
    store = (lambda v: half_store(v, half_sigma(n))) if half_basis else (lambda v: v)
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    f32 = np.float32
    x = np.asarray(x0, dtype=np.float64).copy()
    r = b - spmv(A, x, np.float64)
    gamma = float(np.linalg.norm(r))
    out = GmresOutcome(x, False, 0, 0, gamma / bnorm)
    out.history.append(gamma / bnorm)
    it = 0
    cycles = 0
    while gamma / bnorm > tol and it < max_iters and (max_cycles is None or cycles < max_cycles):
        v = (r / gamma).astype(f32)
        beta0 = np.sqrt(v @ v)
        V = np.zeros((n, m + 1), dtype=f32)
        H = np.zeros((m + 1, m))
        cs, sn, g = np.zeros(m), np.zeros(m), np.zeros(m + 1)
        vj = v / beta0
        V[:, 0] = store(vj)
        g[0] = float(beta0)
        k = 0
        for j in range(m):
            z = prec32(vj) if prec32 else vj
            w = spmv(A, z, f32)
            w, h1, h2, beta = cgs2(V, j + 1, w)
            H[: j + 1, j] = h1.astype(np.float64) + h2.astype(np.float64)
            H[j + 1, j] = float(beta)
            res = apply_givens_column(H[:, j], cs, sn, g, j)
            it += 1
            k = j + 1
            out.implicit_history.append(gamma * res / bnorm)
            brk = _is_breakdown(beta, f32)
            if not brk:
                vj = w / beta
                V[:, j + 1] = store(vj)
            if brk or it >= max_iters:
                break
        y = back_substitute(H[:k, :k], g[:k])
        t = V[:, :k] @ y.astype(f32)
        if prec32:
            t = prec32(t)
        x = x + gamma * t.astype(np.float64)
        cycles += 1
        r = b - spmv(A, x, np.float64)
        gamma = float(np.linalg.norm(r))
        out.history.append(gamma / bnorm)
        if not np.isfinite(gamma):
            break
    out.x, out.iters, out.cycles = x, it, cycles
    out.rel_res = gamma / bnorm
    out.converged = out.rel_res <= tol
    return out


# ---------------------------------------------------------------------------
# O5b: GMRES-FD (§III-C, option 1, the method of the switch-point study in
# §V-A): GMRES(m) in float32 (float32 copies of A, b and x0) for
# ``switch_iters`` iterations, then GMRES(m) in float64 started from the
# float32 iterate widened to float64, until the float64 residual test holds.
# ``max_iters`` caps both phases together.  Returns (float32 phase or None
# when switch_iters is 0, float64 phase).
# ---------------------------------------------------------------------------
def gmres_fd(A, b, x0, m: int, tol: float, switch_iters: int, max_iters: int):
    first = None
    x = np.asarray(x0, dtype=np.float64)
    used = 0
    if switch_iters > 0:
        first = gmres(A, b, x0, m, tol, switch_iters, dt=np.float32)
        x = first.x.astype(np.float64)
        used = first.iters
    second = gmres(A, b, x, m, tol, max_iters - used, dt=np.float64)
    return first, second


# ---------------------------------------------------------------------------
# O5c: a float32 preconditioner inside float64 GMRES (§III-D option (a)): each
# application casts its float64 input to float32, applies M in float32 and
# casts the result back to float64.
# ---------------------------------------------------------------------------
def cast_wrapped(prec32: Callable) -> Callable:
    return lambda v: np.asarray(prec32(np.asarray(v).astype(np.float32)), dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# O5d: float16 storage of a float32 basis vector (the third precision of
# §VI): entries of a unit vector are about 1/sqrt(n), below float16's normal
# range for large n, so the vector is scaled by a power of two sigma ~ sqrt(n)
# before rounding (round to nearest even) and unscaled after; both scalings
# are exact.
# ---------------------------------------------------------------------------
def half_sigma(n: int) -> float:
    return float(2.0 ** min(15, max(0, int(round(0.5 * np.log2(n))))))


def half_store(v: np.ndarray, sigma: float) -> np.ndarray:
    f32 = np.float32
    return ((np.asarray(v, dtype=f32) * f32(sigma)).astype(np.float16).astype(f32)) / f32(sigma)
