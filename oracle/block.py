"""Oracle: block GMRES(m)-IR for several right-hand sides of one system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's solver handles one right-hand side (§IV); the batched workload
solves p right-hand sides of each system at once.  This project reads that as
block GMRES: the Krylov space of the residual block R (n x p) is built block
by block, each new block W = A V_j is orthogonalised against all previous
blocks by two classical block Gram-Schmidt passes (the block form of the two
CGS passes of §III-A) and then within itself by Cholesky QR done twice.  The
block Hessenberg least-squares problem min ||E1 R0 - Hbar Y||_F is solved
column by column with numpy's lstsq.  GMRES-IR (Alg. 2) wraps it: the inner
block GMRES runs in float32 on float32 A for exactly m block steps, the
residual and the update are float64, and every right-hand side column is
scaled by its own residual norm before the cast.  With a float64 inner solve
the same loop is plain restarted block GMRES(m).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from .krylov import spmv


def spmm(A, X: np.ndarray, dt) -> np.ndarray:
    """Y = A X for a multivector X (n x p), column by column with the O1 SpMV."""
    return np.stack([spmv(A, X[:, c].astype(dt), dt) for c in range(X.shape[1])], axis=1)


def cholqr2(W: np.ndarray, tau: float = 1e-5):
    """Cholesky QR applied twice: W = Q R with Q^T Q = I to working accuracy.
    Returns (Q, R, ok); ok is False when a column of W is (nearly) dependent
    on the earlier ones: a pivot of the first Cholesky factorisation at most
    tau times the column's squared norm (this project's breakdown rule)."""
    dt = W.dtype
    G = (W.T @ W).astype(np.float64)
    if np.any(dependent_columns(G, tau)):
        return W, None, False
    try:
        R1 = np.linalg.cholesky(G).T
    except np.linalg.LinAlgError:
        return W, None, False
    Q = (W @ np.linalg.inv(R1).astype(dt)).astype(dt)
    G2 = (Q.T @ Q).astype(np.float64)
    try:
        R2 = np.linalg.cholesky(G2).T
    except np.linalg.LinAlgError:
        return W, None, False
    Q = (Q @ np.linalg.inv(R2).astype(dt)).astype(dt)
    return Q, R2 @ R1, True


def block_arnoldi(A, V0: np.ndarray, m: int, dt):
    """m block steps from the orthonormal block V0 (n x p).  Returns the list of
    blocks V_0..V_k and the block Hessenberg Hbar ((k+1)p x kp, float64)."""
    n, p = V0.shape
    blocks = [V0.astype(dt)]
    H = np.zeros(((m + 1) * p, m * p))
    k = 0
    for j in range(m):
        W = spmm(A, blocks[j], dt)
        Vj = np.concatenate(blocks, axis=1)
        C1 = Vj.T @ W
        W = W - Vj @ C1
        C2 = Vj.T @ W
        W = W - Vj @ C2
        Q, R, ok = cholqr2(W)
        H[: (j + 1) * p, j * p:(j + 1) * p] = C1.astype(np.float64) + C2.astype(np.float64)
        k = j + 1
        if not ok:
            # breakdown: block column j is kept with the Cholesky factor that
            # skips the dependent columns, and the cycle ends there
            H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = skip_cholesky((W.T @ W).astype(np.float64))[0]
            break
        H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = R
        blocks.append(Q)
    return blocks, H[: (k + 1) * p, : k * p], k


DEP_TAU = 1e-5


def skip_cholesky(G: np.ndarray, tau: float = DEP_TAU):
    """Cholesky factor R (upper) of G = W^T W that skips, instead of stopping
    at, a column whose pivot is at most tau times its squared norm: such a
    column gets a zero row in R and is flagged dependent.  The columns of W
    satisfy W = Q R for the orthonormal basis Q of the kept columns, up to the
    skipped components."""
    p = G.shape[0]
    R = np.zeros((p, p))
    dep = np.zeros(p, dtype=bool)
    for c in range(p):
        d = G[c, c] - np.sum(R[:c, c] ** 2)
        if not (d > tau * G[c, c]):
            dep[c] = True
            R[c, c + 1:] = 0.0
            continue
        R[c, c] = np.sqrt(d)
        R[c, c + 1:] = (G[c, c + 1:] - R[:c, c] @ R[:c, c + 1:]) / R[c, c]
    return R, dep


def dependent_columns(G: np.ndarray, tau: float = DEP_TAU) -> np.ndarray:
    """Columns of W (Gram matrix G = W^T W) whose component orthogonal to the
    earlier kept columns has relative squared norm <= tau."""
    return skip_cholesky(G, tau)[1]


START_TAU = 1e-12
# Dependency threshold of a start block with a float32 inner solve: the kept
# columns then have parts outside the span of the earlier ones of relative
# squared norm > 1e-3, which bounds the block's condition number to the range
# (about u^-1/2 in float32) where Cholesky QR twice is reliable; float64 keeps 1e-5.
START_DEP_TAU_F32 = 1e-3


def start_block(W: np.ndarray, Z: np.ndarray):
    """Orthonormal start block of a cycle: columns of W that (nearly) depend on
    earlier ones are replaced by the matching columns of the random block Z
    before Cholesky QR twice; R0 = V0^T W then represents every column of W."""
    tau = START_DEP_TAU_F32 if W.dtype == np.float32 else DEP_TAU
    dep = dependent_columns((W.T @ W).astype(np.float64), tau)
    Wp = W.copy()
    Wp[:, dep] = Z[:, dep].astype(W.dtype)
    V0, _, ok = cholqr2(Wp, START_TAU)
    R0 = (V0.T @ W).astype(np.float64)
    return V0, R0, ok, dep


@dataclass
class BlockOutcome:
    X: np.ndarray
    converged: bool
    cycles: int
    rel_res: np.ndarray                      # per column, float64 explicit
    history: List[np.ndarray] = field(default_factory=list)


def block_gmres_ir(A, B: np.ndarray, m: int, tol: float, max_cycles: int,
                   Z: np.ndarray = None, inner=np.float32) -> BlockOutcome:
    """Block GMRES(m)-IR: float32 inner block GMRES(m), float64 outer refinement.
    Z (n x p) is the random block that replaces dependent start columns.
    inner=np.float64 runs the same loop with the inner block GMRES in float64,
    i.e. plain restarted block GMRES(m) in float64 (the baseline of §V-B)."""
    n, p = B.shape
    f32 = inner
    if Z is None:
        Z = np.random.default_rng(0).uniform(-1, 1, (n, p))
    X = np.zeros((n, p))
    bn = np.linalg.norm(B, axis=0)
    R = B - spmm(A, X, np.float64)
    gam = np.linalg.norm(R, axis=0)
    out = BlockOutcome(X, False, 0, gam / bn)
    out.history.append(gam / bn)
    cycles = 0
    while np.any(gam / bn > tol) and cycles < max_cycles:
        W = (R / gam).astype(f32)
        V0, R0, ok, _ = start_block(W, Z)
        if not ok:
            break
        blocks, Hbar, k = block_arnoldi(A, V0, m, f32)
        if k == 0:
            break
        E = np.zeros(((k + 1) * p, p))
        E[:p, :p] = R0
        Y = np.linalg.lstsq(Hbar, E, rcond=None)[0]
        Vk = np.concatenate(blocks[:k], axis=1)  # the blocks that carry the solution
        U = (Vk @ Y.astype(f32)).astype(np.float64)
        X = X + U * gam
        cycles += 1
        R = B - spmm(A, X, np.float64)
        gam = np.linalg.norm(R, axis=0)
        out.history.append(gam / bn)
    out.X, out.cycles, out.rel_res = X, cycles, gam / bn
    out.converged = bool(np.all(out.rel_res <= tol))
    return out
