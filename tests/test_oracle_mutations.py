"""Plant plausible mistakes in the oracle (CPU only) and require the pins to catch them."""
import numpy as np
import pytest

import oracle
import oracle.krylov as K
import oracle.poly as P
import oracle.block as O_blk
import oracle.precond as O_pre
import oracle.features as O_feat
import pins


def _patch(monkeypatch, name, fn, modules=(oracle, K, P, O_pre, O_blk, O_feat)):
    for m in modules:
        if hasattr(m, name):
            monkeypatch.setattr(m, name, fn)


def _fails(checks):
    failed = []
    for c in checks:
        try:
            c()
        except Exception:  # AssertionError or a numerical error caused by the mutation
            failed.append(c.__name__)
    return failed


def spmv_drop_last(A, x, dt=None):
    dt = np.dtype(dt or x.dtype)
    val = A.val.astype(dt)
    x = np.asarray(x).astype(dt)
    y = np.zeros(A.n, dt)
    for r in range(A.n):
        for k in range(A.row_ptr[r], A.row_ptr[r + 1] - 1):
            y[r] += val[k] * x[A.col_idx[k]]
    return y


def spmv_row_index(A, x, dt=None):
    dt = np.dtype(dt or x.dtype)
    y = np.zeros(A.n, dt)
    for r in range(A.n):
        for k in range(A.row_ptr[r], A.row_ptr[r + 1]):
            y[r] += A.val[k] * x[r]
    return y


def cgs_single_pass(V, j, w):
    Vj = V[:, :j]
    h1 = Vj.T @ w
    w = w - Vj @ h1
    return w, h1, np.zeros_like(h1), np.sqrt(w @ w)


def cgs2_stale_w(V, j, w):
    Vj = V[:, :j]
    h1 = Vj.T @ w
    w1 = w - Vj @ h1
    h2 = Vj.T @ w            # mistake: dots against the unupdated vector
    w2 = w1 - Vj @ h2
    return w2, h1, h2, np.sqrt(w2 @ w2)


def givens_wrong_sign(h, cs, sn, g, j):
    for i in range(j):
        hi, hi1 = h[i], h[i + 1]
        h[i] = cs[i] * hi + sn[i] * hi1
        h[i + 1] = sn[i] * hi + cs[i] * hi1          # mistake: sign of the sine
    a, b = h[j], h[j + 1]
    rho = float(np.hypot(a, b))
    cs[j], sn[j] = (1.0, 0.0) if rho == 0 else (a / rho, b / rho)
    h[j], h[j + 1] = rho, 0.0
    g[j + 1] = -sn[j] * g[j]
    g[j] = cs[j] * g[j]
    return abs(g[j + 1])


def backsolve_transposed(R, g):
    k = R.shape[0]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        s = g[i]
        for c in range(i + 1, k):
            s -= R[c, i] * y[c]                      # mistake: transposed operand
        y[i] = s / R[i, i]
    return y


def poly_apply_half_a(A, roots, x, dt=np.float64):
    r = np.array([complex(z.real * (0.5 if z.imag != 0 else 1.0), z.imag) for z in roots])
    return _orig_poly_apply(A, r, x, dt)


def harmonic_unsquared(H, k):
    Hk = H[:k, :k].copy()
    ek = np.zeros(k)
    ek[-1] = 1.0
    f = np.linalg.solve(Hk.T, ek)
    Hk[:, k - 1] += H[k, k - 1] * f                  # mistake: h_{k+1,k} not squared
    return np.linalg.eigvals(Hk)


_orig_poly_apply = P.poly_apply


def fd_phase2_from_x0(A, b, x0, m, tol, switch_iters, max_iters):
    first = K.gmres(A, b, x0, m, tol, switch_iters, dt=np.float32) if switch_iters > 0 else None
    second = K.gmres(A, b, np.asarray(x0, np.float64), m, tol,  # mistake: drops the float32 iterate
                     max_iters - (first.iters if first else 0), dt=np.float64)
    return first, second


def fd_phase1_float64(A, b, x0, m, tol, switch_iters, max_iters):
    first = K.gmres(A, b, x0, m, tol, switch_iters, dt=np.float64) if switch_iters > 0 else None  # mistake
    x = first.x if first else np.asarray(x0, np.float64)
    second = K.gmres(A, b, x, m, tol, max_iters - (first.iters if first else 0), dt=np.float64)
    return first, second

def poly_apply_f64_always(A, roots, x, dt=np.float64):
    return _orig_poly_apply(A, roots, x, np.float64)  # mistake: ignores the working precision


def bjac_transposed(A, block, v, dt=np.float64):
    dt = np.dtype(dt)
    v = np.asarray(v).astype(dt)
    z = np.zeros(A.n, dtype=dt)
    for r0 in range(0, A.n, block):
        r1 = min(r0 + block, A.n)
        z[r0:r1] = np.linalg.solve(O_pre.diagonal_block(A, r0, r1).astype(dt).T, v[r0:r1])  # mistake
    return z


def bjac_short_blocks(A, block, v, dt=np.float64):
    dt = np.dtype(dt)
    v = np.asarray(v).astype(dt)
    z = np.zeros(A.n, dtype=dt)
    for r0 in range(0, A.n, block):
        r1 = min(r0 + block - 1, A.n)   # mistake: drops the last row of every block
        z[r0:r1] = np.linalg.solve(O_pre.diagonal_block(A, r0, r1).astype(dt), v[r0:r1])
    return z


def half_store_unscaled(v, sigma):
    return np.asarray(v, dtype=np.float32).astype(np.float16).astype(np.float32)  # mistake: no scaling


def half_store_identity(v, sigma):
    return np.asarray(v, dtype=np.float32)  # mistake: the basis is never rounded


def leja_by_modulus(theta):
    # mistake: decreasing modulus instead of the distance-product rule
    # (pairs still adjacent, positive imaginary part first)
    out = []
    for t in sorted((complex(z) for z in theta if complex(z).imag >= 0), key=lambda z: -abs(z)):
        out.append(t)
        if t.imag != 0.0:
            out.append(t.conjugate())
    return np.array(out)


def block_arnoldi_zero_r(A, V0, m, dt):
    # mistake: at a breakdown the last block row of Hbar is left zero
    n, p = V0.shape
    blocks = [V0.astype(dt)]
    H = np.zeros(((m + 1) * p, m * p))
    k = 0
    for j in range(m):
        W_ = O_blk.spmm(A, blocks[j], dt)
        Vj = np.concatenate(blocks, axis=1)
        C1 = Vj.T @ W_
        W_ = W_ - Vj @ C1
        C2 = Vj.T @ W_
        W_ = W_ - Vj @ C2
        Q, R, ok = O_blk.cholqr2(W_)
        H[: (j + 1) * p, j * p:(j + 1) * p] = C1 + C2
        k = j + 1
        if not ok:
            break
        H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p] = R
        blocks.append(Q)
    return blocks, H[: (k + 1) * p, : k * p], k


def row_stats_with_diagonal(A):
    # mistake: the diagonal counted in the off-diagonal sum r_i
    D = A.to_dense()
    d = np.diag(D).copy()
    r = np.array([sum(abs(D[i, j]) for j in range(A.n) if D[i, j] != 0.0) for i in range(A.n)])
    return dict(d=d, r=r, nnz_row=np.diff(A.row_ptr), fro2=float((D * D).sum()),
                skew2=float(((D - D.T) ** 2).sum()))


MUTATIONS = {
    "spmv_drop_last": ("spmv", spmv_drop_last),
    "spmv_row_index": ("spmv", spmv_row_index),
    "cgs_single_pass": ("cgs2", cgs_single_pass),
    "cgs2_stale_w": ("cgs2", cgs2_stale_w),
    "givens_wrong_sign": ("apply_givens_column", givens_wrong_sign),
    "backsolve_transposed": ("back_substitute", backsolve_transposed),
    "poly_apply_half_a": ("poly_apply", poly_apply_half_a),
    "harmonic_unsquared": ("harmonic_ritz_values", harmonic_unsquared),
    "fd_phase2_from_x0": ("gmres_fd", fd_phase2_from_x0),
    "fd_phase1_float64": ("gmres_fd", fd_phase1_float64),
    "poly_apply_f64_always": ("poly_apply", poly_apply_f64_always),
    "bjac_transposed": ("bjac_apply", bjac_transposed),
    "bjac_short_blocks": ("bjac_apply", bjac_short_blocks),
    "half_store_unscaled": ("half_store", half_store_unscaled),
    "half_store_identity": ("half_store", half_store_identity),
    "leja_by_modulus": ("leja_order", leja_by_modulus),
    "block_arnoldi_zero_r": ("block_arnoldi", block_arnoldi_zero_r),
    "features_diag_in_offdiag_sum": ("row_stats", row_stats_with_diagonal),
}

FAST_CHECKS = [c for c in pins.ALL_CHECKS if c.__name__ not in
               ("check_gmres_config1_counts", "check_gmres_ir_config1", "check_spmv_integer_exact")]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(monkeypatch, name):
    attr, fn = MUTATIONS[name]
    _patch(monkeypatch, attr, fn)
    failed = _fails(FAST_CHECKS)
    assert failed, f"mutation {name} passed every pin"
