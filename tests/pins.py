"""Checks that tie the oracle to facts outside itself.

Each check raises AssertionError when the oracle disagrees with the paper,
a closed form, a library routine or brute force.  ``test_oracle_pins`` runs
them on the oracle as written; ``test_oracle_mutations`` plants plausible
mistakes in the oracle (on the CPU) and requires at least one check to fail.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import workloads as W


def rng(seed):
    return np.random.default_rng(seed)


def random_csr(n, density, seed, diag_shift=0.0):
    r = rng(seed)
    D = r.standard_normal((n, n)) * (r.random((n, n)) < density)
    D += diag_shift * np.eye(n)
    rows, cols = np.nonzero(D)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return W.CSR(n, row_ptr, cols.astype(np.int32), D[rows, cols]), D


def dense_csr(D):
    rows, cols = np.nonzero(D)
    n = D.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return W.CSR(n, np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), D[rows, cols])


# --- O1 SpMV -----------------------------------------------------------------
def check_spmv_matches_dense():
    A, D = random_csr(60, 0.15, 1)
    x = rng(2).standard_normal(60)
    y = O.spmv(A, x)
    assert np.allclose(y, D @ x, rtol=0, atol=1e-13 * (np.abs(D) @ np.abs(x)).max()), "spmv != dense"
    # an empty row and a full row
    D2 = D.copy()
    D2[5, :] = 0.0
    D2[7, :] = rng(3).standard_normal(60)
    A2 = dense_csr(D2)
    assert np.allclose(O.spmv(A2, x), D2 @ x, rtol=1e-13, atol=1e-12)


def check_spmv_integer_exact():
    # b = A * ones of the 2D Laplacian is 4 - #neighbours: 2 corners, 1 edges, 0 inside
    N = 64
    A = W.laplace2d(N)
    b = O.spmv(A, np.ones(A.n))
    i = np.arange(A.n) % N
    j = np.arange(A.n) // N
    nb = (i > 0).astype(int) + (i < N - 1) + (j > 0) + (j < N - 1)
    assert np.array_equal(b, 4.0 - nb), "integer SpMV not exact"
    assert np.isclose(np.linalg.norm(b) ** 2, 264.0, rtol=0, atol=1e-12)


def check_spmv_f32_bound():
    # componentwise bound |y^ - y| <= gamma_w |A||x| (inner-product bound)
    A = W.laplace3d(10)
    x = rng(4).uniform(-1, 1, A.n).astype(np.float32)
    y32 = O.spmv(A, x, np.float32).astype(np.float64)
    y64 = O.spmv(A, x.astype(np.float64), np.float64)
    absA = W.CSR(A.n, A.row_ptr, A.col_idx, np.abs(A.val.astype(np.float32)).astype(np.float64))
    u = 2.0 ** -24
    w = 7
    gam = (w + 1) * u / (1 - (w + 1) * u)   # +1: the float32 rounding of A's values
    bound = gam * O.spmv(absA, np.abs(x).astype(np.float64), np.float64)
    assert np.all(np.abs(y32 - y64) <= bound + 1e-30), "float32 SpMV outside its bound"


# --- O2 CGS2 / Arnoldi -----------------------------------------------------
def _nonsym(n, seed):
    r = rng(seed)
    D = np.eye(n) * 4 + r.standard_normal((n, n)) / np.sqrt(n)
    return dense_csr(D), D


def check_arnoldi_orthogonal_and_hessenberg():
    A, D = _nonsym(40, 5)
    v0 = rng(6).standard_normal(40)
    V, H, k = O.arnoldi(A, v0, 12)
    assert k == 12
    orth = np.linalg.norm(V.T @ V - np.eye(13))
    assert orth < 1e-12, f"||V^T V - I|| = {orth}"
    rel = np.linalg.norm(D @ V[:, :12] - V @ H) / (np.linalg.norm(D) * np.linalg.norm(V[:, :12]))
    assert rel < 1e-14, f"Hessenberg relation {rel}"
    assert np.all(np.diag(H, -1) > 0)


def check_arnoldi_equals_qr_of_krylov():
    A, D = _nonsym(12, 7)
    v0 = rng(8).standard_normal(12)
    k = 5
    V, H, _ = O.arnoldi(A, v0, k)
    K = np.empty((12, k + 1))
    K[:, 0] = v0
    for c in range(1, k + 1):
        K[:, c] = D @ K[:, c - 1]
    Q, R = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(R))
    assert np.allclose(V, Q, atol=1e-10), "Arnoldi basis != QR of the Krylov matrix"


# --- O3 Givens least squares --------------------------------------------------
def check_givens_matches_lstsq():
    r = rng(9)
    m = 15
    Hbar = np.triu(r.standard_normal((m + 1, m)), -1)
    Hbar[np.arange(1, m + 1), np.arange(m)] = np.abs(Hbar[np.arange(1, m + 1), np.arange(m)]) + 0.1
    gamma = 2.5
    Hr = Hbar.copy()
    cs, sn, g = np.zeros(m), np.zeros(m), np.zeros(m + 1)
    g[0] = gamma
    for j in range(m):
        res = O.apply_givens_column(Hr[:, j], cs, sn, g, j)
        yj = O.back_substitute(Hr[: j + 1, : j + 1], g[: j + 1])
        rhs = np.zeros(j + 2)
        rhs[0] = gamma
        yl, *_ = np.linalg.lstsq(Hbar[: j + 2, : j + 1], rhs, rcond=None)
        assert np.allclose(yj, yl, rtol=1e-10, atol=1e-12), "Givens y != lstsq"
        true_res = np.linalg.norm(rhs - Hbar[: j + 2, : j + 1] @ yl)
        assert np.isclose(res, true_res, rtol=1e-10, atol=1e-14), "implicit residual wrong"


def check_back_substitute():
    r = rng(10)
    R = np.triu(r.standard_normal((9, 9))) + 3 * np.eye(9)
    g = r.standard_normal(9)
    assert np.allclose(O.back_substitute(R, g), np.linalg.solve(R, g), rtol=1e-12)


# --- O4 GMRES ---------------------------------------------------------------
def check_gmres_tiny_dense_solve():
    A, D = _nonsym(30, 11)
    b = rng(12).standard_normal(30)
    out = O.gmres(A, b, np.zeros(30), 10, 1e-10, 500)
    assert out.converged
    x = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(out.x - x) / np.linalg.norm(x) <= 10 * kappa * 1e-10


def check_gmres_brute_force_minimisation():
    A, D = _nonsym(24, 13)
    b = rng(14).standard_normal(24)
    out = O.gmres(A, b, np.zeros(24), 24, 1e-14, 8, max_cycles=1)
    K = np.empty((24, 8))
    K[:, 0] = b
    for c in range(1, 8):
        K[:, c] = D @ K[:, c - 1]
    bn = np.linalg.norm(b)
    for j in range(1, 9):
        AK = D @ K[:, :j]
        c, *_ = np.linalg.lstsq(AK, b, rcond=None)
        best = np.linalg.norm(b - AK @ c) / bn
        assert np.isclose(out.implicit_history[j - 1], best, rtol=1e-7, atol=1e-15), \
            f"step {j}: GMRES residual {out.implicit_history[j-1]} != Krylov minimum {best}"


def check_gmres_finite_termination():
    # A diagonal with 6 distinct eigenvalues: GMRES is exact after 6 steps
    d = np.repeat([1.0, 2.0, 3.5, 5.0, 7.0, 11.0], 5)
    D = np.diag(d)
    A = dense_csr(D)
    b = rng(15).uniform(0.5, 1.5, 30)
    out = O.gmres(A, b, np.zeros(30), 20, 1e-12, 100)
    assert out.converged and out.iters == 6, (out.iters, out.rel_res)


def check_gmres_config1_counts():
    p = W.config1_laplace2d()
    out = O.gmres(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 5000)
    assert out.converged and out.rel_res <= 1e-10
    assert out.iters % 50 != 0  # mid-cycle stop of the float64 solver
    err = np.linalg.norm(out.x - 1.0) / np.sqrt(p.A.n)
    assert err <= 2e3 * 1e-10 * 10
    return out


# --- O5 GMRES-IR --------------------------------------------------------------
def check_gmres_ir_config1():
    p = W.config1_laplace2d()
    d64 = O.gmres(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 5000)
    ir = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 5000)
    assert ir.converged and ir.rel_res <= 1e-10
    assert ir.iters % 50 == 0
    assert ir.iters <= d64.iters + 3 * 50
    # residual curves track: at each restart IR is within 100x of float64 GMRES at the same iteration
    imp = np.array(d64.implicit_history)
    for c, rr in enumerate(ir.history[1:-1], start=1):
        it = c * 50
        if it <= len(imp):
            assert rr <= 100 * imp[it - 1] + 1e-12, (c, rr, imp[it - 1])
    # single precision alone stalls well above 1e-10
    f32 = O.gmres(p.A, p.b.astype(np.float32), np.zeros(p.A.n), 50, 1e-10, 1500, dt=np.float32)
    assert not f32.converged and 1e-8 < min(f32.history) < 1e-5


# --- O6 polynomial ------------------------------------------------------------
def check_poly_residual_identity():
    A, D = _nonsym(40, 16)
    v = rng(17).standard_normal(40)
    for d in (0, 3, 7):
        roots = O.poly_roots(A, d, v)
        pv = O.poly_apply(A, roots, v)
        lhs = np.linalg.norm(v - D @ pv)
        K = np.empty((40, d + 1))
        K[:, 0] = v
        for c in range(1, d + 1):
            K[:, c] = D @ K[:, c - 1]
        AK = D @ K
        c, *_ = np.linalg.lstsq(AK, v, rcond=None)
        best = np.linalg.norm(v - AK @ c)
        assert np.isclose(lhs, best, rtol=1e-8), (d, lhs, best)


def check_poly_inverse_on_few_eigenvalues():
    d = np.repeat([0.5, 1.0, 2.0, 4.0, 6.0], 4)
    A = dense_csr(np.diag(d))
    v = rng(18).uniform(0.5, 1.5, 20)
    roots = O.poly_roots(A, 4, v)
    pv = O.poly_apply(A, roots, v)
    assert np.allclose(d * pv, v, rtol=1e-9), "p(A) != A^-1 with d+1 distinct eigenvalues"


def check_poly_degree0():
    A, D = _nonsym(25, 19)
    v = rng(20).standard_normal(25)
    roots = O.poly_roots(A, 0, v)
    Av = D @ v
    assert np.isclose(1.0 / roots[0].real, (Av @ v) / (Av @ Av), rtol=1e-12)
    assert np.allclose(O.poly_apply(A, roots, v), (Av @ v) / (Av @ Av) * v, rtol=1e-12)


def check_poly_spd_real_positive():
    A = W.laplace2d(10)
    v = rng(21).standard_normal(A.n)
    roots = O.poly_roots(A, 10, v)
    assert np.all(np.abs(roots.imag) < 1e-8) and np.all(roots.real > 0)
    lam = W.laplacian_eigs_closed_form(10, 2)
    assert np.all(roots.real < lam.max() * (1 + 1e-9)) and np.all(roots.real > lam.min() * (1 - 1e-9))


def check_poly_roots_form_equals_monomial():
    A, D = _nonsym(8, 22)
    v = rng(23).standard_normal(8)
    d = 4
    roots = O.poly_roots(A, d, v)
    pi = np.real(np.poly(roots))                    # coefficients of prod (z - theta), highest first
    pi = pi / pi[-1]                                 # normalise so pi(0) = 1
    c = -pi[:-1]                                     # p(z) = (1 - pi(z))/z, highest power first
    P = np.zeros_like(D)
    for ck in c:                                     # Horner
        P = P @ D + ck * np.eye(8)
    assert np.allclose(O.poly_apply(A, roots, v), P @ v, rtol=1e-9, atol=1e-12)


def check_leja_properties():
    A, D = _nonsym(30, 24)
    v = rng(25).standard_normal(30)
    roots = O.poly_roots(A, 9, v)
    assert np.isclose(abs(roots[0]), np.max(np.abs(roots)))
    i = 0
    while i < len(roots):
        if roots[i].imag != 0:
            assert roots[i].imag > 0 and roots[i + 1] == np.conj(roots[i])
            i += 2
        else:
            i += 1
    # harmonic Ritz values are the roots of the GMRES residual polynomial
    # (brute force on a low degree, where the monomial Krylov basis is still
    # well conditioned)
    d = 4
    roots = O.poly_roots(A, d, v)
    K = np.empty((30, d + 1))
    K[:, 0] = v
    for c in range(1, d + 1):
        K[:, c] = D @ K[:, c - 1]
    c, *_ = np.linalg.lstsq(D @ K, v, rcond=None)
    poly = np.concatenate([-c[::-1], [1.0]])          # 1 - z sum c_i z^i, highest first
    ref = np.roots(poly)
    assert np.allclose(np.sort_complex(ref), np.sort_complex(roots), rtol=1e-7, atol=1e-9)


ALL_CHECKS = [
    check_spmv_matches_dense, check_spmv_integer_exact, check_spmv_f32_bound,
    check_arnoldi_orthogonal_and_hessenberg, check_arnoldi_equals_qr_of_krylov,
    check_givens_matches_lstsq, check_back_substitute,
    check_gmres_tiny_dense_solve, check_gmres_brute_force_minimisation,
    check_gmres_finite_termination, check_gmres_config1_counts, check_gmres_ir_config1,
    check_poly_residual_identity, check_poly_inverse_on_few_eigenvalues, check_poly_degree0,
    check_poly_spd_real_positive, check_poly_roots_form_equals_monomial, check_leja_properties,
]


def check_arnoldi_f32_orthogonality():
    # CGS2 keeps a float32 basis orthogonal to working accuracy even when the
    # Krylov basis is ill conditioned ("twice is enough")
    A = W.laplace2d(20)
    v0 = rng(26).standard_normal(A.n)
    V, H, k = O.arnoldi(A, v0, 40, np.float32)
    orth = np.linalg.norm(V.astype(np.float64).T @ V.astype(np.float64) - np.eye(41))
    assert orth < 2e-5, f"float32 ||V^T V - I|| = {orth}"


ALL_CHECKS.append(check_arnoldi_f32_orthogonality)


# --- O5b GMRES-FD -------------------------------------------------------------
def _dense(A):
    D = np.zeros((A.n, A.n))
    for r in range(A.n):
        D[r, A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]] = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
    return D


def check_gmres_fd():
    # 2D Laplacian, n = 400, GMRES(10), b = A x_true
    A = W.laplace2d(20)
    D = _dense(A)
    xt = rng(31).uniform(-1, 1, A.n)
    b = D @ xt
    bn = np.linalg.norm(b)
    tol = 1e-10
    kappa = np.linalg.cond(D)
    x0 = np.zeros(A.n)
    # switch 0: float64 GMRES(10) alone, which reaches the dense solution
    f, s = O.gmres_fd(A, b, x0, 10, tol, 0, 5000)
    assert f is None and s.converged and s.history[0] == 1.0
    assert np.linalg.norm(b - D @ s.x) / bn <= tol
    for sw in (40, 400):
        f, s = O.gmres_fd(A, b, x0, 10, tol, sw, 5000)
        # the float32 phase runs to the switch point: float32 cannot reach 1e-10
        assert f.iters == sw and not f.converged
        rf = np.linalg.norm(b - D @ f.x.astype(np.float64)) / bn
        assert rf > 1e-9, f"float32 phase reached {rf}: not float32 arithmetic"
        # the float64 phase starts from the widened float32 iterate
        assert np.isclose(s.history[0], rf, rtol=1e-9, atol=0), (s.history[0], rf)
        # and ends at the float64 tolerance, near the dense solution
        assert s.converged and np.linalg.norm(b - D @ s.x) / bn <= tol
        assert np.linalg.norm(s.x - xt) / np.linalg.norm(xt) <= 10 * kappa * tol
        assert s.iters + f.iters <= 5000
    # switching after the float32 phase has stalled: float32 iterations make no progress
    f150, _ = O.gmres_fd(A, b, x0, 10, tol, 150, 5000)
    r150 = np.linalg.norm(b - D @ f150.x.astype(np.float64)) / bn
    r400 = np.linalg.norm(b - D @ f.x.astype(np.float64)) / bn
    assert r400 > 0.1 * r150, (r150, r400)


ALL_CHECKS.append(check_gmres_fd)


# --- O5c float32 preconditioner inside float64 GMRES, loss of accuracy ------
def check_f32_poly_in_f64_gmres_loses_accuracy():
    # 3D Laplacian on 10^3, b = ones, GMRES(50), GMRES polynomial of degree 10
    A = W.laplace3d(10)
    b = np.ones(A.n)
    x0 = np.zeros(A.n)
    v0 = W.poly_start_vector(A.n, 0)
    r64 = O.poly_roots(A, 10, v0, np.float64)
    r32 = O.poly_roots(A, 10, v0.astype(np.float32), np.float32)
    mixed = O.cast_wrapped(lambda v: O.poly_apply(A, r32, v, np.float32))
    y = mixed(rng(33).standard_normal(A.n))
    assert y.dtype == np.float64 and np.array_equal(y.astype(np.float32).astype(np.float64), y)
    # the float32 polynomial is float32 arithmetic: it departs from the same roots
    # applied in float64 by more than one rounding of the result
    v = rng(34).standard_normal(A.n)
    y32, y64 = O.poly_apply(A, r32, v, np.float32), O.poly_apply(A, r32, v, np.float64)
    assert y32.dtype == np.float32
    diff = np.linalg.norm(y32 - y64) / np.linalg.norm(y64)
    assert 1e-7 < diff < 1e-4, diff
    # float64 polynomial: one cycle, implicit and explicit residuals agree
    d = O.gmres(A, b, x0, 50, 1e-10, 500, prec=lambda v: O.poly_apply(A, r64, v, np.float64))
    assert d.converged and d.cycles == 1 and d.loss_of_accuracy == 0
    # float32 polynomial: the first cycle stops on its implicit residual while the
    # explicit one is only float32-accurate (§V-F); a restart from the explicit
    # residual corrects it
    mx = O.gmres(A, b, x0, 50, 1e-10, 500, prec=mixed)
    assert mx.loss_of_accuracy >= 1 and mx.converged
    assert 1e-9 < mx.history[1] < 1e-4, mx.history
    assert np.linalg.norm(b - _dense(A) @ mx.x) / np.linalg.norm(b) <= 1e-10
    st = O.gmres(A, b, x0, 50, 1e-10, 500, prec=mixed, stop_on_loss=True)
    assert st.stopped_on_loss and not st.converged and st.cycles == 1
    assert st.rel_res == mx.history[1]


ALL_CHECKS.append(check_f32_poly_in_f64_gmres_loses_accuracy)


# --- O6b block Jacobi ----------------------------------------------------------
def check_bjac():
    n = 50
    A, D = random_csr(n, 0.15, 35, diag_shift=6.0)
    v = rng(36).standard_normal(n)
    # block 1 is point Jacobi: z = v / diag(A)
    z1 = O.bjac_apply(A, 1, v)
    assert np.allclose(z1, v / np.diag(D), rtol=1e-15, atol=0)
    # block n is the exact inverse
    zn = O.bjac_apply(A, n, v)
    assert np.linalg.norm(D @ zn - v) <= 1e-13 * np.linalg.norm(v)
    for k in (3, 7, 16):
        # z solves blockdiag(A) z = v, with a ragged last block
        mask = np.zeros((n, n), bool)
        for r0 in range(0, n, k):
            mask[r0:r0 + k, r0:r0 + k] = True
        z = O.bjac_apply(A, k, v)
        assert np.linalg.norm((D * mask) @ z - v) <= 1e-13 * np.linalg.norm(v), k
        # on a matrix that is itself block diagonal, M = A^-1 and GMRES needs one iteration
        Ab = dense_csr(D * mask)
        out = O.gmres(Ab, v, np.zeros(n), 10, 1e-12, 10, prec=lambda w, Ab=Ab, k=k: O.bjac_apply(Ab, k, w))
        assert out.converged and out.iters == 1, (k, out.iters)
    # float32: a float32 factorisation, close to the float64 one
    z32 = O.bjac_apply(A, 7, v, np.float32)
    z64 = O.bjac_apply(A, 7, v)
    assert z32.dtype == np.float32
    d = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 0 < d < 1e-5, d


ALL_CHECKS.append(check_bjac)


# --- O5d float16 basis ----------------------------------------------------------
def check_half_basis():
    assert O.half_sigma(3_375_000) == 2048.0 and O.half_sigma(1) == 1.0 and O.half_sigma(2 ** 40) == 2.0 ** 15
    # storage: round to nearest float16 after the power-of-two scaling, so entries far
    # below float16's normal range (1/sqrt(n) at n = 2^24) keep 11 significant bits
    sig = O.half_sigma(2 ** 24)
    v = (rng(37).uniform(0.5, 1.0, 1000) * np.logspace(-7, -1, 1000)).astype(np.float32)
    st = O.half_store(v, sig)
    assert np.array_equal((st * np.float32(sig)).astype(np.float16).astype(np.float32), st * np.float32(sig))
    assert np.max(np.abs(st - v) / v) <= 2.0 ** -11
    # GMRES-IR with the float16 basis: a cycle is only about float16-accurate,
    # the float64 outer loop still reaches 1e-10
    A = W.laplace3d(12)
    xt = W.uniform_pm1(2, A.n)
    b = W.host_matvec(A, xt)
    h32 = O.gmres_ir(A, b, np.zeros(A.n), 20, 1e-10, 2000)
    h16 = O.gmres_ir(A, b, np.zeros(A.n), 20, 1e-10, 2000, half_basis=True)
    assert h16.converged and h32.converged
    assert 2 * h32.history[1] < h16.history[1] < 1e-2, (h32.history[1], h16.history[1])
    assert np.linalg.norm(b - W.host_matvec(A, h16.x)) / np.linalg.norm(b) <= 1e-10


ALL_CHECKS.append(check_half_basis)


# --- O6c Leja order of the polynomial's roots -------------------------------------
def _golden(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)))


def check_leja_golden_order():
    # a hand-derived ordering (tests/golden/leja_order.json) that an order by
    # modulus, or a rule without the distance product, gets wrong
    g = _golden("leja_order.json")
    pts = np.array(g["points_re"]) + 1j * np.array(g["points_im"])
    want = np.array(g["order_re"]) + 1j * np.array(g["order_im"])
    for perm in (np.arange(6), np.arange(6)[::-1], rng(60).permutation(6)):
        got = O.leja_order(pts[perm])
        assert np.array_equal(got, want), (perm, got)


def check_leja_greedy_property():
    # brute force over the candidates at every pick: each real point and each
    # first member of a pair maximises the product of the distances to the
    # points already taken (the conjugate of a taken point follows it)
    A, D = _nonsym(30, 61)
    for d in (5, 9):
        theta = O.poly_roots(A, d, rng(62 + d).standard_normal(30))
        assert len(theta) == d + 1
        assert abs(theta[0]) >= np.max(np.abs(theta)) * (1 - 1e-12)
        i = 1 if theta[0].imag == 0 else 2
        while i < len(theta):
            rest = theta[i:]
            score = [np.sum(np.log(np.abs(z - theta[:i]))) for z in rest]
            assert score[0] >= max(score) - 1e-9 * (1 + abs(max(score))), (d, i, score)
            if theta[i].imag != 0:
                assert theta[i].imag > 0 and theta[i + 1] == np.conj(theta[i])
                i += 2
            else:
                i += 1


def check_leja_float32_apply_stable():
    # the reason for the order: in float32 the roots form of a degree-40
    # polynomial of a 2D Laplacian stays within a few float32 roundings of the
    # float64 apply of the same roots in Leja order, while an order by
    # decreasing modulus loses every digit (growth of the partial products)
    A = W.laplace2d(16)
    v = rng(63).standard_normal(A.n)
    roots = O.poly_roots(A, 40, v)
    y64 = O.poly_apply(A, roots, v)
    y32 = O.poly_apply(A, roots, v, np.float32)
    assert np.linalg.norm(y32 - y64) <= 1e-4 * np.linalg.norm(y64)


ALL_CHECKS += [check_leja_golden_order, check_leja_greedy_property, check_leja_float32_apply_stable]


# --- O8b block Arnoldi at a breakdown -----------------------------------------------
def _block_exhausted_system():
    # A = S diag(lam) S^-1 with five distinct eigenvalues, one of multiplicity 2:
    # for a generic 4-column block the block Krylov space has dimension
    # 4, 8, 12, 16 and then only 18, so the fourth block step finds two of
    # its four columns dependent on the basis
    r = rng(50)
    lam = np.repeat([1.0, 2.0, 3.5, 5.0, 7.0], [10, 10, 10, 2, 8])
    n = lam.size
    S = np.eye(n) + 0.3 * r.standard_normal((n, n)) / np.sqrt(n)
    D = S @ np.diag(lam) @ np.linalg.inv(S)
    return dense_csr(D), D, r.standard_normal((n, 4))


def check_block_arnoldi_breakdown():
    A, D, Bk = _block_exhausted_system()
    p = Bk.shape[1]
    V0, R0, ok = O.cholqr2(Bk)
    assert ok
    blocks, H, k = O.block_arnoldi(A, V0, 10, np.float64)
    assert k == 4 and H.shape == (5 * p, 4 * p), (k, H.shape)
    Vk = np.concatenate(blocks, axis=1)
    assert np.linalg.norm(Vk.T @ Vk - np.eye(k * p)) < 1e-12
    top, bot = H[:k * p], H[k * p:]
    # the rows of the last block row that belong to the dependent columns are zero
    assert np.sum(np.linalg.norm(bot, axis=1) == 0.0) == 2
    # A V_k = V_k H_top + W with W = Q R for an orthonormal Q: W^T W = R^T R
    Wr = D @ Vk - Vk @ top
    assert np.linalg.norm(Wr.T @ Wr - bot.T @ bot) <= 1e-12 * np.linalg.norm(Wr.T @ Wr)
    # the least-squares solution of the cycle is the minimum over the block
    # Krylov space of dimension k (explicit Krylov matrix, brute force)
    E = np.zeros(((k + 1) * p, p))
    E[:p] = R0
    Y = np.linalg.lstsq(H, E, rcond=None)[0]
    res = np.linalg.norm(Bk - D @ (Vk @ Y), axis=0)
    K = np.concatenate([np.linalg.matrix_power(D, i) @ Bk for i in range(k)], axis=1)
    for c in range(p):
        z, *_ = np.linalg.lstsq(D @ K, Bk[:, c], rcond=None)
        best = np.linalg.norm(Bk[:, c] - D @ K @ z)
        assert np.isclose(res[c], best, rtol=1e-9), (c, res[c], best)
    # the restarted float64 block solve, a breakdown in every cycle, reaches the dense solution
    out = O.block_gmres_ir(A, Bk, 10, 1e-12, 40, inner=np.float64)
    Xs = np.linalg.solve(D, Bk)
    assert out.converged and np.allclose(out.X, Xs, rtol=0, atol=1e-9 * np.abs(Xs).max())


ALL_CHECKS.append(check_block_arnoldi_breakdown)


# --- O9b predictor features -------------------------------------------------------
def check_features_hand_matrix():
    # A = [[2, -1, 0], [0, 3, -1], [-1, 0, 4]], worked by hand: diagonal 2, 3, 4,
    # off-diagonal sums 1, 1, 1, dominance 2, 3, 4, ||A||_F^2 = 32,
    # ||A - A^T||_F^2 = 6, diagonal mean 3 and std sqrt(2/3).  Three Arnoldi
    # steps from a generic vector span R^3, so the Ritz values are A's
    # eigenvalues and the run ends with h_{4,3} = 0.
    import oracle.features as F
    D = np.array([[2.0, -1.0, 0.0], [0.0, 3.0, -1.0], [-1.0, 0.0, 4.0]])
    A = dense_csr(D)
    f = F.features(A, np.array([1.0, 0.3, -0.7]))
    lam = np.linalg.eigvals(D)
    want = [np.log10(3), 2.0, 2.0, 2.0, 3.0, 1.0, 1 / 4, 5 / 4, 1 / 4, np.sqrt(6 / 32),
            np.sqrt(2 / 3) / 3, np.abs(lam).max() / 4, np.abs(lam).min() / 4,
            np.log10(np.abs(lam).max() / np.abs(lam).min()), np.abs(lam.imag).max() / np.abs(lam).max(), 0.0]
    assert np.allclose(f, want, rtol=1e-10, atol=1e-12), np.c_[f, want]


def check_features_laplacian_closed_form():
    # 2D Laplacian 4/-1 on N^2: corners dominate with ratio 2, edges 4/3, the
    # interior exactly 1; Gershgorin discs [0, 8] scaled by the diagonal 4;
    # symmetric (nonsymmetry 0, real Ritz values) with a constant diagonal;
    # the Ritz values lie inside the closed-form spectrum
    import oracle.features as F
    N = 12
    A = W.laplace2d(N)
    f = F.features(A, rng(70).standard_normal(A.n))
    n = N * N
    mean_dom = (4 * 2.0 + 4 * (N - 2) * 4 / 3 + (N - 2) ** 2 * 1.0) / n
    assert np.allclose(f[:11], [np.log10(n), (5 * n - 4 * N) / n, 5, 1.0, mean_dom, 1.0, 0.0, 2.0, 1.0, 0.0, 0.0],
                       rtol=1e-12, atol=1e-12), f[:11]
    lam = W.laplacian_eigs_closed_form(N, 2)
    assert lam.min() / 4 * (1 - 1e-12) <= f[12] <= f[11] <= lam.max() / 4 * (1 + 1e-12)
    assert f[14] == 0.0 and f[15] > 0


ALL_CHECKS += [check_features_hand_matrix, check_features_laplacian_closed_form]
