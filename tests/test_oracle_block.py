"""Pins of the block GMRES-IR oracle (batched multi-RHS reading)."""
import numpy as np

import oracle as O
import workloads as W
from pins import _nonsym, dense_csr


def test_block_arnoldi_relation_and_orthogonality():
    A, D = _nonsym(60, 31)
    R = np.random.default_rng(32).standard_normal((60, 4))
    V0, R0, ok = O.cholqr2(R)
    assert ok and np.allclose(V0 @ R0, R, atol=1e-12)
    blocks, H, k = O.block_arnoldi(A, V0, 6, np.float64)
    V = np.concatenate(blocks, axis=1)
    assert k == 6 and V.shape == (60, 28)
    assert np.linalg.norm(V.T @ V - np.eye(28)) < 1e-12
    rel = np.linalg.norm(D @ V[:, :24] - V @ H) / np.linalg.norm(D)
    assert rel < 1e-13


def test_block_gmres_minimises_over_block_krylov_space():
    A, D = _nonsym(30, 33)
    Rb = np.random.default_rng(34).standard_normal((30, 3))
    V0, R0, _ = O.cholqr2(Rb)
    for k in (1, 2, 4):
        blocks, H, kk = O.block_arnoldi(A, V0, k, np.float64)
        E = np.zeros(((kk + 1) * 3, 3))
        E[:3] = R0
        Y = np.linalg.lstsq(H, E, rcond=None)[0]
        U = np.concatenate(blocks[:kk], axis=1) @ Y
        res = np.linalg.norm(Rb - D @ U, axis=0)
        K = np.concatenate([np.linalg.matrix_power(D, i) @ Rb for i in range(k)], axis=1)
        AK = D @ K
        for c in range(3):
            z, *_ = np.linalg.lstsq(AK, Rb[:, c], rcond=None)
            assert np.isclose(res[c], np.linalg.norm(Rb[:, c] - AK @ z), rtol=1e-8), (k, c)


def test_block_with_one_column_is_scalar_gmres_ir():
    p = W.config1_laplace2d(N=20)
    s = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 15, 1e-10, 5000)
    b = O.block_gmres_ir(p.A, p.b[:, None], 15, 1e-10, 100)
    assert b.converged and s.converged and b.cycles == s.cycles
    # same method, different rounding paths (Givens vs lstsq, CGS2 vs BCGS2)
    assert np.allclose(np.log10(np.array(b.history)[:, 0]), np.log10(s.history), atol=0.1)


def test_block_gmres_ir_reaches_tolerance_on_small_batch_system():
    sys = W.config4_batch(count=2, nrhs=4, side_lo=12, side_hi=20)
    for s in sys:
        out = O.block_gmres_ir(s["A"], s["B"], 10, 1e-10, 50)
        assert out.converged
        Xs = np.linalg.solve(s["A"].to_dense(), s["B"])
        assert np.allclose(out.X, Xs, rtol=0, atol=1e-6 * np.abs(Xs).max())


def test_float64_block_gmres_reaches_dense_solution():
    sys = W.config4_batch(count=2, nrhs=4, side_lo=12, side_hi=20, seed=11)
    for s in sys:
        out = O.block_gmres_ir(s["A"], s["B"], 10, 1e-12, 60, inner=np.float64)
        assert out.converged and np.all(out.rel_res <= 1e-12)
        Xs = np.linalg.solve(s["A"].to_dense(), s["B"])
        assert np.allclose(out.X, Xs, rtol=0, atol=1e-8 * np.abs(Xs).max())
        # one float64 cycle from X = 0 reaches the block-Krylov minimum of its
        # restart length (the property pinned on block_arnoldi above)
        one = O.block_gmres_ir(s["A"], s["B"], 3, 1e-30, 1, inner=np.float64)
        D = s["A"].to_dense()
        K = np.concatenate([np.linalg.matrix_power(D, i) @ s["B"] for i in range(3)], axis=1)
        for c in range(4):
            z, *_ = np.linalg.lstsq(D @ K, s["B"][:, c], rcond=None)
            best = np.linalg.norm(s["B"][:, c] - D @ K @ z) / np.linalg.norm(s["B"][:, c])
            assert np.isclose(one.rel_res[c], best, rtol=1e-6), (c, one.rel_res[c], best)


def test_cholqr2_detects_rank_deficiency():
    W_ = np.ones((10, 3))
    _, _, ok = O.cholqr2(W_)
    assert not ok


def test_dependent_columns_rule():
    rng = np.random.default_rng(40)
    Wm = rng.standard_normal((50, 5))
    Wm[:, 3] = 2 * Wm[:, 1] + 1e-5 * rng.standard_normal(50)      # nearly dependent
    Wm[:, 4] = Wm[:, 0] + 0.5 * rng.standard_normal(50)            # independent enough
    dep = O.dependent_columns(Wm.T @ Wm)
    assert list(dep) == [False, False, False, True, False]
    Z = rng.standard_normal((50, 5))
    V0, R0, ok, d = O.start_block(Wm, Z)
    assert ok and np.allclose(V0.T @ V0, np.eye(5), atol=1e-12)
    # R0 represents every column of W to the dependence threshold
    assert np.linalg.norm(V0 @ R0 - Wm) / np.linalg.norm(Wm) < 1e-4
