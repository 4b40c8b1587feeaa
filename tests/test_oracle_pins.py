"""The oracle against the paper, closed forms, library routines and brute force."""
import json
import os

import numpy as np
import pytest

import pins
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(check):
    check()


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: the first three outputs of the published generator
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v) for v in W.splitmix64(0, 3)] == ref
    assert [W.splitmix64_scalar(0, k) for k in (1, 2, 3)] == ref
    z = W.splitmix64(12345, 1000)
    assert all(int(z[k]) == W.splitmix64_scalar(12345, k + 1) for k in (0, 1, 499, 999))
    u = W.uniform_pm1(7, 100000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01


def test_generator_sizes_match_paper():
    sizes = json.load(open(os.path.join(GOLDEN, "paper_sizes.json")))
    for name, s in sizes.items():
        if name.startswith("_"):
            continue
        cf = W.nnz_closed_form_3d(s["N"]) if s["dim"] == 3 else W.nnz_closed_form_2d(s["N"])
        assert cf == s["nnz"], name
        assert s["N"] ** s["dim"] == s["n"]
    for N in (1, 2, 5, 17):
        assert W.laplace2d(N).nnz == W.nnz_closed_form_2d(N)
        assert W.laplace3d(N).nnz == W.nnz_closed_form_3d(N)
        assert W.convdiff2d(N, 0.1, lambda x, y: (np.cos(x), np.sin(y))).nnz == W.nnz_closed_form_2d(N)


def test_generator_laplace3d150_full_size():
    A = W.laplace3d(150)
    assert A.n == 3375000 and A.nnz == 23490000
    assert np.all(np.diff(A.row_ptr) <= 7)


def test_generator_structure():
    for A in (W.laplace2d(7), W.laplace3d(5), W.convdiff2d(9, 0.01, lambda x, y: (np.cos(np.pi * x), np.sin(np.pi * y)))):
        for r in range(A.n):
            cols = A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]
            assert np.all(np.diff(cols) > 0) and r in cols
        D = A.to_dense()
        assert np.all(D.sum(axis=1) >= -1e-15)          # M-matrix rows
        assert np.all(np.diag(D) > 0) and np.all(D - np.diag(np.diag(D)) <= 0)


def test_laplacian_spectrum_closed_form():
    for N, dim in ((6, 2), (4, 3)):
        A = W.laplace2d(N) if dim == 2 else W.laplace3d(N)
        ev = np.sort(np.linalg.eigvalsh(A.to_dense()))
        cf = np.sort(W.laplacian_eigs_closed_form(N, dim))
        assert np.allclose(ev, cf, atol=1e-12)
    lam = W.laplacian_eigs_closed_form(64, 2)
    assert abs(lam.max() / lam.min() - 1711.7) < 0.1
    lam = W.laplacian_eigs_closed_form(150, 3)
    assert abs(lam.max() / lam.min() - 9240.2) < 0.5


def test_convdiff_reduces_to_laplacian_without_wind():
    eps = 0.37
    A = W.convdiff2d(6, eps, lambda x, y: (0.0 * x, 0.0 * y))
    assert np.allclose(A.to_dense(), eps * W.laplace2d(6).to_dense())
    # pure upwind: wind (+1, 0) adds h to the diagonal and -h to the west neighbour
    N = 5
    h = 1.0 / (N + 1)
    B = W.convdiff2d(N, 0.0, lambda x, y: (1.0 + 0 * x, 0 * y)).to_dense()
    r = 2 * N + 2
    assert np.isclose(B[r, r], h) and np.isclose(B[r, r - 1], -h) and np.isclose(B[r, r + 1], 0.0)


def test_spmv_traffic_model_values():
    g = json.load(open(os.path.join(GOLDEN, "spmv_traffic_model.json")))
    # float64 without reuse of x reads (4 + 2*8) w n bytes; float32 with x read once (4 + 4) w n + 4 n
    for w, key in ((5, "ratio_w5"), (7, "ratio_w7")):
        ratio = (4 + 2 * 8) * w / ((4 + 4) * w + 4)
        assert round(ratio, 2) == g[key]
    assert abs(20 * 1e6 / (8 * 1e6 + 4) - g["limit"]) < 1e-5
