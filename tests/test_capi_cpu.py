"""The C-ABI library on the CPU: it loads, exports every declared symbol, its
host routines agree with numpy and the oracle, and bad arguments are
rejected before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2105_07544_amd as G
from paper_2105_07544_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "gmres_ir.h")).read()
    declared = set(re.findall(r"^\s*(?:gmr_status|size_t|void|int32_t|const char\*)\s+(\w+)\s*\(", header, re.M))
    assert declared == set(_capi.EXPORTED), declared ^ set(_capi.EXPORTED)
    lib = G.lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_hessenberg_eigvals_match_numpy():
    rng = np.random.default_rng(0)
    for k in (1, 2, 3, 4, 7, 16, 26, 41, 65):
        H = np.triu(rng.standard_normal((k, k)), -1)
        ev = G.hessenberg_eigvals(H)
        ref = np.linalg.eigvals(H)
        assert np.allclose(np.sort_complex(ev), np.sort_complex(ref), rtol=1e-10, atol=1e-12)
    # repeated and clustered eigenvalues of a symmetric tridiagonal
    T = np.diag(np.full(30, 2.0)) + np.diag(np.full(29, -1.0), 1) + np.diag(np.full(29, -1.0), -1)
    assert np.allclose(np.sort(G.hessenberg_eigvals(T).real), np.sort(np.linalg.eigvalsh(T)), atol=1e-12)


def test_leja_order_matches_oracle():
    rng = np.random.default_rng(1)
    for _ in range(40):
        k = int(rng.integers(1, 45))
        z = np.linalg.eigvals(np.triu(rng.standard_normal((k, k)), -1))
        assert np.allclose(G.leja_order(z), O.leja_order(z))


def test_workspace_query():
    a = G.workspace_bytes(1000, 50, G.GMR_F32)
    b = G.workspace_bytes(1000, 50, G.GMR_F64)
    c = G.workspace_bytes(1000, 100, G.GMR_F32)
    d = G.workspace_bytes(1000, 50, G.GMR_F32, True)
    assert 0 < a < b and a < c and a < d
    p = _capi.gmr_params(600, 1e-10, 10, 0, 0, 0, 0)
    assert G.lib().gmres_workspace_bytes(1000, C.byref(p), 0, 0) == 0
    p = _capi.gmr_params(512, 1e-10, 10, 0, 0, 0, 0)
    assert G.lib().gmres_workspace_bytes(1000, C.byref(p), 0, 0) > c


def test_argument_errors_before_device_work():
    lib = G.lib()
    res = _capi.gmr_result()
    p = _capi.gmr_params(50, 1e-10, 100, 0, 0, 0, 0)
    # null matrix
    assert lib.gmres_solve(None, None, None, None, C.byref(p), None, 0, C.byref(res), None, None) == -1
    assert b"null matrix" in lib.gmr_last_error()
    A = _capi.gmr_csr(10, 28, 16, 32, 48, 1)
    unaligned = _capi.gmr_csr(10, 28, 16, 36, 48, 1)
    assert lib.spmv(C.byref(unaligned), 64, 128, None) == -1
    assert b"aligned" in lib.gmr_last_error()
    bad = _capi.gmr_params(0, 1e-10, 100, 0, 0, 0, 0)
    assert lib.gmres_solve(C.byref(A), None, 8, 16, C.byref(bad), None, 0, C.byref(res), None, None) == -1
    bad = _capi.gmr_params(50, -1.0, 100, 0, 0, 0, 0)
    assert lib.gmres_solve(C.byref(A), None, 8, 16, C.byref(bad), None, 0, C.byref(res), None, None) == -1
    bad = _capi.gmr_params(513, 1e-10, 100, 0, 0, 0, 0)
    assert lib.gmres_solve(C.byref(A), None, 8, 16, C.byref(bad), None, 0, C.byref(res), None, None) == -5
    # dtype mismatch for GMRES-IR
    assert lib.gmres_ir_solve(C.byref(A), C.byref(A), None, 8, 16, C.byref(p), None, 0, C.byref(res),
                              None, None) == -1
    # workspace too small is found before any launch: gmres_solve checks it first
    with pytest.raises(G.GmresError):
        _capi.check(lib.cgs2_orth(0, 10, 0, 1, 10, 1, 1, None, 0, None))
    assert lib.cgs2_orth(0, 10, 600, 1, 10, 1, 1, None, 0, None) == -5
    assert lib.cgs2_orth(0, 10, 3, 1, 5, 1, 1, None, 0, None) == -1
    assert lib.cgs2_orth(0, 10, 3, 1, 10, 1, 1, None, 0, None) == -3
    # the no-allocation variant: its size limit and argument checks come before any HIP call
    assert lib.cgs2_orth_noalloc(2, 10, 3, 1, 10, 1, 1, None) == -1
    assert lib.cgs2_orth_noalloc(0, (1 << 27) + 1, 3, 1, (1 << 27) + 1, 1, 1, None) == -5
    assert lib.cgs2_orth_noalloc(0, 10, 513, 1, 10, 1, 1, None) == -5
    assert lib.cgs2_orth_noalloc(0, 10, 3, 1, 9, 1, 1, None) == -1
    assert lib.cgs2_orth_noalloc(0, 10, 3, None, 10, 1, 1, None) == -1
    assert lib.poly_prec_setup(C.byref(A), 129, 1, None, 0, C.byref(C.c_void_p()), None) == -5
    assert lib.spmv(C.byref(A), 5, 5, None) == -1


def test_fd_host_checks_without_device():
    lib = G.lib()
    res, res32 = _capi.gmr_result(), _capi.gmr_result()
    p = _capi.gmr_params(50, 1e-10, 100, 0, 0, 0, 0)
    A64 = _capi.gmr_csr(10, 28, 16, 32, 48, 1)
    A32 = _capi.gmr_csr(10, 28, 16, 32, 64, 0)
    other = _capi.gmr_csr(11, 28, 16, 32, 64, 0)
    nfd = lib.gmres_fd_workspace_bytes(1000, C.byref(p))
    assert nfd > lib.gmres_workspace_bytes(1000, C.byref(p), 1, 0) >= lib.gmres_workspace_bytes(1000, C.byref(p), 0, 0)
    assert lib.gmres_fd_workspace_bytes(1000, C.byref(_capi.gmr_params(0, 1e-10, 100, 0, 0, 0, 0))) == 0

    def fd(a, b_, sw, prm=p, ws=None, nws=0):
        return lib.gmres_fd_solve(C.byref(a), C.byref(b_), 8, 16, C.byref(prm), sw, ws, nws, C.byref(res),
                                  C.byref(res32), None, None)
    assert fd(A64, A64, 50) == -1 and b"float32" in lib.gmr_last_error()
    assert fd(A64, other, 50) == -1 and b"differ" in lib.gmr_last_error()
    assert fd(A64, A32, -1) == -1
    assert fd(A64, A32, 100) == -1 and b"exceed" in lib.gmr_last_error()
    assert fd(A64, A32, 50, ws=256, nws=16) == -3 and b"workspace" in lib.gmr_last_error()
    assert lib.gmres_fd_solve(C.byref(A64), C.byref(A32), 8, 8, C.byref(p), 10, None, 0, C.byref(res),
                              None, None, None) == -1
    # float32 polynomial inside float64 GMRES: a polynomial is required
    assert lib.gmres_f32prec_solve(C.byref(A64), C.byref(A32), None, 8, 16, C.byref(p), None, 0, C.byref(res),
                                   None, None) == -1
    assert b"float32 polynomial" in lib.gmr_last_error()
    assert lib.gmres_f32prec_solve(C.byref(A64), C.byref(A64), None, 8, 16, C.byref(p), None, 0, C.byref(res),
                                   None, None) == -1
    # the float64 workspace with a polynomial has room for the float32 copies
    assert lib.gmres_workspace_bytes(1000, C.byref(p), 1, 1) >= lib.gmres_workspace_bytes(1000, C.byref(p), 1, 0) + 4 * 8 * 1000 + 2 * 4 * 1000


def test_bjac_host_checks_without_device():
    lib = G.lib()
    assert lib.bjac_prec_bytes(1001, 42, 0) == 256 + 24 * 42 * 42 * 4
    assert lib.bjac_prec_bytes(1001, 42, 1) == 256 + 24 * 42 * 42 * 8
    assert lib.bjac_prec_bytes(10, 1, 1) == 256 + 10 * 8
    assert lib.bjac_prec_bytes(10, 0, 1) == 0 and lib.bjac_prec_bytes(10, 65, 1) == 0
    A = _capi.gmr_csr(10, 28, 16, 32, 48, 1)
    out = C.c_void_p()
    assert lib.bjac_prec_setup(C.byref(A), 0, 256, 1 << 20, C.byref(out), None) == -1
    assert lib.bjac_prec_setup(C.byref(A), 65, 256, 1 << 20, C.byref(out), None) == -5
    assert lib.bjac_prec_setup(C.byref(A), 4, 256, 16, C.byref(out), None) == -3
    assert lib.bjac_prec_setup(C.byref(A), 4, 264, 1 << 20, C.byref(out), None) == -1
    assert b"aligned" in lib.gmr_last_error()
    assert lib.prec_block_size(None) == 0


def test_harmonic_ritz_matches_oracle():
    import workloads as W
    for A, d in ((W.convdiff2d(30, 0.05, W.configs.uniflow_wind), 10), (W.laplace2d(12), 7)):
        v0 = W.poly_start_vector(A.n, 3)
        _, H, _ = O.arnoldi(A, v0, d + 1)
        got = np.sort_complex(G.harmonic_ritz(H))
        ref = np.sort_complex(O.harmonic_ritz_values(H, d + 1))
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_harmonic_ritz_ignores_entries_below_subdiagonal():
    # only the Hessenberg part of the input may be read
    import workloads as W
    A = W.convdiff2d(20, 0.05, W.configs.uniflow_wind)
    _, H, _ = O.arnoldi(A, W.poly_start_vector(A.n, 1), 9)
    junk = H.copy()
    rows, cols = np.tril_indices(10, -2, 9)
    junk[rows, cols] = np.random.default_rng(0).standard_normal(rows.size) * 1e3
    assert np.allclose(np.sort_complex(G.harmonic_ritz(junk)), np.sort_complex(G.harmonic_ritz(H)))
    assert np.allclose(np.sort_complex(G.hessenberg_eigvals(junk[:9, :9])),
                       np.sort_complex(G.hessenberg_eigvals(H[:9, :9])))


def test_batch_host_api_without_device():
    """The batch object is host-side: creation, tiling, graph switch and
    workspace queries run without a GPU, and bad arguments are rejected."""
    lib = G.lib()
    b = G.Batch([300, 1000, 17], restart=8)
    f32, f64 = b.workspace_bytes(G.GMR_F32), b.workspace_bytes(G.GMR_F64)
    assert 0 < f32 < f64
    assert lib.batch_workspace_bytes(b.handle, 7) == 0
    assert lib.batch_workspace_bytes(None, G.GMR_F32) == 0
    assert b.tiling() == (1024, 8)
    for t, g in ((512, 16), (256, 2), (4096, 3), (1024, 5)):
        b.set_tiling(t, g)
        assert b.tiling() == (t, g)
    for t, g in ((255, 8), (1000, 8), (1024, 9), (1024, 0)):
        with pytest.raises(G.GmresError):
            b.set_tiling(t, g)
    b.set_graph(True)
    b.set_graph(False)
    assert lib.batch_set_graph(None, 1) == -1
    # per-system statuses exist only after a solve
    st = np.zeros(3, dtype=np.int32)
    assert lib.batch_system_status(b.handle, st.ctypes.data_as(C.c_void_p)) == -1
    assert lib.batch_system_status(None, st.ctypes.data_as(C.c_void_p)) == -1
    # the features' workspace query is host arithmetic
    assert lib.matrix_features_workspace_bytes(1000, G.GMR_F64) > lib.matrix_features_workspace_bytes(1000, G.GMR_F32) > 0
    assert lib.matrix_features_workspace_bytes(0, G.GMR_F64) == 0
    assert lib.matrix_features_workspace_bytes(10, 5) == 0
    out = C.c_void_p()
    rows = np.array([10, 0], dtype=np.int32)
    assert lib.batch_create(2, rows.ctypes.data_as(C.c_void_p), 16, 8, C.byref(out)) == -1
    rows = np.array([10, 20], dtype=np.int32)
    assert lib.batch_create(2, rows.ctypes.data_as(C.c_void_p), 8, 8, C.byref(out)) == -5
    assert lib.batch_create(2, rows.ctypes.data_as(C.c_void_p), 16, 65, C.byref(out)) == -5
    res = _capi.gmr_batch_result()
    # null arguments and a matrix of the wrong size are found before any launch
    assert lib.batch_gmres_solve(b.handle, None, None, None, None, 1e-10, 10, None, 0, C.byref(res), None, None,
                                 None) == -1
    A = _capi.gmr_csr(1000, 10, 16, 32, 48, 1)  # the batch has 300 + 1000 + 17 rows
    assert lib.batch_gmres_solve(b.handle, C.byref(A), 64, 128, 192, 1e-10, 10, 256, 1 << 40, C.byref(res), None,
                                 None, None) == -1
    assert b"does not match" in lib.gmr_last_error()
    A.n = 300 + 1000 + 17
    assert lib.batch_gmres_solve(b.handle, C.byref(A), 64, 128, 192, 1e-10, 10, 256, 16, C.byref(res), None,
                                 None, None) == -3
