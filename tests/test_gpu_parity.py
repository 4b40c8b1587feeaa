"""GPU parity: the HIP path through the C ABI against the oracle (MI355X)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_2105_07544_amd")

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(A):
    return G.DeviceCSR.from_host(A, DEV)


def t64(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def t32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def random_csr(n, seed, max_row=9, empty_every=0, long_row=None):
    rng = np.random.default_rng(seed)
    rows = []
    for r in range(n):
        if empty_every and r % empty_every == 3:
            rows.append(np.array([], dtype=np.int64))
            continue
        k = int(rng.integers(1, max_row + 1))
        if long_row is not None and r == long_row[0]:
            k = min(long_row[1], n)
        rows.append(np.sort(rng.choice(n, size=min(k, n), replace=False)))
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum([len(c) for c in rows])
    col = np.concatenate(rows).astype(np.int32) if row_ptr[-1] else np.zeros(0, np.int32)
    val = rng.standard_normal(len(col))
    return W.CSR(n, row_ptr, col, val)


# ---------------------------------------------------------------------------
# SpMV: products rounded then summed in ascending k, exactly like the oracle
# ---------------------------------------------------------------------------
SPMV_CASES = {
    "laplace3d_N20": lambda: W.laplace3d(20),
    "convdiff_N37": lambda: W.convdiff2d(37, 1e-2, W.configs.uniflow_wind),
    "random_empty_rows": lambda: random_csr(1000, 3, empty_every=7),
    "random_long_row": lambda: random_csr(5000, 4, long_row=(300, 4500)),
    "one_row": lambda: W.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5])),
    "n_257": lambda: random_csr(257, 5),
}


@pytest.mark.parametrize("name", sorted(SPMV_CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spmv_bit_exact(name, prec):
    say("spmv", name, prec)
    A = SPMV_CASES[name]()
    x = W.uniform_pm1(11, A.n)
    dt = np.float64 if prec == "f64" else np.float32
    Ad = dev(A) if prec == "f64" else dev(A).to_f32()
    xd = t64(x) if prec == "f64" else t32(x)
    y = host(G.spmv(Ad, xd))
    ref = O.spmv(A, x.astype(dt), dt)
    assert np.array_equal(y, ref), np.abs(y - ref).max()


def test_spmv_full_config2_sampled():
    say("spmv full laplace3d N=150")
    A = W.laplace3d(150)
    x = W.uniform_pm1(2, A.n)
    Ad = dev(A)
    A32 = Ad.to_f32()
    y64 = host(G.spmv(Ad, t64(x)))
    y32 = host(G.spmv(A32, t32(x)))
    rows = np.unique(np.concatenate([np.arange(0, 300), W.uniform_int(9, 0, A.n - 1, 2000),
                                     np.arange(A.n - 300, A.n)]))
    for dt, y in ((np.float64, y64), (np.float32, y32)):
        xs = x.astype(dt)
        vals = A.val.astype(dt)
        for r in rows:
            acc = dt(0)
            for k in range(A.row_ptr[r], A.row_ptr[r + 1]):
                acc = dt(acc + vals[k] * xs[A.col_idx[k]])
            assert y[r] == acc, (dt, r)


# ---------------------------------------------------------------------------
# CGS2
# ---------------------------------------------------------------------------
def _basis(n, k, seed, dt):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return Q.astype(dt)


@pytest.mark.parametrize("k", [1, 5, 8, 9, 17, 33, 50, 64, 65, 100, 129, 200, 256, 257, 300, 512])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("aligned", [False, True])
def test_cgs2_orth_matches_oracle(k, prec, aligned):
    # aligned: every column starts on a 256-byte boundary (the four-row vector
    # passes); otherwise ldv is not a multiple of 4 (the one-row passes)
    n = 3001 + 17 * k
    say("cgs2", k, prec, n, aligned)
    dt = np.float64 if prec == "f64" else np.float32
    V = _basis(n, k, k, dt)
    w = np.random.default_rng(100 + k).standard_normal(n).astype(dt)
    ldv = (n + 63) // 64 * 64 if aligned else n + 64 + (1 if n % 2 == 0 else 0)
    Vd = torch.zeros((k, ldv), dtype=torch.float64 if prec == "f64" else torch.float32, device=DEV)
    Vd[:, :n] = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    wd = torch.from_numpy(w.copy()).to(DEV)
    h = host(G.cgs2_orth(Vd, k, wd, ldv=ldv))
    wout = host(wd)
    w_ref, h1, h2, beta = O.cgs2(V, k, w.copy())
    tol = 1e-12 if prec == "f64" else 2e-5
    href = h1.astype(np.float64) + h2.astype(np.float64)
    scale = np.linalg.norm(w.astype(np.float64))
    assert np.allclose(h[:k], href, rtol=0, atol=tol * scale)
    assert abs(h[k] - float(beta)) <= tol * scale
    assert np.allclose(wout, (w_ref / beta).astype(dt), atol=tol * 10)
    orth = np.abs(V.astype(np.float64).T @ wout.astype(np.float64)).max()
    assert orth < (1e-14 if prec == "f64" else 1e-6)


def test_cgs2_twice_is_enough_f32():
    # a nearly dependent w: one pass would leave O(eps * cond) components
    n, k = 20000, 30
    V = _basis(n, k, 7, np.float32)
    c = np.random.default_rng(8).standard_normal(k).astype(np.float32)
    w = (V @ c + 1e-4 * np.random.default_rng(9).standard_normal(n)).astype(np.float32)
    Vd = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    G.cgs2_orth(Vd, k, wd)
    wout = host(wd).astype(np.float64)
    assert np.abs(V.astype(np.float64).T @ wout).max() < 5e-6


# ---------------------------------------------------------------------------
# Solvers
# ---------------------------------------------------------------------------
def _cfg1():
    return W.config1_laplace2d()


def test_gmres_f64_config1_against_oracle():
    say("gmres f64 config1")
    p = _cfg1()
    A = dev(p.A)
    x, res = G.gmres_solve(A, t64(p.b), restart=50, tol=1e-10, max_iters=20000)
    ref = O.gmres(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say(res.iters, res.cycles, res.rel_res, "oracle", ref.iters, ref.cycles, ref.rel_res)
    assert res.converged and res.rel_res <= 1e-10
    xh = host(x)
    true = np.linalg.norm(p.b - O.spmv(p.A, xh)) / np.linalg.norm(p.b)
    assert true <= 1e-10
    assert abs(res.iters - ref.iters) <= max(2, 0.02 * ref.iters)
    assert np.linalg.norm(xh - 1.0) / np.sqrt(p.A.n) <= 1711.7 * 1e-10 * 10


def test_gmres_ir_config1_against_oracle():
    say("gmres-ir config1")
    p = _cfg1()
    A = dev(p.A)
    x, res = G.gmres_ir_solve(A, A.to_f32(), t64(p.b), restart=50, tol=1e-10, max_iters=20000)
    ref = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say(res.iters, res.cycles, res.rel_res, "oracle", ref.iters, ref.cycles, ref.rel_res)
    assert res.converged and res.rel_res <= 1e-10
    assert res.iters % 50 == 0
    assert abs(res.cycles - ref.cycles) <= max(1, 0.1 * ref.cycles)
    xh = host(x)
    assert np.linalg.norm(p.b - O.spmv(p.A, xh)) / np.linalg.norm(p.b) <= 1e-10
    # the per-restart residual history follows the oracle's
    h, hr = np.array(res.history), np.array(ref.history)
    k = min(len(h), len(hr))
    assert np.all(np.abs(np.log10(h[:k]) - np.log10(hr[:k])) < 1.0)


def test_gmres_f32_only_stalls():
    say("gmres f32-only config1")
    p = _cfg1()
    A32 = dev(p.A).to_f32()
    x, res = G.gmres_solve(A32, t32(p.b), restart=50, tol=1e-10, max_iters=2000)
    assert res.status == 1
    assert 1e-8 < min(res.history) < 1e-5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_nonsymmetric_dense_solve(seed):
    rng = np.random.default_rng(seed)
    n = 16 + 8 * seed
    D = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    rows, cols = np.nonzero(D)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    A = W.CSR(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), D[rows, cols])
    b = rng.standard_normal(n)
    xs = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    Ad = dev(A)
    x1, r1 = G.gmres_solve(Ad, t64(b), restart=8, tol=1e-10, max_iters=1000)
    x2, r2 = G.gmres_ir_solve(Ad, Ad.to_f32(), t64(b), restart=8, tol=1e-10, max_iters=1000)
    for x, r in ((x1, r1), (x2, r2)):
        assert r.converged
        assert np.linalg.norm(host(x) - xs) / np.linalg.norm(xs) <= 10 * kappa * 1e-10


def test_determinism_bitwise():
    p = W.config2_laplace3d(N=24)
    A = dev(p.A)
    A32 = A.to_f32()
    xa, ra = G.gmres_ir_solve(A, A32, t64(p.b), restart=30, tol=1e-10, max_iters=5000)
    xb, rb = G.gmres_ir_solve(A, A32, t64(p.b), restart=30, tol=1e-10, max_iters=5000)
    assert np.array_equal(host(xa), host(xb)) and ra.history == rb.history


def test_resume_from_returned_x_is_bitwise_equal():
    p = W.config2_laplace3d(N=20)
    A = dev(p.A)
    A32 = A.to_f32()
    b = t64(p.b)
    xa, ra = G.gmres_ir_solve(A, A32, b, restart=20, tol=1e-10, max_iters=5000)
    xb, rb1 = G.gmres_ir_solve(A, A32, b, restart=20, tol=1e-10, max_iters=5000, max_cycles=3)
    assert rb1.status == 1
    xb, rb2 = G.gmres_ir_solve(A, A32, b, xb, restart=20, tol=1e-10, max_iters=5000)
    assert np.array_equal(host(xa), host(xb))
    assert rb1.cycles + rb2.cycles == ra.cycles


def test_error_paths():
    p = W.config2_laplace3d(N=10)
    A = dev(p.A)
    A32 = A.to_f32()
    b = t64(p.b)
    small = G.alloc_workspace(1024, DEV)
    with pytest.raises(G.GmresError) as e:
        G.gmres_ir_solve(A, A32, b, ws=small)
    assert e.value.status == -3
    bn = b.clone()
    bn[5] = float("nan")
    with pytest.raises(G.GmresError) as e:
        G.gmres_ir_solve(A, A32, bn)
    assert e.value.status == -4
    x, r = G.gmres_ir_solve(A, A32, b, restart=5, max_iters=10)
    assert r.status == 1 and r.iters == 10
    x, r = G.gmres_ir_solve(A, A32, torch.zeros_like(b))
    assert r.status == 0 and float(host(x).max()) == 0.0


def test_ir_self_corrects_a_corrupted_iterate():
    # a damaged x between restarts is repaired by the float64 residual
    p = W.config2_laplace3d(N=16)
    A = dev(p.A)
    A32 = A.to_f32()
    b = t64(p.b)
    x, r1 = G.gmres_ir_solve(A, A32, b, restart=20, max_cycles=2)
    x[::7] += 1.0
    x, r2 = G.gmres_ir_solve(A, A32, b, x, restart=20, max_iters=20000)
    assert r2.converged and r2.rel_res <= 1e-10


# ---------------------------------------------------------------------------
# GMRES polynomial
# ---------------------------------------------------------------------------
def test_poly_roots_and_apply_f64():
    say("poly f64")
    A = W.convdiff2d(30, 0.05, W.configs.uniflow_wind)
    v0 = W.poly_start_vector(A.n, 3)
    Ad = dev(A)
    P = G.poly_prec_setup(Ad, 10, t64(v0))
    roots = P.roots()
    ref = O.poly_roots(A, 10, v0, np.float64)
    assert P.degree == 10
    Hg = P.hessenberg()
    _, Hr, _ = O.arnoldi(A, v0, 11)
    say("max |H_gpu - H_oracle|", np.abs(Hg - Hr).max(), np.abs(Hr).max())
    assert np.allclose(Hg, Hr, rtol=0, atol=1e-12 * np.abs(Hr).max())
    assert np.allclose(np.sort_complex(roots), np.sort_complex(ref), rtol=1e-7, atol=1e-10)
    x = W.uniform_pm1(5, A.n)
    y = host(G.poly_prec_apply(P, Ad, t64(x)))
    yref = O.poly_apply(A, ref, x, np.float64)
    assert np.allclose(y, yref, rtol=1e-8, atol=1e-8 * np.abs(yref).max())
    # pin (i): ||v - A p(A) v|| equals the (d+1)-step GMRES residual from v
    v = v0 / np.linalg.norm(v0)
    pv = host(G.poly_prec_apply(P, Ad, t64(v)))
    res = np.linalg.norm(v - O.spmv(A, pv))
    out = O.gmres(A, v, np.zeros(A.n), 11, 1e-300, 11, max_cycles=1)
    assert np.isclose(res, out.implicit_history[-1] * np.linalg.norm(v), rtol=1e-6)


def test_poly_exact_inverse_diagonal():
    d = np.repeat([0.5, 1.0, 2.0, 4.0, 6.0, 9.0], 50)
    n = d.size
    A = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    Ad = dev(A)
    v = W.uniform01(6, n) + 0.5
    P = G.poly_prec_setup(Ad, 5, t64(v))
    y = host(G.poly_prec_apply(P, Ad, t64(v)))
    assert np.allclose(d * y, v, rtol=1e-9)


def test_poly_f32_apply_close_to_oracle():
    A = W.laplace2d(40)
    v0 = W.poly_start_vector(A.n, 9)
    A32 = dev(A).to_f32()
    P = G.poly_prec_setup(A32, 8, t32(v0))
    r = P.roots()
    assert np.all(np.abs(r.imag) == 0) and np.all(r.real > 0)
    rref = O.poly_roots(A, 8, v0.astype(np.float32), np.float32)
    assert np.allclose(np.sort_complex(r), np.sort_complex(rref), rtol=1e-5, atol=0)
    x = W.uniform_pm1(12, A.n)
    y = host(G.poly_prec_apply(P, A32, t32(x))).astype(np.float64)
    yref = O.poly_apply(A, rref, x, np.float64)
    assert np.allclose(y, yref, rtol=0, atol=2e-4 * np.abs(yref).max())


def test_gmres_ir_poly_small_convdiff():
    say("gmres-ir + poly convdiff N=60")
    p = W.config3_convdiff(N=60, restart=20, degree=8)
    A = dev(p.A)
    A32 = A.to_f32()
    v0 = W.poly_start_vector(p.A.n, p.poly_seed)
    P32 = G.poly_prec_setup(A32, 8, t32(v0))
    x, res = G.gmres_ir_solve(A, A32, t64(p.b), restart=20, tol=1e-10, max_iters=20000, P=P32)
    assert res.converged and res.iters % 20 == 0
    xh = host(x)
    assert np.linalg.norm(p.b - O.spmv(p.A, xh)) / np.linalg.norm(p.b) <= 1e-10
    roots32 = O.poly_roots(p.A, 8, v0.astype(np.float32), np.float32)
    prec = lambda v: O.poly_apply(p.A, roots32, v, np.float32)
    ref = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 20, 1e-10, 20000, prec32=prec)
    say(res.cycles, ref.cycles)
    assert abs(res.cycles - ref.cycles) <= max(1, 0.1 * ref.cycles)
    # float64 GMRES with a float64 polynomial reaches the tolerance too
    P64 = G.poly_prec_setup(A, 8, t64(v0))
    x64, r64 = G.gmres_solve(A, t64(p.b), restart=20, tol=1e-10, max_iters=20000, P=P64)
    assert r64.converged


# ---------------------------------------------------------------------------
# Full-size workloads (properties that hold at any size)
# ---------------------------------------------------------------------------
def test_config2_full_gmres_ir_reaches_1e10():
    say("config2 full gmres-ir")
    p = W.config2_laplace3d()
    A = dev(p.A)
    A32 = A.to_f32()
    x, res = G.gmres_ir_solve(A, A32, t64(p.b), restart=50, tol=1e-10, max_iters=20000)
    say(res.iters, res.cycles, res.rel_res, res.seconds)
    assert res.converged and res.iters % 50 == 0
    xh = host(x)
    assert np.linalg.norm(p.b - O.spmv(p.A, xh)) / np.linalg.norm(p.b) <= 1e-10
    fwd = np.linalg.norm(xh - p.x_true) / np.linalg.norm(p.x_true)
    assert fwd <= 9240.2 * 1e-10 * 10


@pytest.mark.parametrize("fill", [0x00, 0xFF, 0x7F])
def test_poisoned_workspace_gives_identical_results(fill):
    # every workspace byte the solver reads it has written first: a workspace
    # full of NaN (0xFF) or huge values (0x7F) gives the same bits as zeros
    say("poisoned workspace", fill)
    p = W.config3_convdiff(N=40, restart=15, degree=6)
    A = dev(p.A)
    A32 = A.to_f32()
    v0 = t32(W.poly_start_vector(p.A.n, p.poly_seed))
    nb = G.workspace_bytes(p.A.n, 15, G.GMR_F32, True)
    ws = G.alloc_workspace(nb, DEV)
    ws.fill_(fill)
    P32 = G.poly_prec_setup(A32, 6, v0, ws=ws)
    ws.fill_(fill)
    x, res = G.gmres_ir_solve(A, A32, t64(p.b), restart=15, max_iters=3000, P=P32, ws=ws)
    ws0 = G.alloc_workspace(nb, DEV)
    ws0.zero_()
    P0 = G.poly_prec_setup(A32, 6, v0, ws=ws0)
    x0, res0 = G.gmres_ir_solve(A, A32, t64(p.b), restart=15, max_iters=3000, P=P0, ws=ws0)
    assert np.array_equal(P32.roots(), P0.roots())
    assert res.converged and np.array_equal(host(x), host(x0))


def test_config3_full_poly_ir_and_fp64_reach_1e10():
    # 2D upwind convection-diffusion, n = 6.25M, GMRES(100)-IR with a float32
    # degree-25 GMRES polynomial vs float64 GMRES(100) with a float64 one
    say("config3 full: generating")
    p = W.config3_convdiff()
    assert p.A.n == 6250000 and p.A.nnz == 31240000
    A = dev(p.A)
    A32 = A.to_f32()
    b = t64(p.b)
    v0 = W.poly_start_vector(p.A.n, p.poly_seed)
    say("config3 full: poly setup")
    P32 = G.poly_prec_setup(A32, 25, t32(v0))
    P64 = G.poly_prec_setup(A, 25, t64(v0))
    assert P32.degree == 25 and P64.degree == 25
    say("config3 full: GMRES-IR")
    x, res = G.gmres_ir_solve(A, A32, b, restart=100, tol=1e-10, max_iters=5000, P=P32)
    say("IR", res.status_name, res.iters, res.cycles, res.rel_res, res.seconds)
    assert res.converged and res.iters % 100 == 0
    xh = host(x)
    assert np.linalg.norm(p.b - O.spmv(p.A, xh)) / np.linalg.norm(p.b) <= 1e-10
    say("config3 full: FP64 GMRES")
    x64, r64 = G.gmres_solve(A, b, restart=100, tol=1e-10, max_iters=5000, P=P64)
    say("FP64", r64.status_name, r64.iters, r64.cycles, r64.rel_res, r64.seconds)
    assert r64.converged
    x64h = host(x64)
    assert np.linalg.norm(p.b - O.spmv(p.A, x64h)) / np.linalg.norm(p.b) <= 1e-10
    # IR needs at most a few more cycles than float64 GMRES (§III-B, Tables II and III)
    assert res.iters <= r64.iters + 3 * 100


@pytest.mark.parametrize("kind", ["ir", "f64", "ir_poly"])
def test_graph_replay_matches_eager(kind):
    # one restart cycle captured as a hipGraph and replayed every restart (with
    # host synchronisation and copies between replays) gives the eager bits
    say("graph replay", kind)
    p = W.config3_convdiff(N=48, restart=12, degree=5) if kind == "ir_poly" else W.config2_laplace3d(N=22, restart=12)
    A = dev(p.A)
    A32 = A.to_f32()
    b = t64(p.b)
    P = None
    if kind == "ir_poly":
        P = G.poly_prec_setup(A32, 5, t32(W.poly_start_vector(p.A.n, p.poly_seed)))
    out = []
    for graph in (False, True, True):
        if kind == "f64":
            x, r = G.gmres_solve(A, b, restart=12, max_iters=20000, graph=graph)
        else:
            x, r = G.gmres_ir_solve(A, A32, b, restart=12, max_iters=20000, P=P, graph=graph)
        out.append((host(x), r))
    for xg, rg in out[1:]:
        assert rg.converged and rg.cycles == out[0][1].cycles and rg.iters == out[0][1].iters
        assert np.array_equal(xg, out[0][0]) and rg.history == out[0][1].history
    # a capped last cycle (max_iters not a multiple of m) is captured again
    x1, r1 = G.gmres_ir_solve(A, A32, b, restart=12, max_iters=30, P=P, graph=False)
    x2, r2 = G.gmres_ir_solve(A, A32, b, restart=12, max_iters=30, P=P, graph=True)
    assert r1.iters == r2.iters == 30 and np.array_equal(host(x1), host(x2))


# ---------------------------------------------------------------------------
# Persistent single-block cycle (small systems)
# ---------------------------------------------------------------------------
def test_persistent_cycle_small_laplacian_against_oracle():
    say("persistent laplace2d 24x24")
    p = W.config1_laplace2d(N=24)
    A = dev(p.A)
    A32 = A.to_f32()
    x1, r1 = G.gmres_solve(A, t64(p.b), restart=50, tol=1e-10, max_iters=20000, persistent=True)
    ref = O.gmres(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say("f64", r1.iters, r1.cycles, r1.rel_res, "oracle", ref.iters)
    assert r1.converged and abs(r1.iters - ref.iters) <= max(2, 0.02 * ref.iters)
    assert np.linalg.norm(p.b - O.spmv(p.A, host(x1))) / np.linalg.norm(p.b) <= 1e-10
    x2, r2 = G.gmres_ir_solve(A, A32, t64(p.b), restart=50, tol=1e-10, max_iters=20000, persistent=True)
    ref2 = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say("ir", r2.iters, r2.cycles, r2.rel_res, "oracle", ref2.cycles)
    assert r2.converged and r2.iters % 50 == 0
    assert abs(r2.cycles - ref2.cycles) <= max(1, 0.1 * ref2.cycles)
    assert np.linalg.norm(p.b - O.spmv(p.A, host(x2))) / np.linalg.norm(p.b) <= 1e-10
    h, hr = np.array(r2.history), np.array(ref2.history)
    k = min(len(h), len(hr))
    assert np.all(np.abs(np.log10(h[:k]) - np.log10(hr[:k])) < 1.0)


@pytest.mark.parametrize("n_side,restart", [(17, 8), (30, 30), (32, 70), (24, 300)])
def test_persistent_cycle_matches_multikernel(n_side, restart):
    # ragged last SpMV chunk, restart beyond the fused 64-column pass, the largest n (1024)
    say("persistent vs multi-kernel", n_side, restart)
    A_h = W.convdiff2d(n_side, 0.05, lambda x, y: (np.cos(2 * x), np.sin(3 * y)))
    b_h = W.uniform_pm1(77, A_h.n)
    A = dev(A_h)
    A32 = A.to_f32()
    for f in (lambda **k: G.gmres_solve(A, t64(b_h), **k), lambda **k: G.gmres_ir_solve(A, A32, t64(b_h), **k)):
        xa, ra = f(restart=restart, tol=1e-10, max_iters=20000)
        xb, rb = f(restart=restart, tol=1e-10, max_iters=20000, persistent=True)
        say(ra.iters, rb.iters, ra.rel_res, rb.rel_res)
        assert ra.converged and rb.converged
        assert abs(ra.iters - rb.iters) <= max(2, 0.05 * ra.iters)
        assert np.linalg.norm(b_h - O.spmv(A_h, host(xb))) / np.linalg.norm(b_h) <= 1e-10
        # a second persistent run is bitwise the same (deterministic block sums)
        xc, rc = f(restart=restart, tol=1e-10, max_iters=20000, persistent=True)
        assert np.array_equal(host(xb), host(xc)) and rb.history == rc.history


# ---------------------------------------------------------------------------
# Cooperative multi-block cycle (1024 < n <= 6144)
# ---------------------------------------------------------------------------
def test_cooperative_cycle_config1_against_oracle():
    say("cooperative cycle, 2D Laplacian 64x64")
    p = W.config1_laplace2d(N=64)
    A = dev(p.A)
    A32 = A.to_f32()
    x1, r1 = G.gmres_solve(A, t64(p.b), restart=50, tol=1e-10, max_iters=20000, persistent=True)
    ref = O.gmres(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say("f64", r1.iters, r1.cycles, r1.rel_res, "oracle", ref.iters)
    assert r1.converged and abs(r1.iters - ref.iters) <= max(2, 0.02 * ref.iters)
    assert np.linalg.norm(p.b - O.spmv(p.A, host(x1))) / np.linalg.norm(p.b) <= 1e-10
    x2, r2 = G.gmres_ir_solve(A, A32, t64(p.b), restart=50, tol=1e-10, max_iters=20000, persistent=True)
    ref2 = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 50, 1e-10, 20000)
    say("ir", r2.iters, r2.cycles, r2.rel_res, "oracle", ref2.cycles)
    assert r2.converged and r2.iters % 50 == 0
    assert abs(r2.cycles - ref2.cycles) <= max(1, 0.1 * ref2.cycles)
    assert np.linalg.norm(p.b - O.spmv(p.A, host(x2))) / np.linalg.norm(p.b) <= 1e-10
    h, hr = np.array(r2.history), np.array(ref2.history)
    k = min(len(h), len(hr))
    assert np.all(np.abs(np.log10(h[:k]) - np.log10(hr[:k])) < 1.0)


@pytest.mark.parametrize("n_side,restart", [(33, 50), (70, 80), (78, 30), (50, 20)])
def test_cooperative_cycle_matches_multikernel(n_side, restart):
    # 1089 rows (five blocks, ragged last one), 4900 rows with restart beyond
    # the fused 64-column pass, 6084 rows (24 blocks, near the largest n),
    # 2500 rows (ten blocks, a ragged SpMV group)
    say("cooperative vs multi-kernel", n_side, restart)
    A_h = W.convdiff2d(n_side, 0.05, lambda x, y: (np.cos(2 * x), np.sin(3 * y)))
    b_h = W.uniform_pm1(78, A_h.n)
    A = dev(A_h)
    A32 = A.to_f32()
    for f in (lambda **k: G.gmres_solve(A, t64(b_h), **k), lambda **k: G.gmres_ir_solve(A, A32, t64(b_h), **k)):
        xa, ra = f(restart=restart, tol=1e-10, max_iters=40000)
        xb, rb = f(restart=restart, tol=1e-10, max_iters=40000, persistent=True)
        say(ra.iters, rb.iters, ra.rel_res, rb.rel_res)
        assert ra.converged and rb.converged
        assert abs(ra.iters - rb.iters) <= max(2, 0.05 * ra.iters)
        assert np.linalg.norm(b_h - O.spmv(A_h, host(xb))) / np.linalg.norm(b_h) <= 1e-10
        # deterministic: block partials are added in block order
        xc, rc = f(restart=restart, tol=1e-10, max_iters=40000, persistent=True)
        assert np.array_equal(host(xb), host(xc)) and rb.history == rc.history


def test_cooperative_cycle_lucky_breakdown():
    # b = 3 e_8 on a diagonal matrix: v_1 = e_8 exactly, A v_1 = a_88 v_1, and
    # both CGS passes leave w = 0 exactly in either precision, so every cycle
    # ends by breakdown after one column (in GMRES-IR the cooperative cycle
    # takes that column's Givens step after leaving the loop).  a_88 = 5, so
    # the float32 correction 1/5 is inexact and IR needs more than one cycle.
    n = 2000
    d = 2.0 + (np.arange(n) % 5).astype(np.float64)
    A_h = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    b_h = np.zeros(n)
    b_h[8] = 3.0
    A = dev(A_h)
    A32 = A.to_f32()
    for name, f in (("f64", lambda **k: G.gmres_solve(A, t64(b_h), **k)),
                    ("ir", lambda **k: G.gmres_ir_solve(A, A32, t64(b_h), **k))):
        say("lucky breakdown", name)
        xa, ra = f(restart=50, tol=1e-10, max_iters=1000)
        xb, rb = f(restart=50, tol=1e-10, max_iters=1000, persistent=True)
        say(ra.iters, ra.cycles, rb.iters, rb.cycles, rb.rel_res)
        for r in (ra, rb):
            assert r.converged and r.iters == r.cycles
        assert (ra.iters, ra.cycles) == (rb.iters, rb.cycles)
        # one nonzero product per sum: the block order cannot change a bit
        assert np.array_equal(host(xa), host(xb))
        assert np.linalg.norm(b_h - O.spmv(A_h, host(xb))) / np.linalg.norm(b_h) <= 1e-10
        assert np.count_nonzero(host(xb)) == 1
