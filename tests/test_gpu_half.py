"""GPU parity of GMRES-IR with the inner Krylov basis stored in float16."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_2105_07544_amd")

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def t64(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_res(A, b, x):
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return float(np.linalg.norm(b - M @ x) / np.linalg.norm(b))


CASES = {
    # name: (matrix, restart); n odd and not a multiple of 4 or 128 in two of them
    "laplace3d_12_m20": (lambda: W.laplace3d(12), 20),
    "laplace2d_37_m30": (lambda: W.laplace2d(37), 30),
    "convdiff_41_m80": (lambda: W.convdiff2d(41, 1e-2, W.configs.uniflow_wind), 80),   # j > 64 passes
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_half_basis_against_oracle(name):
    say("half basis vs oracle", name)
    make, m = CASES[name]
    A = make()
    xt = W.uniform_pm1(3, A.n)
    b = W.host_matvec(A, xt)
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    x, r = G.gmres_ir_solve(A64, A32, t64(b), restart=m, tol=1e-10, max_iters=40000, half_basis=True)
    ref = O.gmres_ir(A, b, np.zeros(A.n), m, 1e-10, 40000, half_basis=True)
    say(r.iters, r.cycles, r.history[:4], "oracle", ref.iters, ref.cycles, ref.history[:4])
    assert r.converged and rel_res(A, b, host(x)) <= 1e-10
    assert abs(r.cycles - ref.cycles) <= max(1, 0.1 * ref.cycles)
    h, hr = np.array(r.history), np.array(ref.history)
    k = min(len(h), len(hr))
    assert np.all(np.abs(np.log10(h[:k]) - np.log10(hr[:k])) < 0.5)
    # every cycle still cuts the residual by at least the float16 accuracy allows
    assert np.all(h[1:] / h[:-1] < 1e-2) or len(h) > 5


@pytest.mark.parametrize("prec", ["poly", "bjac"])
def test_half_basis_with_preconditioner_against_oracle(prec):
    say("half basis with", prec)
    p = W.config3_convdiff(N=60, restart=20, degree=8)
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    A32 = A64.to_f32()
    v0 = W.poly_start_vector(p.A.n, p.poly_seed)
    if prec == "poly":
        P = G.poly_prec_setup(A32, 8, torch.from_numpy(v0.astype(np.float32)).to(DEV))
        roots = O.poly_roots(p.A, 8, v0.astype(np.float32), np.float32)
        prec32 = lambda v: O.poly_apply(p.A, roots, v, np.float32)  # noqa: E731
    else:
        P = G.bjac_prec_setup(A32, 16)
        prec32 = lambda v: O.bjac_apply(p.A, 16, v, np.float32)  # noqa: E731
    x, r = G.gmres_ir_solve(A64, A32, t64(p.b), restart=20, tol=1e-10, max_iters=20000, P=P, half_basis=True)
    ref = O.gmres_ir(p.A, p.b, np.zeros(p.A.n), 20, 1e-10, 20000, prec32=prec32, half_basis=True)
    say(r.iters, r.cycles, "oracle", ref.iters, ref.cycles)
    assert r.converged and rel_res(p.A, p.b, host(x)) <= 1e-10
    assert abs(r.cycles - ref.cycles) <= max(1, 0.1 * ref.cycles)
    h, hr = np.array(r.history), np.array(ref.history)
    k = min(len(h), len(hr))
    assert np.all(np.abs(np.log10(h[:k]) - np.log10(hr[:k])) < 0.5)


def test_half_basis_graph_replay_is_bitwise_eager():
    p = W.config2_laplace3d(N=22, restart=12)
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    A32 = A64.to_f32()
    out = [G.gmres_ir_solve(A64, A32, t64(p.b), restart=12, max_iters=20000, half_basis=True, graph=g)
           for g in (False, True, True)]
    for x, r in out[1:]:
        assert r.converged and r.iters == out[0][1].iters and r.history == out[0][1].history
        assert np.array_equal(host(x), host(out[0][0]))


def test_half_basis_unsupported_combinations():
    A = W.laplace2d(10)
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    b = t64(np.ones(A.n))
    calls = (lambda: G.gmres_solve(A64, b, restart=10, half_basis=True),
             lambda: G.gmres_solve(A32, b.float(), restart=10, half_basis=True))
    for call in calls:
        with pytest.raises(G.GmresError) as e:
            call()
        assert e.value.status == -5


def test_half_basis_config2_full_size():
    """The 150^3 Laplacian (n = 3,375,000) with the float16 basis reaches 1e-10
    (residual recomputed on the host); the first cycle is float16-limited (about
    4e-4 instead of 1e-5), later ones track the float32 basis, so it needs at most
    20 % more cycles."""
    say("half basis config2 full")
    p = W.config2_laplace3d()
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    A32 = A64.to_f32()
    x, r = G.gmres_ir_solve(A64, A32, t64(p.b), restart=50, tol=1e-10, max_iters=20000, half_basis=True)
    _, r32 = G.gmres_ir_solve(A64, A32, t64(p.b), restart=50, tol=1e-10, max_iters=20000)
    say(r.iters, r.cycles, r.seconds, "float32 basis", r32.iters, r32.cycles, r32.seconds)
    assert r.converged and rel_res(p.A, p.b, host(x)) <= 1e-10
    assert r.cycles <= 1.2 * r32.cycles


def test_half_basis_ignores_the_persistent_flag():
    # the single-block cycle has no float16 form: the flag is ignored, same bits
    A = W.laplace2d(20)
    b = W.host_matvec(A, W.uniform_pm1(5, A.n))
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    x0, r0 = G.gmres_ir_solve(A64, A32, t64(b), restart=20, half_basis=True)
    x1, r1 = G.gmres_ir_solve(A64, A32, t64(b), restart=20, half_basis=True, persistent=True)
    assert r0.converged and r0.iters == r1.iters and np.array_equal(host(x0), host(x1))


@pytest.mark.parametrize("fill", [0x00, 0xFF, 0x7C])
def test_half_basis_poisoned_workspace_gives_identical_results(fill):
    """Odd n: the float16 passes read the padding row of each basis column and must
    not let its contents (never written; NaN or Inf patterns here) reach the result."""
    A = W.laplace2d(37)   # n = 1369, odd
    b = W.host_matvec(A, W.uniform_pm1(6, A.n))
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    ws = G.alloc_workspace(G.workspace_bytes(A.n, 30, G.GMR_F32), DEV)
    ws.fill_(0)
    x0, r0 = G.gmres_ir_solve(A64, A32, t64(b), restart=30, ws=ws, half_basis=True)
    ws.fill_(fill)
    x1, r1 = G.gmres_ir_solve(A64, A32, t64(b), restart=30, ws=ws, half_basis=True)
    assert r0.converged and r1.converged and r0.iters == r1.iters
    assert np.array_equal(host(x0), host(x1))
