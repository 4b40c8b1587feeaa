"""GPU parity of float64 GMRES with a float32 polynomial preconditioner, and of the
loss-of-accuracy handling (implicit residual met, explicit residual not)."""
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


def t32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_res(A, b, x):
    M = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))
    return float(np.linalg.norm(b - M @ x) / np.linalg.norm(b))


@pytest.mark.parametrize("degree", [5, 10, 20])
def test_f32_poly_in_f64_gmres_against_oracle(degree):
    say("f32 poly in f64 gmres, laplace3d 10^3, degree", degree)
    A = W.laplace3d(10)
    b = np.ones(A.n)
    v0 = W.poly_start_vector(A.n, 0)
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    P32 = G.poly_prec_setup(A32, degree, t32(v0))
    P64 = G.poly_prec_setup(A64, degree, t64(v0))
    x, r = G.gmres_f32prec_solve(A64, A32, P32, t64(b), restart=50, tol=1e-10, max_iters=500)
    r32 = O.poly_roots(A, degree, v0.astype(np.float32), np.float32)
    ref = O.gmres(A, b, np.zeros(A.n), 50, 1e-10, 500,
                  prec=O.cast_wrapped(lambda v: O.poly_apply(A, r32, v, np.float32)))
    say(r.iters, r.cycles, r.loss_of_accuracy, r.history, "oracle", ref.iters, ref.cycles,
        ref.loss_of_accuracy, ref.history)
    # both stop the first cycle on the implicit residual with a float32-accurate
    # explicit residual, count the loss of accuracy, and correct it on restart
    assert r.converged and r.loss_of_accuracy >= 1 and ref.loss_of_accuracy >= 1
    assert rel_res(A, b, host(x)) <= 1e-10
    assert 1e-9 < r.history[1] < 1e-4
    assert abs(np.log10(r.history[1]) - np.log10(ref.history[1])) < 1.0
    assert abs(r.cycles - ref.cycles) <= 1 and abs(r.iters - ref.iters) <= max(3, 0.2 * ref.iters)
    # the Belos-like policy ends at the first loss of accuracy, x = that iterate
    x2, r2 = G.gmres_f32prec_solve(A64, A32, P32, t64(b), restart=50, tol=1e-10, max_iters=500,
                                   stop_on_loss=True)
    assert r2.status == 3 and r2.cycles == 1 and r2.loss_of_accuracy == 1
    assert np.isclose(rel_res(A, b, host(x2)), r2.rel_res, rtol=1e-6) and r2.rel_res > 1e-10
    # a float64 polynomial shows no loss of accuracy here
    x3, r3 = G.gmres_solve(A64, t64(b), restart=50, tol=1e-10, max_iters=500, P=P64, stop_on_loss=True)
    assert r3.converged and r3.loss_of_accuracy == 0 and r3.cycles == 1


def test_three_preconditioning_options_small_convdiff():
    """float64 GMRES + float64 polynomial, float64 GMRES + float32 polynomial and
    GMRES-IR + float32 polynomial all reach 1e-10 with similar iteration counts."""
    say("three preconditioning options, convdiff 80^2, degree 10")
    p = W.config3_convdiff(N=80, restart=30, degree=10)
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    A32 = A64.to_f32()
    v0 = W.poly_start_vector(p.A.n, p.poly_seed)
    P32 = G.poly_prec_setup(A32, 10, t32(v0))
    P64 = G.poly_prec_setup(A64, 10, t64(v0))
    b = t64(p.b)
    xa, ra = G.gmres_solve(A64, b, restart=30, tol=1e-10, max_iters=20000, P=P64)
    xb, rb = G.gmres_f32prec_solve(A64, A32, P32, b, restart=30, tol=1e-10, max_iters=20000)
    xc, rc = G.gmres_ir_solve(A64, A32, b, restart=30, tol=1e-10, max_iters=20000, P=P32)
    say("iters", ra.iters, rb.iters, rc.iters, "loss", ra.loss_of_accuracy, rb.loss_of_accuracy)
    for x, r in ((xa, ra), (xb, rb), (xc, rc)):
        assert r.converged and rel_res(p.A, p.b, host(x)) <= 1e-10
    assert rb.iters <= 1.5 * ra.iters + 30 and rc.iters <= 1.5 * ra.iters + 30


def test_f32prec_graph_replay_is_bitwise_eager():
    say("f32 poly in f64 gmres, graph replay")
    p = W.config3_convdiff(N=48, restart=12, degree=5)
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    A32 = A64.to_f32()
    P32 = G.poly_prec_setup(A32, 5, t32(W.poly_start_vector(p.A.n, p.poly_seed)))
    out = [G.gmres_f32prec_solve(A64, A32, P32, t64(p.b), restart=12, max_iters=20000, graph=g)
           for g in (False, True, True)]
    for x, r in out[1:]:
        assert r.converged and r.iters == out[0][1].iters
        assert np.array_equal(host(x), host(out[0][0]))


def test_f32prec_rejects_float64_polynomial():
    A = W.laplace2d(8)
    A64 = G.DeviceCSR.from_host(A, DEV)
    P64 = G.poly_prec_setup(A64, 3, t64(W.poly_start_vector(A.n, 1)))
    with pytest.raises(G.GmresError) as e:
        G.gmres_f32prec_solve(A64, A64.to_f32(), P64, t64(np.ones(A.n)))
    assert e.value.status == -1
