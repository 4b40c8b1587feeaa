"""GPU parity of GMRES-FD (float32 GMRES(m), then float64 GMRES(m) from its iterate)."""
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


def scipy_csr(A):
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))


def _problem():
    # 2D Laplacian on 32^2 (n = 1024), b = A x_true with x_true ~ U(-1, 1)
    A = W.laplace2d(32)
    xt = W.uniform_pm1(41, A.n)
    return A, scipy_csr(A) @ xt, xt


@pytest.mark.parametrize("switch", [0, 40, 200, 600])
def test_fd_against_oracle(switch):
    say("fd vs oracle, switch", switch)
    A, b, xt = _problem()
    m, tol = 20, 1e-10
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    x, both, first = G.gmres_fd_solve(A64, A32, t64(b), switch, restart=m, tol=tol, max_iters=20000)
    f_ref, s_ref = O.gmres_fd(A, b, np.zeros(A.n), m, tol, switch, 20000)
    say(switch, first.iters, both.iters, both.rel_res, "oracle",
        f_ref.iters if f_ref else 0, (f_ref.iters if f_ref else 0) + s_ref.iters, s_ref.rel_res)
    # the float32 phase runs exactly to the switch point (float32 cannot reach 1e-10)
    assert first.iters == switch
    assert first.status == (1 if switch else 0)
    # the float64 phase starts from the widened float32 iterate: its first residual
    # follows the oracle's (closely before the float32 stall, within the noise after)
    start, start_ref = both.history[0], s_ref.history[0]
    slack = 0.02 if switch <= 40 else 0.5
    assert abs(np.log10(start) - np.log10(start_ref)) < slack, (start, start_ref)
    # both reach the float64 tolerance with the same amount of work, up to a restart or 10 %
    assert both.converged and both.rel_res <= tol
    xh = host(x)
    assert np.linalg.norm(b - scipy_csr(A) @ xh) / np.linalg.norm(b) <= tol
    kappa = 1.0 / np.tan(np.pi / 66) ** 2   # lambda_max / lambda_min of the 32^2 Laplacian
    assert np.linalg.norm(xh - xt) / np.linalg.norm(xt) <= 10 * kappa * tol
    total_ref = (f_ref.iters if f_ref else 0) + s_ref.iters
    assert abs(both.iters - total_ref) <= max(m, 0.1 * total_ref)
    assert both.cycles >= first.cycles


def test_fd_switch_zero_is_float64_gmres_bitwise():
    say("fd switch 0 == gmres_solve")
    A, b, _ = _problem()
    A64 = G.DeviceCSR.from_host(A, DEV)
    x1, both, first = G.gmres_fd_solve(A64, A64.to_f32(), t64(b), 0, restart=20, tol=1e-10, max_iters=20000)
    x2, r2 = G.gmres_solve(A64, t64(b), restart=20, tol=1e-10, max_iters=20000)
    assert first.iters == 0 and both.iters == r2.iters and both.cycles == r2.cycles
    assert np.array_equal(host(x1), host(x2))


def test_fd_iteration_cap_and_nonconvergence():
    say("fd iteration cap")
    A, b, _ = _problem()
    A64 = G.DeviceCSR.from_host(A, DEV)
    x, both, first = G.gmres_fd_solve(A64, A64.to_f32(), t64(b), 60, restart=20, tol=1e-10, max_iters=90)
    assert first.iters == 60 and both.iters == 90 and both.status == 1
    # the returned iterate is finite and better than x0 = 0
    assert np.isfinite(host(x)).all() and both.rel_res < 1.0


def test_fd_float32_overflow_leaves_x_unchanged():
    say("fd float32 overflow")
    A, b, _ = _problem()
    A64 = G.DeviceCSR.from_host(A, DEV)
    b = b.copy()
    b[5] = 1e39   # not representable in float32
    x0 = t64(np.full(A.n, 0.25))
    with pytest.raises(G.GmresError) as e:
        G.gmres_fd_solve(A64, A64.to_f32(), t64(b), 40, x0, restart=20, tol=1e-10, max_iters=1000)
    assert e.value.status == -4
    assert np.array_equal(host(x0), np.full(A.n, 0.25))


def test_fd_b_zero_gives_zero():
    say("fd b = 0")
    A, _, _ = _problem()
    A64 = G.DeviceCSR.from_host(A, DEV)
    x0 = t64(np.ones(A.n))
    x, both, first = G.gmres_fd_solve(A64, A64.to_f32(), t64(np.zeros(A.n)), 40, x0, restart=20)
    assert both.status == 0 and not host(x).any()


def test_fd_laplace3d200_one_switch_point_full_size():
    """The switch-point problem at its full size (n = 8,000,000), one switch point;
    the residual is recomputed on the host in float64."""
    say("fd laplace3d 200^3, switch 1000")
    p = W.fd_laplace3d(200)
    A64 = G.DeviceCSR.from_host(p.A, DEV)
    x, both, first = G.gmres_fd_solve(A64, A64.to_f32(), t64(p.b), 1000, restart=50, tol=1e-10,
                                      max_iters=20000)
    say(first.iters, both.iters, both.rel_res, both.seconds)
    assert first.iters == 1000 and both.converged
    xh = host(x)
    rel = np.linalg.norm(p.b - scipy_csr(p.A) @ xh) / np.linalg.norm(p.b)
    assert rel <= 1e-10, rel


def test_fd_graph_and_persistent_flags():
    """GMRES-FD under graph replay gives the eager bits; the single-block cycle
    (n <= 1024) reaches the same tolerance with the same iteration split."""
    A, b, _ = _problem()
    A64 = G.DeviceCSR.from_host(A, DEV)
    A32 = A64.to_f32()
    x0, r0, f0 = G.gmres_fd_solve(A64, A32, t64(b), 60, restart=20, tol=1e-10, max_iters=20000)
    x1, r1, f1 = G.gmres_fd_solve(A64, A32, t64(b), 60, restart=20, tol=1e-10, max_iters=20000, graph=True)
    assert np.array_equal(host(x0), host(x1)) and r0.iters == r1.iters and f0.iters == f1.iters == 60
    x2, r2, f2 = G.gmres_fd_solve(A64, A32, t64(b), 60, restart=20, tol=1e-10, max_iters=20000, persistent=True)
    assert r2.converged and f2.iters == 60 and abs(r2.iters - r0.iters) <= 20
