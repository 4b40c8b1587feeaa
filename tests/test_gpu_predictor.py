"""GPU parity of the predictor kernels and an end-to-end check of what the
trained network gains over the fixed GMRES-IR parameters."""
import sys

import numpy as np
import pytest

import oracle.mlp as M
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_2105_07544_amd")
from paper_2105_07544_amd import predictor as PR  # noqa: E402

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch(seed, B):
    r = np.random.default_rng(seed)
    X = (r.standard_normal((B, 16)) * 2 + 0.5)
    y = np.stack([r.integers(0, k, B) for k in M.HEADS], axis=1).astype(np.int32)
    return X, X.mean(0), X.std(0) + 0.1, y


@pytest.mark.parametrize("B", [1, 7, 64, 300])
def test_mlp_forward_and_gradient_match_oracle(B):
    X, mu, sd, y = _batch(B, B)
    th = M.init_params(17) + 0.02 * np.random.default_rng(18).standard_normal(M.NPARAM)
    net = PR.Net(th, mu, sd, DEV)
    L = net.logits(X)
    Lr, _ = M.forward(th.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
                      mu.astype(np.float32), sd.astype(np.float32))
    assert np.allclose(L, Lr, rtol=1e-4, atol=1e-4 * np.abs(Lr).max())
    loss, g = net.loss_grad(X, y)
    lr, gr = M.loss_and_grad(th.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
                             mu.astype(np.float32), sd.astype(np.float32), y)
    assert abs(loss - lr) <= 1e-4 * max(1.0, abs(lr))
    gh = g.cpu().numpy().astype(np.float64)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], M.unpack(gh), M.unpack(gr)):
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 1e-4, (name, rel)


def test_adam_step_matches_oracle():
    X, mu, sd, y = _batch(3, 32)
    th = M.init_params(19)
    net = PR.Net(th, mu, sd, DEV)
    th_o, m_o, v_o = th.astype(np.float32).astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for t in range(1, 6):
        _, g = net.loss_grad(X, y)
        gh = g.cpu().numpy().astype(np.float64)
        net.adam(g, lr=1e-3)
        th_o, m_o, v_o = M.adam_step(th_o, gh, m_o, v_o, t, lr=1e-3)
        assert np.allclose(net.theta.cpu().numpy(), th_o, rtol=1e-5, atol=1e-6)


def _hand3():
    # a_12, a_23 and a_31 have no stored transpose: ||A - A^T||_F^2 counts each twice
    D3 = np.array([[2.0, -1.0, 0.0], [0.0, 3.0, -1.0], [-1.0, 0.0, 4.0]])
    return W.CSR(3, np.array([0, 2, 4, 6], dtype=np.int32), np.array([0, 1, 1, 2, 0, 2], dtype=np.int32),
                 D3[D3 != 0].astype(np.float64))


def test_matrix_stats_match_dense_definitions():
    mats = [W.laplace2d(9), W.laplace3d(5), W.convdiff2d(11, 0.01, lambda x, y: (np.cos(3 * x), np.sin(2 * y))),
            _hand3()]
    for A in mats:
        D = A.to_dense()
        s = PR.matrix_stats(G.DeviceCSR.from_host(A, DEV))
        d = np.diag(D)
        # off-diagonal sums added in ascending column order, as the kernel does,
        # so the ratio >= 1 decision is taken on the same floating-point value
        r = np.zeros(A.n)
        for i in range(A.n):
            for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
                if A.col_idx[k] != i:
                    r[i] += abs(A.val[k])
        ratio = np.abs(d)[r > 0] / r[r > 0]
        ref = [ratio.sum(), ratio.min(), (ratio >= 1).sum(), (r > 0).sum(), (d - r).min(), (d + r).max(),
               r.max(), np.abs(d).max(), d.sum(), (d * d).sum(), (D != 0).sum(1).max(),
               (D * D).sum(), ((D - D.T) ** 2).sum()]
        assert np.allclose(s, ref, rtol=1e-12, atol=1e-12), (s, ref)


def test_matrix_features_match_oracle():
    import oracle.features as F
    # the last two: fewer rows than Arnoldi steps (n = 3, the hand-worked pin) and n = 1
    hand = _hand3()
    one = W.CSR(1, np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32), np.array([3.0]))
    mats = [W.laplace2d(9), W.laplace3d(5), W.convdiff2d(11, 0.01, lambda x, y: (np.cos(3 * x), np.sin(2 * y))),
            W.convdiff2d(40, 1e-3, lambda x, y: (np.cos(np.pi * x), np.sin(np.pi * y))), hand, one]
    for i, A in enumerate(mats):
        v0 = W.uniform_pm1(300 + i, A.n)
        say("features", i, A.n)
        f = PR.features(G.DeviceCSR.from_host(A, DEV), torch.from_numpy(v0).to(DEV))
        ref = F.features(A, v0)
        # the row statistics to rounding; the Ritz features through a float64
        # Arnoldi run on each side and two eigenvalue solvers
        assert np.allclose(f[:11], ref[:11], rtol=1e-12, atol=1e-12), np.c_[f, ref]
        assert np.allclose(f[11:], ref[11:], rtol=1e-7, atol=1e-9), np.c_[f, ref]


def test_trained_network_gains_over_fixed_parameters():
    # the config-5 pipeline at small grid sides: branch-and-bound labels, GPU
    # training, then held-out systems timed live with the predicted and the
    # fixed (m = 50, d = 0, float32) combinations, fallback time included
    train = W.config5_systems(40, seed=50, side2d=(16, 72), side3d=(6, 16))
    test = W.config5_systems(20, seed=51, side2d=(16, 72), side3d=(6, 16))
    say("labelling", len(train), "systems x", len(PR.COMBOS), "combinations")
    recs = [PR.label_system(s, W.uniform_pm1(1000 + i, s["A"].n), DEV, base_cap_s=2.0) for i, s in enumerate(train)]
    for r in recs:
        t = np.array([np.inf if v is None else v for v in r["times"]])
        best = t.min()
        assert np.isfinite(best)
        # a combination is stopped only once it has spent more than the best time
        for k in np.nonzero(r["capped"])[0]:
            assert r["bounds"][k] > best and not np.isfinite(t[k])
    dtr = PR.dataset_from_records(recs)
    mu, sd = dtr.X.mean(0), dtr.X.std(0) + 1e-6
    net = PR.Net(M.init_params(23), mu, sd, DEV)
    hist = net.train(dtr.X, dtr.labels, epochs=300, batch=32, lr=3e-3, order_seed=700)
    say("loss", hist[0], "->", hist[-1])
    assert hist[-1] < hist[0]
    rows = [PR.evaluate_system(net, s, W.uniform_pm1(2000 + i, s["A"].n), DEV, base_cap_s=2.0)
            for i, s in enumerate(test)]
    live = PR.summarize_live(rows)
    say("held out", live)
    # a strict gain on the held-out systems, fallback time included
    assert live["fixed_solves"] >= 15
    assert live["total_pred"] < live["total_fixed"]
    assert live["geomean_ratio"] < 1.0
