"""Host logic of the parameter predictor's labelling and live evaluation
(branch and bound over the 40 combinations, the fallback rule), run on the
CPU with the GPU solver replaced by a model of its timing: a combination k
needs T[k] seconds and reports its time after 1, 2, 4, ... restart cycles of
c[k] seconds each, as the chunked solver does."""
import math
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")
PR = pytest.importorskip("paper_2105_07544_amd.predictor")


class FakeSolver:
    def __init__(self, T, c):
        self.T, self.c = T, c
        self.calls = []

    def __call__(self, A64, A32, b, combo, v0, cap_s, max_iters):
        self.calls.append((combo, cap_s, max_iters))
        k = PR.combo_index(combo)
        spent, chunk, cycles = 0.0, 1, 0
        while True:
            step = chunk * self.c[k]
            if spent + step >= self.T[k]:
                cycles += math.ceil((self.T[k] - spent) / self.c[k])
                return self.T[k], True, 50 * cycles, False
            spent += step
            cycles += chunk
            if spent > cap_s:
                return spent, False, 50 * cycles, True
            chunk *= 2


def _patch(monkeypatch, solver):
    monkeypatch.setattr(PR, "device_system", lambda sysd, device="cuda": (None, None, torch.zeros(1)))
    monkeypatch.setattr(PR, "features", lambda A, v: np.arange(16, dtype=np.float64))
    monkeypatch.setattr(PR, "_chunked_solve", solver)


def _system():
    return dict(A=types.SimpleNamespace(n=4096, nnz=20224), kind="laplace2d", N=64, index=3)


@pytest.mark.parametrize("seed", range(12))
def test_branch_and_bound_label_is_the_exact_argmin(monkeypatch, seed):
    rng = np.random.default_rng(seed)
    n = len(PR.COMBOS)
    T = 10.0 ** rng.uniform(-3, 0, n)
    if seed % 3 == 0:
        T[rng.integers(0, n, 5)] = math.inf  # combinations that never converge
    c = T / rng.integers(1, 40, n)  # time per restart cycle
    c[~np.isfinite(c)] = 0.05
    solver = FakeSolver(T, c)
    _patch(monkeypatch, solver)
    order = [PR.COMBOS[i] for i in rng.permutation(n)]
    r = PR.label_system(_system(), np.zeros(4096), "cpu", base_cap_s=4.0, order=order)
    times = np.array([math.inf if t is None else t for t in r["times"]])
    kb = PR.combo_index(PR.FIXED_COMBO)
    # the warm-up call, then the fixed combination with the base cap, then every other one once
    assert solver.calls[0][0] == PR.FIXED_COMBO and solver.calls[0][1] == 0.0
    assert solver.calls[1][0] == PR.FIXED_COMBO and solver.calls[1][1] == 4.0
    assert sorted(PR.combo_index(cl[0]) for cl in solver.calls[2:]) == sorted(set(range(n)) - {kb})
    # the label is the true fastest combination, with its true time
    assert int(np.argmin(times)) == int(np.argmin(T))
    assert times.min() == T.min()
    best = times.min()
    for k in range(n):
        if np.isfinite(times[k]):
            assert times[k] == T[k] and not r["capped"][k]
        else:
            # stopped only after spending more than the best time found
            assert r["capped"][k] and r["bounds"][k] > best
    # each combination's cap was the best time found before it ran
    running = T[kb] if np.isfinite(T[kb]) and T[kb] <= 4.0 else 4.0
    for combo, cap, _ in solver.calls[2:]:
        assert cap == running
        k = PR.combo_index(combo)
        if T[k] < running:
            running = T[k]


def test_evaluation_charges_the_fallback(monkeypatch):
    n = len(PR.COMBOS)
    T = np.full(n, 0.5)
    T[PR.combo_index(PR.FIXED_COMBO)] = 0.8
    slow = (25, 40, "f64")
    fast = (25, 40, "f32")
    T[PR.combo_index(slow)] = math.inf
    T[PR.combo_index(fast)] = 0.1
    _patch(monkeypatch, FakeSolver(T, np.full(n, 0.01)))
    rows = []
    for pred in (fast, slow, PR.FIXED_COMBO):
        net = types.SimpleNamespace(predict=lambda f, p=pred: [p])
        rows.append(PR.evaluate_system(net, _system(), np.zeros(4096), "cpu", base_cap_s=2.0))
    assert rows[0]["t_pred"] == 0.1 and not rows[0]["fallback"]
    # the predicted combination ran out of its budget: its time plus the fixed one's
    assert rows[1]["fallback"] and rows[1]["pred_converged"]
    assert rows[1]["t_pred"] > 2.0 + 0.8 - 1e-12
    assert rows[2]["t_pred"] == rows[2]["t_fixed"] == 0.8 and not rows[2]["fallback"]
    s = PR.summarize_live(rows)
    assert s["fixed_solves"] == 3 and s["fallbacks"] == 1
    assert s["total_fixed"] == pytest.approx(2.4)
    assert s["total_pred"] == pytest.approx(0.1 + rows[1]["t_pred"] + 0.8)
    assert s["geomean_ratio"] == pytest.approx(np.exp(np.mean(np.log([0.1 / 0.8, rows[1]["t_pred"] / 0.8, 1.0]))))
