"""Learned parameter predictor for GMRES-IR.

Given a matrix, predict the restart length m in {25, 50, 100, 200}, the
GMRES-polynomial degree d in {0, 5, 10, 25, 40} and the inner precision
(float32 GMRES-IR or plain float64 GMRES) that solve A x = b to 1e-10
fastest.  The paper gives rules of thumb for each choice (§V-B, §V-C, §V-E,
§V-F); here a 16-64-64-11 MLP learns them from solver runs.

* features: the library call ``matrix_features`` (11 row statistics from one
  GPU pass over A and 5 Ritz-value features of a 5-step Arnoldi run);
* labels: the fastest (m, d, precision) combination by measured time to
  1e-10, found by branch and bound (a combination is stopped once it has
  spent more than the best time so far, which cannot change the argmin);
* training: the library's forward, backward and Adam kernels;
* solving: the predicted combination, with the fixed combination
  (m = 50, d = 0, float32) as the fallback when the predicted one does not
  converge (its time is charged too).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List

import numpy as np
import torch

from . import DeviceCSR, GMR_F32, GMR_F64, alloc_workspace, gmres_ir_solve, gmres_solve, lib
from . import poly_prec_setup, workspace_bytes
from ._capi import check

RESTARTS = (25, 50, 100, 200)
DEGREES = (0, 5, 10, 25, 40)
PRECISIONS = ("f32", "f64")
COMBOS = [(m, d, p) for m in RESTARTS for d in DEGREES for p in PRECISIONS]
FIXED_COMBO = (50, 0, "f32")
NFEAT = 16
# layer shapes of the network, in the order of the flat parameter vector
LAYERS = [(64, NFEAT), (64,), (64, 64), (64,), (11, 64), (11,)]


def init_params(seed: int) -> np.ndarray:
    """He-uniform initial weights (seeded draws), zero biases."""
    from workloads import he_uniform_params
    return he_uniform_params(seed, LAYERS)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


def matrix_stats(A: DeviceCSR) -> np.ndarray:
    out = np.zeros(13)
    G = min((A.n + 255) // 256, 1024)
    ws = alloc_workspace(8 * 13 * (G + 1), A.device)
    st = A.struct()
    check(lib().matrix_stats(C.byref(st), out.ctypes.data_as(C.c_void_p), _ptr(ws), ws.numel(),
                             _stream(A.device)))
    return out


def features(A: DeviceCSR, v0: torch.Tensor) -> np.ndarray:
    """The 16 features of A (library call matrix_features); v0 (A's dtype) is
    the start vector of the 5-step Arnoldi run."""
    out = np.zeros(NFEAT)
    dt = GMR_F64 if A.val.dtype == torch.float64 else GMR_F32
    ws = alloc_workspace(lib().matrix_features_workspace_bytes(A.n, dt), A.device)
    st = A.struct()
    check(lib().matrix_features(C.byref(st), _ptr(v0), out.ctypes.data_as(C.c_void_p), _ptr(ws), ws.numel(),
                                _stream(A.device)))
    return out


@dataclass
class Dataset:
    X: np.ndarray           # systems x 16 features
    times: np.ndarray       # systems x 40 measured seconds (inf: not converged)
    spent: np.ndarray       # systems x 40 wall seconds of the attempt, converged or not
    labels: np.ndarray      # systems x 3 class indices of the fastest combination


def combo_index(combo) -> int:
    return COMBOS.index(combo)


def labels_from_times(times: np.ndarray) -> np.ndarray:
    best = np.argmin(times, axis=1)
    out = np.zeros((times.shape[0], 3), dtype=np.int32)
    for i, k in enumerate(best):
        m, d, p = COMBOS[k]
        out[i] = (RESTARTS.index(m), DEGREES.index(d), PRECISIONS.index(p))
    return out


def device_system(sysd, device="cuda"):
    A64 = DeviceCSR.from_host(sysd["A"], device)
    return A64, A64.to_f32(), torch.from_numpy(sysd["b"]).to(device)


class Net:
    """Parameters, Adam state and the training / inference calls (GPU kernels)."""

    def __init__(self, theta0: np.ndarray, mu: np.ndarray, sigma: np.ndarray, device="cuda"):
        n = int(lib().mlp_param_count())
        assert theta0.size == n
        self.device = device
        self.theta = torch.from_numpy(theta0.astype(np.float32)).to(device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.mu = torch.from_numpy(mu.astype(np.float32)).to(device)
        self.sigma = torch.from_numpy(sigma.astype(np.float32)).to(device)
        self.step = 0

    def loss_grad(self, X: np.ndarray, labels: np.ndarray):
        B = X.shape[0]
        Xd = torch.from_numpy(X.astype(np.float32)).to(self.device)
        Ld = torch.from_numpy(labels.astype(np.int32)).to(self.device)
        g = torch.empty_like(self.theta)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = alloc_workspace(lib().mlp_workspace_bytes(B), self.device)
        check(lib().mlp_loss_grad(_ptr(self.theta), _ptr(Xd), _ptr(self.mu), _ptr(self.sigma), _ptr(Ld), B,
                                  _ptr(g), _ptr(loss), _ptr(ws), ws.numel(), _stream(self.device)))
        return float(loss.item()), g

    def adam(self, g: torch.Tensor, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        check(lib().mlp_adam_step(_ptr(self.theta), _ptr(g), _ptr(self.m), _ptr(self.v), self.step, lr, b1, b2,
                                  eps, _stream(self.device)))

    def logits(self, X: np.ndarray) -> np.ndarray:
        B = X.shape[0]
        Xd = torch.from_numpy(X.astype(np.float32)).to(self.device)
        out = torch.empty((B, 11), dtype=torch.float32, device=self.device)
        check(lib().mlp_forward(_ptr(self.theta), _ptr(Xd), _ptr(self.mu), _ptr(self.sigma), B, _ptr(out),
                                _stream(self.device)))
        return out.cpu().numpy()

    def predict(self, X: np.ndarray) -> List[tuple]:
        L = self.logits(X)
        out = []
        for row in L:
            out.append((RESTARTS[int(np.argmax(row[0:4]))], DEGREES[int(np.argmax(row[4:9]))],
                        PRECISIONS[int(np.argmax(row[9:11]))]))
        return out

    def train(self, X: np.ndarray, labels: np.ndarray, epochs: int, batch: int, lr: float, order_seed: int):
        """Mini-batch Adam; the sample order of every epoch comes from a seeded permutation."""
        from workloads import uniform01
        n = X.shape[0]
        hist = []
        for e in range(epochs):
            perm = np.argsort(uniform01(order_seed + e, n))
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                loss, g = self.loss_grad(X[idx], labels[idx])
                self.adam(g, lr=lr)
            hist.append(loss)
        return hist


def evaluate(net: Net, ds: Dataset):
    """Time to solution with the predicted combination (plus the fixed
    combination when the predicted one fails, both charged) against the fixed
    combination alone, over the systems the fixed combination solves."""
    pred = net.predict(ds.X)
    kb = combo_index(FIXED_COMBO)
    tb = ds.times[:, kb]
    tp = np.empty(len(pred))
    fallbacks = 0
    for i, c in enumerate(pred):
        k = combo_index(c)
        if np.isfinite(ds.times[i, k]):
            tp[i] = ds.times[i, k]
        else:
            fallbacks += 1
            tp[i] = ds.spent[i, k] + tb[i]
    ok = np.isfinite(tb)
    best = np.min(ds.times, axis=1)
    return dict(total_pred=float(tp[ok].sum()), total_base=float(tb[ok].sum()),
                total_best=float(best[ok].sum()),
                geomean_ratio=float(np.exp(np.mean(np.log(tp[ok] / tb[ok])))),
                fallbacks=fallbacks, systems=int(ok.sum()),
                accuracy=float(np.mean([combo_index(c) == int(np.argmin(ds.times[i])) for i, c in enumerate(pred)])),
                predictions=[list(c) for c in pred])


# ---------------------------------------------------------------------------
# Labelling at scale: branch and bound over the 40 combinations
# ---------------------------------------------------------------------------
def _chunked_solve(A64, A32, b, combo, v0, cap_s: float, max_iters: int):
    """Solve from x0 = 0 with one combination, in calls of 1, 2, 4, ... restart
    cycles, each continuing from the previous call's iterate (a restarted
    solver's cycles depend only on the iterate, so the sequence is the same as
    one uninterrupted solve; each call adds one residual product).  Stops once
    the summed solve time exceeds cap_s.  The polynomial setup is outside the
    timing (§V-C).  Returns (seconds, converged, iterations, capped)."""
    m, d, prec = combo
    if prec == "f32":
        P = poly_prec_setup(A32, d, v0.float()) if d > 0 else None
    else:
        P = poly_prec_setup(A64, d, v0.double()) if d > 0 else None
    x = torch.zeros_like(b)
    ws = alloc_workspace(workspace_bytes(A64.n, m, GMR_F32 if prec == "f32" else GMR_F64, d > 0), b.device)
    spent, iters, chunk = 0.0, 0, 1
    while True:
        left = max_iters - iters
        if prec == "f32":
            _, r = gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=left, max_cycles=chunk,
                                  P=P, ws=ws)
        else:
            _, r = gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=left, max_cycles=chunk, P=P, ws=ws)
        spent += r.seconds
        iters += r.iters
        if r.converged:
            return spent, True, iters, False
        if r.status_name not in ("GMR_NOT_CONVERGED",) or iters >= max_iters:
            return spent, False, iters, False
        if spent > cap_s:
            return spent, False, iters, True
        chunk *= 2


def label_system(sysd, v0: np.ndarray, device="cuda", base_cap_s: float = 4.0, max_iters: int = 100000,
                 order=None, log=None) -> dict:
    """Features and the measured time to 1e-10 of the 40 combinations of one
    system, by branch and bound: the fixed combination first (capped at
    base_cap_s), then the others in the given order, each stopped as soon as
    its time exceeds the best time so far.  A stopped combination cannot be the
    fastest, so the label (the argmin) is exact; its entry in `times` is inf and
    `bounds` holds the time it had spent (a lower bound of its time)."""
    A64, A32, b = device_system(sysd, device)
    v = torch.from_numpy(v0).to(device)
    feats = features(A64, v.double())
    _chunked_solve(A64, A32, b, FIXED_COMBO, v, 0.0, 50)  # warm-up of the kernels at this size
    times = np.full(len(COMBOS), math.inf)
    bounds = np.zeros(len(COMBOS))
    iters = np.zeros(len(COMBOS), dtype=np.int64)
    capped = np.zeros(len(COMBOS), dtype=bool)
    kb = combo_index(FIXED_COMBO)
    t, ok, it, cp = _chunked_solve(A64, A32, b, FIXED_COMBO, v, base_cap_s, max_iters)
    bounds[kb], iters[kb], capped[kb] = t, it, cp
    if ok:
        times[kb] = t
    best = t if ok else base_cap_s
    for c in (order or COMBOS):
        k = combo_index(c)
        if k == kb:
            continue
        t, ok, it, cp = _chunked_solve(A64, A32, b, c, v, best, max_iters)
        bounds[k], iters[k], capped[k] = t, it, cp
        if ok and t < best:
            times[k] = t
            best = t
        elif ok:
            times[k] = t
    out = dict(n=int(sysd["A"].n), nnz=int(sysd["A"].nnz), kind=sysd["kind"], N=int(sysd["N"]),
               features=feats.tolist(), times=[None if not np.isfinite(x) else float(x) for x in times],
               bounds=bounds.tolist(), iters=iters.tolist(), capped=capped.tolist())
    if log:
        kbest = int(np.argmin(times))
        log(f"n={out['n']} {out['kind']} best={COMBOS[kbest]} {times[kbest]:.4f}s "
            f"fixed={times[kb]:.4f}s labelled in {bounds.sum():.1f}s")
    return out


def dataset_from_records(records) -> Dataset:
    """Dataset of labelled systems (label_system records)."""
    X = np.array([r["features"] for r in records], dtype=np.float64)
    T = np.array([[math.inf if t is None else t for t in r["times"]] for r in records])
    S = np.array([r["bounds"] for r in records])
    return Dataset(X, T, S, labels_from_times(T))


def evaluate_system(net: "Net", sysd, v0: np.ndarray, device="cuda", base_cap_s: float = 4.0,
                    max_iters: int = 100000) -> dict:
    """Time to 1e-10 of one unseen system with the predicted combination and
    with the fixed one, each given the same budget base_cap_s; when the
    predicted one does not converge within it, the fixed combination runs
    after it and both times are charged (the fallback)."""
    A64, A32, b = device_system(sysd, device)
    v = torch.from_numpy(v0).to(device)
    f = features(A64, v.double())
    pred = net.predict(f[None, :])[0]
    _chunked_solve(A64, A32, b, FIXED_COMBO, v, 0.0, 50)  # warm-up of the kernels at this size
    tb, okb, itb, _ = _chunked_solve(A64, A32, b, FIXED_COMBO, v, base_cap_s, max_iters)
    if pred == FIXED_COMBO:
        tp, okp, itp, fb = tb, okb, itb, False
    else:
        tp, okp, itp, _ = _chunked_solve(A64, A32, b, pred, v, base_cap_s, max_iters)
        fb = not okp
        if fb:
            tp, okp = tp + tb, okb
    return dict(index=int(sysd.get("index", -1)), n=int(sysd["A"].n), kind=sysd["kind"], N=int(sysd["N"]),
                predicted=list(pred), t_pred=tp, pred_converged=bool(okp), fallback=fb,
                t_fixed=tb, fixed_converged=bool(okb), iters_pred=int(itp), iters_fixed=int(itb))


def summarize_live(rows) -> dict:
    """Totals and the geometric mean of time(predicted, fallback included) /
    time(fixed) over the systems the fixed combination solves within its
    budget; the others are counted apart."""
    ok = [r for r in rows if r["fixed_converged"]]
    tp = np.array([r["t_pred"] for r in ok])
    tb = np.array([r["t_fixed"] for r in ok])
    return dict(systems=len(rows), fixed_solves=len(ok), total_pred=float(tp.sum()), total_fixed=float(tb.sum()),
                gain_total=float(tb.sum() / tp.sum()) if len(ok) else None,
                geomean_ratio=float(np.exp(np.mean(np.log(tp / tb)))) if len(ok) else None,
                fallbacks=int(sum(r["fallback"] for r in rows)),
                fixed_failed_pred_solved=int(sum((not r["fixed_converged"]) and r["pred_converged"] for r in rows)))
