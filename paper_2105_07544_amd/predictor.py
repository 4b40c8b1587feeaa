"""Learned parameter predictor for GMRES-IR.

Given a matrix, predict the restart length m in {25, 50, 100, 200}, the
GMRES-polynomial degree d in {0, 5, 10, 25, 40} and the inner precision
(float32 GMRES-IR or plain float64 GMRES) that solve A x = b to 1e-10
fastest.  The paper gives rules of thumb for each choice (§V-B, §V-C, §V-E,
§V-F); here a 16-64-64-11 MLP learns them from solver runs.

* features: 11 row statistics from one GPU pass over A (``matrix_stats``) and
  5 Ritz-value features from a 5-step Arnoldi run on the GPU;
* labels: the measured time-to-solution of every (m, d, precision)
  combination, the fastest one being the label;
* training: the library's forward, backward and Adam kernels;
* solving: the predicted combination, with the fixed combination
  (m = 50, d = 0, float32) as the fallback when the predicted one does not
  converge (its time is charged too).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import DeviceCSR, GMR_F32, GMR_F64, alloc_workspace, gmres_ir_solve, gmres_solve, lib
from . import hessenberg_eigvals, poly_prec_setup, workspace_bytes
from ._capi import check

RESTARTS = (25, 50, 100, 200)
DEGREES = (0, 5, 10, 25, 40)
PRECISIONS = ("f32", "f64")
COMBOS = [(m, d, p) for m in RESTARTS for d in DEGREES for p in PRECISIONS]
BASELINE = (50, 0, "f32")
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
    """16 features of A; v0 is the start vector of the 5-step Arnoldi run."""
    s = matrix_stats(A)
    n, nnz = A.n, A.nnz
    maxd = max(s[7], 1e-300)
    rows_off = max(s[3], 1.0)
    mean_d = s[8] / n
    var_d = max(s[9] / n - mean_d * mean_d, 0.0)
    P = poly_prec_setup(A, 4, v0)
    H = P.hessenberg()
    k = H.shape[1]
    theta = hessenberg_eigvals(H[:k, :k])
    amax = float(np.max(np.abs(theta)))
    amin = float(np.min(np.abs(theta)))
    f = [
        math.log10(n),
        nnz / n,
        s[10],
        s[1] if s[3] > 0 else 10.0,
        s[0] / rows_off,
        s[2] / n,
        s[4] / maxd,
        s[5] / maxd,
        s[6] / maxd,
        math.sqrt(s[12] / max(s[11], 1e-300)),
        math.sqrt(var_d) / max(abs(mean_d), 1e-300),
        amax / maxd,
        amin / maxd,
        math.log10(amax / max(amin, 1e-300)),
        float(np.max(np.abs(theta.imag))) / amax,
        float(H[k, k - 1]) / amax if H.shape[0] > k else 0.0,
    ]
    return np.nan_to_num(np.array(f, dtype=np.float64), nan=0.0, posinf=1e6, neginf=-1e6)


def solve_combo(A64: DeviceCSR, A32: DeviceCSR, b: torch.Tensor, combo, v0: torch.Tensor,
                max_iters: int = 20000):
    """Time one (m, d, precision) solve from x0 = 0; the polynomial setup is
    outside the timed solve (as in §V-C).  Returns (seconds or inf, result)."""
    m, d, prec = combo
    if prec == "f32":
        P = poly_prec_setup(A32, d, v0.float()) if d > 0 else None
        x, r = gmres_ir_solve(A64, A32, b, restart=m, tol=1e-10, max_iters=max_iters,
                              stagnation_cycles=20, P=P)
    else:
        P = poly_prec_setup(A64, d, v0.double()) if d > 0 else None
        x, r = gmres_solve(A64, b, restart=m, tol=1e-10, max_iters=max_iters, P=P)
    return (r.seconds if r.converged else math.inf), r


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


def build_dataset(systems, start_vectors, device="cuda", max_iters: int = 6000, log=None) -> Dataset:
    """Features and the measured time of all 40 combinations for each system
    (an attempt that does not converge within max_iters, or stagnates, is
    recorded as inf, with the time it spent)."""
    X = np.zeros((len(systems), NFEAT))
    T = np.full((len(systems), len(COMBOS)), math.inf)
    S = np.zeros((len(systems), len(COMBOS)))
    for i, s in enumerate(systems):
        A64, A32, b = device_system(s, device)
        v0 = torch.from_numpy(start_vectors[i]).to(device)
        X[i] = features(A64, v0.double())
        solve_combo(A64, A32, b, BASELINE, v0, max_iters=200)  # warm-up
        for c in COMBOS:
            t, r = solve_combo(A64, A32, b, c, v0, max_iters=max_iters)
            T[i, combo_index(c)] = t
            S[i, combo_index(c)] = r.seconds
        if log:
            log(f"system {i}: n={s['A'].n} best={COMBOS[int(np.argmin(T[i]))]} "
                f"t={np.min(T[i]):.4f}s baseline={T[i, combo_index(BASELINE)]:.4f}s")
    return Dataset(X, T, S, labels_from_times(T))


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
    kb = combo_index(BASELINE)
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
