"""cgs2_orth_noalloc (the entry point whose scratch is the library's static
device array) against cgs2_orth with a caller workspace and against the
oracle's CGS2 step (§III-A: two classical Gram-Schmidt passes), on two calls
in a row, the second one smaller, in both precisions."""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_2105_07544_amd")

DEV = "cuda"


def _case(n, k, prec, seed):
    dt = np.float64 if prec == "f64" else np.float32
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    V = V.astype(dt)
    w = rng.standard_normal(n).astype(dt)
    ldv = n + 64 + (1 if n % 2 == 0 else 0)
    tdt = torch.float64 if prec == "f64" else torch.float32
    Vd = torch.zeros((k, ldv), dtype=tdt, device=DEV)
    Vd[:, :n] = torch.from_numpy(np.ascontiguousarray(V.T)).to(DEV)
    return V, w, Vd, ldv


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_workspace_entry_point(prec):
    dt = np.float64 if prec == "f64" else np.float32
    tol = 1e-12 if prec == "f64" else 2e-5
    for n, k, seed in ((40013, 61, 7), (3001, 9, 8)):   # the second call is smaller
        print("noalloc", prec, n, k, flush=True)
        sys.stdout.flush()
        V, w, Vd, ldv = _case(n, k, prec, seed)
        w_ws = torch.from_numpy(w.copy()).to(DEV)
        h_ws = G.cgs2_orth(Vd, k, w_ws, ldv=ldv)
        w_na = torch.from_numpy(w.copy()).to(DEV)
        h_na = torch.full((k + 1,), float("nan"), dtype=torch.float64, device=DEV)
        G.cgs2_orth_noalloc(Vd, k, w_na, h_na, ldv=ldv)
        torch.cuda.synchronize()
        # same kernels, same reduction order: the same bits
        assert torch.equal(h_na, h_ws)
        assert torch.equal(w_na, w_ws)
        # and the oracle's CGS2 step within the parity tolerance
        w_ref, h1, h2, beta = O.cgs2(V, k, w.copy())
        h = h_na.cpu().numpy()
        scale = np.linalg.norm(w.astype(np.float64))
        assert np.allclose(h[:k], h1.astype(np.float64) + h2.astype(np.float64), rtol=0, atol=tol * scale)
        assert abs(h[k] - float(beta)) <= tol * scale
        assert np.allclose(w_na.cpu().numpy(), (w_ref / beta).astype(dt), atol=tol * 10)
