"""GPU parity of the batched block GMRES-IR (16 right-hand sides per system)."""
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def batch_inputs(systems, seed=9):
    A = W.block_diag([s["A"] for s in systems])
    B = W.stack_rows([s["B"] for s in systems])
    Z = W.uniform_pm1(seed, A.n * 16).reshape(A.n, 16)
    A64 = G.DeviceCSR.from_host(A, DEV)
    return A, B, Z, A64, A64.to_f32()


@pytest.mark.parametrize("tile_rows,gb", [(256, 4), (1024, 8), (512, 16), (256, 2), (1024, 3), (512, 5), (512, 6), (1024, 7)])
def test_block_gram_schmidt_step_matches_numpy(tile_rows, gb):
    # uneven systems, row counts that are not multiples of 4 or 16, several tiles each
    rows = [300, 1000, 17, 2049, 64, 777]
    nblk = 3
    b = G.Batch(rows, restart=4)
    b.set_tiling(tile_rows, gb)
    ws = G.alloc_workspace(b.workspace_bytes(), DEV)
    n = sum(rows)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((nblk, n, 16)).astype(np.float32)
    Wm = rng.standard_normal((n, 16)).astype(np.float32)
    Vd = torch.from_numpy(V).to(DEV)
    Wd = torch.from_numpy(Wm.copy()).to(DEV)
    C = host(b.bcgs_step(Vd, nblk, Wd, ws))
    Wout = host(Wd)
    off = 0
    for s, ns in enumerate(rows):
        Vs = V[:, off:off + ns, :].astype(np.float64)          # nblk x ns x 16
        Ws = Wm[off:off + ns].astype(np.float64)
        ref = np.einsum("bri,rc->bic", Vs, Ws)
        scale = np.sqrt(ns) * 16
        assert np.allclose(C[s], ref, rtol=0, atol=2e-5 * scale), (s, np.abs(C[s] - ref).max())
        Cf = C[s].astype(np.float32).astype(np.float64)
        wref = Ws - np.einsum("bri,bic->rc", Vs, Cf)
        assert np.allclose(Wout[off:off + ns], wref, rtol=0, atol=2e-4 * scale), s
        off += ns


def test_small_batch_matches_oracle():
    systems = W.config4_batch(count=5, nrhs=16, side_lo=12, side_hi=30, seed=14)
    A, B, Z, A64, A32 = batch_inputs(systems)
    m = 8
    b = G.Batch([s["A"].n for s in systems], restart=m)
    ws = G.alloc_workspace(b.workspace_bytes(), DEV)
    Bd = torch.from_numpy(B).to(DEV)
    X = torch.zeros_like(Bd)
    Zd = torch.from_numpy(Z.astype(np.float32)).to(DEV)
    out = b.solve(A64, A32, Bd, X, Zd, ws, tol=1e-10, max_cycles=200)
    say(out["status_name"], out["cycles"], out["max_rel_res"], list(out["sys_cycles"]))
    assert out["status"] == 0 and out["max_rel_res"] <= 1e-10
    Xh = host(X)
    off = 0
    for s, sy in enumerate(systems):
        ns = sy["A"].n
        Xs = Xh[off:off + ns]
        res = np.linalg.norm(sy["B"] - O.spmm(sy["A"], Xs, np.float64), axis=0) / np.linalg.norm(sy["B"], axis=0)
        assert np.all(res <= 1e-10), (s, res.max())
        ref = O.block_gmres_ir(sy["A"], sy["B"], m, 1e-10, 200, Z=Z[off:off + ns])
        say("system", s, "cycles gpu", out["sys_cycles"][s], "oracle", ref.cycles)
        assert ref.converged
        assert abs(int(out["sys_cycles"][s]) - ref.cycles) <= max(2, 0.3 * ref.cycles)
        off += ns


def test_float64_batched_solve_matches_oracle():
    systems = W.config4_batch(count=4, nrhs=16, side_lo=12, side_hi=28, seed=16)
    A, B, Z, A64, A32 = batch_inputs(systems)
    m = 8
    b = G.Batch([s["A"].n for s in systems], restart=m)
    assert b.workspace_bytes(G.GMR_F64) > b.workspace_bytes(G.GMR_F32) > 0
    ws = G.alloc_workspace(b.workspace_bytes(G.GMR_F64), DEV)
    Bd = torch.from_numpy(B).to(DEV)
    X = torch.zeros_like(Bd)
    Zd = torch.from_numpy(Z.astype(np.float32)).to(DEV)
    out = b.solve(A64, None, Bd, X, Zd, ws, tol=1e-12, max_cycles=200)
    say(out["status_name"], out["cycles"], out["max_rel_res"], list(out["sys_cycles"]))
    assert out["status"] == 0 and out["max_rel_res"] <= 1e-12
    Xh = host(X)
    off = 0
    for s, sy in enumerate(systems):
        ns = sy["A"].n
        res = np.linalg.norm(sy["B"] - O.spmm(sy["A"], Xh[off:off + ns], np.float64), axis=0) / \
            np.linalg.norm(sy["B"], axis=0)
        assert np.all(res <= 1e-12), (s, res.max())
        ref = O.block_gmres_ir(sy["A"], sy["B"], m, 1e-12, 200, Z=Z[off:off + ns].astype(np.float32),
                               inner=np.float64)
        say("system", s, "cycles gpu", out["sys_cycles"][s], "oracle", ref.cycles)
        assert ref.converged
        assert abs(int(out["sys_cycles"][s]) - ref.cycles) <= max(1, 0.1 * ref.cycles)
        off += ns


def test_float64_workspace_too_small_is_an_error():
    systems = W.config4_batch(count=2, nrhs=16, side_lo=12, side_hi=16, seed=17)
    A, B, Z, A64, A32 = batch_inputs(systems)
    b = G.Batch([s["A"].n for s in systems], restart=4)
    ws = G.alloc_workspace(b.workspace_bytes(G.GMR_F32), DEV)  # the float32 size
    Bd = torch.from_numpy(B).to(DEV)
    with pytest.raises(G.GmresError):
        b.solve(A64, None, Bd, torch.zeros_like(Bd), torch.from_numpy(Z.astype(np.float32)).to(DEV), ws)


@pytest.mark.parametrize("inner", ["f32", "f64"])
def test_graph_replay_matches_eager(inner):
    systems = W.config4_batch(count=5, nrhs=16, side_lo=12, side_hi=40, seed=18)
    A, B, Z, A64, A32 = batch_inputs(systems)
    b = G.Batch([s["A"].n for s in systems], restart=6)
    code = G.GMR_F32 if inner == "f32" else G.GMR_F64
    ws = G.alloc_workspace(b.workspace_bytes(code), DEV)
    Bd = torch.from_numpy(B).to(DEV)
    Zd = torch.from_numpy(Z.astype(np.float32)).to(DEV)
    Ain = A32 if inner == "f32" else None
    X0 = torch.zeros_like(Bd)
    ref = b.solve(A64, Ain, Bd, X0, Zd, ws, tol=1e-10, max_cycles=300)
    assert ref["status"] == 0
    Xref = host(X0)
    # eager launches are repeatable bit for bit
    X2 = torch.zeros_like(Bd)
    b.solve(A64, Ain, Bd, X2, Zd, ws, tol=1e-10, max_cycles=300)
    assert np.array_equal(host(X2), Xref)
    # the captured cycle builds the tile table of the active systems on the
    # device, as the eager cycle does: every replay gives the eager bits
    b.set_graph(True)
    for rep in range(3):  # replays of a freshly captured graph, with eager work in between
        torch.cuda.synchronize()
        _ = (Bd * 2.0).sum().item()
        X1 = torch.zeros_like(Bd)
        out = b.solve(A64, Ain, Bd, X1, Zd, ws, tol=1e-10, max_cycles=300)
        say("graph", inner, rep, out["status_name"], out["cycles"], out["block_iters"])
        assert out["status"] == 0 and out["max_rel_res"] <= 1e-10
        assert out["cycles"] == ref["cycles"] and out["block_iters"] == ref["block_iters"]
        assert np.array_equal(host(X1), Xref)
        assert np.array_equal(out["sys_cycles"], ref["sys_cycles"])
    b.set_graph(False)


@pytest.mark.parametrize("graph", [False, True])
def test_failed_system_is_frozen_and_the_others_converge(graph):
    # system 2's right-hand sides are 16 copies of one vector, so 15 start
    # columns depend on the first and are replaced from Z, whose rows for that
    # system are zero: its start block cannot be orthonormalised.  The solve
    # freezes it at x0 and finishes the other systems.
    systems = W.config4_batch(count=5, nrhs=16, side_lo=12, side_hi=30, seed=19)
    bad = 2
    systems[bad]["B"] = np.repeat(systems[bad]["B"][:, :1], 16, axis=1)
    A, B, Z, A64, A32 = batch_inputs(systems)
    offs = np.concatenate([[0], np.cumsum([s["A"].n for s in systems])])
    Z[offs[bad]:offs[bad + 1]] = 0.0
    m = 8
    b = G.Batch([s["A"].n for s in systems], restart=m)
    b.set_graph(graph)
    ws = G.alloc_workspace(b.workspace_bytes(), DEV)
    Bd = torch.from_numpy(B).to(DEV)
    X = torch.zeros_like(Bd)
    out = b.solve(A64, A32, Bd, X, torch.from_numpy(Z.astype(np.float32)).to(DEV), ws, tol=1e-10, max_cycles=200)
    say("graph", graph, out["status_name"], list(out["sys_status"]), list(out["sys_cycles"]), out["max_rel_res"])
    assert out["status_name"] == "GMR_SYSTEMS_FAILED"
    assert list(out["sys_status"]) == [0, 0, -4, 0, 0]
    assert out["max_rel_res"] <= 1e-10
    Xh = host(X)
    assert np.all(Xh[offs[bad]:offs[bad + 1]] == 0.0)
    for s, sy in enumerate(systems):
        if s == bad:
            continue
        Xs = Xh[offs[s]:offs[s + 1]]
        res = np.linalg.norm(sy["B"] - O.spmm(sy["A"], Xs, np.float64), axis=0) / np.linalg.norm(sy["B"], axis=0)
        assert np.all(res <= 1e-10), (s, res.max())
        ref = O.block_gmres_ir(sy["A"], sy["B"], m, 1e-10, 200, Z=Z[offs[s]:offs[s + 1]])
        say("system", s, "cycles gpu", out["sys_cycles"][s], "oracle", ref.cycles)
        assert ref.converged
        assert abs(int(out["sys_cycles"][s]) - ref.cycles) <= max(2, 0.3 * ref.cycles)
    b.set_graph(False)


def test_autotune_picks_a_candidate_and_solves():
    systems = W.config4_batch(count=6, nrhs=16, side_lo=20, side_hi=60, seed=15)
    A, B, Z, A64, A32 = batch_inputs(systems)
    b = G.Batch([s["A"].n for s in systems], restart=6)
    ws = G.alloc_workspace(b.workspace_bytes(), DEV)
    t, g, ms = b.autotune(ws)
    say("autotune", t, g, ms)
    assert t in (512, 1024, 2048, 4096) and g in (4, 8, 16, 2, 3, 5, 6, 7) and ms > 0
    assert b.tiling() == (t, g)
    Bd = torch.from_numpy(B).to(DEV)
    X = torch.zeros_like(Bd)
    out = b.solve(A64, A32, Bd, X, torch.from_numpy(Z.astype(np.float32)).to(DEV), ws, tol=1e-10, max_cycles=300)
    assert out["status"] == 0 and out["max_rel_res"] <= 1e-10


def test_config4_full_batch_reaches_1e10():
    say("config4 full: generating")
    systems = W.config4_batch()
    A, B, Z, A64, A32 = batch_inputs(systems)
    m = 50
    b = G.Batch([s["A"].n for s in systems], restart=m)
    ws = G.alloc_workspace(b.workspace_bytes(), DEV)
    Bd = torch.from_numpy(B).to(DEV)
    X = torch.zeros_like(Bd)
    say("config4 full: solving")
    out = b.solve(A64, A32, Bd, X, torch.from_numpy(Z.astype(np.float32)).to(DEV), ws, tol=1e-10,
                  max_cycles=100)
    say(out["status_name"], out["cycles"], out["block_iters"], out["max_rel_res"], out["seconds"])
    assert out["status"] == 0 and out["max_rel_res"] <= 1e-10
    Xh = host(X)
    offs = np.concatenate([[0], np.cumsum([s["A"].n for s in systems])])
    sizes = np.array([s["A"].n for s in systems])
    sample = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes))] + list(range(0, 256, 37))))
    for s in sample:
        sy = systems[s]
        Xs = Xh[offs[s]:offs[s + 1]]
        res = np.linalg.norm(sy["B"] - O.spmm(sy["A"], Xs, np.float64), axis=0) / np.linalg.norm(sy["B"], axis=0)
        assert np.all(res <= 1e-10), (s, res.max())
