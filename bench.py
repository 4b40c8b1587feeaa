#!/usr/bin/env python3
"""Benchmark: time to a 1e-10 relative residual, GMRES-IR vs float64 GMRES, one MI355X.

Default workload (``--workload laplace3d``): 3D 7-point Laplacian on a 150^3 grid
(n = 3,375,000, nnz = 23,490,000, the size of the paper's Laplace3D150),
b = A x_true with x_true ~ U(-1,1) (seed 2), x0 = 0, restart m = 50, tol 1e-10.
One step = one complete GMRES-IR solve (float32 inner GMRES(50) with CGS2,
float64 residual and update) with the inputs already resident in HBM.  The
float32 copy of A is made before the timed region (the paper excludes it too).

Other workloads (each prints its own line; the default line is the one above):
  convdiff   upwind convection-diffusion on 2500^2, GMRES(100)-IR with a float32
             degree-25 GMRES polynomial vs float64 GMRES(100) with a float64 one
  laplace2d  2D Laplacian 64^2, GMRES(50)
  batch      256 convection-diffusion systems x 16 right-hand sides, batched
             block GMRES(50)-IR on the matrix cores
  predictor  the learned parameter predictor: train on the GPU on the labelled
             config-5 systems, then time held-out systems live with the
             predicted (m, degree, precision) and with the fixed (50, 0, f32)
  predictor-label  label config-5 training systems by branch and bound
  fd         GMRES-FD switch-point sweep on the 3D Laplacian 200^3 (b = ones):
             float32 GMRES(50) for s iterations, then float64 GMRES(50)
  prec32     polynomial degrees 10..70 on the same Laplacian: float64 GMRES with
             a float64 or a float32 polynomial (loss of accuracy), and GMRES-IR
  bjac       block Jacobi (block 1 and 42) on the 2500^2 convection-diffusion
             matrix: GMRES-IR with float32 blocks vs float64 GMRES
  restart    restart lengths 25..400 on the 3D Laplacian 150^3 (b = ones)

Extra fields of the default line: the float64 GMRES time on the same GPU and
the ratio, the per-restart residual table (GMRES-IR's explicit residual beside
float64 GMRES's at the same restart), the float32-only GMRES residual,
per-kernel-family time and GB/s (the analogue of the paper's Table I), the
roofline of the dominant kernel from separately bracketed solves, the oracle's
time on one host core (extrapolated, with a check of the fit), and `configs`:
the same IR-vs-float64 record for the 2D Laplacian 64^2, the 2500^2
convection-diffusion problem with the degree-25 polynomials, and the batch of
256 systems x 16 right-hand sides (--no-configs leaves them out).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-1e-10 residual (GMRES-IR vs FP64 GMRES, same GPU); SpMV/CGS2 HBM GB/s")
HBM_PEAK_GBS = 8000.0
FAMILIES = ["spmv", "cgs_dots", "cgs_update_dots", "cgs_update_norm", "poly_step", "residual"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_csr(A):
    """scipy view of a CSR matrix, for the float64 residual checks on the host."""
    import scipy.sparse as sp
    return sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.n, A.n))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2105_07544_amd", "csrc", f) for f in ("kernels.hpp", "device_common.hpp")]


def kernel_source_hash() -> str:
    """sha256 of the single-system kernel sources: a stored counter figure is
    used only while these are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the hardware-counter
    summary, or None when there is none or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            entry = json.load(fh)[workload][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if entry.get("source_sha256") != kernel_source_hash():
        return None
    return entry["bytes_per_launch"]


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, kernel: str, patterns, calib_mib: int):
    """Turns two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) into bytes per launch of the kernel family: each counter is scaled
    by what it reads for the element-wise negation of calib_mib MiB (which
    reads and writes exactly that much).  Writes the entry to the traffic file
    and prints a markdown table."""
    import csv
    from collections import defaultdict

    def load(path):
        d = defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return d
    f, w = load(fetch_csv), load(write_csv)
    calib = [n for n in f if "neg_kernel" in n]
    if not calib:
        raise SystemExit("no calibration kernel in the counter runs (run bench.py with --copy-calibration)")
    known_kib = calib_mib * 1024.0
    ff = known_kib / (sum(f[calib[0]]) / len(f[calib[0]]))
    fw = known_kib / (sum(w[calib[0]]) / len(w[calib[0]]))
    rows, tot, cnt = [], 0.0, 0
    for name in sorted(n for n in f if any(p in n for p in patterns)):
        vf, vw = f[name], w.get(name, [])
        if len(vf) != len(vw):
            raise SystemExit(f"dispatch counts differ between the two runs for {name}")
        b = [1024.0 * (a * ff + c * fw) for a, c in zip(vf, vw)]
        tot += sum(b)
        cnt += len(b)
        rows.append((name.split("(")[0].replace("void ", ""), len(b), sum(vf) / len(vf), sum(vw) / len(vw),
                     sum(b) / len(b)))
    per_launch = tot / cnt
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    data.setdefault(workload, {})[kernel] = {
        "bytes_per_launch": per_launch, "launches": cnt, "fetch_scale": ff, "write_scale": fw,
        "source_sha256": kernel_source_hash()}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(f"scale factors (negation of {calib_mib} MiB): FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {fw:.4f}\n")
    print("| kernel | launches | FETCH_SIZE KiB/launch | WRITE_SIZE KiB/launch | HBM bytes/launch (scaled) |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| `{r[0]}` | {r[1]} | {r[2]:.1f} | {r[3]:.1f} | {r[4]:.4g} |")
    print(f"\nall {kernel} launches ({', '.join(patterns)}): {cnt}, mean HBM bytes per launch {per_launch:.6g}")
    # the SpMV in both precisions (the cache model of §V-D): reads and writes apart
    sp = [(p, [n for n in f if p in n]) for p in ("spmv_kernel<float", "spmv_kernel<double")]
    if all(names for _, names in sp):
        print("\n| SpMV | launches | HBM bytes read/launch | HBM bytes written/launch |")
        print("|---|---|---|---|")
        reads = {}
        for p, names in sp:
            vf = [v for n in names for v in f[n]]
            vw = [v for n in names for v in w.get(n, [])]
            reads[p] = 1024.0 * ff * sum(vf) / len(vf)
            print(f"| `{p}>` | {len(vf)} | {reads[p]:.4g} | {1024.0 * fw * sum(vw) / max(1, len(vw)):.4g} |")
        print(f"\nread ratio float64 / float32: {reads['spmv_kernel<double'] / reads['spmv_kernel<float']:.3f}")


def cpu_baseline(problem, cycles_full: int, m: int, prec32=None, ks=(1, 4, 10)):
    """The oracle on one host core (BLAS held to one thread; the oracle's SpMV
    is a single-threaded numpy loop): prefix runs of a few inner iterations of
    the same solve fix a per-iteration cost a + b*j (j = basis size) and the
    per-run overhead, and the full solve is extrapolated to the GPU's cycle
    count.  The same fit is then checked once against a complete oracle solve
    of the 3D Laplacian at N = 60 (fit from prefixes, measured to 1e-10)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    import workloads as W

    def fit(prob, cycles, mm, pre, kk):
        A, b = prob.A, prob.b
        t0 = time.perf_counter()
        O.spmv(A, b, np.float64)
        t_res = time.perf_counter() - t0
        ts = []
        for k in kk:
            t0 = time.perf_counter()
            O.gmres_ir(A, b, np.zeros(A.n), mm, 1e-10, k, prec32=pre)
            ts.append(time.perf_counter() - t0)
            log(f"cpu_baseline: oracle GMRES-IR (n={A.n}) prefix of {k} iterations: {ts[-1]:.2f} s")
        # T(k) = c0 + a k + b k(k+1)/2
        M = np.array([[1.0, k, k * (k + 1) / 2.0] for k in kk])
        c0, a, bb = np.linalg.solve(M, np.array(ts))
        t_cycle = (c0 + a * mm + bb * mm * (mm + 1) / 2.0) - t_res
        return t_res + cycles * t_cycle, sum(ts)

    with threadpool_limits(limits=1):
        est, spent = fit(problem, cycles_full, m, prec32, ks)
        small = W.config2_laplace3d(N=60, restart=50)
        t0 = time.perf_counter()
        ref = O.gmres_ir(small.A, small.b, np.zeros(small.A.n), 50, 1e-10, 100000)
        t_full = time.perf_counter() - t0
        pred, spent_small = fit(small, ref.cycles, 50, None, (3, 10, 24))
    log(f"cpu_baseline: fit check at N=60: predicted {pred:.2f} s, measured {t_full:.2f} s")
    return {"value": float(est), "unit": "s", "cores": 1, "kind": "oracle", "extrapolated": True,
            "sample": (f"oracle GMRES-IR on the same workload on one core, prefixes of {list(ks)} inner "
                       f"iterations ({spent:.1f} s of CPU work); cost a+b*j per iteration and the "
                       f"per-run overhead fitted, extrapolated to {cycles_full} cycles of m={m}"),
            "sample_seconds": float(spent),
            "host_cores": os.cpu_count(),
            "fit_check": {"workload": "3D Laplacian 60^3, GMRES(50)-IR to 1e-10, oracle on one core",
                          "cycles": int(ref.cycles), "predicted_s": round(pred, 3),
                          "measured_s": round(t_full, 3), "rel_error": round(pred / t_full - 1.0, 4),
                          "sample_seconds": round(spent_small + t_full, 2)}}


def residual_table(ir, f64, m: int):
    """Per restart k: GMRES-IR's explicit ||b - A x_k|| / ||b|| beside float64
    GMRES(m)'s explicit residual at the end of its k-th cycle (iteration k*m,
    or its mid-cycle stop in the last cycle); both histories start at x0."""
    rows = []
    for k in range(max(len(ir.history), len(f64.history))):
        rows.append({"k": k, "iter": min(k * m, ir.iters) if k < len(ir.history) else None,
                     "ir": ir.history[k] if k < len(ir.history) else None,
                     "fp64": f64.history[k] if k < len(f64.history) else None})
    return rows


def single_system(args, kind, steps=None, warmup=None, breakdown=True, extras=True, cpu=True):
    """One single-system config: GMRES-IR (float32 inner) against float64
    GMRES on the same GPU.  `value` is the mean of `steps` unprofiled IR solves;
    the roofline comes from separate solves whose dominant-kernel launches are
    bracketed by HIP events on the solver's stream."""
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = "cuda:0"
    log(f"bench: building the workload ({kind})")
    if kind == "laplace3d":
        N = args.grid or 150
        prob = W.config2_laplace3d(N=N, restart=args.restart or 50)
        desc = (f"GMRES({prob.restart})-IR, 3D Laplacian 6/-1 on {N}^3 (n={prob.A.n}, nnz={prob.A.nnz}), "
                f"b=A*x_true, x_true~U(-1,1) seed 2, x0=0, tol 1e-10")
    elif kind == "convdiff":
        N = args.grid or 2500
        prob = W.config3_convdiff(N=N, restart=args.restart or 100, degree=25)
        desc = (f"GMRES({prob.restart})-IR + float32 GMRES polynomial of degree 25 vs float64 "
                f"GMRES({prob.restart}) + float64 polynomial; upwind convection-diffusion eps=1e-3, wind "
                f"(cos pi x, sin pi y) on {N}^2 (n={prob.A.n}, nnz={prob.A.nnz}), b=A*x_true seed 3, "
                f"x0=0, tol 1e-10")
    else:
        N = args.grid or 64
        prob = W.config1_laplace2d(N=N, restart=args.restart or 50)
        desc = (f"GMRES({prob.restart})-IR vs float64 GMRES({prob.restart}), 2D Laplacian 4/-1 on {N}^2 "
                f"(n={prob.A.n}), b=A*1, x0=0, tol 1e-10")
    degree = prob.poly_degree
    dominant = "poly_step" if degree else "cgs_update_dots"
    m = prob.restart
    A64 = G.DeviceCSR.from_host(prob.A, dev)
    A32 = A64.to_f32()
    b = torch.from_numpy(prob.b).to(dev)
    P32 = P64 = None
    if degree:
        v0 = W.poly_start_vector(prob.A.n, prob.poly_seed)
        log("bench: polynomial setup (outside the timed region)")
        P32 = G.poly_prec_setup(A32, degree, torch.from_numpy(v0.astype(np.float32)).to(dev))
        P64 = G.poly_prec_setup(A64, degree, torch.from_numpy(v0).to(dev))
    ws_ir = G.alloc_workspace(G.workspace_bytes(prob.A.n, m, G.GMR_F32, degree > 0), dev)
    ws_64 = G.alloc_workspace(G.workspace_bytes(prob.A.n, m, G.GMR_F64, degree > 0), dev)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    graph = bool(args.graph)
    Ah = host_csr(prob.A)

    def host_err():
        xh = x.cpu().numpy()
        rel = float(np.linalg.norm(prob.b - Ah @ xh) / np.linalg.norm(prob.b))
        fwd = (float(np.linalg.norm(xh - prob.x_true) / np.linalg.norm(prob.x_true))
               if prob.x_true is not None else None)
        return rel, fwd

    # small and mid-size systems run each restart cycle as one launch: one
    # block up to n = 1024, a cooperative multi-block grid up to n = 6144
    pers = (args.persistent == 1) or (args.persistent < 0 and prob.A.n <= 6144)

    def ir(prof="none", g=None):
        x.zero_()
        return G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_ir,
                                P=P32, prof=prof, graph=graph if g is None else g, persistent=pers)[1]

    def f64(prof="none", g=None):
        x.zero_()
        return G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_64, P=P64,
                             prof=prof, graph=graph if g is None else g, persistent=pers)[1]

    log("bench: warmup")
    for _ in range(warmup):
        ir()
    # timed region: `steps` complete GMRES-IR solves, nothing bracketed
    log(f"bench: timing {steps} GMRES-IR solves")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [ir() for _ in range(steps)]
    torch.cuda.synchronize()
    t_ir = (time.perf_counter() - t0) / steps
    last = res[-1]
    assert all(r.converged for r in res), [r.status_name for r in res]
    rel, fwd = host_err()
    log(f"bench: IR {t_ir:.4f} s/solve, {last.iters} iters, {last.cycles} cycles")

    log("bench: float64 GMRES")
    f64()
    nf = max(1, min(steps, 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r64 = [f64() for _ in range(nf)]
    torch.cuda.synchronize()
    t_64 = (time.perf_counter() - t0) / nf
    assert all(r.converged for r in r64), [r.status_name for r in r64]
    rel64, fwd64 = host_err()

    # the roofline of the dominant kernel: separate solves, every launch of it
    # bracketed by events (graph replay and the single-block cycle have none)
    npro = max(1, min(steps, 5))
    pres = [ir(prof=dominant, g=False) for _ in range(npro)]
    prof_ms = sum(r.prof_ms for r in pres)
    prof_bytes = sum(r.prof_bytes for r in pres)
    prof_launches = sum(r.prof_launches for r in pres)
    achieved = prof_bytes / (prof_ms * 1e-3) / 1e9 if prof_ms > 0 else 0.0

    half = None
    if extras and not degree and prob.A.n > 1024:
        # the third precision (float16 basis), reported beside the paper's method
        log("bench: GMRES-IR with the float16 basis")
        x.zero_()
        G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_ir, half_basis=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rh = [G.gmres_ir_solve(A64, A32, b, x.zero_(), restart=m, tol=1e-10, max_iters=200000, ws=ws_ir,
                               half_basis=True)[1] for _ in range(nf)]
        t_h = (time.perf_counter() - t0) / nf
        rel16, _ = host_err()
        half = {"seconds": round(t_h, 5), "iters": rh[-1].iters, "cycles": rh[-1].cycles, "rel_res": rel16,
                "speedup_vs_fp64": round(t_64 / t_h, 3), "speedup_vs_f32_basis": round(t_ir / t_h, 3)}
        assert all(r.converged for r in rh) and rel16 <= 1e-10, half
        if breakdown and not args.no_breakdown:
            for fam in ("spmv", "cgs_dots", "cgs_update_dots", "cgs_update_norm"):
                x.zero_()
                rp = G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_ir,
                                      half_basis=True, prof=fam)[1]
                half[fam + "_gbs"] = round(rp.prof_bytes / (rp.prof_ms * 1e-3) / 1e9, 1) if rp.prof_ms else None
                half[fam + "_ms"] = round(rp.prof_ms, 3)
    if extras and degree and prob.A.n > 1024:
        log("bench: GMRES-IR + float32 polynomial with the float16 basis")
        x.zero_()
        t0 = time.perf_counter()
        _, rh = G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_ir, P=P32,
                                 half_basis=True)
        t_h = time.perf_counter() - t0
        rel16, _ = host_err()
        half = {"seconds": round(t_h, 5), "iters": rh.iters, "cycles": rh.cycles, "rel_res": rel16,
                "speedup_vs_fp64": round(t_64 / t_h, 3), "speedup_vs_f32_basis": round(t_ir / t_h, 3)}
        assert rh.converged and rel16 <= 1e-10, half
    mixed = None
    if extras and degree:
        # the middle option of §V-C: float64 GMRES with the float32 polynomial
        log("bench: float64 GMRES with the float32 polynomial")
        x.zero_()
        t0 = time.perf_counter()
        _, rmx = G.gmres_f32prec_solve(A64, A32, P32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws_64)
        mixed = {"seconds": round(time.perf_counter() - t0, 5), "status": rmx.status_name, "iters": rmx.iters,
                 "loss_of_accuracy": rmx.loss_of_accuracy}
    # float32-only GMRES(m) on the same system: where float32 arithmetic alone
    # stalls (§V-B), which is what the float64 outer loop of IR removes
    f32only = None
    if not degree:
        b32 = b.float()
        x32 = torch.zeros_like(b32)
        _, r32 = G.gmres_solve(A32, b32, x32, restart=m, tol=1e-10, max_iters=40 * m, ws=ws_ir)
        xh = x32.double().cpu().numpy()
        f32only = {"status": r32.status_name, "iters": r32.iters,
                   "rel_res": float(np.linalg.norm(prob.b - Ah @ xh) / np.linalg.norm(prob.b))}
    breakdown_d = {}
    if breakdown and not args.no_breakdown:
        log("bench: per-kernel breakdown")
        for fam in FAMILIES:
            if fam == "poly_step" and not degree:
                continue
            ri, rd = ir(prof=fam, g=False), f64(prof=fam, g=False)
            breakdown_d[fam] = {
                "ir_ms": round(ri.prof_ms, 3), "ir_launches": ri.prof_launches,
                "ir_gbs": round(ri.prof_bytes / (ri.prof_ms * 1e-3) / 1e9, 1) if ri.prof_ms > 0 else None,
                "f64_ms": round(rd.prof_ms, 3), "f64_launches": rd.prof_launches,
                "f64_gbs": round(rd.prof_bytes / (rd.prof_ms * 1e-3) / 1e9, 1) if rd.prof_ms > 0 else None,
            }
    out = {
        "metric": METRIC, "value": round(t_ir, 5), "unit": "s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(t_ir * 1e3, 3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "n": prob.A.n, "nnz": prob.A.nnz, "restart": m, "tol": 1e-10,
                   "poly_degree": degree, "inner": "f32", "outer": "f64"},
        "fp64_gmres_s": round(t_64, 5), "ir_speedup_vs_fp64": round(t_64 / t_ir, 3),
        "ir_iters": last.iters, "ir_cycles": last.cycles,
        "fp64_iters": r64[-1].iters, "fp64_cycles": r64[-1].cycles,
        "rel_res": rel, "forward_error": fwd, "fp64_rel_res": rel64, "fp64_forward_error": fwd64,
        "residual_table": residual_table(last, r64[-1], m),
        **({"fp32_only_gmres": f32only} if f32only else {}),
        "graph": graph, "persistent_cycle": pers,
        **({"fp64_gmres_f32poly": mixed} if mixed else {}),
        **({"ir_half_basis": half} if half else {}),
        "roofline": {"kernel": dominant, "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": stored_traffic(dominant, kind), "launches": prof_launches,
                     "avg_launch_us": round(1e3 * prof_ms / max(1, prof_launches), 2),
                     "bytes_per_launch": round(prof_bytes / max(1, prof_launches)),
                     "solves": npro},
        **({"kernel_breakdown": breakdown_d} if breakdown_d else {}),
    }
    if cpu and not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        prec32, ks = None, (3, 10, 24)
        import oracle as O
        if degree:
            # the oracle builds its own float32 polynomial from the same start vector
            v0 = W.poly_start_vector(prob.A.n, prob.poly_seed).astype(np.float32)
            roots = O.poly_roots(prob.A, degree, v0, np.float32)
            prec32 = lambda v: O.poly_apply(prob.A, roots, v, np.float32)  # noqa: E731
            ks = (1, 2, 3)
        out["cpu_baseline"] = cpu_baseline(prob, last.cycles, m, prec32, ks)
    del A64, A32, ws_ir, ws_64, P32, P64, b, x
    torch.cuda.empty_cache()
    return out


def fd_sweep(args):
    """GMRES-FD switch-point sweep (§V-A): float32 GMRES(m) for s iterations, then
    float64 GMRES(m) from its iterate, for s = 0, stride, 2*stride, ...; beside it
    one GMRES-IR solve and one float64 GMRES(m) solve of the same system."""
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    dev = "cuda:0"
    N = args.grid or 200
    log("bench: building the workload")
    prob = W.fd_laplace3d(N, restart=args.restart or 50)
    m = prob.restart
    desc = (f"GMRES-FD switch-point sweep vs GMRES({m})-IR vs float64 GMRES({m}): 3D Laplacian 6/-1 "
            f"on {N}^3 (n={prob.A.n}, nnz={prob.A.nnz}), b=ones, x0=0, tol 1e-10")
    A64 = G.DeviceCSR.from_host(prob.A, dev)
    A32 = A64.to_f32()
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros_like(b)
    ws = G.alloc_workspace(G.fd_workspace_bytes(prob.A.n, m), dev)
    Ah = host_csr(prob.A)

    def host_rel():
        xh = x.cpu().numpy()
        return float(np.linalg.norm(prob.b - Ah @ xh) / np.linalg.norm(prob.b))

    def ir(prof="none"):
        x.zero_()
        return G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws, prof=prof)[1]

    log("bench: warmup")
    for _ in range(args.warmup):
        ir()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    log(f"bench: timing {steps} GMRES-IR solves")
    t0 = time.perf_counter()
    rir = [ir() for _ in range(steps)]
    t_ir = (time.perf_counter() - t0) / steps
    assert all(r.converged for r in rir), [r.status_name for r in rir]
    rel_ir = host_rel()
    log(f"bench: IR {t_ir:.3f} s, {rir[-1].iters} iters")
    pr = ir(prof="cgs_update_dots")
    achieved = pr.prof_bytes / (pr.prof_ms * 1e-3) / 1e9 if pr.prof_ms > 0 else 0.0
    x.zero_()
    t0 = time.perf_counter()
    _, r64 = G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=200000, ws=ws)
    t_64 = time.perf_counter() - t0
    assert r64.converged, r64.status_name
    log(f"bench: float64 GMRES {t_64:.3f} s, {r64.iters} iters")
    stride = args.fd_stride or 5 * m
    smax = args.fd_max or -(-r64.iters // m) * m
    sweep = []
    for sw in range(0, smax + 1, stride):
        x.zero_()
        t0 = time.perf_counter()
        _, both, first = G.gmres_fd_solve(A64, A32, b, sw, x, restart=m, tol=1e-10, max_iters=200000, ws=ws)
        sec = time.perf_counter() - t0
        row = {"switch": sw, "f32_iters": first.iters, "f64_iters": both.iters - first.iters,
               "total_iters": both.iters, "seconds": round(sec, 4), "converged": both.converged,
               "rel_res": both.rel_res,
               "f64_start_rel_res": both.history[0] if both.history else None}
        sweep.append(row)
        log(f"bench: FD switch {sw}: {row['total_iters']} iters ({row['f32_iters']} f32), {sec:.3f} s, "
            f"f64 start residual {row['f64_start_rel_res']:.3e}")
    assert all(r["converged"] for r in sweep)
    best = min(sweep, key=lambda r: r["seconds"])
    x.zero_()
    G.gmres_fd_solve(A64, A32, b, best["switch"], x, restart=m, tol=1e-10, max_iters=200000, ws=ws)
    rel_fd = host_rel()
    return {
        "metric": METRIC, "value": round(t_ir, 5), "unit": "s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(t_ir * 1e3, 3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": desc, "n": prob.A.n, "nnz": prob.A.nnz, "restart": m, "tol": 1e-10,
                   "fd_stride": stride, "fd_max": smax},
        "ir_iters": rir[-1].iters, "ir_rel_res": rel_ir,
        "fp64_gmres_s": round(t_64, 5), "fp64_iters": r64.iters, "ir_speedup_vs_fp64": round(t_64 / t_ir, 3),
        "fd_best": {**best, "host_rel_res": rel_fd}, "ir_speedup_vs_best_fd": round(best["seconds"] / t_ir, 3),
        "fd_sweep": sweep,
        "roofline": {"kernel": "cgs_update_dots", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "launches": pr.prof_launches,
                     "avg_launch_us": round(1e3 * pr.prof_ms / max(1, pr.prof_launches), 2)},
    }


def prec32_sweep(args):
    """§V-F: float64 GMRES(m) on the 3D Laplacian 200^3 (b = ones) with a GMRES
    polynomial of degree 10..70 built and applied in float64, or built and applied
    in float32 (corrected by restarting from the explicit residual after a loss of
    accuracy, or stopped there), beside GMRES-IR with the float32 polynomial."""
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    dev = "cuda:0"
    N = args.grid or 200
    log("bench: building the workload")
    prob = W.fd_laplace3d(N, restart=args.restart or 50)
    m = prob.restart
    A64 = G.DeviceCSR.from_host(prob.A, dev)
    A32 = A64.to_f32()
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros_like(b)
    ws = G.alloc_workspace(G.workspace_bytes(prob.A.n, m, G.GMR_F64, True), dev)
    v0 = W.poly_start_vector(prob.A.n, 0)
    Ah = host_csr(prob.A)
    degrees = [int(d) for d in args.degrees.split(",")]
    rows = []
    cap = 5000   # iterations; a float32 polynomial that cannot reach 1e-10 also stops after 20 stagnant restarts

    def run(fn):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = fn()
        sec = time.perf_counter() - t0
        xh = x.cpu().numpy()
        rel = float(np.linalg.norm(prob.b - Ah @ xh) / np.linalg.norm(prob.b))
        return {"status": r.status_name, "iters": r.iters, "cycles": r.cycles, "seconds": round(sec, 4),
                "rel_res": rel, "loss_of_accuracy": r.loss_of_accuracy}

    for d in degrees:
        log(f"bench: degree {d}: polynomial setup (outside the timed solves)")
        P64 = G.poly_prec_setup(A64, d, torch.from_numpy(v0).to(dev))
        P32 = G.poly_prec_setup(A32, d, torch.from_numpy(v0.astype(np.float32)).to(dev))
        row = {"degree": d}
        row["f64_f64poly"] = run(lambda: G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=cap, ws=ws, P=P64))
        row["f64_f32poly"] = run(lambda: G.gmres_f32prec_solve(A64, A32, P32, b, x, restart=m, tol=1e-10,
                                                               max_iters=cap, stagnation_cycles=20, ws=ws))
        row["f64_f32poly_stop_on_loss"] = run(lambda: G.gmres_f32prec_solve(A64, A32, P32, b, x, restart=m,
                                                                            tol=1e-10, max_iters=cap, ws=ws,
                                                                            stop_on_loss=True))
        row["ir_f32poly"] = run(lambda: G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=cap,
                                                         stagnation_cycles=20, ws=ws, P=P32))
        rows.append(row)
        log("bench: " + json.dumps(row))
        del P64, P32
    best_ir = min(r["ir_f32poly"]["seconds"] for r in rows if r["ir_f32poly"]["status"] == "GMR_OK")
    best_64 = min(r["f64_f64poly"]["seconds"] for r in rows if r["f64_f64poly"]["status"] == "GMR_OK")
    return {
        "metric": METRIC, "value": round(best_ir, 5), "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(best_ir * 1e3, 3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"polynomial degree sweep {degrees}: float64 GMRES({m}) with a float64 or a "
                                f"float32 GMRES polynomial, GMRES({m})-IR with the float32 one; 3D Laplacian "
                                f"6/-1 on {N}^3 (n={prob.A.n}), b=ones, x0=0, tol 1e-10"),
                   "n": prob.A.n, "nnz": prob.A.nnz, "restart": m, "tol": 1e-10},
        "best_fp64_f64poly_s": round(best_64, 5), "ir_speedup_vs_best_fp64": round(best_64 / best_ir, 3),
        "sweep": rows,
    }


def bjac_leg(args):
    """Block Jacobi (§III-D, "J k" of §V-G) on the 2500^2 convection-diffusion matrix:
    float64 GMRES(m) with float64 blocks, float64 GMRES(m) with float32 blocks, and
    GMRES(m)-IR with float32 blocks, for block sizes 1 and 42."""
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    dev = "cuda:0"
    N = args.grid or 2500
    m = args.restart or 50
    log("bench: building the workload")
    prob = W.config3_convdiff(N=N, restart=m, degree=0)
    A64 = G.DeviceCSR.from_host(prob.A, dev)
    A32 = A64.to_f32()
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros_like(b)
    ws = G.alloc_workspace(G.workspace_bytes(prob.A.n, m, G.GMR_F64, True), dev)
    Ah = host_csr(prob.A)
    cap = 20000

    def run(fn):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = fn()
        sec = time.perf_counter() - t0
        xh = x.cpu().numpy()
        rel = float(np.linalg.norm(prob.b - Ah @ xh) / np.linalg.norm(prob.b))
        return {"status": r.status_name, "iters": r.iters, "cycles": r.cycles, "seconds": round(sec, 4),
                "rel_res": rel, "loss_of_accuracy": r.loss_of_accuracy}

    rows = []
    for k in [int(v) for v in args.blocks.split(",")]:
        log(f"bench: block Jacobi {k}: setup (outside the timed solves)")
        J64 = G.bjac_prec_setup(A64, k)
        J32 = G.bjac_prec_setup(A32, k)
        row = {"block": k}
        row["f64_f64blocks"] = run(lambda: G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=cap, ws=ws, P=J64))
        row["f64_f32blocks"] = run(lambda: G.gmres_f32prec_solve(A64, A32, J32, b, x, restart=m, tol=1e-10,
                                                                 max_iters=cap, ws=ws))
        row["ir_f32blocks"] = run(lambda: G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=cap,
                                                           ws=ws, P=J32))
        x.zero_()
        _, pr = G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=cap, ws=ws, P=J32, prof="bjac")
        row["bjac_apply_f32"] = {"launches": pr.prof_launches,
                                 "avg_launch_us": round(1e3 * pr.prof_ms / max(1, pr.prof_launches), 2),
                                 "gbs": round(pr.prof_bytes / (pr.prof_ms * 1e-3) / 1e9, 1) if pr.prof_ms else None}
        x.zero_()
        _, pr = G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=cap, ws=ws, P=J64, prof="bjac")
        row["bjac_apply_f64"] = {"launches": pr.prof_launches,
                                 "avg_launch_us": round(1e3 * pr.prof_ms / max(1, pr.prof_launches), 2),
                                 "gbs": round(pr.prof_bytes / (pr.prof_ms * 1e-3) / 1e9, 1) if pr.prof_ms else None}
        row["ir_speedup_vs_fp64"] = round(row["f64_f64blocks"]["seconds"] / row["ir_f32blocks"]["seconds"], 3)
        rows.append(row)
        log("bench: " + json.dumps(row))
        del J64, J32
    best = min(rows, key=lambda r: r["ir_f32blocks"]["seconds"])
    return {
        "metric": METRIC, "value": best["ir_f32blocks"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(1e3 * best["ir_f32blocks"]["seconds"], 3), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"block Jacobi sizes {args.blocks}: GMRES({m})-IR with float32 blocks vs float64 "
                                f"GMRES({m}) with float64 or float32 blocks; upwind convection-diffusion eps=1e-3, "
                                f"wind (cos pi x, sin pi y) on {N}^2 (n={prob.A.n}), b=A*x_true seed 3, x0=0, tol 1e-10"),
                   "n": prob.A.n, "nnz": prob.A.nnz, "restart": m, "tol": 1e-10},
        "sweep": rows,
    }


def restart_sweep(args):
    """The restart-length study of §V-E on the 3D Laplacian 150^3 (b = ones):
    float64 GMRES(m) and GMRES(m)-IR for m = 25 .. 400."""
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    dev = "cuda:0"
    N = args.grid or 150
    log("bench: building the workload")
    prob = W.fd_laplace3d(N)
    A64 = G.DeviceCSR.from_host(prob.A, dev)
    A32 = A64.to_f32()
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros_like(b)
    Ah = host_csr(prob.A)
    ms = [int(v) for v in args.restarts.split(",")]
    ws = G.alloc_workspace(G.workspace_bytes(prob.A.n, max(ms), G.GMR_F64), dev)

    def run(fn):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, r = fn()
        sec = time.perf_counter() - t0
        rel = float(np.linalg.norm(prob.b - Ah @ x.cpu().numpy()) / np.linalg.norm(prob.b))
        return {"status": r.status_name, "iters": r.iters, "cycles": r.cycles, "seconds": round(sec, 4),
                "rel_res": rel}

    rows = []
    G.gmres_ir_solve(A64, A32, b, x, restart=50, tol=1e-10, max_iters=20000, ws=ws)  # warm-up
    for m in ms:
        row = {"restart": m,
               "f64": run(lambda: G.gmres_solve(A64, b, x, restart=m, tol=1e-10, max_iters=20000, ws=ws)),
               "ir": run(lambda: G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=20000,
                                                  stagnation_cycles=20, ws=ws)),
               "ir_half_basis": run(lambda: G.gmres_ir_solve(A64, A32, b, x, restart=m, tol=1e-10, max_iters=20000,
                                                             stagnation_cycles=20, ws=ws, half_basis=True))}
        row["ir_speedup_vs_fp64"] = round(row["f64"]["seconds"] / row["ir"]["seconds"], 3)
        rows.append(row)
        log("bench: " + json.dumps(row))
    ok = [r for r in rows if r["ir"]["status"] == "GMR_OK"]
    best = min(ok, key=lambda r: r["ir"]["seconds"])
    return {
        "metric": METRIC, "value": best["ir"]["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1e3 * best["ir"]["seconds"], 3), "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"restart sweep {ms}: float64 GMRES(m) vs GMRES(m)-IR, 3D Laplacian 6/-1 on {N}^3 "
                                f"(n={prob.A.n}), b=ones, x0=0, tol 1e-10"),
                   "n": prob.A.n, "nnz": prob.A.nnz, "tol": 1e-10},
        "best_ir_restart": best["restart"], "sweep": rows,
    }


def batch(args):
    import numpy as np
    import torch

    import paper_2105_07544_amd as G
    import workloads as W

    dev = "cuda:0"
    log("bench: building 256 systems x 16 right-hand sides")
    systems = W.config4_batch()
    A = W.block_diag([s["A"] for s in systems])
    B = W.stack_rows([s["B"] for s in systems])
    Z = W.uniform_pm1(9, A.n * 16).reshape(A.n, 16).astype(np.float32)
    A64 = G.DeviceCSR.from_host(A, dev)
    A32 = A64.to_f32()
    m = args.restart or 50
    bt = G.Batch([s["A"].n for s in systems], restart=m)
    bt.set_graph(args.batch_graph != 0)
    ws = G.alloc_workspace(bt.workspace_bytes(), dev)
    if args.tiling:
        tr, gb = (int(v) for v in args.tiling.split(","))
        bt.set_tiling(tr, gb)
        tiling = (tr, gb, None)
    else:
        tiling = bt.autotune(ws)
    log(f"bench: autotuned tiling {tiling}")
    Bd = torch.from_numpy(B).to(dev)
    Zd = torch.from_numpy(Z).to(dev)
    X = torch.zeros_like(Bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = bt.solve(A64, A32, Bd, X, Zd, ws, tol=1e-10, max_cycles=500)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    assert out["status"] == 0, out["status_name"]
    Xh = X.cpu().numpy()
    del ws
    log(f"bench: batched GMRES-IR {t:.2f} s; float64 batched block GMRES")
    ws64 = G.alloc_workspace(bt.workspace_bytes(G.GMR_F64), dev)
    X64 = torch.zeros_like(Bd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out64 = bt.solve(A64, None, Bd, X64, Zd, ws64, tol=1e-10, max_cycles=500)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    assert out64["status"] == 0, out64["status_name"]
    del ws64
    offs = np.concatenate([[0], np.cumsum([s["A"].n for s in systems])])
    worst = 0.0
    for s in range(0, len(systems), 17):
        sy = systems[s]
        r = np.linalg.norm(sy["B"] - host_csr(sy["A"]) @ Xh[offs[s]:offs[s + 1]], axis=0)
        worst = max(worst, float(np.max(r / np.linalg.norm(sy["B"], axis=0))))
    # roofline of the block Gram-Schmidt pair on the matrix cores (block dots
    # C = V^T W, then W -= V C) at the mean basis size of a cycle, timed with
    # events on the stream it runs on: algorithmic bytes = the nblk basis
    # blocks read twice, W read twice and written once (16 float32 columns per
    # row), plus the float64 coefficients written and read back
    nblk = (m + 1) // 2
    wsr = G.alloc_workspace(bt.workspace_bytes(), dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    Vin = torch.rand(nblk * A.n * 16, generator=gen, device=dev) * 2 - 1
    Wb = torch.rand(A.n * 16, generator=gen, device=dev) * 2 - 1
    bt.bcgs_step(Vin, nblk, Wb, wsr)
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bt.bcgs_step(Vin, nblk, Wb, wsr)
    e1.record()
    torch.cuda.synchronize()
    step_us = e0.elapsed_time(e1) * 1e3 / reps
    step_bytes = 2.0 * nblk * A.n * 64 + 3.0 * A.n * 64 + 2.0 * len(systems) * nblk * 256 * 8
    gbs = step_bytes / (step_us * 1e-6) / 1e9
    del Vin, Wb, wsr
    torch.cuda.empty_cache()
    return {"metric": METRIC, "value": round(t, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": round(t * 1e3, 2), "higher_is_better": False, "scaling": "strong",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"batched block GMRES({m})-IR, 256 upwind convection-diffusion systems "
                                   f"(side U{{32..256}}, eps 10^U(-3,0), random wind angle) x 16 right-hand "
                                   f"sides, rows={A.n}, nnz={A.nnz}, tol 1e-10 per column",
                       "systems": len(systems), "rhs": 16, "rows": A.n, "nnz": A.nnz, "restart": m},
            "rhs_solved_per_s": round(len(systems) * 16 / t, 2), "tiling": list(tiling[:2]),
            "graph": args.batch_graph != 0,
            "cycles_slowest_system": out["cycles"], "block_iters": out["block_iters"],
            "max_rel_res": out["max_rel_res"], "sampled_host_rel_res": worst,
            "fp64_batched_s": round(t64, 4), "ir_speedup_vs_fp64": round(t64 / t, 3),
            "fp64_cycles_slowest_system": out64["cycles"], "fp64_block_iters": out64["block_iters"],
            "fp64_max_rel_res": out64["max_rel_res"],
            "roofline": {"kernel": "block Gram-Schmidt pair (bdots + bgemm)", "bound": "hbm",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "avg_launch_us": round(step_us, 2), "bytes_per_launch": round(step_bytes),
                         "basis_blocks": nblk}}


LABELS_FILE = os.path.join(ROOT, "paper_2105_07544_amd", "predictor_data", "config5_train.jsonl")


def predictor_label(args):
    """Labels training systems start .. start+count-1 of the config-5
    distribution (seed 5) by branch and bound over the 40 combinations and
    appends one JSON record per system to --label-out (default: the committed
    training file)."""
    import numpy as np

    import workloads as W
    from paper_2105_07544_amd import predictor as PR

    out_path = args.label_out or LABELS_FILE
    systems = W.config5_systems(args.label_count, seed=5, start=args.label_start)
    t0 = time.perf_counter()
    recs = []
    wins = {}
    for s in systems:
        # combinations that won on the systems labelled so far go first (a
        # tighter bound sooner); the label does not depend on the order
        order = sorted(PR.COMBOS, key=lambda c: -wins.get(c, 0))
        v0 = W.uniform_pm1(10000 + s["index"], s["A"].n)
        t1 = time.perf_counter()
        r = PR.label_system(s, v0, "cuda:0", base_cap_s=args.base_cap, order=order, log=log)
        r["index"] = s["index"]
        r["label_seconds"] = round(time.perf_counter() - t1, 3)
        best = PR.COMBOS[int(np.argmin([np.inf if t is None else t for t in r["times"]]))]
        wins[best] = wins.get(best, 0) + 1
        recs.append(r)
        with open(out_path, "a") as fh:
            fh.write(json.dumps(r) + "\n")
        log(f"bench: labelled system {s['index']} ({r['label_seconds']} s)")
    return {"metric": "labelled config-5 training systems", "value": len(recs), "unit": "systems",
            "start": args.label_start, "count": args.label_count, "seconds": round(time.perf_counter() - t0, 1),
            "file": os.path.relpath(out_path, ROOT)}


def predictor(args):
    """Trains the network on the GPU on the labelled training systems, then
    times held-out systems start .. start+count-1 (seed 6) live with the
    predicted combination and with the fixed one (m = 50, d = 0, float32)."""
    import numpy as np

    import workloads as W
    from paper_2105_07544_amd import predictor as PR

    with open(args.labels or LABELS_FILE) as fh:
        recs = [json.loads(line) for line in fh if line.strip()]
    recs.sort(key=lambda r: r["index"])
    dtr = PR.dataset_from_records(recs)
    mu, sd = dtr.X.mean(0), dtr.X.std(0) + 1e-6
    net = PR.Net(PR.init_params(23), mu, sd, "cuda:0")
    epochs = 400
    t0 = time.perf_counter()
    hist = net.train(dtr.X, dtr.labels, epochs=epochs, batch=64, lr=3e-3, order_seed=700)
    t_train = time.perf_counter() - t0
    fit = PR.evaluate(net, dtr)
    fit.pop("predictions")
    test = W.config5_systems(args.test, seed=6, start=args.test_start)
    rows = []
    for s in test:
        v0 = W.uniform_pm1(20000 + s["index"], s["A"].n)
        r = PR.evaluate_system(net, s, v0, "cuda:0", base_cap_s=args.base_cap)
        rows.append(r)
        log(f"bench: held-out {s['index']} n={r['n']} {r['kind']} pred={tuple(r['predicted'])} "
            f"{r['t_pred']:.4f}s fixed={r['t_fixed']:.4f}s")
        if args.test_out:
            with open(args.test_out, "a") as fh:
                fh.write(json.dumps(r) + "\n")
    live = PR.summarize_live(rows)
    kinds = {k: sum(r["kind"] == k for r in recs) for k in ("convdiff", "laplace2d", "laplace3d")}
    return {"metric": METRIC, "value": round(live["total_pred"], 5), "unit": "s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(live["total_pred"] * 1e3, 3),
            "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": (f"learned (m, degree, precision) predictor: trained on {len(recs)} labelled "
                                    "systems (half upwind convection-diffusion, a quarter 2D and a quarter 3D "
                                    "Laplacians; 2D side U{64..1024}, 3D side U{16..101}), held-out systems "
                                    f"{args.test_start}..{args.test_start + args.test - 1} timed live"),
                       "train": len(recs), "test": len(rows), "train_kinds": kinds,
                       "grid_side_2d": [64, 1024], "grid_side_3d": [16, 101], "fixed_budget_s": args.base_cap},
            "held_out": live, "gain_vs_fixed": live["gain_total"], "train_fit": fit,
            "train_samples_per_s": round(epochs * len(recs) / t_train, 1),
            "loss_first_last": [hist[0], hist[-1]]}


def copy_calibration(mib: int):
    """Plain streaming kernels of known size, for a hardware-counter run: three
    device-to-device copies and three element-wise negations of `mib` MiB, each
    reading and writing exactly `mib` MiB.  Their FETCH_SIZE / WRITE_SIZE give
    the scale factor from the counters to bytes."""
    import torch
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"bench: copy calibration, 3 copies and 3 negations of {mib} MiB")
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="laplace3d",
                    choices=["laplace3d", "convdiff", "laplace2d", "batch", "predictor", "predictor-label", "fd",
                             "prec32", "bjac", "restart"])
    ap.add_argument("--grid", type=int, default=0, help="grid side (0: the workload's own)")
    ap.add_argument("--restart", type=int, default=0, help="restart length (0: the workload's own)")
    ap.add_argument("--test", type=int, default=32, help="predictor: held-out systems timed live")
    ap.add_argument("--test-start", type=int, default=0, help="predictor: first held-out system")
    ap.add_argument("--test-out", default="", help="predictor: append per-system held-out records here")
    ap.add_argument("--labels", default="", help="predictor: labelled training file (default: the committed one)")
    ap.add_argument("--label-start", type=int, default=0, help="predictor-label: first training system")
    ap.add_argument("--label-count", type=int, default=8, help="predictor-label: systems to label")
    ap.add_argument("--label-out", default="", help="predictor-label: output file (default: the committed one)")
    ap.add_argument("--base-cap", type=float, default=4.0,
                    help="predictor: time budget (s) of the fixed combination and of a predicted one")
    ap.add_argument("--fd-stride", type=int, default=0, help="fd: switch-point stride (0: 5 restarts)")
    ap.add_argument("--fd-max", type=int, default=0, help="fd: last switch point (0: float64 GMRES's count)")
    ap.add_argument("--degrees", default="10,20,30,40,50,60,70", help="prec32: polynomial degrees")
    ap.add_argument("--blocks", default="1,42", help="bjac: block sizes")
    ap.add_argument("--restarts", default="25,50,100,200,300,400", help="restart: restart lengths")
    ap.add_argument("--tiling", default="", help="batch: 'rows,variant' instead of the autotuner")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="default workload: the headline line only, without the other configs' records")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run three plain copies of MIB MiB first (counter scale factor)")
    ap.add_argument("--persistent", type=int, default=-1,
                    help="one launch per restart cycle (1), off (0), or -1: on for n <= 6144")
    ap.add_argument("--batch-graph", type=int, default=1,
                    help="batch: replay each restart cycle as a hipGraph (1, default) or launch eagerly (0)")
    ap.add_argument("--graph", type=int, default=0,
                    help="replay each restart cycle as a hipGraph (no per-kernel events then)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no run: turn two counter runs of this script into the stored traffic figure")
    args = ap.parse_args()
    if args.summarize_pmc:
        dom = "poly_step" if args.workload == "convdiff" else "cgs_update_dots"
        pats = {"poly_step": ["poly_real_kernel<float", "poly_pair1_kernel<float", "poly_pair2_kernel<float"],
                "cgs_update_dots": ["cgs_update_dots_kernel<float"]}[dom]
        summarize_pmc(*args.summarize_pmc, args.workload, dom, pats, args.copy_calibration or 1024)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import paper_2105_07544_amd as G
    G.lib()  # fails loudly when the HIP library is not built
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
    if args.workload == "batch":
        out = batch(args)
    elif args.workload == "predictor":
        out = predictor(args)
    elif args.workload == "predictor-label":
        out = predictor_label(args)
    elif args.workload == "fd":
        out = fd_sweep(args)
    elif args.workload == "prec32":
        out = prec32_sweep(args)
    elif args.workload == "bjac":
        out = bjac_leg(args)
    elif args.workload == "restart":
        out = restart_sweep(args)
    elif args.workload == "laplace3d" and not args.no_configs and not args.grid and not args.restart:
        # the headline (3D Laplacian 150^3) with the other configs' IR-vs-float64
        # records beside it, each measured in this run
        out = single_system(args, "laplace3d")
        out["configs"] = {}
        for key, fn in (("laplace2d_64", lambda: single_system(args, "laplace2d", steps=5, warmup=2,
                                                                breakdown=False, extras=False, cpu=False)),
                        ("convdiff_2500", lambda: single_system(args, "convdiff", steps=1, warmup=1,
                                                                 breakdown=False, extras=False, cpu=False)),
                        ("batch_256x16", lambda: batch(args))):
            rec = fn()
            out["configs"][key] = {k: v for k, v in rec.items()
                                   if k not in ("metric", "n_gpus", "higher_is_better", "scaling",
                                                "vs_baseline", "data")}
    else:
        out = single_system(args, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
