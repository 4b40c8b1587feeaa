"""MI355X GMRES(m) / GMRES-IR hot path: Python binding of libgmresir.so.

Torch supplies device memory and the current HIP stream; every step of the
solvers runs in the library's HIP kernels.  The names follow the C ABI in
include/gmres_ir.h.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import _capi
from ._capi import GMR_F32, GMR_F64, GmresError, PROF, check

__all__ = ["DeviceCSR", "Poly", "SolveResult", "workspace_bytes", "alloc_workspace", "spmv",
           "cgs2_orth", "cgs2_orth_noalloc", "poly_prec_setup", "bjac_prec_setup", "poly_prec_apply", "gmres_solve", "gmres_ir_solve", "gmres_f32prec_solve", "gmres_fd_solve",
           "fd_workspace_bytes",
           "hessenberg_eigvals", "harmonic_ritz", "leja_order", "Batch", "GmresError", "GMR_F32", "GMR_F64", "lib"]


def lib():
    return _capi.load()


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return GMR_F64
    if t == torch.float32:
        return GMR_F32
    raise ValueError(f"unsupported dtype {t}")


class DeviceCSR:
    """A CSR matrix whose arrays live in device memory (int32 indices)."""

    def __init__(self, row_ptr, col_idx, val, device="cuda"):
        self.row_ptr = torch.as_tensor(np.asarray(row_ptr) if not torch.is_tensor(row_ptr) else row_ptr,
                                       dtype=torch.int32).to(device).contiguous()
        self.col_idx = torch.as_tensor(np.asarray(col_idx) if not torch.is_tensor(col_idx) else col_idx,
                                       dtype=torch.int32).to(device).contiguous()
        v = val if torch.is_tensor(val) else torch.from_numpy(np.ascontiguousarray(val))
        if v.dtype not in (torch.float32, torch.float64):
            v = v.to(torch.float64)
        self.val = v.to(device).contiguous()
        self.n = int(self.row_ptr.numel()) - 1
        self.nnz = int(self.col_idx.numel())
        self.device = self.val.device

    @classmethod
    def from_host(cls, A, device="cuda"):
        """From any object with n, row_ptr, col_idx, val (numpy)."""
        return cls(A.row_ptr, A.col_idx, A.val, device)

    @property
    def dtype(self) -> int:
        return _dtype_code(self.val.dtype)

    def struct(self) -> _capi.gmr_csr:
        return _capi.gmr_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                             self.val.data_ptr(), self.dtype)

    def to_f32(self) -> "DeviceCSR":
        """Float32 copy of the values (round to nearest) by the library's cast kernel;
        the index arrays are shared."""
        out = DeviceCSR.__new__(DeviceCSR)
        out.row_ptr, out.col_idx, out.n, out.nnz, out.device = (self.row_ptr, self.col_idx, self.n,
                                                                 self.nnz, self.device)
        out.val = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        if self.val.dtype == torch.float32:
            out.val.copy_(self.val)
        else:
            check(lib().csr_values_to_f32(_ptr(self.val), _ptr(out.val), self.nnz, _stream(self.device)))
        return out


def workspace_bytes(n: int, restart: int, dtype: int, with_poly: bool = False) -> int:
    p = _capi.gmr_params(restart, 1e-10, 1, 0, 0, 0, 0)
    nb = lib().gmres_workspace_bytes(n, C.byref(p), dtype, int(bool(with_poly)))
    if nb == 0:
        raise GmresError(-1, "invalid workspace query")
    return int(nb)


def fd_workspace_bytes(n: int, restart: int) -> int:
    """Workspace bytes of gmres_fd_solve (also enough for gmres_solve and gmres_ir_solve
    without a polynomial)."""
    p = _capi.gmr_params(restart, 1e-10, 1, 0, 0, 0, 0)
    nb = lib().gmres_fd_workspace_bytes(n, C.byref(p))
    if nb == 0:
        raise GmresError(-1, "invalid workspace query")
    return int(nb)


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def spmv(A: DeviceCSR, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x (asynchronous on the current stream)."""
    if y is None:
        y = torch.empty(A.n, dtype=A.val.dtype, device=A.device)
    st = A.struct()
    check(lib().spmv(C.byref(st), _ptr(x), _ptr(y), _stream(A.device)))
    return y


def cgs2_orth(V: torch.Tensor, k: int, w: torch.Tensor, ws: Optional[torch.Tensor] = None,
              ldv: Optional[int] = None) -> torch.Tensor:
    """Orthogonalise w against the first k columns of V (column-major n x >=k,
    given as a (cols, ldv) row-major tensor) by CGS2 and normalise it in place.
    Returns h (float64, k+1): h[:k] = h1 + h2, h[k] = ||w|| before normalising."""
    n = w.numel()
    ld = ldv if ldv is not None else V.shape[-1]
    dt = _dtype_code(w.dtype)
    if ws is None:
        ws = alloc_workspace(workspace_bytes(n, max(k, 1), dt), w.device)
    h = torch.empty(k + 1, dtype=torch.float64, device=w.device)
    check(lib().cgs2_orth(dt, n, k, _ptr(V), ld, _ptr(w), _ptr(h), _ptr(ws), ws.numel(),
                          _stream(w.device)))
    return h


def cgs2_orth_noalloc(V: torch.Tensor, k: int, w: torch.Tensor, h: torch.Tensor,
                      ldv: Optional[int] = None) -> torch.Tensor:
    """cgs2_orth with the library's static scratch array instead of a workspace:
    the call itself allocates nothing (h, float64 with k+1 entries, is the
    caller's).  Calls that overlap on one device race."""
    n = w.numel()
    ld = ldv if ldv is not None else V.shape[-1]
    check(lib().cgs2_orth_noalloc(_dtype_code(w.dtype), n, k, _ptr(V), ld, _ptr(w), _ptr(h),
                                  _stream(w.device)))
    return h


class Poly:
    """Handle of a right preconditioner: a GMRES polynomial (poly_prec_setup) or
    block Jacobi (bjac_prec_setup, which keeps its device buffer alive here)."""

    def __init__(self, handle: C.c_void_p, dtype: int, keep=None):
        self._h = handle
        self.dtype = dtype
        self._keep = keep

    @property
    def block(self) -> int:
        """Rows per diagonal block for block Jacobi, 0 for a polynomial."""
        return int(lib().prec_block_size(self._h))

    @property
    def handle(self):
        return self._h

    @property
    def degree(self) -> int:
        return int(lib().poly_prec_degree(self._h))

    def roots(self) -> np.ndarray:
        k = self.degree + 1
        re = np.zeros(k)
        im = np.zeros(k)
        check(lib().poly_prec_roots(self._h, re.ctypes.data_as(C.c_void_p), im.ctypes.data_as(C.c_void_p)))
        return re + 1j * im

    def hessenberg(self) -> np.ndarray:
        """(s+1) x s Hessenberg matrix of the Arnoldi run that built the polynomial."""
        s = self.degree + 1
        H = np.zeros((s + 1) * s)
        check(lib().poly_prec_hessenberg(self._h, H.ctypes.data_as(C.c_void_p)))
        return H.reshape(s, s + 1).T.copy()

    def __del__(self):
        try:
            if self._h:
                lib().poly_prec_destroy(self._h)
                self._h = None
        except Exception:
            pass


def poly_prec_setup(A: DeviceCSR, degree: int, v0: torch.Tensor, ws: Optional[torch.Tensor] = None) -> Poly:
    if ws is None:
        ws = alloc_workspace(workspace_bytes(A.n, degree + 1, A.dtype, True), A.device)
    out = C.c_void_p()
    st = A.struct()
    check(lib().poly_prec_setup(C.byref(st), degree, _ptr(v0), _ptr(ws), ws.numel(), C.byref(out),
                                _stream(A.device)))
    return Poly(out, A.dtype)


def bjac_prec_setup(A: DeviceCSR, block: int) -> Poly:
    """Block Jacobi M = blockdiag(A)^-1 with `block` rows per diagonal block, inverted on
    the device in A's precision."""
    nb = lib().bjac_prec_bytes(A.n, int(block), A.dtype)
    if nb == 0:
        raise GmresError(-1 if block < 1 else -5, f"bjac_prec_setup: unsupported block size {block}")
    inv = alloc_workspace(nb, A.device)
    out = C.c_void_p()
    st = A.struct()
    check(lib().bjac_prec_setup(C.byref(st), int(block), _ptr(inv), inv.numel(), C.byref(out), _stream(A.device)))
    return Poly(out, A.dtype, keep=inv)


def poly_prec_apply(P: Poly, A: DeviceCSR, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                    ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    if y is None:
        y = torch.empty_like(x)
    if ws is None:
        ws = alloc_workspace(workspace_bytes(A.n, 1, A.dtype, True), A.device)
    st = A.struct()
    check(lib().poly_prec_apply(P.handle, C.byref(st), _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                _stream(A.device)))
    return y


@dataclass
class SolveResult:
    status: int
    status_name: str
    iters: int
    cycles: int
    rel_res: float
    implicit_rel_res: float
    seconds: float
    history: List[float] = field(default_factory=list)
    prof_ms: float = 0.0
    prof_launches: int = 0
    prof_bytes: float = 0.0
    loss_of_accuracy: int = 0

    @property
    def converged(self) -> bool:
        return self.status == 0


def _params(restart, tol, max_iters, max_cycles, stagnation_cycles, prof, graph=False, persistent=False,
            stop_on_loss=False, half_basis=False):
    flags = ((_capi.GMR_FLAG_GRAPH if graph else 0) | (_capi.GMR_FLAG_PERSISTENT if persistent else 0)
             | (_capi.GMR_FLAG_STOP_ON_LOSS if stop_on_loss else 0)
             | (_capi.GMR_FLAG_HALF_BASIS if half_basis else 0))
    return _capi.gmr_params(int(restart), float(tol), int(max_iters), int(max_cycles),
                            int(stagnation_cycles), PROF[prof] if isinstance(prof, str) else int(prof), flags)


def _result(res: _capi.gmr_result, hist: np.ndarray) -> SolveResult:
    return SolveResult(res.status, _capi.STATUS.get(res.status, str(res.status)), int(res.iters),
                       int(res.cycles), float(res.rel_res), float(res.implicit_rel_res),
                       float(res.seconds), list(hist[: res.history_len]), float(res.prof_ms),
                       int(res.prof_launches), float(res.prof_bytes), int(res.loss_of_accuracy))


def gmres_solve(A: DeviceCSR, b: torch.Tensor, x: Optional[torch.Tensor] = None, *, restart: int = 50,
                tol: float = 1e-10, max_iters: int = 100000, max_cycles: int = 0,
                P: Optional[Poly] = None, ws: Optional[torch.Tensor] = None, prof="none",
                graph: bool = False, persistent: bool = False, stop_on_loss: bool = False,
                half_basis: bool = False):
    """Restarted GMRES(m) in A's precision.  x (x0, updated in place) defaults to 0.
    persistent: one launch per restart cycle (one block up to n = 1024, a cooperative grid up to n = 6144).
    stop_on_loss: end at the first loss of accuracy instead of restarting.
    half_basis: passed through as GMR_FLAG_HALF_BASIS (only GMRES-IR supports it)."""
    if x is None:
        x = torch.zeros_like(b)
    prm = _params(restart, tol, max_iters, max_cycles, 0, prof, graph, persistent, stop_on_loss, half_basis)
    if ws is None:
        ws = alloc_workspace(workspace_bytes(A.n, restart, A.dtype, P is not None), A.device)
    cap = max_cycles + 1 if max_cycles > 0 else 4096
    hist = np.zeros(cap)
    res = _capi.gmr_result()
    st = A.struct()
    status = lib().gmres_solve(C.byref(st), P.handle if P else None, _ptr(b), _ptr(x), C.byref(prm),
                               _ptr(ws), ws.numel(), C.byref(res), hist.ctypes.data_as(C.c_void_p),
                               _stream(A.device))
    check(status)
    return x, _result(res, hist)


def gmres_ir_solve(A64: DeviceCSR, A32: DeviceCSR, b: torch.Tensor, x: Optional[torch.Tensor] = None, *,
                   restart: int = 50, tol: float = 1e-10, max_iters: int = 100000, max_cycles: int = 0,
                   stagnation_cycles: int = 0, P: Optional[Poly] = None,
                   ws: Optional[torch.Tensor] = None, prof="none", graph: bool = False,
                   persistent: bool = False, half_basis: bool = False):
    """GMRES-IR: float32 inner GMRES(m) on A32, float64 residual and update on A64.
    persistent: one launch per restart cycle (one block up to n = 1024, a cooperative grid up to n = 6144).
    half_basis: store the inner Krylov basis in float16 (no preconditioner)."""
    if x is None:
        x = torch.zeros_like(b)
    prm = _params(restart, tol, max_iters, max_cycles, stagnation_cycles, prof, graph, persistent,
                  half_basis=half_basis)
    if ws is None:
        ws = alloc_workspace(workspace_bytes(A64.n, restart, GMR_F32, P is not None), A64.device)
    cap = max_cycles + 1 if max_cycles > 0 else 4096
    hist = np.zeros(cap)
    res = _capi.gmr_result()
    s64, s32 = A64.struct(), A32.struct()
    status = lib().gmres_ir_solve(C.byref(s64), C.byref(s32), P.handle if P else None, _ptr(b), _ptr(x),
                                  C.byref(prm), _ptr(ws), ws.numel(), C.byref(res),
                                  hist.ctypes.data_as(C.c_void_p), _stream(A64.device))
    check(status)
    return x, _result(res, hist)


def gmres_f32prec_solve(A64: DeviceCSR, A32: DeviceCSR, P32: Poly, b: torch.Tensor,
                        x: Optional[torch.Tensor] = None, *, restart: int = 50, tol: float = 1e-10,
                        max_iters: int = 100000, max_cycles: int = 0, stagnation_cycles: int = 0,
                        ws: Optional[torch.Tensor] = None, prof="none", graph: bool = False,
                        stop_on_loss: bool = False):
    """Float64 GMRES(m) on A64 with the float32 polynomial P32 (built on A32) as right
    preconditioner: each application casts to float32, applies p(A32), widens back."""
    if x is None:
        x = torch.zeros_like(b)
    prm = _params(restart, tol, max_iters, max_cycles, stagnation_cycles, prof, graph, False, stop_on_loss)
    if ws is None:
        ws = alloc_workspace(workspace_bytes(A64.n, restart, GMR_F64, True), A64.device)
    cap = max_cycles + 1 if max_cycles > 0 else 4096
    hist = np.zeros(cap)
    res = _capi.gmr_result()
    s64, s32 = A64.struct(), A32.struct()
    status = lib().gmres_f32prec_solve(C.byref(s64), C.byref(s32), P32.handle, _ptr(b), _ptr(x), C.byref(prm),
                                       _ptr(ws), ws.numel(), C.byref(res), hist.ctypes.data_as(C.c_void_p),
                                       _stream(A64.device))
    check(status)
    return x, _result(res, hist)


def gmres_fd_solve(A64: DeviceCSR, A32: DeviceCSR, b: torch.Tensor, switch_iters: int,
                   x: Optional[torch.Tensor] = None, *, restart: int = 50, tol: float = 1e-10,
                   max_iters: int = 100000, max_cycles: int = 0, stagnation_cycles: int = 0,
                   ws: Optional[torch.Tensor] = None, prof="none", graph: bool = False,
                   persistent: bool = False, stop_on_loss: bool = False):
    """GMRES-FD: float32 GMRES(m) on A32 for switch_iters iterations, then float64
    GMRES(m) on A64 from the float32 iterate.  Returns (x, result of both phases,
    result of the float32 phase); the first history is the float64 phase's residuals,
    the second the float32 phase's."""
    if x is None:
        x = torch.zeros_like(b)
    prm = _params(restart, tol, max_iters, max_cycles, stagnation_cycles, prof, graph, persistent, stop_on_loss)
    if ws is None:
        ws = alloc_workspace(fd_workspace_bytes(A64.n, restart), A64.device)
    cap = max_cycles + 1 if max_cycles > 0 else 4096
    hist = np.zeros(2 * cap)
    res, res32 = _capi.gmr_result(), _capi.gmr_result()
    s64, s32 = A64.struct(), A32.struct()
    status = lib().gmres_fd_solve(C.byref(s64), C.byref(s32), _ptr(b), _ptr(x), C.byref(prm), int(switch_iters),
                                  _ptr(ws), ws.numel(), C.byref(res), C.byref(res32),
                                  hist.ctypes.data_as(C.c_void_p), _stream(A64.device))
    check(status)
    n1 = res32.history_len
    both = _result(res, hist)
    both.history = list(hist[n1: res.history_len])
    return x, both, _result(res32, hist)


def hessenberg_eigvals(H: np.ndarray) -> np.ndarray:
    """Eigenvalues of an upper Hessenberg matrix (host routine of the library)."""
    k = H.shape[0]
    Hc = np.asfortranarray(H, dtype=np.float64)
    re = np.zeros(k)
    im = np.zeros(k)
    check(lib().gmr_hessenberg_eigvals(k, Hc.ctypes.data_as(C.c_void_p), re.ctypes.data_as(C.c_void_p),
                                       im.ctypes.data_as(C.c_void_p)))
    return re + 1j * im


def harmonic_ritz(H: np.ndarray) -> np.ndarray:
    """Harmonic Ritz values of a (k+1) x k Hessenberg matrix (host routine of the library)."""
    k = H.shape[1]
    Hc = np.asfortranarray(H, dtype=np.float64)
    re = np.zeros(k)
    im = np.zeros(k)
    check(lib().gmr_harmonic_ritz(k, Hc.ctypes.data_as(C.c_void_p), k + 1, re.ctypes.data_as(C.c_void_p),
                                  im.ctypes.data_as(C.c_void_p)))
    return re + 1j * im


def leja_order(z: np.ndarray) -> np.ndarray:
    """Modified Leja ordering (host routine of the library)."""
    re = np.ascontiguousarray(np.real(z), dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(z), dtype=np.float64).copy()
    check(lib().gmr_leja_order(len(re), re.ctypes.data_as(C.c_void_p), im.ctypes.data_as(C.c_void_p)))
    return re + 1j * im


class Batch:
    """Batched block GMRES-IR over many systems with 16 right-hand sides each.

    The systems are the diagonal blocks of one block-diagonal CSR matrix (global
    column indices); multivectors are row-major (rows x 16)."""

    def __init__(self, sys_rows, restart: int = 50, nrhs: int = 16):
        rows = np.ascontiguousarray(np.asarray(sys_rows, dtype=np.int32))
        h = C.c_void_p()
        check(lib().batch_create(len(rows), rows.ctypes.data_as(C.c_void_p), nrhs, restart, C.byref(h)))
        self._h = h
        self.nsys = len(rows)
        self.rows = int(rows.sum())
        self.restart = restart

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, inner: int = GMR_F32) -> int:
        """Workspace of the float32-inner solve (and autotune, bcgs_step), or of
        the float64 one with inner=GMR_F64."""
        return int(lib().batch_workspace_bytes(self._h, int(inner)))

    def set_tiling(self, tile_rows: int, group_blocks: int):
        check(lib().batch_set_tiling(self._h, tile_rows, group_blocks))

    def set_graph(self, on: bool):
        """Replay each restart cycle as a captured hipGraph (same results)."""
        check(lib().batch_set_graph(self._h, 1 if on else 0))

    def tiling(self):
        t, g = C.c_int32(), C.c_int32()
        check(lib().batch_get_tiling(self._h, C.byref(t), C.byref(g)))
        return t.value, g.value

    def autotune(self, ws: torch.Tensor):
        t, g, ms = C.c_int32(), C.c_int32(), C.c_double()
        check(lib().batch_autotune(self._h, _ptr(ws), ws.numel(), C.byref(t), C.byref(g), C.byref(ms),
                                   _stream(ws.device)))
        return t.value, g.value, ms.value

    def solve(self, A64: DeviceCSR, A32: Optional[DeviceCSR], B: torch.Tensor, X: torch.Tensor,
              Z: torch.Tensor, ws: torch.Tensor, tol: float = 1e-10, max_cycles: int = 100):
        """GMRES-IR with the float32 inner solve on A32, or, with A32=None, plain
        float64 block GMRES (workspace_bytes(GMR_F64))."""
        res = _capi.gmr_batch_result()
        cyc = np.zeros(self.nsys, dtype=np.int32)
        rel = np.zeros(self.nsys * 16)
        s64 = A64.struct()
        cp, rp = cyc.ctypes.data_as(C.c_void_p), rel.ctypes.data_as(C.c_void_p)
        if A32 is None:
            status = lib().batch_gmres_solve(self._h, C.byref(s64), _ptr(B), _ptr(X), _ptr(Z), float(tol),
                                             int(max_cycles), _ptr(ws), ws.numel(), C.byref(res), cp, rp,
                                             _stream(B.device))
        else:
            s32 = A32.struct()
            status = lib().batch_gmres_ir_solve(self._h, C.byref(s64), C.byref(s32), _ptr(B), _ptr(X), _ptr(Z),
                                                float(tol), int(max_cycles), _ptr(ws), ws.numel(), C.byref(res),
                                                cp, rp, _stream(B.device))
        check(status)
        sys_status = np.zeros(self.nsys, dtype=np.int32)
        check(lib().batch_system_status(self._h, sys_status.ctypes.data_as(C.c_void_p)))
        return {"status": res.status, "status_name": _capi.STATUS.get(res.status, str(res.status)),
                "cycles": res.cycles, "block_iters": res.block_iters, "max_rel_res": res.max_rel_res,
                "seconds": res.seconds, "sys_cycles": cyc, "sys_rel_res": rel.reshape(self.nsys, 16),
                "sys_status": sys_status}

    def bcgs_step(self, Vin: torch.Tensor, nblk: int, W: torch.Tensor, ws: torch.Tensor) -> torch.Tensor:
        Cout = torch.empty((self.nsys, nblk, 16, 16), dtype=torch.float64, device=W.device)
        check(lib().batch_bcgs_step(self._h, _ptr(Vin), nblk, _ptr(W), _ptr(Cout), _ptr(ws), ws.numel(),
                                    _stream(W.device)))
        return Cout

    def __del__(self):
        try:
            if self._h:
                lib().batch_destroy(self._h)
                self._h = None
        except Exception:
            pass
