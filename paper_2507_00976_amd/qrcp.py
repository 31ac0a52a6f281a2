"""Thin ctypes binding of ``libqrcp.so`` (declared in include/qrcp.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
supplies device memory and the current stream.  Matrices are column-major: a
torch tensor ``A`` of shape (m, n) with ``A.stride(0) == 1`` (for example
``X.t()`` of a contiguous (n, m) tensor, or ``colmajor(A)``).

If the shared library is missing the import fails loudly: there is no CPU or
PyTorch fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqrcp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_2507_00976_amd.build` "
        "(hipcc, gfx950).  The QRCP path has no fallback implementation.")

_lib = ctypes.CDLL(LIB_PATH)

QRCP_OK = 0
QRCP_ERR_WORKSPACE = 1
QRCP_ERR_HIP = 2
QRCP_ERR_NONFINITE = 3
QRCP_ERR_UNSUPPORTED = 4
QRCP_ERR_TIMEOUT = 5

_i64, _u64, _i32, _u32, _dbl, _sz, _vp = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32,
                                          ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p)


class QrcpOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("cholqr_passes", ctypes.c_int32),
                ("sketch_precision", ctypes.c_int32), ("trailing_precision", ctypes.c_int32),
                ("pivot_base", ctypes.c_int32), ("pivot_steps", ctypes.c_int32),
                ("qr_tall", ctypes.c_int32), ("qrcp_wide", ctypes.c_int32),
                ("max_rank", ctypes.c_int64)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("qrcp_workspace_size", _sz, _i64, _i64, _i64, _dbl, ctypes.POINTER(QrcpOpts))
_sig("qrcp_factor", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _dbl, _u64, _dbl, _vp, _vp,
     ctypes.POINTER(_i64), ctypes.POINTER(QrcpOpts), _vp, _sz, _vp)
_sig("qrcp_factor_async", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _dbl, _u64, _dbl, _vp, _vp,
     _vp, _vp, ctypes.POINTER(QrcpOpts), _vp, _sz, _vp)
_sig("qrcp_noalloc_max_bytes", _sz)
_sig("qrcp_factor_noalloc", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _dbl, _u64, _dbl, _vp, _vp,
     ctypes.POINTER(_i64), ctypes.POINTER(QrcpOpts), _vp)
_sig("qrcp_geqrf_workspace_size", _sz, _i64, _i64, _i64)
_sig("qrcp_geqrf", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("qrcp_status_string", ctypes.c_char_p, ctypes.c_int)
_sig("qrcp_last_error", ctypes.c_char_p)
_sig("qrcp_sketch_operator", ctypes.c_int, _vp, _i64, _i64, _i64, _u64, _vp)
_sig("qrcp_philox", ctypes.c_int, _vp, _i64, _u32, _u32, _vp, _vp)
_sig("qrcp_sketch", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _u64, _i32, _vp, _i64, _vp, _sz, _vp)
_sig("qrcp_lu_workspace_size", _sz, _i64, _i64)
_sig("qrcp_lu_pivots", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _sz, _vp)
_sig("qrcp_sketch_qr_workspace_size", _sz, _i64, _i64)
_sig("qrcp_sketch_qr", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("qrcp_panel_workspace_size", _sz, _i64, _i64)
_sig("qrcp_cholqr", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _i32,
     ctypes.POINTER(_i64), _vp, _sz, _vp)
_sig("qrcp_reconstruct", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _sz, _vp)
_sig("qrcp_apply_qt_workspace_size", _sz, _i64, _i64, _i64)
_sig("qrcp_apply_qt", ctypes.c_int, _vp, _i64, _i64, _i64, _vp, _vp, _i64, _i64, _i32, _vp, _sz, _vp)
_sig("qrcp_sketch_update", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp)
_sig("qrcp_sketch_update_chol", ctypes.c_int, _vp, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _i64,
     _vp, _sz, _vp)



class ServerCfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("device", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("block_size", ctypes.c_int64),
                ("sketch_factor", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("tol", ctypes.c_double), ("A", ctypes.c_void_p), ("jpiv", ctypes.c_void_p),
                ("tau", ctypes.c_void_p), ("opts", QrcpOpts)]


class Result(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rank", ctypes.c_int64), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


_sig("qrcp_server_create", _vp, ctypes.POINTER(ServerCfg))
_sig("qrcp_server_submit", ctypes.c_int, _vp, ctypes.POINTER(Request), ctypes.POINTER(_u64))
_sig("qrcp_server_poll", ctypes.c_int, _vp, _u64, ctypes.POINTER(Result))
_sig("qrcp_server_wait", ctypes.c_int, _vp, _u64, ctypes.POINTER(Result))
_sig("qrcp_server_pending", ctypes.c_int, _vp)
_sig("qrcp_server_destroy", None, _vp)

_sig("qrcp_profile_enable", ctypes.c_int, _i32)
_sig("qrcp_profile_num_stages", _i32)
_sig("qrcp_profile_stage_name", ctypes.c_char_p, _i32)
_sig("qrcp_profile_read", ctypes.c_int, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
     ctypes.POINTER(ctypes.c_double))

EXPORTED = ["qrcp_profile_enable", "qrcp_profile_num_stages", "qrcp_profile_stage_name",
            "qrcp_profile_read", "qrcp_workspace_size", "qrcp_factor", "qrcp_factor_async", "qrcp_noalloc_max_bytes",
            "qrcp_factor_noalloc", "qrcp_geqrf_workspace_size", "qrcp_geqrf",
            "qrcp_status_string", "qrcp_last_error", "qrcp_sketch_operator", "qrcp_philox",
            "qrcp_sketch", "qrcp_lu_workspace_size", "qrcp_lu_pivots",
            "qrcp_sketch_qr_workspace_size", "qrcp_sketch_qr", "qrcp_panel_workspace_size",
            "qrcp_cholqr", "qrcp_reconstruct", "qrcp_apply_qt_workspace_size", "qrcp_apply_qt",
            "qrcp_sketch_update", "qrcp_sketch_update_chol", "qrcp_server_create", "qrcp_server_submit", "qrcp_server_poll",
            "qrcp_server_wait", "qrcp_server_pending", "qrcp_server_destroy"]


class QrcpError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.qrcp_status_string(code).decode()
        last = _lib.qrcp_last_error().decode()
        super().__init__(f"{where}: status {code} ({msg}){' - ' + last if last else ''}")
        self.code = code


def status_string(code: int) -> str:
    return _lib.qrcp_status_string(code).decode()


def _check(code: int, where: str):
    if code != QRCP_OK:
        raise QrcpError(code, where)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def colmajor(a: torch.Tensor) -> torch.Tensor:
    """A column-major copy (stride(0) == 1) of a 2-D tensor."""
    return a.t().contiguous().t()


def _cm(a: torch.Tensor, name: str, dtype=torch.float64):
    if a.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if a.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not a.is_cuda:
        raise ValueError(f"{name} must be a CUDA/HIP tensor")
    m, n = a.shape
    # the row stride matters only with two or more rows and columns (torch keeps
    # any stride on a dimension of size 1)
    if n > 1 and m > 1 and a.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1); use colmajor()")
    ld = a.stride(1) if n > 1 else max(m, 1)
    return a.data_ptr(), m, n, max(ld, max(m, 1))


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _opts(cholqr_passes=1, sketch_precision=0, trailing_precision=0, pivot_base=0,
          pivot_steps=0, qr_tall=0, qrcp_wide=0, max_rank=0) -> QrcpOpts:
    return QrcpOpts(ctypes.sizeof(QrcpOpts), cholqr_passes, sketch_precision, trailing_precision,
                    pivot_base, pivot_steps, qr_tall, qrcp_wide, max_rank)


# ---------------------------------------------------------------- full method
def workspace_size(m, n, block_size, sketch_factor=1.25, **opts) -> int:
    o = _opts(**opts)
    return int(_lib.qrcp_workspace_size(m, n, block_size, sketch_factor, ctypes.byref(o)))


def factor(A: torch.Tensor, block_size: int, sketch_factor: float = 1.25, seed: int = 42,
           tol: float = 0.0, *, workspace: torch.Tensor | None = None, stream=None, **opts):
    """qrcp_factor: A (m x n, column-major, overwritten) -> (A, jpiv, tau, rank).
    ``opts`` are qrcp_opts fields: cholqr_passes, sketch_precision,
    trailing_precision, pivot_base, pivot_steps, qr_tall, qrcp_wide, max_rank."""
    ptr, m, n, lda = _cm(A, "A")
    o = _opts(**opts)
    need = int(_lib.qrcp_workspace_size(m, n, block_size, sketch_factor, ctypes.byref(o)))
    if workspace is None:
        workspace = _ws(need, A.device)
    jpiv = torch.empty(n, dtype=torch.int64, device=A.device)
    tau = torch.empty(min(m, n), dtype=torch.float64, device=A.device)
    rank = _i64(0)
    rc = _lib.qrcp_factor(ptr, m, n, lda, block_size, sketch_factor, seed, tol, jpiv.data_ptr(),
                          tau.data_ptr(), ctypes.byref(rank), ctypes.byref(o), workspace.data_ptr(),
                          workspace.numel(), _stream(stream))
    _check(rc, "qrcp_factor")
    return A, jpiv, tau, int(rank.value)


def factor_async(A: torch.Tensor, block_size: int, sketch_factor: float = 1.25, seed: int = 42,
                 tol: float = 0.0, *, workspace: torch.Tensor | None = None, stream=None, **opts):
    """qrcp_factor_async: enqueues the whole factorization on the stream and
    returns at once -> (A, jpiv, tau, rank_dev, status_dev); rank_dev (int64)
    and status_dev (int32) are one-element device tensors, valid once the
    stream has passed the call.  The returned tensors and the workspace must
    stay alive until then."""
    ptr, m, n, lda = _cm(A, "A")
    o = _opts(**opts)
    need = int(_lib.qrcp_workspace_size(m, n, block_size, sketch_factor, ctypes.byref(o)))
    if workspace is None:
        workspace = _ws(need, A.device)
    jpiv = torch.empty(n, dtype=torch.int64, device=A.device)
    tau = torch.empty(min(m, n), dtype=torch.float64, device=A.device)
    rank_dev = torch.empty(1, dtype=torch.int64, device=A.device)
    status_dev = torch.empty(1, dtype=torch.int32, device=A.device)
    rc = _lib.qrcp_factor_async(ptr, m, n, lda, block_size, sketch_factor, seed, tol,
                                jpiv.data_ptr(), tau.data_ptr(), rank_dev.data_ptr(),
                                status_dev.data_ptr(), ctypes.byref(o), workspace.data_ptr(),
                                workspace.numel(), _stream(stream))
    _check(rc, "qrcp_factor_async")
    return A, jpiv, tau, rank_dev, status_dev


def noalloc_max_bytes() -> int:
    return int(_lib.qrcp_noalloc_max_bytes())


def factor_noalloc(A: torch.Tensor, block_size: int, sketch_factor: float = 1.25, seed: int = 42,
                   tol: float = 0.0, *, jpiv: torch.Tensor, tau: torch.Tensor, stream=None, **opts):
    """qrcp_factor_noalloc: as factor(), with the library's fixed device
    workspace; the caller passes the jpiv (int64, n) and tau (float64,
    min(m, n)) outputs.  Returns (A, jpiv, tau, rank)."""
    ptr, m, n, lda = _cm(A, "A")
    assert jpiv.is_cuda and jpiv.dtype == torch.int64 and jpiv.numel() >= n
    assert tau.is_cuda and tau.dtype == torch.float64 and tau.numel() >= min(m, n)
    o = _opts(**opts)
    rank = _i64(0)
    rc = _lib.qrcp_factor_noalloc(ptr, m, n, lda, block_size, sketch_factor, seed, tol,
                                  jpiv.data_ptr(), tau.data_ptr(), ctypes.byref(rank),
                                  ctypes.byref(o), _stream(stream))
    _check(rc, "qrcp_factor_noalloc")
    return A, jpiv, tau, int(rank.value)


def geqrf_workspace_size(m, n, nb) -> int:
    return int(_lib.qrcp_geqrf_workspace_size(m, n, nb))


def geqrf(A: torch.Tensor, nb: int = 256, workspace: torch.Tensor | None = None, stream=None):
    """qrcp_geqrf: unpivoted Householder QR in place -> (A, tau)."""
    ptr, m, n, lda = _cm(A, "A")
    if workspace is None:
        workspace = _ws(_lib.qrcp_geqrf_workspace_size(m, n, nb), A.device)
    tau = torch.empty(min(m, n), dtype=torch.float64, device=A.device)
    rc = _lib.qrcp_geqrf(ptr, m, n, lda, tau.data_ptr(), nb, workspace.data_ptr(), workspace.numel(),
                         _stream(stream))
    _check(rc, "qrcp_geqrf")
    return A, tau


# ---------------------------------------------------------------- steps
def sketch_operator(m: int, d: int, seed: int, device="cuda") -> torch.Tensor:
    """S^T (m x d, column-major) of the Gaussian sketching operator."""
    st = colmajor(torch.empty(m, d, dtype=torch.float64, device=device))
    _check(_lib.qrcp_sketch_operator(st.data_ptr(), m, d, max(m, 1), seed, _stream()),
           "qrcp_sketch_operator")
    return st


def philox(ctr: torch.Tensor, key0: int, key1: int) -> torch.Tensor:
    """Raw Philox4x32-10 blocks; ctr is an int32 tensor (count, 4) holding uint32 bits."""
    assert ctr.dtype == torch.int32 and ctr.is_cuda and ctr.is_contiguous() and ctr.shape[1] == 4
    out = torch.empty_like(ctr)
    _check(_lib.qrcp_philox(ctr.data_ptr(), ctr.shape[0], key0, key1, out.data_ptr(), _stream()),
           "qrcp_philox")
    return out


def sketch(A: torch.Tensor, d: int, seed: int, precision: int = 0) -> torch.Tensor:
    ptr, m, n, lda = _cm(A, "A")
    msk = colmajor(torch.empty(d, n, dtype=torch.float64, device=A.device))
    ws = _ws(m * d * 8 + (40 << 20) + 1024, A.device)
    _check(_lib.qrcp_sketch(ptr, m, n, lda, d, seed, precision, msk.data_ptr(), d, ws.data_ptr(),
                            ws.numel(), _stream()), "qrcp_sketch")
    return msk


def lu_pivots(Msk: torch.Tensor):
    ptr, d, ni, ld = _cm(Msk, "Msk")
    ipiv = torch.empty(min(d, ni), dtype=torch.int64, device=Msk.device)
    jsk = torch.empty(ni, dtype=torch.int64, device=Msk.device)
    ws = _ws(_lib.qrcp_lu_workspace_size(d, ni), Msk.device)
    _check(_lib.qrcp_lu_pivots(ptr, d, ni, ld, ipiv.data_ptr(), jsk.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream()), "qrcp_lu_pivots")
    return ipiv, jsk


def sketch_qr(B: torch.Tensor) -> torch.Tensor:
    ptr, d, ni, ld = _cm(B, "B")
    r = colmajor(torch.empty(d, ni, dtype=torch.float64, device=B.device))
    ws = _ws(_lib.qrcp_sketch_qr_workspace_size(d, ni), B.device)
    _check(_lib.qrcp_sketch_qr(ptr, d, ni, ld, r.data_ptr(), d, ws.data_ptr(), ws.numel(), _stream()),
           "qrcp_sketch_qr")
    return r


def cholqr(P: torch.Tensor, Rs: torch.Tensor, passes: int = 1):
    """P (mi x k) is overwritten by Q; returns (P, Rc, keff)."""
    ptr, mi, k, ldp = _cm(P, "P")
    rptr, _, _, ldrs = _cm(Rs, "Rs")
    rc = colmajor(torch.zeros(k, k, dtype=torch.float64, device=P.device))
    keff = _i64(0)
    ws = _ws(_lib.qrcp_panel_workspace_size(mi, k), P.device)
    _check(_lib.qrcp_cholqr(ptr, mi, k, ldp, rptr, ldrs, rc.data_ptr(), max(k, 1), passes,
                            ctypes.byref(keff), ws.data_ptr(), ws.numel(), _stream()), "qrcp_cholqr")
    return P, rc, int(keff.value)


def reconstruct(Q: torch.Tensor):
    """Q (mi x k) -> Y below / U on+above the diagonal in place; returns (Q, tau, dsig)."""
    ptr, mi, k, ldq = _cm(Q, "Q")
    tau = torch.empty(k, dtype=torch.float64, device=Q.device)
    dsig = torch.empty(k, dtype=torch.float64, device=Q.device)
    ws = _ws(_lib.qrcp_panel_workspace_size(mi, k), Q.device)
    _check(_lib.qrcp_reconstruct(ptr, mi, k, ldq, tau.data_ptr(), dsig.data_ptr(), ws.data_ptr(),
                                 ws.numel(), _stream()), "qrcp_reconstruct")
    return Q, tau, dsig


def apply_qt(Y: torch.Tensor, tau: torch.Tensor, C: torch.Tensor, precision: int = 0) -> torch.Tensor:
    yptr, mi, k, ldy = _cm(Y, "Y")
    cptr, mc, nc, ldc = _cm(C, "C")
    assert mc == mi
    ws = _ws(_lib.qrcp_apply_qt_workspace_size(mi, k, nc), C.device)
    _check(_lib.qrcp_apply_qt(yptr, mi, k, ldy, tau.data_ptr(), cptr, nc, ldc, precision,
                              ws.data_ptr(), ws.numel(), _stream()), "qrcp_apply_qt")
    return C


def sketch_update(Rsk: torch.Tensor, b: int, R11: torch.Tensor, R12: torch.Tensor) -> torch.Tensor:
    ptr, d, cols, ld = _cm(Rsk, "Rsk")
    p11, _, _, ld11 = _cm(R11, "R11")
    p12, _, nt, ld12 = _cm(R12, "R12")
    assert cols == b + nt
    ws = _ws(2 * b * b * 8 + 2048, Rsk.device)
    _check(_lib.qrcp_sketch_update(ptr, d, b, nt, ld, p11, ld11, p12, ld12, ws.data_ptr(), ws.numel(),
                                   _stream()), "qrcp_sketch_update")
    return Rsk


def sketch_update_chol(Rsk: torch.Tensor, b: int, Rc: torch.Tensor, dsig: torch.Tensor,
                       R12: torch.Tensor) -> torch.Tensor:
    """The one-pass form of the sample update: Rsk12 - Rc^{-1} diag(D) R12."""
    ptr, d, cols, ld = _cm(Rsk, "Rsk")
    pc, _, _, ldc = _cm(Rc, "Rc")
    p12, _, nt, ld12 = _cm(R12, "R12")
    assert cols == b + nt and dsig.is_cuda and dsig.dtype == torch.float64
    ws = _ws(2 * b * b * 8 + 2048, Rsk.device)
    _check(_lib.qrcp_sketch_update_chol(ptr, d, b, nt, ld, pc, ldc, dsig.data_ptr(), p12, ld12,
                                        ws.data_ptr(), ws.numel(), _stream()),
           "qrcp_sketch_update_chol")
    return Rsk


# ---------------------------------------------------------------- timing
def profile_enable(mode: int) -> None:
    _check(_lib.qrcp_profile_enable(mode), "qrcp_profile_enable")


def profile_read() -> dict:
    """{stage: (ms, launches, flops)} of everything timed since profile_enable()."""
    out = {}
    for st in range(int(_lib.qrcp_profile_num_stages())):
        ms, cnt, fl = ctypes.c_double(0), _i64(0), ctypes.c_double(0)
        _check(_lib.qrcp_profile_read(st, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(fl)),
               "qrcp_profile_read")
        out[_lib.qrcp_profile_stage_name(st).decode()] = (ms.value, int(cnt.value), fl.value)
    return out



# ---------------------------------------------------------------- request server
class Server:
    """qrcp_server_*: concurrent factorizations of independent requests.

    ``submit`` hands the library a column-major FP64 device matrix (overwritten in
    place, as ``factor``) and returns a ticket; ``poll``/``wait`` return
    ``(A, jpiv, tau, rank, timing)`` once the request is done, where timing holds
    the server-clock submit/start/end times in ms.  The tensors of a request are
    kept alive here until it is collected.
    """

    def __init__(self, slots: int = 8, hbm_budget: int = 0, device: int = 0):
        cfg = ServerCfg(ctypes.sizeof(ServerCfg), slots, hbm_budget, device)
        self._h = _lib.qrcp_server_create(ctypes.byref(cfg))
        if not self._h:
            raise QrcpError(QRCP_ERR_HIP, "qrcp_server_create")
        self._live = {}

    def submit(self, A: torch.Tensor, block_size: int, sketch_factor: float = 1.25,
               seed: int = 42, tol: float = 0.0, **opts) -> int:
        ptr, m, n, lda = _cm(A, "A")
        jpiv = torch.empty(n, dtype=torch.int64, device=A.device)
        tau = torch.empty(min(m, n), dtype=torch.float64, device=A.device)
        # the caller's pending work on A (e.g. its initialization) must be done
        # before a server stream reads it
        torch.cuda.current_stream(A.device).synchronize()
        req = Request(ctypes.sizeof(Request), m, n, lda, block_size, sketch_factor, seed, tol,
                      ptr, jpiv.data_ptr(), tau.data_ptr(), _opts(**opts))
        t = _u64(0)
        _check(_lib.qrcp_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "qrcp_server_submit")
        self._live[t.value] = (A, jpiv, tau)
        return t.value

    def _done(self, ticket, res):
        A, jpiv, tau = self._live.pop(ticket)
        _check(res.status, "qrcp_server request")
        return A, jpiv, tau, int(res.rank), {"submit_ms": res.submit_ms,
                                             "start_ms": res.start_ms, "end_ms": res.end_ms}

    def poll(self, ticket: int):
        res = Result()
        rc = _lib.qrcp_server_poll(self._h, ticket, ctypes.byref(res))
        if rc == 1:
            return None
        if rc != 0:
            raise KeyError(ticket)
        return self._done(ticket, res)

    def wait(self, ticket: int):
        res = Result()
        if _lib.qrcp_server_wait(self._h, ticket, ctypes.byref(res)) != 0:
            raise KeyError(ticket)
        return self._done(ticket, res)

    def pending(self) -> int:
        return int(_lib.qrcp_server_pending(self._h))

    def close(self):
        if self._h:
            _lib.qrcp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
