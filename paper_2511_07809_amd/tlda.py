"""Thin ctypes binding of libtlda (include/tlda.h), function for function.

Argument marshalling only: every call goes straight to the HIP library; there
is no CPU implementation behind any of these names.  PyTorch supplies device
memory and the current HIP stream.  Importing this module without a built
libtlda.so raises immediately.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # loads the HIP runtime libtlda.so binds to (same soname)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlda.so")

TLDA_OK = 0
STATUS_NAMES = {0: "TLDA_OK", 1: "TLDA_ERR_ARG", 2: "TLDA_ERR_SHAPE", 3: "TLDA_ERR_CSR",
                4: "TLDA_ERR_STATE", 5: "TLDA_ERR_NUMERIC", 6: "TLDA_ERR_OOM",
                7: "TLDA_ERR_DEVICE"}
TLDA_VALIDATE_CSR = 0x1
TLDA_BF16 = 0x2
TLDA_CLASSIC = 0x4
TLDA_REFRESH_W = 0x1
TLDA_RESET = 0x2
TLDA_RELEASE = 0x4
TLDA_REFRESH_WARM = 0x8
TLDA_PROJECT_SIMPLEX = 0x1
TLDA_MAX_D = 256
TLDA_MAX_K = 256
TLDA_MAX_DK = 16384
TLDA_MLP_MAX_WIDTH = 1024

EXPORTED = ("tlda_create", "tlda_destroy", "tlda_status_str", "tlda_last_error",
            "tlda_update_moments", "tlda_whiten_batch", "tlda_cp_step", "tlda_whiten_cp_step",
            "tlda_whiten_cp_step_noalloc",
            "tlda_unwhiten",
            "tlda_infer_doc_topics", "tlda_infer_doc_topics_whitened", "tlda_stage_batch", "tlda_stage_batch_u16", "tlda_get_stats",
            "tlda_get_whitening", "tlda_set_whitening", "tlda_rebase_phi",
            "tlda_set_timing_events",
            "tlda_save_state", "tlda_load_state",
            "tlda_mlp_param_count", "tlda_mlp_create", "tlda_mlp_destroy", "tlda_mlp_last_error",
            "tlda_mlp_set_params", "tlda_mlp_get_params", "tlda_mlp_forward",
            "tlda_mlp_gradients", "tlda_mlp_train_step", "tlda_infer_doc_topics_mlp",
            "tlda_multi_create", "tlda_multi_destroy", "tlda_multi_last_error",
            "tlda_multi_set_blocks", "tlda_multi_get_blocks", "tlda_multi_set_tile",
            "tlda_multi_get_tile", "tlda_multi_step",
            "tlda_multi_autotune", "tlda_graph_capture", "tlda_graph_capture_steps",
            "tlda_graph_launch",
            "tlda_graph_destroy")


class tlda_config(ctypes.Structure):
    _fields_ = [("V", ctypes.c_int32), ("K", ctypes.c_int32), ("D", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("alpha0", ctypes.c_double),
                ("theta", ctypes.c_double), ("eig_iters", ctypes.c_int32),
                ("eig_block", ctypes.c_int32), ("eig_seed", ctypes.c_uint64),
                ("eig_warm_iters", ctypes.c_int32)]


class tlda_csr_batch(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("slot", ctypes.c_int32),
                ("first_doc", ctypes.c_int64)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libtlda.so is not built at {path}; run "
                          "`python -m paper_2511_07809_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    sig = {
        "tlda_create": ([ctypes.POINTER(tlda_config), vp, ctypes.POINTER(vp)], i32),
        "tlda_destroy": ([vp], None),
        "tlda_status_str": ([i32], ctypes.c_char_p),
        "tlda_last_error": ([vp], ctypes.c_char_p),
        "tlda_update_moments": ([vp, ctypes.POINTER(tlda_csr_batch), u32], i32),
        "tlda_whiten_batch": ([vp, ctypes.POINTER(tlda_csr_batch), vp, vp], i32),
        "tlda_cp_step": ([vp, vp, i32, vp, ctypes.c_float, vp, vp], i32),
        "tlda_whiten_cp_step": ([vp, ctypes.POINTER(tlda_csr_batch), ctypes.c_float, vp, vp, vp,
                                 vp], i32),
        "tlda_whiten_cp_step_noalloc": ([vp, ctypes.POINTER(tlda_csr_batch), ctypes.c_float, vp,
                                         vp, vp, vp], i32),
        "tlda_unwhiten": ([vp, vp, vp, vp, vp, u32], i32),
        "tlda_infer_doc_topics": ([vp, ctypes.POINTER(tlda_csr_batch), vp, i32, ctypes.c_float,
                                   vp], i32),
        "tlda_infer_doc_topics_whitened": ([vp, vp, i32, vp, i32, ctypes.c_float, vp], i32),
        "tlda_stage_batch": ([vp, ctypes.POINTER(tlda_csr_batch), i32,
                              ctypes.POINTER(tlda_csr_batch)], i32),
        "tlda_stage_batch_u16": ([vp, vp, i32, ctypes.POINTER(tlda_csr_batch)], i32),
        "tlda_get_stats": ([vp, vp, vp, vp], i32),
        "tlda_get_whitening": ([vp, vp, vp, vp], i32),
        "tlda_set_whitening": ([vp, vp, vp], i32),
        "tlda_rebase_phi": ([vp, vp], i32),
        "tlda_set_timing_events": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32], i32),
        "tlda_save_state": ([vp, vp, ctypes.POINTER(ctypes.c_size_t)], i32),
        "tlda_mlp_param_count": ([i32, i32, i32], ctypes.c_int64),
        "tlda_multi_create": ([i32, ctypes.POINTER(vp), ctypes.POINTER(tlda_csr_batch),
                               ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_float), vp,
                               ctypes.POINTER(vp)], i32),
        "tlda_multi_destroy": ([vp], None),
        "tlda_multi_last_error": ([vp], ctypes.c_char_p),
        "tlda_multi_set_blocks": ([vp, i32], i32),
        "tlda_multi_get_blocks": ([vp, ctypes.POINTER(i32)], i32),
        "tlda_multi_set_tile": ([vp, i32, i32], i32),
        "tlda_multi_get_tile": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "tlda_multi_step": ([vp], i32),
        "tlda_multi_autotune": ([vp, i32, ctypes.POINTER(i32)], i32),
        "tlda_graph_capture": ([ctypes.POINTER(vp), i32, ctypes.POINTER(vp)], i32),
        "tlda_graph_capture_steps": ([vp, vp, i32, ctypes.c_float, vp, ctypes.POINTER(vp)], i32),
        "tlda_graph_launch": ([vp], i32),
        "tlda_graph_destroy": ([vp], None),
        "tlda_mlp_create": ([i32, i32, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "tlda_mlp_destroy": ([vp], None),
        "tlda_mlp_last_error": ([vp], ctypes.c_char_p),
        "tlda_mlp_set_params": ([vp, vp], i32),
        "tlda_mlp_get_params": ([vp, vp], i32),
        "tlda_mlp_forward": ([vp, vp, ctypes.c_int64, vp], i32),
        "tlda_mlp_gradients": ([vp, vp, vp, i32, vp, vp], i32),
        "tlda_mlp_train_step": ([vp, vp, vp, i32, ctypes.c_float, vp], i32),
        "tlda_infer_doc_topics_mlp": ([vp, vp, vp, i32, vp, ctypes.c_float, i32, i32, vp, vp],
                                      i32),
        "tlda_load_state": ([vp, vp, ctypes.c_size_t], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_LIB = load_library()


class TldaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """Owns a tlda_ctx* created on a HIP stream."""

    def __init__(self, handle: int, cfg: tlda_config, stream: torch.cuda.Stream):
        self.handle = handle
        self.cfg = cfg
        self.stream = stream

    @property
    def V(self) -> int:
        return self.cfg.V

    @property
    def K(self) -> int:
        return self.cfg.K

    @property
    def D(self) -> int:
        return self.cfg.D

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _LIB is not None:          # (None while the interpreter shuts down)
            _LIB.tlda_destroy(h)


def _check(ctx: Optional[Context], status: int) -> None:
    if status != TLDA_OK:
        msg = _LIB.tlda_last_error(ctx.handle if ctx else None) or b""
        raise TldaError(status, msg.decode() or _LIB.tlda_status_str(status).decode())


class CsrBatch:
    """A CSR batch whose arrays live in device (or pinned host) memory."""

    def __init__(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor,
                 slot: int = -1, first_doc: int = 0):
        assert row_ptr.dtype == torch.int32 and col_idx.dtype == torch.int32
        assert val.dtype == torch.float32
        assert row_ptr.is_contiguous() and col_idx.is_contiguous() and val.is_contiguous()
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val
        self.n_rows = row_ptr.numel() - 1
        self.nnz = col_idx.numel()
        self.slot = slot
        self.first_doc = int(first_doc)

    @classmethod
    def from_numpy(cls, row_ptr, col_idx, val, device="cuda", pin=False, first_doc=0):
        rp = torch.from_numpy(row_ptr.astype("int32", copy=False))
        ci = torch.from_numpy(col_idx.astype("int32", copy=False))
        va = torch.from_numpy(val.astype("float32", copy=False))
        if pin:
            return cls(rp.pin_memory(), ci.pin_memory(), va.pin_memory(), first_doc=first_doc)
        return cls(rp.to(device), ci.to(device), va.to(device), first_doc=first_doc)

    def struct(self) -> tlda_csr_batch:
        return tlda_csr_batch(self.n_rows, self.nnz, self.row_ptr.data_ptr(),
                              self.col_idx.data_ptr() if self.nnz else None,
                              self.val.data_ptr() if self.nnz else None, self.slot,
                              self.first_doc)


class tlda_csr_batch_u16(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("first_doc", ctypes.c_int64)]


class CsrBatchU16:
    """A CSR batch in the compact staging format (pinned host memory):
    int32 row pointers, 16-bit column indices and counts."""

    def __init__(self, row_ptr, col_idx, val, first_doc: int = 0):
        import numpy as np
        self.first_doc = int(first_doc)
        assert col_idx.size == 0 or int(col_idx.max()) < 65536
        assert val.size == 0 or (float(val.min()) >= 1 and float(val.max()) <= 65535)
        self.n_rows = int(row_ptr.shape[0]) - 1
        self.nnz = int(col_idx.shape[0])
        self.row_ptr = torch.from_numpy(row_ptr.astype("int32")).pin_memory()
        self.col_idx = torch.from_numpy(col_idx.astype(np.uint16).view(np.int16)).pin_memory()
        self.val = torch.from_numpy(val.astype(np.uint16).view(np.int16)).pin_memory()

    def struct(self) -> tlda_csr_batch_u16:
        return tlda_csr_batch_u16(self.n_rows, self.nnz, self.row_ptr.data_ptr(),
                                  self.col_idx.data_ptr() if self.nnz else None,
                                  self.val.data_ptr() if self.nnz else None, self.first_doc)


class _StagedBatch(CsrBatch):
    def __init__(self, s: tlda_csr_batch, owner: CsrBatch):
        self._s = s
        self._owner = owner          # keeps the pinned host arrays alive
        self.n_rows, self.nnz, self.slot, self.first_doc = s.n_rows, s.nnz, s.slot, s.first_doc

    def struct(self) -> tlda_csr_batch:
        return self._s


# ---------------------------------------------------------------------------
# The C ABI, one Python function per C function.
# ---------------------------------------------------------------------------
def tlda_create(V: int, K: int, D: int, alpha0: float, theta: float = 0.0, *,
                validate_csr: bool = False, bf16: bool = False, classic: bool = False,
                eig_iters: int = 0, eig_warm_iters: int = 0,
                eig_block: int = 0, eig_seed: int = 0,
                stream: Optional[torch.cuda.Stream] = None) -> Context:
    if not torch.cuda.is_available():
        raise RuntimeError("libtlda needs a ROCm GPU; none is visible")
    stream = stream or torch.cuda.current_stream()
    flags = ((TLDA_VALIDATE_CSR if validate_csr else 0) | (TLDA_BF16 if bf16 else 0)
             | (TLDA_CLASSIC if classic else 0))
    cfg = tlda_config(V, K, D, flags, float(alpha0), float(theta), eig_iters, eig_block, eig_seed,
                      eig_warm_iters)
    h = ctypes.c_void_p()
    _check(None, _LIB.tlda_create(ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream),
                                  ctypes.byref(h)))
    return Context(h.value, cfg, stream)


def tlda_update_moments(ctx: Context, batch: Optional[CsrBatch], flags: int = 0) -> None:
    s = batch.struct() if batch is not None else None
    _check(ctx, _LIB.tlda_update_moments(ctx.handle, ctypes.byref(s) if s else None, flags))


def tlda_whiten_batch(ctx: Context, batch: CsrBatch, X: Optional[torch.Tensor] = None,
                      n_kept: Optional[torch.Tensor] = None):
    if X is None:
        X = torch.empty((batch.n_rows, ctx.D), dtype=torch.float32, device="cuda")
    if n_kept is None:
        n_kept = torch.empty(1, dtype=torch.int32, device="cuda")
    assert X.dtype == torch.float32 and X.is_contiguous() and X.numel() >= batch.n_rows * ctx.D
    s = batch.struct()
    _check(ctx, _LIB.tlda_whiten_batch(ctx.handle, ctypes.byref(s), _ptr(X), _ptr(n_kept)))
    return X, n_kept


def tlda_cp_step(ctx: Context, X: torch.Tensor, n_rows: int, n_kept: Optional[torch.Tensor],
                 beta: float, Phi: torch.Tensor, grad: Optional[torch.Tensor] = None) -> None:
    assert Phi.dtype == torch.float32 and Phi.is_contiguous() and Phi.numel() == ctx.D * ctx.K
    assert X.dtype == torch.float32 and X.is_contiguous() and X.numel() >= n_rows * ctx.D
    _check(ctx, _LIB.tlda_cp_step(ctx.handle, _ptr(X), n_rows, _ptr(n_kept), float(beta),
                                  _ptr(Phi), _ptr(grad)))


def tlda_whiten_cp_step(ctx: Context, batch: CsrBatch, beta: float, Phi: torch.Tensor,
                        grad: Optional[torch.Tensor] = None, X_out: Optional[torch.Tensor] = None,
                        n_kept: Optional[torch.Tensor] = None) -> None:
    assert Phi.dtype == torch.float32 and Phi.is_contiguous() and Phi.numel() == ctx.D * ctx.K
    if X_out is not None:
        assert X_out.dtype == torch.float32 and X_out.numel() >= batch.n_rows * ctx.D
    s = batch.struct()
    _check(ctx, _LIB.tlda_whiten_cp_step(ctx.handle, ctypes.byref(s), float(beta), _ptr(Phi),
                                         _ptr(grad), _ptr(X_out), _ptr(n_kept)))


def tlda_whiten_cp_step_noalloc(ctx: Context, batch: CsrBatch, beta: float, Phi: torch.Tensor,
                                grad: Optional[torch.Tensor] = None,
                                X_out: Optional[torch.Tensor] = None,
                                n_kept: Optional[torch.Tensor] = None) -> None:
    assert Phi.dtype == torch.float32 and Phi.is_contiguous() and Phi.numel() == ctx.D * ctx.K
    if X_out is not None:
        assert X_out.dtype == torch.float32 and X_out.numel() >= batch.n_rows * ctx.D
    s = batch.struct()
    _check(ctx, _LIB.tlda_whiten_cp_step_noalloc(ctx.handle, ctypes.byref(s), float(beta),
                                                 _ptr(Phi), _ptr(grad), _ptr(X_out),
                                                 _ptr(n_kept)))


def tlda_unwhiten(ctx: Context, Phi: torch.Tensor, flags: int = 0):
    mu = torch.empty((ctx.V, ctx.K), dtype=torch.float64, device="cuda")
    alpha = torch.empty(ctx.K, dtype=torch.float64, device="cuda")
    lam = torch.empty(ctx.K, dtype=torch.float64, device="cuda")
    _check(ctx, _LIB.tlda_unwhiten(ctx.handle, _ptr(Phi), _ptr(mu), _ptr(alpha), _ptr(lam),
                                   flags))
    return mu, alpha, lam


def tlda_infer_doc_topics(ctx: Context, batch: CsrBatch, mu: torch.Tensor, max_iter: int,
                          tol: float = 0.0, theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    if theta is None:
        theta = torch.empty((batch.n_rows, ctx.K), dtype=torch.float32, device="cuda")
    assert mu.dtype == torch.float64 and mu.is_contiguous()
    s = batch.struct()
    _check(ctx, _LIB.tlda_infer_doc_topics(ctx.handle, ctypes.byref(s), _ptr(mu), max_iter,
                                           float(tol), _ptr(theta)))
    return theta


def tlda_infer_doc_topics_whitened(ctx: Context, X: torch.Tensor, n_rows: int, mu: torch.Tensor,
                                   max_iter: int, tol: float = 0.0,
                                   theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    if theta is None:
        theta = torch.empty((n_rows, ctx.K), dtype=torch.float32, device="cuda")
    assert mu.dtype == torch.float64 and mu.is_contiguous()
    _check(ctx, _LIB.tlda_infer_doc_topics_whitened(ctx.handle, _ptr(X), n_rows, _ptr(mu),
                                                    max_iter, float(tol), _ptr(theta)))
    return theta


def tlda_stage_batch(ctx: Context, host_batch: CsrBatch, slot: int) -> CsrBatch:
    h = host_batch.struct()
    out = tlda_csr_batch()
    _check(ctx, _LIB.tlda_stage_batch(ctx.handle, ctypes.byref(h), slot, ctypes.byref(out)))
    return _StagedBatch(out, host_batch)


def tlda_stage_batch_u16(ctx: Context, host_batch: CsrBatchU16, slot: int) -> CsrBatch:
    h = host_batch.struct()
    out = tlda_csr_batch()
    _check(ctx, _LIB.tlda_stage_batch_u16(ctx.handle, ctypes.byref(h), slot, ctypes.byref(out)))
    return _StagedBatch(out, host_batch)


def tlda_get_stats(ctx: Context):
    import numpy as np
    N = ctypes.c_int64()
    sk = ctypes.c_int64()
    tot = np.zeros(ctx.V, dtype=np.int64)
    _check(ctx, _LIB.tlda_get_stats(ctx.handle, ctypes.addressof(N), ctypes.addressof(sk),
                                    tot.ctypes.data))
    return int(N.value), int(sk.value), tot


def tlda_get_whitening(ctx: Context):
    import numpy as np
    W = np.zeros((ctx.V, ctx.D))
    eig = np.zeros(ctx.D)
    m = np.zeros(ctx.V)
    _check(ctx, _LIB.tlda_get_whitening(ctx.handle, W.ctypes.data, eig.ctypes.data, m.ctypes.data))
    return W, eig, m


def tlda_set_whitening(ctx: Context, W, M1) -> None:
    import numpy as np
    W = np.ascontiguousarray(W, dtype=np.float64)
    M1 = np.ascontiguousarray(M1, dtype=np.float64)
    assert W.shape == (ctx.V, ctx.D) and M1.shape == (ctx.V,)
    _check(ctx, _LIB.tlda_set_whitening(ctx.handle, W.ctypes.data, M1.ctypes.data))


def tlda_rebase_phi(ctx: Context, Phi: torch.Tensor) -> None:
    assert Phi.dtype == torch.float32 and Phi.is_contiguous() and Phi.numel() == ctx.D * ctx.K
    _check(ctx, _LIB.tlda_rebase_phi(ctx.handle, _ptr(Phi)))


def tlda_set_timing_events(ctx: Context, starts, stops) -> None:
    """starts/stops: equal-length lists of torch.cuda.Event(enable_timing=True),
    each already recorded once (torch creates an event on its first record).
    Empty lists turn the hook off.  The events must outlive the hook."""
    assert len(starts) == len(stops)
    n = len(starts)
    arr = ctypes.c_void_p * max(n, 1)
    a = arr(*[ctypes.c_void_p(e.cuda_event) for e in starts])
    b = arr(*[ctypes.c_void_p(e.cuda_event) for e in stops])
    ctx._timing_refs = (list(starts), list(stops))
    _check(ctx, _LIB.tlda_set_timing_events(ctx.handle, a, b, n))


def tlda_save_state(ctx: Context) -> bytes:
    n = ctypes.c_size_t(0)
    _check(ctx, _LIB.tlda_save_state(ctx.handle, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(ctx, _LIB.tlda_save_state(ctx.handle, buf, ctypes.byref(n)))
    return buf.raw[:n.value]


def tlda_load_state(ctx: Context, data: bytes) -> None:
    buf = ctypes.create_string_buffer(data, len(data))
    _check(ctx, _LIB.tlda_load_state(ctx.handle, buf, len(data)))


# ---------------------------------------------------------------------------
# Document-topic encoder
# ---------------------------------------------------------------------------
class Mlp:
    """Owns a tlda_mlp* created on a HIP stream."""

    def __init__(self, handle: int, d_in: int, hidden: int, k_out: int, max_batch: int,
                 stream: torch.cuda.Stream):
        self.handle = handle
        self.d_in, self.hidden, self.k_out, self.max_batch = d_in, hidden, k_out, max_batch
        self.stream = stream
        self.n_params = int(_LIB.tlda_mlp_param_count(d_in, hidden, k_out))

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.tlda_mlp_destroy(self.handle)
            self.handle = None


def _check_mlp(m: Mlp, status: int) -> None:
    if status != TLDA_OK:
        msg = _LIB.tlda_mlp_last_error(m.handle) or b""
        raise TldaError(status, msg.decode() or _LIB.tlda_status_str(status).decode())


def tlda_mlp_param_count(d_in: int, hidden: int, k_out: int) -> int:
    return int(_LIB.tlda_mlp_param_count(d_in, hidden, k_out))


def tlda_mlp_create(d_in: int, hidden: int, k_out: int, max_batch: int,
                    stream: Optional[torch.cuda.Stream] = None) -> Mlp:
    if not torch.cuda.is_available():
        raise RuntimeError("libtlda needs a ROCm GPU; none is visible")
    stream = stream or torch.cuda.current_stream()
    h = ctypes.c_void_p()
    st = _LIB.tlda_mlp_create(d_in, hidden, k_out, max_batch, ctypes.c_void_p(stream.cuda_stream),
                              ctypes.byref(h))
    if st != TLDA_OK:
        raise TldaError(st, _LIB.tlda_status_str(st).decode())
    return Mlp(h.value, d_in, hidden, k_out, max_batch, stream)


def tlda_mlp_set_params(m: Mlp, params) -> None:
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.shape == (m.n_params,)
    _check_mlp(m, _LIB.tlda_mlp_set_params(m.handle, p.ctypes.data))


def tlda_mlp_get_params(m: Mlp):
    import numpy as np
    p = np.empty(m.n_params, dtype=np.float32)
    _check_mlp(m, _LIB.tlda_mlp_get_params(m.handle, p.ctypes.data))
    return p


def tlda_mlp_forward(m: Mlp, X: torch.Tensor, theta: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = X.shape[0]
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[1] == m.d_in
    if theta is None:
        theta = torch.empty((n, m.k_out), dtype=torch.float32, device="cuda")
    _check_mlp(m, _LIB.tlda_mlp_forward(m.handle, _ptr(X), n, _ptr(theta)))
    return theta


def tlda_mlp_gradients(m: Mlp, X: torch.Tensor, T: torch.Tensor):
    n = X.shape[0]
    assert X.is_contiguous() and T.is_contiguous() and T.shape == (n, m.k_out)
    g = torch.empty(m.n_params, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check_mlp(m, _LIB.tlda_mlp_gradients(m.handle, _ptr(X), _ptr(T), n, _ptr(g), _ptr(loss)))
    return g, loss


def tlda_mlp_train_step(m: Mlp, X: torch.Tensor, T: torch.Tensor, lr: float,
                        loss: Optional[torch.Tensor] = None) -> None:
    n = X.shape[0]
    assert X.is_contiguous() and T.is_contiguous() and T.shape == (n, m.k_out)
    _check_mlp(m, _LIB.tlda_mlp_train_step(m.handle, _ptr(X), _ptr(T), n, float(lr), _ptr(loss)))


def tlda_infer_doc_topics_mlp(ctx: Context, m: Optional[Mlp], X: torch.Tensor, n_rows: int,
                              mu: torch.Tensor, gap_tol: float, max_iter: int,
                              theta: Optional[torch.Tensor] = None,
                              n_stepped: Optional[torch.Tensor] = None, min_steps: int = 0):
    if theta is None:
        theta = torch.empty((n_rows, ctx.K), dtype=torch.float32, device="cuda")
    if n_stepped is None:
        n_stepped = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert mu.dtype == torch.float64 and mu.is_contiguous()
    _check(ctx, _LIB.tlda_infer_doc_topics_mlp(ctx.handle, m.handle if m is not None else None,
                                               _ptr(X), n_rows, _ptr(mu), float(gap_tol),
                                               min_steps, max_iter, _ptr(theta),
                                               _ptr(n_stepped)))
    return theta, n_stepped


# ---------------------------------------------------------------------------
# Batched time slices
# ---------------------------------------------------------------------------
class Multi:
    """Owns a tlda_multi* (a step plan over several slices).  Keeps the
    contexts, batches and Phi tensors it refers to alive."""

    def __init__(self, handle: int, refs):
        self.handle = handle
        self._refs = refs

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.tlda_multi_destroy(self.handle)
            self.handle = None


class Graph:
    def __init__(self, handle: int, refs):
        self.handle = handle
        self._refs = refs

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.tlda_graph_destroy(self.handle)
            self.handle = None


def _check_multi(p: Multi, status: int) -> None:
    if status != TLDA_OK:
        msg = _LIB.tlda_multi_last_error(p.handle) or b""
        raise TldaError(status, msg.decode() or _LIB.tlda_status_str(status).decode())


def tlda_multi_create(ctxs, batches, Phis, betas, n_kept: Optional[torch.Tensor] = None) -> Multi:
    n = len(ctxs)
    assert len(batches) == n and len(Phis) == n and len(betas) == n
    c_ctx = (ctypes.c_void_p * n)(*[c.handle for c in ctxs])
    c_b = (tlda_csr_batch * n)(*[b.struct() for b in batches])
    c_p = (ctypes.c_void_p * n)(*[P.data_ptr() for P in Phis])
    c_beta = (ctypes.c_float * n)(*[float(x) for x in betas])
    h = ctypes.c_void_p()
    st = _LIB.tlda_multi_create(n, c_ctx, c_b, c_p, c_beta, _ptr(n_kept), ctypes.byref(h))
    if st != TLDA_OK:
        raise TldaError(st, _LIB.tlda_status_str(st).decode())
    return Multi(h.value, (list(ctxs), list(batches), list(Phis), n_kept))


def tlda_multi_set_blocks(p: Multi, total_blocks: int) -> None:
    _check_multi(p, _LIB.tlda_multi_set_blocks(p.handle, total_blocks))


def tlda_multi_get_blocks(p: Multi) -> int:
    v = ctypes.c_int32(0)
    _check_multi(p, _LIB.tlda_multi_get_blocks(p.handle, ctypes.byref(v)))
    return int(v.value)


def tlda_multi_set_tile(p: Multi, rows_per_tile: int, waves_per_block: int) -> None:
    _check_multi(p, _LIB.tlda_multi_set_tile(p.handle, rows_per_tile, waves_per_block))


def tlda_multi_get_tile(p: Multi):
    r, w = ctypes.c_int32(0), ctypes.c_int32(0)
    _check_multi(p, _LIB.tlda_multi_get_tile(p.handle, ctypes.byref(r), ctypes.byref(w)))
    return int(r.value), int(w.value)


def tlda_multi_step(p: Multi) -> None:
    _check_multi(p, _LIB.tlda_multi_step(p.handle))


def tlda_multi_autotune(p: Multi, reps: int = 3) -> int:
    v = ctypes.c_int32(0)
    _check_multi(p, _LIB.tlda_multi_autotune(p.handle, reps, ctypes.byref(v)))
    return int(v.value)


def tlda_graph_capture(plans) -> Graph:
    n = len(plans)
    arr = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    h = ctypes.c_void_p()
    st = _LIB.tlda_graph_capture(arr, n, ctypes.byref(h))
    if st != TLDA_OK:
        raise TldaError(st, _LIB.tlda_status_str(st).decode())
    return Graph(h.value, list(plans))


def tlda_graph_capture_steps(ctx: Context, batches, beta: float, Phi: torch.Tensor) -> Graph:
    """One HIP graph of len(batches) fused steps of ctx (device batches)."""
    assert Phi.dtype == torch.float32 and Phi.is_contiguous() and Phi.numel() == ctx.D * ctx.K
    n = len(batches)
    arr = (tlda_csr_batch * n)(*[b.struct() for b in batches])
    h = ctypes.c_void_p()
    _check(ctx, _LIB.tlda_graph_capture_steps(ctx.handle, arr, n, float(beta), _ptr(Phi),
                                              ctypes.byref(h)))
    return Graph(h.value, [ctx, list(batches), Phi])


def tlda_graph_launch(g: Graph) -> None:
    st = _LIB.tlda_graph_launch(g.handle)
    if st != TLDA_OK:
        raise TldaError(st, _LIB.tlda_status_str(st).decode())
