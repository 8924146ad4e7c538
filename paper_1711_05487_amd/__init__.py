"""Python binding of libcsrspmv (matrix-adaptive CSR SpMV for MI355X).

Argument marshalling only: every step of the SpMV path runs in the HIP
library, reached through its C ABI (include/csrspmv.h) with ctypes. torch
provides device memory and streams. If the library has not been built the
import of this binding fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcsrspmv.so")

F64, F32, BF16 = 0, 1, 2
STORAGE = {"f64": F64, "f32": F32, "bf16": BF16}

OPT_DELTA, OPT_PREFETCH, OPT_DECOMP, OPT_MERGE, OPT_UNROLL = 1, 2, 4, 8, 16
OPT_NAMES = {OPT_DELTA: "delta", OPT_PREFETCH: "prefetch", OPT_DECOMP: "decomp",
             OPT_MERGE: "merge", OPT_UNROLL: "unroll"}
CLS_MB, CLS_ML, CLS_IMB, CLS_CMP = 1, 2, 4, 8

SEL_PLAIN, SEL_PROFILE, SEL_LEARNED, SEL_EXHAUSTIVE, SEL_FORCED, SEL_TREE = 0, 1, 2, 3, 4, 5
SELECT = {"plain": SEL_PLAIN, "profile": SEL_PROFILE, "learned": SEL_LEARNED,
          "exhaustive": SEL_EXHAUSTIVE, "forced": SEL_FORCED, "tree": SEL_TREE}

(DEBUG_VALUES, DEBUG_CODES, DEBUG_TILE_I, DEBUG_TILE_J, DEBUG_LONG_ROWS, DEBUG_PLAN,
 DEBUG_MERGE_CODES, DEBUG_TILE_BASE, DEBUG_WINDOW_DICT, DEBUG_WINDOW_LEN,
 DEBUG_WINDOW_CODES, DEBUG_CB_ROWPTR, DEBUG_CB_COL, DEBUG_CB_VAL,
 DEBUG_MLP_BOUNDS, DEBUG_MLP_TIMES, DEBUG_MLP_RATIOS, DEBUG_IMB_SPANS,
 DEBUG_BANDWIDTH, DEBUG_WINDOW_RUNS, DEBUG_CB_ROWS, DEBUG_CB_ROWLIST_PTR) = range(22)

STATUS = ["CSR_OK", "CSR_ERR_INVALID_ARG", "CSR_ERR_INVALID_MATRIX", "CSR_ERR_OUT_OF_MEMORY",
          "CSR_ERR_DEVICE", "CSR_ERR_UNSUPPORTED", "CSR_ERR_NOT_READY"]

# Every entry point declared in include/csrspmv.h.
EXPORTS = ("csr_config_default", "csr_create", "csr_destroy", "csr_inspect", "csr_select",
           "csr_spmv", "csr_spmv_batched", "csr_status_str", "csr_last_error", "csr_query",
           "csr_debug_copy", "csr_debug_probe", "csr_triad", "csr_device_bandwidth",
           "csr_debug_triad", "csr_time_spmv", "csr_mlp_load", "csr_mlp_unload",
           "csr_mlp_forward", "csr_mlp_grad", "csr_mlp_train", "csr_mlp_normalize",
           "csr_tree_load", "csr_tree_unload", "csr_jit_compile", "csr_spmv_noalloc",
           "csr_debug_alloc", "csr_classify")


class CsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")


class Config(ctypes.Structure):
    _fields_ = [("t_ml", ctypes.c_double), ("t_imb", ctypes.c_double), ("t_mb", ctypes.c_double),
                ("long_row_factor", ctypes.c_double), ("long_row_floor", ctypes.c_int32),
                ("forced_opts", ctypes.c_int32), ("rows_per_group", ctypes.c_int32),
                ("merge_items", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("timing_calls", ctypes.c_int32), ("rows_in_flight", ctypes.c_int32),
                ("exhaustive_set", ctypes.c_int32), ("dynamic_rows", ctypes.c_int32),
                ("ml_partitions", ctypes.c_int32), ("t_ml_part", ctypes.c_double),
                ("jit_tiles", ctypes.c_int32), ("window_runs", ctypes.c_int32),
                ("remedy_map", ctypes.c_int32), ("split_row_blocks", ctypes.c_int32),
                ("ood_z", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("opts", ctypes.c_int32), ("classes", ctypes.c_int32),
                ("variant_id", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32),
                ("merge_items", ctypes.c_int32), ("delta_bits", ctypes.c_int32),
                ("n_long_rows", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("merge_slack", ctypes.c_int32), ("window_codes", ctypes.c_int32),
                ("column_blocks", ctypes.c_int32), ("dynamic_rows", ctypes.c_int32),
                ("ml_partitions", ctypes.c_int32), ("ml_parts_flagged", ctypes.c_int32),
                ("jit", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("p_csr", ctypes.c_double), ("p_mb", ctypes.c_double), ("p_ml", ctypes.c_double),
                ("p_imb", ctypes.c_double), ("p_cmp", ctypes.c_double),
                ("p_peak", ctypes.c_double), ("b_max", ctypes.c_double),
                ("t_select_ms", ctypes.c_double), ("t_prep_ms", ctypes.c_double),
                ("format_bytes", ctypes.c_double), ("ml_part_max", ctypes.c_double),
                ("feature_z_max", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Features(ctypes.Structure):
    _fields_ = [("f", ctypes.c_double * 16), ("isum", ctypes.c_int64 * 8),
                ("rows_sorted", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load libcsrspmv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1711_05487_amd.build` (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sig = {
            "csr_config_default": (None, [ctypes.POINTER(Config)]),
            "csr_create": (ctypes.c_int, [ctypes.POINTER(P), i32, i32, i64, P, P, P, i32, P]),
            "csr_destroy": (None, [P]),
            "csr_inspect": (ctypes.c_int, [P, ctypes.POINTER(Features), P]),
            "csr_select": (ctypes.c_int, [P, i32, ctypes.POINTER(Config), ctypes.POINTER(PlanInfo), P]),
            "csr_spmv": (ctypes.c_int, [P, P, P, P]),
            "csr_spmv_batched": (ctypes.c_int, [i32, P, P, P, P]),
            "csr_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "csr_last_error": (ctypes.c_char_p, []),
            "csr_query": (ctypes.c_int, [P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                         ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "csr_debug_copy": (ctypes.c_int, [P, i32, P, sz, ctypes.POINTER(sz), P]),
            "csr_triad": (ctypes.c_int, [sz, i32, ctypes.POINTER(ctypes.c_double), P]),
            "csr_device_bandwidth": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                                    ctypes.POINTER(ctypes.c_double), P]),
            "csr_debug_triad": (ctypes.c_int, [P, P, P, i64, ctypes.c_double, i32, P]),
            "csr_debug_probe": (ctypes.c_int, [P, i32, P, P, P]),
            "csr_time_spmv": (ctypes.c_int, [P, P, P, i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), ctypes.c_char_p, sz, P]),
            "csr_mlp_load": (ctypes.c_int, [P, i32, P, P]),
            "csr_mlp_unload": (ctypes.c_int, []),
            "csr_mlp_forward": (ctypes.c_int, [P, i32, P, i32, P, P]),
            "csr_mlp_grad": (ctypes.c_int, [P, i32, P, P, i32, P, P, P]),
            "csr_mlp_train": (ctypes.c_int, [P, P, P, i32, P, P, P, i32, i32, i32, ctypes.c_float,
                                             ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P]),
            "csr_mlp_normalize": (ctypes.c_int, [P, P, P, i64, P, P]),
            "csr_tree_load": (ctypes.c_int, [i32, P, P, P, P, P]),
            "csr_tree_unload": (ctypes.c_int, []),
            "csr_jit_compile": (ctypes.c_int, [i32, i32, i32, i32, i32, P, sz, ctypes.POINTER(sz)]),
            "csr_spmv_noalloc": (ctypes.c_int, [i32, i32, i64, P, P, P, P, P, P]),
            "csr_classify": (ctypes.c_int, [P, ctypes.POINTER(Config), i32, ctypes.POINTER(i32),
                                            ctypes.POINTER(i32)]),
            "csr_debug_alloc": (ctypes.c_int, [i32, i64, i64, ctypes.POINTER(i64),
                                               ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise CsrError(st, lib().csr_last_error().decode())


def _stream(stream):
    """HIP stream handle as void*: an explicit torch stream, an int, or torch's
    current stream."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def default_config() -> Config:
    c = Config()
    lib().csr_config_default(ctypes.byref(c))
    return c


def x_dtype(storage: int):
    import torch
    return torch.float64 if storage == F64 else torch.float32


class CsrMatrix:
    """Handle of a CSR matrix living in device memory owned by the library."""

    def __init__(self, row_ptr, col_idx, val, n_cols: int | None = None, storage="f64",
                 stream=None):
        import torch
        storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        dev = torch.device("cuda", torch.cuda.current_device())
        rp = torch.as_tensor(np.asarray(row_ptr) if not torch.is_tensor(row_ptr) else row_ptr,
                             dtype=torch.int32).to(dev).contiguous()
        ci = torch.as_tensor(np.asarray(col_idx) if not torch.is_tensor(col_idx) else col_idx,
                             dtype=torch.int32).to(dev).contiguous()
        va = torch.as_tensor(np.asarray(val) if not torch.is_tensor(val) else val,
                             dtype=torch.float64).to(dev).contiguous()
        n_rows = rp.numel() - 1
        if n_cols is None:
            n_cols = n_rows
        self.n_rows, self.n_cols, self.nnz, self.storage = n_rows, int(n_cols), ci.numel(), storage
        h = ctypes.c_void_p()
        _check(lib().csr_create(ctypes.byref(h), n_rows, int(n_cols), self.nnz, _ptr(rp), _ptr(ci),
                                _ptr(va), storage, _stream(stream)))
        self._h = h
        self.info = None

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().csr_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def x_dtype(self):
        return x_dtype(self.storage)

    def spmv(self, x, y=None, stream=None):
        """y = A x on the device (asynchronous on `stream`)."""
        import torch
        if y is None:
            y = torch.empty(self.n_rows, dtype=x.dtype, device=x.device)
        want = self.x_dtype()
        if x.dtype != want or y.dtype != want:
            raise TypeError(f"x and y must be {want}")
        if not (x.is_contiguous() and y.is_contiguous()):
            raise ValueError("x and y must be contiguous")
        if x.numel() < self.n_cols or y.numel() < self.n_rows:
            raise ValueError("vector too short")
        _check(lib().csr_spmv(self._h, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def select(self, mode="plain", config: Config | None = None, stream=None, **overrides) -> dict:
        cfg = config if config is not None else default_config()
        for k, v in overrides.items():
            setattr(cfg, k, v)
        info = PlanInfo()
        m = SELECT[mode] if isinstance(mode, str) else int(mode)
        _check(lib().csr_select(self._h, m, ctypes.byref(cfg), ctypes.byref(info), _stream(stream)))
        self.info = info.as_dict()
        return self.info

    def inspect(self, stream=None):
        f = Features()
        _check(lib().csr_inspect(self._h, ctypes.byref(f), _stream(stream)))
        return np.array(f.f[:], dtype=np.float64), np.array(f.isum[:], dtype=np.int64), f.rows_sorted

    def debug_copy(self, what: int, dtype, stream=None):
        need = ctypes.c_size_t(0)
        st = lib().csr_debug_copy(self._h, what, None, 0, ctypes.byref(need), _stream(stream))
        if need.value == 0:
            _check(st)
            return np.zeros(0, dtype=dtype)
        out = np.empty(need.value // np.dtype(dtype).itemsize, dtype=dtype)
        _check(lib().csr_debug_copy(self._h, what, out.ctypes.data_as(ctypes.c_void_p),
                                    need.value, None, _stream(stream)))
        return out

    def time_spmv(self, x, y, calls: int, stream=None):
        """(dominant-kernel ms, whole-call ms, kernel name) averaged over
        `calls` SpMVs, from HIP events on the launch stream."""
        k, c = ctypes.c_double(), ctypes.c_double()
        name = ctypes.create_string_buffer(128)
        _check(lib().csr_time_spmv(self._h, _ptr(x), _ptr(y), calls, ctypes.byref(k),
                                   ctypes.byref(c), name, 128, _stream(stream)))
        return k.value, c.value, name.value.decode()

    def probe(self, which: int, x, y=None, stream=None):
        """Run the P_ML (1) or P_CMP (2) micro-benchmark kernel on x."""
        import torch
        if y is None:
            y = torch.empty(self.n_rows, dtype=x.dtype, device=x.device)
        _check(lib().csr_debug_probe(self._h, which, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def query(self):
        a, b, d, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        n = ctypes.c_int64()
        _check(lib().csr_query(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n),
                               ctypes.byref(d), ctypes.byref(e)))
        return {"n_rows": a.value, "n_cols": b.value, "nnz": n.value, "storage": d.value,
                "rows_sorted": e.value}


def spmv_noalloc(n_rows: int, n_cols: int, row_ptr, col_idx, val, x, y, stream=None):
    """y = A x on device CSR tensors (int32 row_ptr/col_idx, float64 val, x,
    y) without a handle and without allocating (csr_spmv_noalloc)."""
    _check(lib().csr_spmv_noalloc(n_rows, n_cols, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
                                  _ptr(val), _ptr(x), _ptr(y), _stream(stream)))
    return y


def spmv_batched(mats, xs, ys, stream=None):
    n = len(mats)
    hA = (ctypes.c_void_p * n)(*[m.handle for m in mats])
    hx = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    hy = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
    _check(lib().csr_spmv_batched(n, hA, hx, hy, _stream(stream)))


def triad(bytes_per_array: int = 1 << 30, reps: int = 5, stream=None) -> float:
    """Sustained triad bandwidth in bytes/s (B_max probe)."""
    out = ctypes.c_double()
    _check(lib().csr_triad(bytes_per_array, reps, ctypes.byref(out), _stream(stream)))
    return out.value


def classify(bounds, has_long_rows: bool, config: Config | None = None, **overrides):
    """(classes, opts) of the profile-guided rule on bounds = (P_CSR, P_MB,
    P_ML, P_IMB, P_CMP, P_peak), as csr_select('profile') decides them."""
    cfg = config if config is not None else default_config()
    for k, v in overrides.items():
        setattr(cfg, k, v)
    p = np.ascontiguousarray(bounds, dtype=np.float64)
    if p.shape != (6,):
        raise ValueError("six bounds")
    c, o = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().csr_classify(p.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cfg),
                              1 if has_long_rows else 0, ctypes.byref(c), ctypes.byref(o)))
    return c.value, o.value


def debug_alloc(arm: bool = False, fail_from: int = 0, fail_count: int = 0):
    """(live device buffers, live bytes, allocation attempts since the last
    arming) of the library; with arm=True then re-arm the failure injector so
    that attempts fail_from .. fail_from + fail_count - 1 from now fail."""
    b, n, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().csr_debug_alloc(1 if arm else 0, fail_from, fail_count, ctypes.byref(b),
                                 ctypes.byref(n), ctypes.byref(a)))
    return b.value, n.value, a.value


def device_bandwidth(stream=None):
    """(HBM, cache) triad bandwidths in bytes/s that PROFILE takes B_max from."""
    h, c = ctypes.c_double(), ctypes.c_double()
    _check(lib().csr_device_bandwidth(ctypes.byref(h), ctypes.byref(c), _stream(stream)))
    return h.value, c.value


def debug_triad(a, b, c, scalar: float, streaming: bool, stream=None):
    """One pass of the B_max triad kernel: a = b + scalar * c (FP64 tensors)."""
    _check(lib().csr_debug_triad(_ptr(a), _ptr(b), _ptr(c), a.numel(), float(scalar),
                                 1 if streaming else 0, _stream(stream)))
    return a


# ---------------------------------------------------------------------------
# Learned selector (MLP kernels in the library)
# ---------------------------------------------------------------------------

def mlp_load(params: np.ndarray, K: int, mu: np.ndarray, sigma: np.ndarray):
    """Install a trained model on the current device for select("learned")."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    _check(lib().csr_mlp_load(p.ctypes.data_as(ctypes.c_void_p), K,
                              m.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p)))


def mlp_unload():
    _check(lib().csr_mlp_unload())


def tree_load(tree: dict):
    """Install a decision tree (flat arrays feature, threshold, left, right,
    value) for select("tree")."""
    n = len(tree["feature"])
    arr = {k: np.ascontiguousarray(tree[k], dtype=np.float64 if k == "threshold" else np.int32)
           for k in ("feature", "threshold", "left", "right", "value")}
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().csr_tree_load(n, vp(arr["feature"]), vp(arr["threshold"]), vp(arr["left"]),
                               vp(arr["right"]), vp(arr["value"])))


def tree_unload():
    _check(lib().csr_tree_unload())


def mlp_forward(params, K, X, stream=None):
    import torch
    B = X.shape[0]
    logits = torch.empty((B, K), dtype=torch.float32, device=X.device)
    _check(lib().csr_mlp_forward(_ptr(params), K, _ptr(X), B, _ptr(logits), _stream(stream)))
    return logits


def mlp_grad(params, K, X, labels, stream=None):
    import torch
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().csr_mlp_grad(_ptr(params), K, _ptr(X), _ptr(labels), X.shape[0], _ptr(g),
                              _ptr(loss), _stream(stream)))
    return g, loss


def mlp_train(params, m, v, K, X, labels, order, B, t0=0, lr=1e-3, betas=(0.9, 0.999),
              eps=1e-8, stream=None):
    """Adam steps over the batches listed in `order` (steps*B row indices);
    params, m, v are updated in place. Returns the per-step losses."""
    import torch
    steps = order.numel() // B
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device=X.device)
    _check(lib().csr_mlp_train(_ptr(params), _ptr(m), _ptr(v), K, _ptr(X), _ptr(labels),
                               _ptr(order), B, steps, t0, lr, betas[0], betas[1], eps,
                               _ptr(losses), _stream(stream)))
    return losses[:steps]


def mlp_normalize(F, mu, sigma, stream=None):
    import torch
    out = torch.empty(F.shape, dtype=torch.float32, device=F.device)
    _check(lib().csr_mlp_normalize(_ptr(F), _ptr(mu), _ptr(sigma), F.shape[0], _ptr(out),
                                   _stream(stream)))
    return out


STORAGES = {"f64": 0, "f32": 1, "bf16": 2}


def jit_compile(storage="f64", merge_items=768, index_mode=0, streaming=True,
                row_aligned=True) -> bytes:
    """Compile the merge-path kernel for a tile size (run-time specialization,
    csr_jit_compile; needs no GPU) and return its code object."""
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    need = ctypes.c_size_t(0)
    args = (st, merge_items, index_mode, int(streaming), int(row_aligned))
    _check(lib().csr_jit_compile(*args, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().csr_jit_compile(*args, ctypes.cast(buf, ctypes.c_void_p), need.value, None))
    return buf.raw
