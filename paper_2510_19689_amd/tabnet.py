"""Python binding of libtabnet (include/tabnet.h): argument marshalling only.

Every step of the forward runs in the HIP library; this module resolves pointers and
streams from torch tensors and turns status codes into exceptions.  There is no other
execution path: if libtabnet.so is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TABNET_LIB") or os.path.join(HERE, "libtabnet.so")
# the product library plus the host-only test hooks (include/tabnet_internal.h)
TEST_LIB_PATH = os.path.join(HERE, "libtabnet_test.so")

OK, E_INVALID, E_OOM, E_HIP, E_IO, E_ADMISSION, E_TIMEOUT, E_STOPPED, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
FP32, BF16, FP8_E4M3, INT8, MXFP8, MXFP4, MXFP6, MXFP8_E5M2, MXFP6_E3M2, FP8_WEIGHTS = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3, "int8": INT8, "mxfp8": MXFP8, "mxfp4": MXFP4,
              "mxfp6": MXFP6, "mxfp8_e5m2": MXFP8_E5M2, "mxfp6_e3m2": MXFP6_E3M2, "fp8w": FP8_WEIGHTS}


class TabNetError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("n_d", ctypes.c_int32), ("n_a", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_shared", ctypes.c_int32),
                ("n_indep", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("bn_eps", ctypes.c_double)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_rows_per_launch", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("with_step_masks", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("mask_stats_window", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "admitted", "completed", "rejected",
                                                "cancelled", "rows_completed", "launches")] + \
               [(n, ctypes.c_double) for n in ("p50_us", "p99_us", "p999_us", "max_us", "mean_us",
                                                "rows_per_s", "mean_rows_per_launch")] + \
               [("inflight_bytes", ctypes.c_uint64), ("peak_inflight_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_test_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libtabnet.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _lib = _open(LIB_PATH)
    return _lib


def test_lib() -> ctypes.CDLL:
    """The test library (libtabnet.so's code plus the host-only hooks of
    include/tabnet_internal.h): for tests only."""
    global _test_lib
    if _test_lib is None:
        L = _open(TEST_LIB_PATH)
        _declare_hooks(L)
        _test_lib = L
    return _test_lib


def _open(path: str) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{os.path.basename(path)} not found at {path}; build it with "
                           "`python -m paper_2510_19689_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.tabnet_load.argtypes = [ctypes.c_char_p, i32, i32, ctypes.POINTER(vp)]
    L.tabnet_load.restype = i32
    L.tabnet_get_config.argtypes = [vp, ctypes.POINTER(Config)]
    L.tabnet_get_config.restype = i32
    L.tabnet_get_precision.argtypes = [vp]
    L.tabnet_get_precision.restype = i32
    L.tabnet_forward.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.tabnet_forward.restype = i32
    L.tabnet_set_embeddings.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    L.tabnet_set_embeddings.restype = i32
    L.tabnet_forward_raw.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.tabnet_forward_raw.restype = i32
    L.tabnet_free.argtypes = [vp]
    L.tabnet_free.restype = None
    L.tabnet_last_error.argtypes = []
    L.tabnet_last_error.restype = ctypes.c_char_p
    L.tabnet_abi_version.restype = i32
    L.tabnet_serve_start.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ServeOpts), ctypes.POINTER(vp)]
    L.tabnet_serve_start.restype = i32
    L.tabnet_serve_submit.argtypes = [vp, i32, vp, i64, vp, vp, vp, i64, ctypes.POINTER(ctypes.c_uint64)]
    L.tabnet_serve_submit.restype = i32
    L.tabnet_serve_wait.argtypes = [vp, ctypes.c_uint64, i64]
    L.tabnet_serve_wait.restype = i32
    L.tabnet_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.tabnet_serve_poll.restype = i32
    L.tabnet_serve_get_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    L.tabnet_serve_get_stats.restype = i32
    L.tabnet_serve_get_model_stats.argtypes = [vp, i32, ctypes.POINTER(ServeStats)]
    L.tabnet_serve_get_model_stats.restype = i32
    L.tabnet_serve_reset_stats.argtypes = [vp]
    L.tabnet_serve_reset_stats.restype = i32
    L.tabnet_serve_mask_stats.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i64)]
    L.tabnet_serve_mask_stats.restype = i32
    L.tabnet_mask_stats_workspace_bytes.argtypes = [i64, ctypes.c_int32]
    L.tabnet_mask_stats_workspace_bytes.restype = ctypes.c_size_t
    L.tabnet_mask_stats.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp, ctypes.c_size_t, vp]
    L.tabnet_mask_stats.restype = i32
    L.tabnet_mask_stats_noalloc_max_bytes.argtypes = []
    L.tabnet_mask_stats_noalloc_max_bytes.restype = ctypes.c_size_t
    L.tabnet_mask_stats_noalloc.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp]
    L.tabnet_mask_stats_noalloc.restype = i32
    L.tabnet_serve_now_ns.argtypes = []
    L.tabnet_serve_now_ns.restype = i64
    L.tabnet_serve_stop.argtypes = [vp]
    L.tabnet_serve_stop.restype = i32
    return L


def _declare_hooks(L) -> None:
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.tabnet_hook_bf16_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_bf16_bits.restype = ctypes.c_uint16
    L.tabnet_hook_e4m3_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_e4m3_bits.restype = ctypes.c_uint8
    L.tabnet_hook_e2m1_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_e2m1_bits.restype = ctypes.c_uint8
    L.tabnet_hook_e2m3_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_e2m3_bits.restype = ctypes.c_uint8
    L.tabnet_hook_e5m2_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_e5m2_bits.restype = ctypes.c_uint8
    L.tabnet_hook_e3m2_bits.argtypes = [ctypes.c_double]
    L.tabnet_hook_e3m2_bits.restype = ctypes.c_uint8
    L.tabnet_hook_mx_exponent.argtypes = [ctypes.c_double, i32]
    L.tabnet_hook_mx_exponent.restype = i32
    L.tabnet_hook_int8_rows.argtypes = [vp, i32, i32, vp]
    L.tabnet_hook_int8_rows.restype = None
    L.tabnet_hook_parse.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(Config)]
    L.tabnet_hook_parse.restype = i32
    L.tabnet_hook_fold.argtypes = [vp, ctypes.c_size_t, i32, vp, vp,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.tabnet_hook_fold.restype = i32
    L.tabnet_hook_packed_sizes.argtypes = [vp, ctypes.c_size_t, i32,
                                           ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.tabnet_hook_packed_sizes.restype = i32
    L.tabnet_hook_serve_start_fake.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(ServeOpts), i32, i32, i32,
                                               ctypes.POINTER(vp)]
    L.tabnet_hook_serve_start_fake.restype = i32


def check(status: int, L=None) -> None:
    """Raise TabNetError for a non-OK status, with the message of the library L (default
    libtabnet.so) that returned it."""
    if status != OK:
        msg = (L or lib()).tabnet_last_error().decode(errors="replace")
        raise TabNetError(status, msg)


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_tensor(t, name: str, shape, device: int, dtype=None) -> None:
    """t must be a contiguous tensor of `dtype` (float32 by default) and exactly `shape`
    on GPU `device`: a host tensor's address must never reach a kernel."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must be a CUDA tensor on cuda:{device}")
    if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}{'' if t.is_contiguous() else ' (not contiguous)'}")


def _check_host(a, name: str, shape) -> None:
    """a must be a C-contiguous float32 numpy array of exactly `shape`."""
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"] \
            or tuple(a.shape) != tuple(shape):
        got = f"{a.dtype} {a.shape}" if isinstance(a, np.ndarray) else type(a).__name__
        raise ValueError(f"{name} must be a C-contiguous float32 array of shape {tuple(shape)}, got {got}")


class Model:
    """A TabNet model resident on one GPU (tabnet_load / tabnet_free)."""

    def __init__(self, path: str, precision="fp32", device: int = 0):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        check(lib().tabnet_load(os.fsencode(path), prec, device, ctypes.byref(h)))
        self._h = h
        self.device = device
        self.precision = prec
        c = Config()
        check(lib().tabnet_get_config(self._h, ctypes.byref(c)))
        self.config = c

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().tabnet_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def forward_into(self, X, logits, masks_agg, masks_step=None, stream=None) -> None:
        """tabnet_forward on caller-provided device tensors (float32, contiguous, on the
        model's GPU): X [B, D], logits [B, n_out], masks_agg [B, D], masks_step [S, B, D]."""
        c = self.config
        B = int(X.shape[0]) if hasattr(X, "shape") and len(X.shape) == 2 else -1
        _check_tensor(X, "X", (B, c.D), self.device)
        _check_tensor(logits, "logits", (B, c.n_out), self.device)
        _check_tensor(masks_agg, "masks_agg", (B, c.D), self.device)
        if masks_step is not None:
            _check_tensor(masks_step, "masks_step", (c.n_steps, B, c.D), self.device)
        check(lib().tabnet_forward(self._h, X.data_ptr(), B, logits.data_ptr(),
                                   masks_agg.data_ptr(),
                                   None if masks_step is None else masks_step.data_ptr(),
                                   _stream_ptr(stream)))

    def set_embeddings(self, cards, dims, tables) -> None:
        """tabnet_set_embeddings: cards / dims per raw column (int32), tables the categorical
        columns' [card, dim] tables concatenated (float32)."""
        import numpy as np
        cards = np.ascontiguousarray(cards, dtype=np.int32)
        dims = np.ascontiguousarray(dims, dtype=np.int32)
        tables = np.ascontiguousarray(tables, dtype=np.float32)
        if cards.shape != dims.shape or cards.ndim != 1:
            raise ValueError("cards and dims must be 1-D arrays of equal length")
        check(lib().tabnet_set_embeddings(self._h, int(cards.size), cards.ctypes.data, dims.ctypes.data,
                                          tables.ctypes.data if tables.size else None))
        self.n_cols = int(cards.size)

    def forward_raw_into(self, X_raw, logits, masks_agg_cols, masks_step_cols=None, stream=None) -> None:
        """tabnet_forward_raw on caller-provided device tensors (float32, contiguous, on the
        model's GPU): X_raw [B, C], logits [B, n_out], masks [B, C] and [S, B, C]."""
        c = self.config
        B = int(X_raw.shape[0]) if hasattr(X_raw, "shape") and len(X_raw.shape) == 2 else -1
        # before set_embeddings the library itself refuses the call (TABNET_E_INVALID)
        C = getattr(self, "n_cols", None)
        if C is None:
            C = int(X_raw.shape[1]) if B >= 0 else -1
        _check_tensor(X_raw, "X_raw", (B, C), self.device)
        _check_tensor(logits, "logits", (B, c.n_out), self.device)
        _check_tensor(masks_agg_cols, "masks_agg", (B, C), self.device)
        if masks_step_cols is not None:
            _check_tensor(masks_step_cols, "masks_step", (c.n_steps, B, C), self.device)
        check(lib().tabnet_forward_raw(self._h, X_raw.data_ptr(), int(X_raw.shape[0]), logits.data_ptr(),
                                       masks_agg_cols.data_ptr(),
                                       None if masks_step_cols is None else masks_step_cols.data_ptr(),
                                       _stream_ptr(stream)))

    def forward_raw(self, X_raw, with_steps: bool = True, stream=None) -> Tuple:
        """Returns (logits[B, n_out], masks_agg[B, C], masks_step[S, B, C] or None)."""
        import torch
        C = getattr(self, "n_cols", 0)
        B = int(X_raw.shape[0]) if hasattr(X_raw, "shape") and len(X_raw.shape) == 2 else -1
        _check_tensor(X_raw, "X_raw (after set_embeddings)", (B, C), self.device)
        c = self.config
        dev = X_raw.device
        lo = torch.empty((B, c.n_out), dtype=torch.float32, device=dev)
        ag = torch.empty((B, C), dtype=torch.float32, device=dev)
        ms = torch.empty((c.n_steps, B, C), dtype=torch.float32, device=dev) if with_steps else None
        self.forward_raw_into(X_raw, lo, ag, ms, stream)
        return lo, ag, ms

    def outputs(self, B: int, with_steps: bool = True):
        import torch
        c = self.config
        dev = torch.device("cuda", self.device)
        lo = torch.empty((B, c.n_out), dtype=torch.float32, device=dev)
        ag = torch.empty((B, c.D), dtype=torch.float32, device=dev)
        ms = torch.empty((c.n_steps, B, c.D), dtype=torch.float32, device=dev) if with_steps else None
        return lo, ag, ms

    def forward(self, X, with_steps: bool = True, stream=None) -> Tuple:
        """Returns (logits[B, n_out], masks_agg[B, D], masks_step[S, B, D] or None)."""
        B = int(X.shape[0]) if hasattr(X, "shape") and len(X.shape) == 2 else -1
        _check_tensor(X, "X", (B, self.config.D), self.device)
        lo, ag, ms = self.outputs(B, with_steps)
        self.forward_into(X, lo, ag, ms, stream)
        return lo, ag, ms


def mask_stats_workspace_bytes(B: int, D: int) -> int:
    return int(lib().tabnet_mask_stats_workspace_bytes(int(B), int(D)))


def mask_stats_into(masks, mean, var, workspace, stream=None) -> None:
    """tabnet_mask_stats on caller-provided device tensors: masks float32 [B, D],
    mean / var float64 [D], workspace a device tensor of at least
    mask_stats_workspace_bytes(B, D) bytes."""
    _check_stats_args(masks, mean, var)
    if not workspace.is_cuda or workspace.device != masks.device or not workspace.is_contiguous():
        raise ValueError(f"workspace must be a contiguous tensor on {masks.device}")
    B, D = int(masks.shape[0]), int(masks.shape[1])
    check(lib().tabnet_mask_stats(masks.data_ptr(), B, D, mean.data_ptr(), var.data_ptr(),
                                  workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                  _stream_ptr(stream)))


def _check_stats_args(masks, mean, var) -> None:
    """masks: contiguous float32 [B, D] on a GPU; mean / var: contiguous float64 [D] on the
    same GPU (a host tensor's address must never reach the kernels)."""
    import torch
    if masks.dtype != torch.float32 or masks.dim() != 2 or not masks.is_contiguous() or not masks.is_cuda:
        raise ValueError("masks must be a contiguous float32 [B, D] CUDA tensor")
    D = int(masks.shape[1])
    for name, t in (("mean", mean), ("var", var)):
        if (t.dtype != torch.float64 or t.dim() != 1 or int(t.shape[0]) != D or not t.is_contiguous()
                or t.device != masks.device):
            raise ValueError(f"{name} must be a contiguous float64 [{D}] tensor on {masks.device}")


def mask_stats_noalloc_max_bytes() -> int:
    return int(lib().tabnet_mask_stats_noalloc_max_bytes())


def mask_stats_noalloc_into(masks, mean, var, stream=None) -> None:
    """tabnet_mask_stats_noalloc on caller-provided device tensors: masks float32 [B, D],
    mean / var float64 [D]; the partial sums go to the library's own device scratch."""
    _check_stats_args(masks, mean, var)
    B, D = int(masks.shape[0]), int(masks.shape[1])
    check(lib().tabnet_mask_stats_noalloc(masks.data_ptr(), B, D, mean.data_ptr(), var.data_ptr(),
                                          _stream_ptr(stream)))


def mask_stats(masks, stream=None):
    """Per-column mean and population variance (float64 [D] tensors) of a device
    float32 [B, D] mask matrix."""
    import torch
    if masks.dtype != torch.float32 or masks.dim() != 2 or not masks.is_contiguous() or not masks.is_cuda:
        raise ValueError("masks must be a contiguous float32 [B, D] CUDA tensor")
    B, D = int(masks.shape[0]), int(masks.shape[1])
    mean = torch.empty(D, dtype=torch.float64, device=masks.device)
    var = torch.empty(D, dtype=torch.float64, device=masks.device)
    ws = torch.empty(max(mask_stats_workspace_bytes(B, D), 1), dtype=torch.uint8, device=masks.device)
    mask_stats_into(masks, mean, var, ws, stream)
    return mean, var


class Server:
    """Continuous-batching server over resident models (tabnet_serve_*).

    Host buffers passed to submit() must stay alive until the request is waited on;
    the caller keeps references (numpy arrays) for that long.
    """

    def __init__(self, models=None, mem_budget_bytes: int = 0, max_rows_per_launch: int = 0,
                 slots: int = 0, with_step_masks: bool = False, use_graph: bool = True,
                 mask_stats_window: int = 0, fake_configs=None, fake_delay_us: int = 0,
                 fake_fail_launch: int = -1, fake_fail_wait: int = -1):
        o = ServeOpts(mem_budget_bytes=mem_budget_bytes, max_rows_per_launch=max_rows_per_launch,
                      slots=slots, with_step_masks=int(with_step_masks), use_graph=int(use_graph),
                      mask_stats_window=int(mask_stats_window))
        h = ctypes.c_void_p()
        if fake_configs is not None:
            self._L = test_lib()
            arr = (Config * len(fake_configs))(*fake_configs)
            check(self._L.tabnet_hook_serve_start_fake(arr, len(fake_configs), ctypes.byref(o), fake_delay_us,
                                                       fake_fail_launch, fake_fail_wait, ctypes.byref(h)), self._L)
            self.configs = list(fake_configs)
        else:
            self._L = lib()
            hs = (ctypes.c_void_p * len(models))(*[m.handle.value for m in models])
            check(self._L.tabnet_serve_start(hs, len(models), ctypes.byref(o), ctypes.byref(h)), self._L)
            self.configs = [m.config for m in models]
        self._s = h
        self.with_step_masks = with_step_masks
        self._live = {}      # request id -> the host arrays the library writes to

    def submit(self, model: int, X, logits, masks_agg, masks_step=None, arrival_ns: int = 0) -> int:
        """Queue a request on host arrays (C-contiguous float32): X [rows, D], logits
        [rows, n_out], masks_agg [rows, D] and, if given, masks_step [S, rows, D].  The
        arrays are kept referenced here until wait() or poll() reports the request done."""
        if not 0 <= model < len(self.configs):
            raise ValueError(f"model index {model} out of range")
        c = self.configs[model]
        rows = int(X.shape[0]) if getattr(X, "ndim", 0) == 2 else -1
        _check_host(X, "X", (rows, c.D))
        _check_host(logits, "logits", (rows, c.n_out))
        _check_host(masks_agg, "masks_agg", (rows, c.D))
        if masks_step is not None:
            _check_host(masks_step, "masks_step", (c.n_steps, rows, c.D))
        rid = ctypes.c_uint64()
        check(self._L.tabnet_serve_submit(self._s, model, X.ctypes.data, rows, logits.ctypes.data,
                                        masks_agg.ctypes.data,
                                        None if masks_step is None else masks_step.ctypes.data,
                                        int(arrival_ns), ctypes.byref(rid)), self._L)
        self._live[rid.value] = (X, logits, masks_agg, masks_step)
        return rid.value

    def wait(self, rid: int, timeout_us: int = -1) -> int:
        st = self._L.tabnet_serve_wait(self._s, rid, timeout_us)
        if st != E_TIMEOUT:
            self._live.pop(rid, None)
        return st

    def poll(self, rid: int):
        d = ctypes.c_int()
        st = self._L.tabnet_serve_poll(self._s, rid, ctypes.byref(d))
        if st != OK or d.value:
            self._live.pop(rid, None)
        return st, bool(d.value)

    def stats(self) -> dict:
        st = ServeStats()
        check(self._L.tabnet_serve_get_stats(self._s, ctypes.byref(st)), self._L)
        return st.as_dict()

    def model_stats(self, model: int) -> dict:
        """Statistics of one model's requests (tabnet_serve_get_model_stats)."""
        st = ServeStats()
        check(self._L.tabnet_serve_get_model_stats(self._s, int(model), ctypes.byref(st)), self._L)
        return st.as_dict()

    def reset_stats(self) -> None:
        check(self._L.tabnet_serve_reset_stats(self._s), self._L)

    def mask_stats(self, model: int):
        """(mean [D], var [D], rows) of masks_agg over the model's last mask_stats_window
        launches (numpy float64)."""
        import numpy as np
        D = self.configs[model].D
        mean = np.zeros(D, np.float64)
        var = np.zeros(D, np.float64)
        rows = ctypes.c_int64()
        check(self._L.tabnet_serve_mask_stats(self._s, model, mean.ctypes.data, var.ctypes.data,
                                            ctypes.byref(rows)), self._L)
        return mean, var, rows.value

    @staticmethod
    def now_ns() -> int:
        return lib().tabnet_serve_now_ns()

    def stop(self) -> None:
        if self._s is not None and self._s.value:
            check(self._L.tabnet_serve_stop(self._s), self._L)
            self._s = ctypes.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
