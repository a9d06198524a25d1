"""Python binding of the C-ABI library ``liblpbatch.so`` (include/lpbatch.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Batch arrays are torch tensors on the GPU (PyTorch supplies device
memory and streams); m[] and n[] are host int32 arrays.  If the library is not
built this module raises on first use -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpbatch.so")

LP_LE, LP_GE, LP_EQ = 0, 1, 2
OPTIMAL, INFEASIBLE, UNBOUNDED, ITERATION_LIMIT, NUMERICAL, INVALID_INPUT = range(6)
PREC_FP64, PREC_FP32_CERT64 = 0, 1
PLACE_AUTO, PLACE_LDS, PLACE_HBM = 0, 1, 2
PRICE_DANTZIG, PRICE_STEEPEST_EDGE = 0, 1
FLAG_SYNC, FLAG_TIME_KERNELS, FLAG_AUTOTUNE = 1, 2, 4
STATS_WIDTH = 8
LP_OK, LP_ERR_ARG, LP_ERR_NOMEM, LP_ERR_HIP = 0, -1, -2, -3

# Every symbol include/lpbatch.h declares.
EXPORTS = ("lp_batch_solve", "lp_ctx_create", "lp_ctx_destroy", "lp_options_init",
           "lp_batch_solve_ex", "lp_ctx_kernel_times", "lp_last_error",
           "lp_mlp_init", "lp_mlp_set_params", "lp_mlp_get_params", "lp_mlp_infer",
           "lp_mlp_grads", "lp_mlp_train_step", "lp_mlp_save", "lp_mlp_load",
           "lp_hyperbox_support", "lp_ctx_tuning", "lp_batch_solve_host", "lp_batch_scale",
           "lp_measure_peaks", "lp_batch_solve_noalloc")
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_NUM_PARAMS = 20, 256, 120, 102008


class LPOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("tol_piv", ctypes.c_double), ("tol_opt", ctypes.c_double),
                ("tol_feas", ctypes.c_double), ("k_deg", ctypes.c_int32),
                ("placement", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("stats", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("shared", ctypes.c_int32),
                ("row_subset", ctypes.c_void_p), ("subset_m", ctypes.c_int32),
                ("scaling", ctypes.c_int32), ("pricing", ctypes.c_int32)]


class LPPeaks(ctypes.Structure):
    _fields_ = [("lds_read", ctypes.c_double), ("lds_write", ctypes.c_double),
                ("lds_read_write", ctypes.c_double), ("lds_broadcast", ctypes.c_double),
                ("hbm_copy", ctypes.c_double), ("clock_hz", ctypes.c_double),
                ("num_cu", ctypes.c_int32)]


class LPBatchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblpbatch error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Open liblpbatch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1802_08557_amd.build_lib` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.lp_batch_solve.argtypes = [i64] + [vp] * 9
    lib.lp_batch_solve.restype = i32
    lib.lp_ctx_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.lp_ctx_create.restype = i32
    lib.lp_ctx_destroy.argtypes = [vp]
    lib.lp_ctx_destroy.restype = None
    lib.lp_options_init.argtypes = [ctypes.POINTER(LPOptions)]
    lib.lp_options_init.restype = None
    lib.lp_batch_solve_ex.argtypes = [vp, i64] + [vp] * 9 + [ctypes.POINTER(LPOptions)]
    lib.lp_batch_solve_ex.restype = i32
    lib.lp_ctx_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(ctypes.c_float), i32]
    lib.lp_ctx_kernel_times.restype = i32
    lib.lp_last_error.argtypes = []
    lib.lp_last_error.restype = ctypes.c_char_p
    lib.lp_mlp_init.argtypes = [vp, ctypes.c_uint64]
    lib.lp_mlp_set_params.argtypes = [vp, vp, vp]
    lib.lp_mlp_get_params.argtypes = [vp, vp, vp]
    lib.lp_mlp_infer.argtypes = [vp, i64, vp, vp, vp, ctypes.c_int32, vp]
    lib.lp_mlp_grads.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    lib.lp_mlp_train_step.argtypes = [vp, i64, vp, vp, ctypes.c_float, ctypes.c_float, vp, vp]
    lib.lp_mlp_save.argtypes = [vp, ctypes.c_char_p]
    lib.lp_mlp_load.argtypes = [vp, ctypes.c_char_p]
    lib.lp_hyperbox_support.argtypes = [vp, i64, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    lib.lp_hyperbox_support.restype = i32
    lib.lp_ctx_tuning.argtypes = [vp, vp, i32]
    lib.lp_ctx_tuning.restype = i32
    lib.lp_batch_solve_host.argtypes = [vp, i64] + [vp] * 9 + [ctypes.POINTER(LPOptions), i64]
    lib.lp_batch_solve_host.restype = i32
    lib.lp_batch_scale.argtypes = [vp, i64] + [vp] * 5 + [ctypes.c_int32, ctypes.c_int32] + [vp] * 6
    lib.lp_batch_scale.restype = i32
    lib.lp_measure_peaks.argtypes = [vp, ctypes.POINTER(LPPeaks)]
    lib.lp_measure_peaks.restype = i32
    lib.lp_batch_solve_noalloc.argtypes = [vp, i64] + [vp] * 4 + [ctypes.c_int32] * 2 + [vp] * 5
    lib.lp_batch_solve_noalloc.restype = i32
    for nm in ("lp_mlp_init", "lp_mlp_set_params", "lp_mlp_get_params", "lp_mlp_infer",
               "lp_mlp_grads", "lp_mlp_train_step", "lp_mlp_save", "lp_mlp_load",
           "lp_hyperbox_support", "lp_ctx_tuning"):
        getattr(lib, nm).restype = i32
    _lib = lib
    return lib


def last_error() -> str:
    return load().lp_last_error().decode()


def _check(rc):
    if rc != LP_OK:
        raise LPBatchError(rc, last_error())
    return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _require(t, dtype, numel):
    """A contiguous device tensor of the given dtype and element count."""
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != f"torch.{dtype}" or t.numel() != numel:
        raise ValueError(f"expected a contiguous {dtype} device tensor of {numel} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")


@dataclass
class DeviceBatch:
    """A batch resident on the GPU: A, b, c (float64), sense (int8) as torch
    tensors, m, n as host int32 numpy arrays."""
    A: object
    b: object
    c: object
    sense: object
    m: np.ndarray
    n: np.ndarray

    @property
    def num_lps(self):
        return int(self.m.shape[0])

    shared: bool = False  # A, b, sense hold one LP used by every LP of the batch

    @classmethod
    def from_host(cls, batch, device="cuda"):
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        return cls(t(batch.A, np.float64), t(batch.b, np.float64), t(batch.c, np.float64),
                   t(batch.sense, np.int8), np.ascontiguousarray(batch.m, np.int32),
                   np.ascontiguousarray(batch.n, np.int32))

    @classmethod
    def shared_from_host(cls, A, b, sense, c, device="cuda"):
        """N LPs over one constraint set: A [m, n], b [m], sense [m]; c [N, n]."""
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        A = np.asarray(A)
        N = int(np.asarray(c).shape[0])
        m, n = A.shape
        return cls(t(A.reshape(-1), np.float64), t(b, np.float64), t(np.asarray(c).reshape(-1), np.float64),
                   t(sense, np.int8), np.full(N, m, np.int32), np.full(N, n, np.int32), shared=True)


@dataclass
class Solution:
    status: object   # torch int32 [N]
    x: object        # torch float64 [sum n]
    obj: object      # torch float64 [N]
    stats: object    # torch int32 [N, 8] or None


class Context:
    """An lp_ctx on one device (scratch, plans, timing events)."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        _check(self.lib.lp_ctx_create(ctypes.byref(h), int(device)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            self.lib.lp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, batch: DeviceBatch, *, precision=PREC_FP64, max_iters=0, tol_piv=0.0,
              tol_opt=0.0, tol_feas=0.0, k_deg=50, placement=PLACE_AUTO, block_threads=0,
              stats=False, stream=None, sync=False, time_kernels=False, out=None,
              row_subset=None, autotune=False, scaling=0, pricing=0) -> Solution:
        """Queue lp_batch_solve_ex on `stream` (default: torch's current stream).
        row_subset: int32 device tensor [N, subset_m] for a screened solve of a
        shared batch.  scaling: passes of power-of-two scaling (0: off).
        pricing: PRICE_DANTZIG or PRICE_STEEPEST_EDGE."""
        import torch
        dev = batch.A.device
        N = batch.num_lps
        if out is None:
            status = torch.empty(N, dtype=torch.int32, device=dev)
            x = torch.empty(int(batch.n.sum()), dtype=torch.float64, device=dev)
            obj = torch.empty(N, dtype=torch.float64, device=dev)
            st = torch.empty((N, STATS_WIDTH), dtype=torch.int32, device=dev) if stats else None
        else:
            status, x, obj, st = out.status, out.x, out.obj, out.stats
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        o = LPOptions()
        self.lib.lp_options_init(ctypes.byref(o))
        o.precision, o.max_iters = precision, max_iters
        o.tol_piv, o.tol_opt, o.tol_feas = tol_piv, tol_opt, tol_feas
        o.k_deg, o.placement, o.block_threads = k_deg, placement, block_threads
        o.stats = st.data_ptr() if st is not None else None
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        o.flags = ((FLAG_SYNC if sync else 0) | (FLAG_TIME_KERNELS if time_kernels else 0)
                   | (FLAG_AUTOTUNE if autotune else 0))
        o.shared = 1 if batch.shared else 0
        o.scaling = scaling
        o.pricing = pricing
        if row_subset is not None:
            if row_subset.dim() != 2 or row_subset.shape[0] != N:
                raise ValueError("row_subset must be [num_lps, subset_m]")
            _require(row_subset, "int32", row_subset.numel())
            o.row_subset = row_subset.data_ptr()
            o.subset_m = int(row_subset.shape[1])
        m = np.ascontiguousarray(batch.m, np.int32)
        n = np.ascontiguousarray(batch.n, np.int32)
        _check(self.lib.lp_batch_solve_ex(
            self.handle, N, _ptr(batch.A), _ptr(batch.b), _ptr(batch.c), _ptr(batch.sense),
            m.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
            _ptr(status), _ptr(x), _ptr(obj), ctypes.byref(o)))
        return Solution(status, x, obj, st)

    def solve_noalloc(self, batch: DeviceBatch, *, stats=False, stream=None, out=None) -> Solution:
        """Queue lp_batch_solve_noalloc (FP64, default options, one m x n shape
        taken by the one-wavefront kernel; nothing is allocated by the library;
        outputs are allocated here unless `out` is given)."""
        import torch
        dev = batch.A.device
        N = batch.num_lps
        if N and not (np.all(batch.m == batch.m[0]) and np.all(batch.n == batch.n[0])):
            raise ValueError("solve_noalloc needs every LP of one shape")
        m0 = int(batch.m[0]) if N else 1
        n0 = int(batch.n[0]) if N else 1
        if out is None:
            status = torch.empty(N, dtype=torch.int32, device=dev)
            x = torch.empty(N * n0, dtype=torch.float64, device=dev)
            obj = torch.empty(N, dtype=torch.float64, device=dev)
            st = torch.empty((N, STATS_WIDTH), dtype=torch.int32, device=dev) if stats else None
        else:
            status, x, obj, st = out.status, out.x, out.obj, out.stats
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self.lib.lp_batch_solve_noalloc(
            self.handle, N, _ptr(batch.A), _ptr(batch.b), _ptr(batch.c), _ptr(batch.sense), m0, n0,
            _ptr(status), _ptr(x), _ptr(obj), st.data_ptr() if st is not None else None,
            ctypes.c_void_p(stream.cuda_stream)))
        return Solution(status, x, obj, st)

    def scale(self, batch: DeviceBatch, passes: int, stream=None):
        """lp_batch_scale: (A', b', c', row_exp, col_exp) as device tensors,
        queued on `stream` (default: torch's current stream)."""
        import torch
        dev = batch.A.device
        N = batch.num_lps
        m = np.ascontiguousarray(batch.m, np.int32)
        n = np.ascontiguousarray(batch.n, np.int32)
        if batch.shared:
            rows, cols, nc = int(m[0]), int(n[0]), N * int(n[0])
        else:
            rows, cols = int(m.astype(np.int64).sum()), int(n.astype(np.int64).sum())
            nc = cols
        A2 = torch.empty(batch.A.numel(), dtype=torch.float64, device=dev)
        b2 = torch.empty(batch.b.numel(), dtype=torch.float64, device=dev)
        c2 = torch.empty(nc, dtype=torch.float64, device=dev)
        rexp = torch.empty(rows, dtype=torch.int32, device=dev)
        cexp = torch.empty(cols, dtype=torch.int32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        _check(self.lib.lp_batch_scale(
            self.handle, N, _ptr(batch.A), _ptr(batch.b), _ptr(batch.c),
            m.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p), int(passes),
            1 if batch.shared else 0, _ptr(A2), _ptr(b2), _ptr(c2), _ptr(rexp), _ptr(cexp),
            ctypes.c_void_p(stream.cuda_stream)))
        return A2, b2, c2, rexp, cexp

    def solve_host(self, A, b, c, sense, m, n, *, precision=PREC_FP64, chunk_lps=0, out=None,
                   time_kernels=False, scaling=0, pricing=0):
        """lp_batch_solve_host on a batch in host memory: A, b, c, sense are
        numpy arrays or CPU torch tensors (pinned tensors are copied directly,
        pageable memory is staged by the library); m, n numpy int32.  Returns
        (status, x, obj) as numpy arrays, or fills `out` = (status, x, obj)
        (numpy arrays or CPU torch tensors, pinned or not)."""
        m = np.ascontiguousarray(m, np.int32)
        n = np.ascontiguousarray(n, np.int32)
        N = int(m.shape[0])

        def host_ptr(a, dtype, count, name):
            if isinstance(a, np.ndarray):
                if a.dtype != np.dtype(dtype) or not a.flags.c_contiguous or a.size < count:
                    raise ValueError(f"{name}: need a contiguous {dtype} array of >= {count} entries")
                return ctypes.c_void_p(a.ctypes.data)
            import torch
            if a.device.type != "cpu" or a.dtype != getattr(torch, dtype) or not a.is_contiguous() \
                    or a.numel() < count:
                raise ValueError(f"{name}: need a contiguous CPU {dtype} tensor of >= {count} entries")
            return ctypes.c_void_p(a.data_ptr())

        rows, cols, cells = int(m.sum()), int(n.sum()), int((m.astype(np.int64) * n).sum())
        if out is None:
            out = (np.empty(N, np.int32), np.empty(cols, np.float64), np.empty(N, np.float64))
        status, x, obj = out
        o = LPOptions()
        self.lib.lp_options_init(ctypes.byref(o))
        o.precision = precision
        o.scaling = scaling
        o.pricing = pricing
        o.flags = FLAG_TIME_KERNELS if time_kernels else 0
        _check(self.lib.lp_batch_solve_host(
            self.handle, N, host_ptr(A, "float64", cells, "A"), host_ptr(b, "float64", rows, "b"),
            host_ptr(c, "float64", cols, "c"), host_ptr(sense, "int8", rows, "sense"),
            m.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
            host_ptr(status, "int32", N, "status"), host_ptr(x, "float64", cols, "x"),
            host_ptr(obj, "float64", N, "obj"), ctypes.byref(o), int(chunk_lps)))
        return status, x, obj

    # Warm-start network (lp_mlp_*): tensors are torch tensors on this device.
    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(stream.cuda_stream)

    def mlp_init(self, seed: int):
        _check(self.lib.lp_mlp_init(self.handle, ctypes.c_uint64(seed)))

    def mlp_set_params(self, params, stream=None):
        """params: float32 [MLP_NUM_PARAMS] device tensor (copied)."""
        _require(params, "float32", MLP_NUM_PARAMS)
        _check(self.lib.lp_mlp_set_params(self.handle, _ptr(params), self._stream(stream)))

    def mlp_get_params(self, stream=None):
        import torch
        out = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device=f"cuda:{self.device}")
        _check(self.lib.lp_mlp_get_params(self.handle, _ptr(out), self._stream(stream)))
        return out

    def mlp_infer(self, dirs, k=0, scores=True, stream=None):
        """dirs: float32 [B, 20] device tensor.  Returns (scores [B, 120] or
        None, top_k [B, k] int32 or None)."""
        import torch
        B = int(dirs.shape[0])
        _require(dirs, "float32", B * MLP_IN)
        dev = dirs.device
        S = torch.empty((B, MLP_OUT), dtype=torch.float32, device=dev) if scores else None
        T = torch.empty((B, k), dtype=torch.int32, device=dev) if k else None
        _check(self.lib.lp_mlp_infer(self.handle, B, _ptr(dirs), _ptr(S), _ptr(T), int(k),
                                     self._stream(stream)))
        return S, T

    def mlp_grads(self, dirs, tight, stream=None):
        """Returns (grad float32 [MLP_NUM_PARAMS], loss float32 [1]) device tensors."""
        import torch
        B = int(dirs.shape[0])
        _require(dirs, "float32", B * MLP_IN)
        _require(tight, "uint8", B * MLP_OUT)
        g = torch.empty(MLP_NUM_PARAMS, dtype=torch.float32, device=dirs.device)
        L = torch.empty(1, dtype=torch.float32, device=dirs.device)
        _check(self.lib.lp_mlp_grads(self.handle, B, _ptr(dirs), _ptr(tight), _ptr(g), _ptr(L),
                                     self._stream(stream)))
        return g, L

    def mlp_train_step(self, dirs, tight, lr, weight_decay=0.0, loss=None, stream=None):
        """One AdamW step; the loss before it goes to `loss` (float32 [1] device
        tensor) when given."""
        B = int(dirs.shape[0])
        _require(dirs, "float32", B * MLP_IN)
        _require(tight, "uint8", B * MLP_OUT)
        _check(self.lib.lp_mlp_train_step(self.handle, B, _ptr(dirs), _ptr(tight), float(lr),
                                          float(weight_decay), _ptr(loss), self._stream(stream)))

    def mlp_save(self, path: str):
        _check(self.lib.lp_mlp_save(self.handle, os.fsencode(path)))

    def mlp_load(self, path: str):
        _check(self.lib.lp_mlp_load(self.handle, os.fsencode(path)))

    def hyperbox_support(self, lo, hi, l, want_x=False, stream=None):
        """Closed-form box LPs: l float64 [num, n]; lo, hi float64 [num, n] or
        [n] (one box for every direction).  Returns (value [num], x or None)."""
        import torch
        num, n = int(l.shape[0]), int(l.shape[1])
        shared_box = lo.dim() == 1
        _require(l, "float64", num * n)
        _require(lo, "float64", n if shared_box else num * n)
        _require(hi, "float64", n if shared_box else num * n)
        value = torch.empty(num, dtype=torch.float64, device=l.device)
        x = torch.empty((num, n), dtype=torch.float64, device=l.device) if want_x else None
        _check(self.lib.lp_hyperbox_support(self.handle, num, n, _ptr(lo), _ptr(hi), _ptr(l),
                                            1 if shared_box else 0, _ptr(value), _ptr(x),
                                            self._stream(stream)))
        return value, x

    def measure_peaks(self):
        """lp_measure_peaks: measured LDS and HBM bandwidths (bytes/s), the
        shader clock (Hz) during the LDS runs and the CU count, as a dict."""
        p = LPPeaks()
        _check(self.lib.lp_measure_peaks(self.handle, ctypes.byref(p)))
        return {name: getattr(p, name) for name, _ in LPPeaks._fields_}

    def tuning(self):
        """[(bin, fp32, workgroup size, hbm)] of the context's autotuned launches."""
        cnt = self.lib.lp_ctx_tuning(self.handle, None, 0)
        if cnt < 0:
            raise LPBatchError(cnt, last_error())
        buf = (ctypes.c_int32 * (4 * max(cnt, 1)))()
        self.lib.lp_ctx_tuning(self.handle, buf, cnt)
        return [tuple(buf[4 * i:4 * i + 4]) for i in range(cnt)]

    def kernel_times(self, cap=4096):
        """[(name, ms)] of every kernel of the solves made with time_kernels=True
        since the previous call (the context then forgets them)."""
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_float * cap)()
        cnt = self.lib.lp_ctx_kernel_times(self.handle, names, ms, cap)
        if cnt < 0:
            raise LPBatchError(cnt, last_error())
        return [(names[i].decode(), float(ms[i])) for i in range(min(cnt, cap))]


def batch_solve(batch: DeviceBatch):
    """lp_batch_solve: synchronous FP64 solve with the library's default context."""
    import torch
    lib = load()
    dev = batch.A.device
    N = batch.num_lps
    status = torch.empty(N, dtype=torch.int32, device=dev)
    x = torch.empty(int(batch.n.sum()), dtype=torch.float64, device=dev)
    obj = torch.empty(N, dtype=torch.float64, device=dev)
    m = np.ascontiguousarray(batch.m, np.int32)
    n = np.ascontiguousarray(batch.n, np.int32)
    torch.cuda.synchronize(dev)
    _check(lib.lp_batch_solve(N, _ptr(batch.A), _ptr(batch.b), _ptr(batch.c), _ptr(batch.sense),
                              m.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
                              _ptr(status), _ptr(x), _ptr(obj)))
    return Solution(status, x, obj, None)

