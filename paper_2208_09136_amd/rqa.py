"""ctypes binding of librqa.so (include/rqa.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Series live in device memory as torch CUDA tensors
(torch serves for device memory and streams); thresholds, targets and all
results are host numpy arrays.  The functions carry the names of the C calls.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqa.so")

RQA_MAX_K = 128
RQA_NORM_MAX = 0
RQA_NORM_EUCLIDEAN = 1
RQA_SEL_AUTO = 0
RQA_SEL_PLAIN = 16
RQA_SEL_LEARNED = 1
RQA_FULL_HIST = 2
RQA_SEL_SAMPLE = 4
RQA_SEL_WINDOW = 8

STATUS = {0: "RQA_OK", -1: "RQA_ERR_INVALID_ARG", -2: "RQA_ERR_TOO_SHORT",
          -3: "RQA_ERR_NONFINITE", -4: "RQA_ERR_DEVICE", -5: "RQA_ERR_NOMEM",
          -6: "RQA_ERR_UNSUPPORTED"}

PHASES = ("select_pass1", "select_pass2", "select_pass3", "sweep", "other", "histogram")


class RqaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class rqa_params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint32), ("tau", ctypes.c_uint32), ("norm", ctypes.c_uint32),
                ("theiler", ctypes.c_uint32), ("lmin", ctypes.c_uint32)]


_lib = None
_u32, _u64, _i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_vp = ctypes.c_void_p
_fp = ctypes.POINTER(ctypes.c_float)
_dp = ctypes.POINTER(ctypes.c_double)
_up = ctypes.POINTER(ctypes.c_uint64)
_pp = ctypes.POINTER(rqa_params)

SIGNATURES = {
    "rqa_create": (_i32, [ctypes.POINTER(_vp), _i32, _vp]),
    "rqa_destroy": (None, [_vp]),
    "rqa_select_thresholds": (_i32, [_vp, _vp, _u64, _pp, _dp, _u32, _u32, _fp, _up, _up]),
    "rqa_det_curve": (_i32, [_vp, _vp, _u64, _pp, _fp, _u32, _u32, _up, _dp, _dp, _dp, _up, _u64]),
    "rqa_run": (_i32, [_vp, _vp, _u64, _pp, _dp, _u32, _u32, _fp, _up, _up, _dp, _dp, _dp]),
    "rqa_batch": (_i32, [_vp, _u32, _vp, _up, _pp, _dp, _u32, _u32, _fp, _dp, _dp, _dp, _up]),
    "rqa_batch_static": (_i32, [_vp, _u32, _vp, _up, _pp, _dp, _u32, _u32, _fp, _dp, _dp, _dp, _up]),
    "rqa_batch_hist": (_i32, [_vp, _u32, _vp, _up, _pp, _dp, _u32, _u32, _fp, _dp, _dp, _dp, _up, _up, _u64]),
    "rqa_phase_times": (_i32, [_vp, _dp, _i32]),
    "rqa_set_timing": (_i32, [_vp, _i32]),
    "rqa_valu_rate": (_i32, [_vp, _u32, _dp, _dp]),
    "rqa_set_shape": (_i32, [_vp, _u32, _u32]),
    "rqa_set_grid": (_i32, [_vp, _u32]),
    "rqa_autotune": (_i32, [_vp, _vp, _u64, _pp, _dp, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "rqa_autotune_batch": (_i32, [_vp, _u32, _vp, _up, _pp, _dp, _u32, ctypes.POINTER(_u32)]),
    "rqa_sketch_batch": (_i32, [_vp, _u32, _vp, _up, _pp, _u64, _fp, ctypes.POINTER(_u32)]),
    "rqa_sketch_sample": (_i32, [_vp, _u32, _vp, _up, _pp, _u64, ctypes.POINTER(_u32)]),
    "rqa_mlp_init": (_i32, [_vp, _u64]),
    "rqa_mlp_set_params": (_i32, [_vp, _fp, _u64]),
    "rqa_mlp_get_params": (_i32, [_vp, _fp, _u64]),
    "rqa_mlp_forward": (_i32, [_vp, _vp, _u32, _vp]),
    "rqa_mlp_gradients": (_i32, [_vp, _vp, _vp, _u32, _fp, _dp]),
    "rqa_mlp_train_step": (_i32, [_vp, _vp, _vp, _u32, ctypes.c_float, _dp]),
    "rqa_mlp_set_bracket": (_i32, [_vp, _fp, _u32]),
    "rqa_set_window": (_i32, [_vp, ctypes.c_float, ctypes.c_float]),
    "rqa_set_sample_width": (_i32, [_vp, ctypes.c_float]),
    "rqa_selection_stats": (_i32, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    "rqa_averaged_det": (_i32, [_dp, _u32, _dp]),
    "rqa_line_measures": (_i32, [_up, _u32, _u64, _u32, _dp, _up]),
    "rqa_tune_save": (_i32, [_vp, ctypes.c_char_p]),
    "rqa_tune_load": (_i32, [_vp, ctypes.c_char_p]),
    "rqa_status_string": (ctypes.c_char_p, [_i32]),
    "rqa_last_error": (ctypes.c_char_p, []),
}


def load():
    """Load librqa.so; raise loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2208_09136_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(st):
    if st != 0:
        raise RqaError(st, load().rqa_last_error().decode())


def _params(p):
    if isinstance(p, rqa_params):
        return p
    if isinstance(p, dict):
        return rqa_params(p["m"], p["tau"], p["norm"], p.get("theiler", p.get("w", 1)), p["lmin"])
    return rqa_params(*p)


def _series_ptr(series):
    """(device pointer, length) of a contiguous float32 CUDA tensor."""
    import torch
    if not isinstance(series, torch.Tensor) or not series.is_cuda:
        raise TypeError("series must be a CUDA torch tensor (device memory)")
    if series.dtype != torch.float32 or not series.is_contiguous():
        raise TypeError("series must be contiguous float32")
    return series.data_ptr(), series.numel()


def _a(x, dtype):
    return np.ascontiguousarray(x, dtype=dtype)


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def rqa_status_string(status):
    return load().rqa_status_string(status).decode()


def rqa_last_error():
    return load().rqa_last_error().decode()


def rqa_create(device=0, stream=None):
    """Context on `device`; `stream` is a torch.cuda.Stream, a raw hipStream_t
    integer, or None for a context-owned stream."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    ctx = _vp()
    _check(load().rqa_create(ctypes.byref(ctx), device, _vp(stream) if stream else None))
    return ctx


def rqa_destroy(ctx):
    load().rqa_destroy(ctx)


def rqa_set_timing(ctx, enable=True):
    _check(load().rqa_set_timing(ctx, 1 if enable else 0))


VALU_PROBES = {"v_add_f32": 0, "v_add_u32": 1, "v_max_u32": 2, "v_add_u32_sgpr": 3}


def rqa_valu_rate(ctx, kind):
    """Measured VALU rate of one instruction class: (lane-ops/s, ms)."""
    rate, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load().rqa_valu_rate(ctx, VALU_PROBES.get(kind, kind), ctypes.byref(rate), ctypes.byref(ms)))
    return rate.value, ms.value


def rqa_phase_times(ctx):
    out = np.zeros(len(PHASES), dtype=np.float64)
    n = load().rqa_phase_times(ctx, _p(out, ctypes.c_double), len(PHASES))
    return dict(zip(PHASES[:n], out[:n].tolist()))


def rqa_set_shape(ctx, segment=0, chunk_tiles=0):
    _check(load().rqa_set_shape(ctx, segment, chunk_tiles))


def rqa_set_grid(ctx, workgroups=0):
    _check(load().rqa_set_grid(ctx, workgroups))


def rqa_autotune(ctx, series, params, rr):
    """Tune the launch shape on one series; returns (segment, chunk_tiles)."""
    ptr, n = _series_ptr(series)
    rrt = _a(rr, np.float64)
    seg, chunk = _u32(0), _u32(0)
    prm = _params(params)
    _check(load().rqa_autotune(ctx, ptr, n, ctypes.byref(prm), _p(rrt, ctypes.c_double), len(rrt),
                               ctypes.byref(seg), ctypes.byref(chunk)))
    return seg.value, chunk.value


def rqa_autotune_batch(ctx, concat, offsets, params, rr):
    """Tune per-bucket segment lengths and the batch chunk size; returns the
    chunk size."""
    ptr, _ = _series_ptr(concat)
    offs = _a(offsets, np.uint64)
    S = len(offs) - 1
    rrt = _a(rr, np.float64)
    prm = (rqa_params * S)(*[_params(p) for p in params])
    chunk = _u32(0)
    _check(load().rqa_autotune_batch(ctx, S, ptr, _p(offs, ctypes.c_uint64), prm, _p(rrt, ctypes.c_double),
                                     rrt.shape[1], ctypes.byref(chunk)))
    return chunk.value


SKETCH_FEATURES = 66


def rqa_sketch_batch(ctx, concat, offsets, params, seed):
    """Sketch features (S, 66) float32 and scales (S,) uint32 of S series."""
    ptr, _ = _series_ptr(concat)
    offs = _a(offsets, np.uint64)
    S = len(offs) - 1
    prm = (rqa_params * S)(*[_params(p) for p in params])
    feats = np.zeros((S, SKETCH_FEATURES), np.float32)
    scale = np.zeros(S, np.uint32)
    _check(load().rqa_sketch_batch(ctx, S, ptr, _p(offs, ctypes.c_uint64), prm, int(seed),
                                   _p(feats, ctypes.c_float), scale.ctypes.data_as(ctypes.POINTER(_u32))))
    return feats, scale


SKETCH_PAIRS = 4096


def rqa_sketch_sample(ctx, concat, offsets, params, seed):
    """Sorted sampled key bit patterns (S, 4096) uint32 of the sketch of S series."""
    ptr, _ = _series_ptr(concat)
    offs = _a(offsets, np.uint64)
    S = len(offs) - 1
    prm = (rqa_params * S)(*[_params(p) for p in params])
    out = np.zeros((S, SKETCH_PAIRS), np.uint32)
    _check(load().rqa_sketch_sample(ctx, S, ptr, _p(offs, ctypes.c_uint64), prm, int(seed),
                                    out.ctypes.data_as(ctypes.POINTER(_u32))))
    return out


MLP_INPUTS, MLP_OUTPUTS, MLP_PARAMS = 66, 20, 27668


def _dev_matrix(t, cols):
    """(device pointer, rows) of a contiguous float32 CUDA tensor [rows, cols]."""
    ptr, n = _series_ptr(t)
    if n % cols:
        raise ValueError(f"tensor size {n} is not a multiple of {cols}")
    return ptr, n // cols


def rqa_mlp_init(ctx, seed):
    _check(load().rqa_mlp_init(ctx, int(seed)))


def rqa_mlp_set_params(ctx, params):
    p = _a(params, np.float32)
    _check(load().rqa_mlp_set_params(ctx, _p(p, ctypes.c_float), p.size))


def rqa_mlp_get_params(ctx):
    p = np.zeros(MLP_PARAMS, np.float32)
    _check(load().rqa_mlp_get_params(ctx, _p(p, ctypes.c_float), p.size))
    return p


def rqa_mlp_forward(ctx, x, y):
    """y[B, 20] = network(x[B, 66]); x and y are CUDA float32 tensors."""
    xp, B = _dev_matrix(x, MLP_INPUTS)
    yp, By = _dev_matrix(y, MLP_OUTPUTS)
    if By != B:
        raise ValueError("x and y rows differ")
    _check(load().rqa_mlp_forward(ctx, xp, B, yp))


def rqa_mlp_gradients(ctx, x, t):
    """(gradient float32[27668], loss) of the MSE on the batch."""
    xp, B = _dev_matrix(x, MLP_INPUTS)
    tp, Bt = _dev_matrix(t, MLP_OUTPUTS)
    if Bt != B:
        raise ValueError("x and t rows differ")
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float64)
    _check(load().rqa_mlp_gradients(ctx, xp, tp, B, _p(g, ctypes.c_float), _p(loss, ctypes.c_double)))
    return g, float(loss[0])


def rqa_mlp_train_step(ctx, x, t, lr):
    xp, B = _dev_matrix(x, MLP_INPUTS)
    tp, Bt = _dev_matrix(t, MLP_OUTPUTS)
    if Bt != B:
        raise ValueError("x and t rows differ")
    loss = np.zeros(1, np.float64)
    _check(load().rqa_mlp_train_step(ctx, xp, tp, B, float(lr), _p(loss, ctypes.c_double)))
    return float(loss[0])


def rqa_mlp_set_bracket(ctx, delta):
    d = _a(delta, np.float32)
    _check(load().rqa_mlp_set_bracket(ctx, _p(d, ctypes.c_float), d.size))


def rqa_set_window(ctx, lo, hi):
    _check(load().rqa_set_window(ctx, float(lo), float(hi)))


def rqa_set_sample_width(ctx, z):
    _check(load().rqa_set_sample_width(ctx, float(z)))


def rqa_selection_stats(ctx):
    a, b, c = _u32(0), _u32(0), _u32(0)
    _check(load().rqa_selection_stats(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"full_passes": a.value, "series_fallback": b.value, "targets_missed": c.value}


def rqa_averaged_det(det):
    """Averaged-DET curve over an ordered RR set: element r is the mean of
    det[0..r] (left fold in double, in the library)."""
    d = _a(det, np.float64)
    out = np.zeros(d.size, np.float64)
    _check(load().rqa_averaged_det(_p(d, ctypes.c_double), d.size, _p(out, ctypes.c_double)))
    return out


def rqa_line_measures(hist, lmin):
    """(L, L_max) per row of a (K, hist_len) line histogram, in the library."""
    h = _a(hist, np.uint64)
    if h.ndim != 2:
        raise ValueError("hist must be (K, hist_len)")
    K, n = h.shape
    L = np.zeros(K, np.float64)
    lmax = np.zeros(K, np.uint64)
    _check(load().rqa_line_measures(_p(h, ctypes.c_uint64), K, n, lmin, _p(L, ctypes.c_double),
                                    _p(lmax, ctypes.c_uint64)))
    return L, lmax


def rqa_tune_save(ctx, path):
    _check(load().rqa_tune_save(ctx, os.fsencode(path)))


def rqa_tune_load(ctx, path):
    _check(load().rqa_tune_load(ctx, os.fsencode(path)))


def rqa_select_thresholds(ctx, series, params, rr, flags=RQA_SEL_AUTO):
    """Exact thresholds for the RR targets: (eps float32[K], k uint64[K],
    count uint64[K])."""
    ptr, n = _series_ptr(series)
    rr = _a(rr, np.float64)
    K = len(rr)
    eps = np.zeros(K, np.float32)
    k = np.zeros(K, np.uint64)
    cnt = np.zeros(K, np.uint64)
    prm = _params(params)
    _check(load().rqa_select_thresholds(ctx, ptr, n, ctypes.byref(prm), _p(rr, ctypes.c_double), K, flags,
                                        _p(eps, ctypes.c_float), _p(k, ctypes.c_uint64),
                                        _p(cnt, ctypes.c_uint64)))
    return eps, k, cnt


def rqa_det_curve(ctx, series, params, eps, flags=0, hist_len=0):
    """RR and DET at the given thresholds: dict(count, rr, det, det_mean,
    hist).  hist_len > 0 sets RQA_FULL_HIST and returns hist, a (K, hist_len)
    uint64 array of P_r(l) (the last entry collects longer lines); else hist
    is None."""
    ptr, n = _series_ptr(series)
    eps = _a(eps, np.float32)
    K = len(eps)
    cnt = np.zeros(K, np.uint64)
    rr = np.zeros(K, np.float64)
    det = np.zeros(K, np.float64)
    dm = np.zeros(1, np.float64)
    hist = np.zeros((K, hist_len), np.uint64) if hist_len else None
    if hist_len:
        flags |= RQA_FULL_HIST
    prm = _params(params)
    _check(load().rqa_det_curve(ctx, ptr, n, ctypes.byref(prm), _p(eps, ctypes.c_float), K, flags,
                                _p(cnt, ctypes.c_uint64), _p(rr, ctypes.c_double), _p(det, ctypes.c_double),
                                _p(dm, ctypes.c_double), _p(hist, ctypes.c_uint64) if hist_len else None,
                                hist_len))
    return {"count": cnt, "rr": rr, "det": det, "det_mean": float(dm[0]), "hist": hist}


def rqa_run(ctx, series, params, rr, flags=RQA_SEL_AUTO):
    """Thresholds for the targets, then RR/DET at them: dict(eps, k, count,
    rr, det, det_mean)."""
    ptr, n = _series_ptr(series)
    rrt = _a(rr, np.float64)
    K = len(rrt)
    eps = np.zeros(K, np.float32)
    k = np.zeros(K, np.uint64)
    cnt = np.zeros(K, np.uint64)
    rro = np.zeros(K, np.float64)
    det = np.zeros(K, np.float64)
    dm = np.zeros(1, np.float64)
    prm = _params(params)
    _check(load().rqa_run(ctx, ptr, n, ctypes.byref(prm), _p(rrt, ctypes.c_double), K, flags,
                          _p(eps, ctypes.c_float), _p(k, ctypes.c_uint64), _p(cnt, ctypes.c_uint64),
                          _p(rro, ctypes.c_double), _p(det, ctypes.c_double), _p(dm, ctypes.c_double)))
    return {"eps": eps, "k": k, "count": cnt, "rr": rro, "det": det, "det_mean": float(dm[0])}


def rqa_batch(ctx, concat, offsets, params, rr, flags=RQA_SEL_AUTO, _entry="rqa_batch"):
    """S series back to back in one device tensor.  offsets: S+1 element
    offsets; params: S parameter sets; rr: (S, K) targets.  Returns dict of
    (S, K) arrays eps, rr, det, count and det_mean (S,)."""
    ptr, _ = _series_ptr(concat)
    offs = _a(offsets, np.uint64)
    S = len(offs) - 1
    rrt = _a(rr, np.float64)
    if rrt.ndim != 2 or rrt.shape[0] != S:
        raise ValueError("rr must have shape (S, K)")
    K = rrt.shape[1]
    prm = (rqa_params * S)(*[_params(p) for p in params])
    eps = np.zeros((S, K), np.float32)
    rro = np.zeros((S, K), np.float64)
    det = np.zeros((S, K), np.float64)
    cnt = np.zeros((S, K), np.uint64)
    dm = np.zeros(S, np.float64)
    fn = getattr(load(), _entry)
    _check(fn(ctx, S, ptr, _p(offs, ctypes.c_uint64), prm, _p(rrt, ctypes.c_double), K, flags,
              _p(eps, ctypes.c_float), _p(rro, ctypes.c_double), _p(det, ctypes.c_double),
              _p(dm, ctypes.c_double), _p(cnt, ctypes.c_uint64)))
    return {"eps": eps, "rr": rro, "det": det, "det_mean": dm, "count": cnt}


RQA_STATIC_SCRATCH_BYTES = 64 << 20


def rqa_batch_hist(ctx, concat, offsets, params, rr, hist_len, flags=RQA_SEL_AUTO):
    """rqa_batch plus the full line-length histogram at every selected
    threshold: the dict also holds "hist", an (S, K, hist_len) uint64 array."""
    ptr, _ = _series_ptr(concat)
    offs = _a(offsets, np.uint64)
    S = len(offs) - 1
    rrt = _a(rr, np.float64)
    if rrt.ndim != 2 or rrt.shape[0] != S:
        raise ValueError("rr must have shape (S, K)")
    K = rrt.shape[1]
    prm = (rqa_params * S)(*[_params(p) for p in params])
    eps = np.zeros((S, K), np.float32)
    rro = np.zeros((S, K), np.float64)
    det = np.zeros((S, K), np.float64)
    cnt = np.zeros((S, K), np.uint64)
    dm = np.zeros(S, np.float64)
    hist = np.zeros((S, K, int(hist_len)), np.uint64)
    _check(load().rqa_batch_hist(ctx, S, ptr, _p(offs, ctypes.c_uint64), prm, _p(rrt, ctypes.c_double), K, flags,
                                 _p(eps, ctypes.c_float), _p(rro, ctypes.c_double), _p(det, ctypes.c_double),
                                 _p(dm, ctypes.c_double), _p(cnt, ctypes.c_uint64), _p(hist, ctypes.c_uint64),
                                 int(hist_len)))
    return {"eps": eps, "rr": rro, "det": det, "det_mean": dm, "count": cnt, "hist": hist}


def rqa_batch_static(ctx, concat, offsets, params, rr, flags=RQA_SEL_AUTO):
    """rqa_batch with device scratch from the library's static area: the call
    allocates no device memory (see include/rqa.h)."""
    return rqa_batch(ctx, concat, offsets, params, rr, flags, _entry="rqa_batch_static")


class Context:
    """Owns an rqa context; methods mirror the C calls."""

    def __init__(self, device=0, stream=None):
        self.ctx = rqa_create(device, stream)

    def close(self):
        if self.ctx:
            rqa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def select_thresholds(self, series, params, rr, flags=RQA_SEL_AUTO):
        return rqa_select_thresholds(self.ctx, series, params, rr, flags)

    def det_curve(self, series, params, eps, flags=0, hist_len=0):
        return rqa_det_curve(self.ctx, series, params, eps, flags, hist_len)

    def run(self, series, params, rr, flags=RQA_SEL_AUTO):
        return rqa_run(self.ctx, series, params, rr, flags)

    def batch(self, concat, offsets, params, rr, flags=RQA_SEL_AUTO):
        return rqa_batch(self.ctx, concat, offsets, params, rr, flags)

    def batch_static(self, concat, offsets, params, rr, flags=RQA_SEL_AUTO):
        return rqa_batch_static(self.ctx, concat, offsets, params, rr, flags)

    def batch_hist(self, concat, offsets, params, rr, hist_len, flags=RQA_SEL_AUTO):
        return rqa_batch_hist(self.ctx, concat, offsets, params, rr, hist_len, flags)

    def set_timing(self, enable=True):
        rqa_set_timing(self.ctx, enable)

    def valu_rate(self, kind):
        return rqa_valu_rate(self.ctx, kind)

    def phase_times(self):
        return rqa_phase_times(self.ctx)

    def set_shape(self, segment=0, chunk_tiles=0):
        rqa_set_shape(self.ctx, segment, chunk_tiles)

    def set_grid(self, workgroups=0):
        rqa_set_grid(self.ctx, workgroups)

    def autotune(self, series, params, rr):
        return rqa_autotune(self.ctx, series, params, rr)

    def autotune_batch(self, concat, offsets, params, rr):
        return rqa_autotune_batch(self.ctx, concat, offsets, params, rr)

    def sketch_batch(self, concat, offsets, params, seed):
        return rqa_sketch_batch(self.ctx, concat, offsets, params, seed)

    def sketch_sample(self, concat, offsets, params, seed):
        return rqa_sketch_sample(self.ctx, concat, offsets, params, seed)

    def mlp_init(self, seed):
        rqa_mlp_init(self.ctx, seed)

    def mlp_set_params(self, params):
        rqa_mlp_set_params(self.ctx, params)

    def mlp_get_params(self):
        return rqa_mlp_get_params(self.ctx)

    def mlp_forward(self, x, y):
        rqa_mlp_forward(self.ctx, x, y)

    def mlp_gradients(self, x, t):
        return rqa_mlp_gradients(self.ctx, x, t)

    def mlp_train_step(self, x, t, lr):
        return rqa_mlp_train_step(self.ctx, x, t, lr)

    def mlp_set_bracket(self, delta):
        rqa_mlp_set_bracket(self.ctx, delta)

    def set_window(self, lo, hi):
        rqa_set_window(self.ctx, lo, hi)

    def set_sample_width(self, z):
        rqa_set_sample_width(self.ctx, z)

    def selection_stats(self):
        return rqa_selection_stats(self.ctx)

    def tune_save(self, path):
        rqa_tune_save(self.ctx, path)

    def tune_load(self, path):
        rqa_tune_load(self.ctx, path)
