"""CPU oracle for averaged RQA (arXiv 2208.09136).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The GPU library never loads it and
shares no code with it.

The arithmetic lives in ``rqa_oracle.c`` (plain C, built without FMA
contraction); this module is a ctypes wrapper around it plus the pure-numpy
MLP reference in ``mlp.py``.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rqa_oracle.c")
LIB = os.path.join(HERE, "librqa_oracle.so")

NORM_MAX = 0
NORM_EUCLID = 1

OK = 0
ERR_INVALID = -1
ERR_TOO_SHORT = -2
ERR_NONFINITE = -3


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def build(force=False):
    """Compile the oracle with gcc: no FMA contraction, no fast-math."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        fp = ctypes.POINTER(ctypes.c_float)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        lib.orc_num_vectors.restype = u64
        lib.orc_num_vectors.argtypes = [u64, u32, u32]
        lib.orc_num_pairs.restype = u64
        lib.orc_num_pairs.argtypes = [u64, u32]
        lib.orc_rank.restype = u64
        lib.orc_rank.argtypes = [ctypes.c_double, u64]
        lib.orc_key.restype = ctypes.c_float
        lib.orc_key.argtypes = [fp, u32, u32, u32, u64, u64]
        lib.orc_keys.restype = i32
        lib.orc_keys.argtypes = [fp, u64, u32, u32, u32, u32, fp]
        lib.orc_count.restype = i32
        lib.orc_count.argtypes = [fp, u64, u32, u32, u32, u32, fp, u32, up, up]
        lib.orc_select.restype = i32
        lib.orc_select.argtypes = [fp, u64, u32, u32, u32, u32, dp, u32, i32, fp, up, up]
        lib.orc_lines.restype = i32
        lib.orc_lines.argtypes = [fp, u64, u32, u32, u32, u32, u32, fp, u32, up, u64,
                                  up, dp, dp, dp]
        lib.orc_num_threads.restype = i32
        lib.orc_num_threads.argtypes = []
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def num_vectors(n, m, tau):
    return int(_load().orc_num_vectors(n, m, tau))


def num_pairs(nv, w):
    return int(_load().orc_num_pairs(nv, w))


def rank(rr, M):
    return int(_load().orc_rank(float(rr), int(M)))


def key(y, m, tau, norm, i, j):
    y = _f32(y)
    return np.float32(_load().orc_key(_ptr(y, ctypes.c_float), m, tau, norm, i, j))


def keys(y, m, tau, norm, w):
    """All keys, diagonal-major: d = w..nv-1, then t = 0..nv-1-d."""
    y = _f32(y)
    nv = num_vectors(len(y), m, tau)
    M = num_pairs(nv, w)
    out = np.empty(max(M, 1), dtype=np.float32)
    st = _load().orc_keys(_ptr(y, ctypes.c_float), len(y), m, tau, norm, w,
                          _ptr(out, ctypes.c_float))
    if st:
        raise OracleError(st, "keys")
    return out[:M]


def count(y, m, tau, norm, w, values):
    """(#{key < v}, #{key <= v}) for each v in values."""
    y = _f32(y)
    v = _f32(values)
    lt = np.zeros(len(v), dtype=np.uint64)
    le = np.zeros(len(v), dtype=np.uint64)
    st = _load().orc_count(_ptr(y, ctypes.c_float), len(y), m, tau, norm, w,
                           _ptr(v, ctypes.c_float), len(v), _ptr(lt, ctypes.c_uint64),
                           _ptr(le, ctypes.c_uint64))
    if st:
        raise OracleError(st, "count")
    return lt, le


def select(y, m, tau, norm, w, rr, method=0):
    """Exact thresholds: returns (eps float32[K], k uint64[K], count uint64[K])."""
    y = _f32(y)
    rr = np.ascontiguousarray(rr, dtype=np.float64)
    K = len(rr)
    eps = np.zeros(K, dtype=np.float32)
    k = np.zeros(K, dtype=np.uint64)
    c = np.zeros(K, dtype=np.uint64)
    st = _load().orc_select(_ptr(y, ctypes.c_float), len(y), m, tau, norm, w,
                            _ptr(rr, ctypes.c_double), K, method,
                            _ptr(eps, ctypes.c_float), _ptr(k, ctypes.c_uint64),
                            _ptr(c, ctypes.c_uint64))
    if st:
        raise OracleError(st, "select")
    return eps, k, c


def lines(y, m, tau, norm, w, lmin, eps, hist_len=0):
    """Line statistics per threshold.

    Returns dict(count, rr, det, det_mean, hist) where hist is None unless
    hist_len > 0 (then a (K, hist_len) uint64 array of P_r(l))."""
    y = _f32(y)
    e = _f32(eps)
    K = len(e)
    c = np.zeros(K, dtype=np.uint64)
    rr = np.zeros(K, dtype=np.float64)
    det = np.zeros(K, dtype=np.float64)
    dm = np.zeros(1, dtype=np.float64)
    hist = np.zeros((K, hist_len), dtype=np.uint64) if hist_len else None
    hp = _ptr(hist, ctypes.c_uint64) if hist_len else None
    st = _load().orc_lines(_ptr(y, ctypes.c_float), len(y), m, tau, norm, w, lmin,
                           _ptr(e, ctypes.c_float), K, hp, hist_len,
                           _ptr(c, ctypes.c_uint64), _ptr(rr, ctypes.c_double),
                           _ptr(det, ctypes.c_double), _ptr(dm, ctypes.c_double))
    if st:
        raise OracleError(st, "lines")
    return {"count": c, "rr": rr, "det": det, "det_mean": float(dm[0]), "hist": hist}


def run(y, m, tau, norm, w, lmin, rr, method=0, hist_len=0):
    """Whole path: exact thresholds, then line statistics at those thresholds."""
    eps, k, c = select(y, m, tau, norm, w, rr, method)
    out = lines(y, m, tau, norm, w, lmin, eps, hist_len)
    out.update(eps=eps, k=k, count_select=c)
    return out


def line_measures(hist, lmin):
    """Average diagonal line length L and longest line L_max per row of a line
    histogram (rows P_r(l), l = 0 .. hist_len - 1; the last entry holds the
    lines of that length or longer).  The paper derives DET, L and L_max from
    the histogram (section on the GPU implementation) without printing the
    last two; the standard RQA definitions are used:
      L_r = sum_{l >= lmin} l P_r(l) / sum_{l >= lmin} P_r(l)  (NaN without
            such a line), summed in increasing l in float64;
      L_max_r = the largest l with P_r(l) > 0 (0 without a line).
    Plain Python loops over the entries."""
    hist = np.asarray(hist, dtype=np.uint64)
    K, n = hist.shape
    L = np.zeros(K, dtype=np.float64)
    lmax = np.zeros(K, dtype=np.uint64)
    for r in range(K):
        num = 0
        den = 0
        for l in range(n):
            c = int(hist[r, l])
            if c:
                lmax[r] = l
            if l >= lmin:
                num += l * c
                den += c
        L[r] = float(num) / float(den) if den else float("nan")
    return L, lmax


def sorting_rate(measure):
    """Sorting rate S of Eq. 5 in percent.  measure[i][j] is the measure of
    realisation i's series of SNR index j (SNRs ascending).  x_j is the
    position (1-based) of series j when realisation i's series are ordered by
    ascending measure (equal values keep their SNR order; NaN after every
    number), y_j = j and z the reversed y:
      S = 100 (sum_i sum_j |z_j - y_j| - sum_i sum_j |x_j - y_j|)
              / sum_i sum_j |z_j - y_j|.
    Plain loops: the position of series j counts the series before it."""
    def before(a, ka, b, kb):
        # does (value a, index ka) sort before (value b, index kb)?
        na, nb = a != a, b != b
        if na != nb:
            return nb
        if not na and a != b:
            return a < b
        return ka < kb
    worst = 0
    dep = 0
    for row in measure:
        n = len(row)
        for j in range(n):
            pos = 1 + sum(1 for k in range(n) if k != j and before(float(row[k]), k, float(row[j]), j))
            dep += abs(pos - (j + 1))
            worst += abs((n - j) - (j + 1))
    return 100.0 * (worst - dep) / worst


def grid_select(y, m, tau, norm, w, targets, n_grid=400):
    """The grid-threshold variant (a commented-out paragraph of the Averaged
    RQA section): y rescaled to [0, 1] (float64, then float32), RR at the
    thresholds i / n_grid (i = 1..n_grid; squared for the Euclidean key),
    and per target the grid threshold whose RR is closest (the first on
    ties).  Returns (eps, rr, |rr - target|) per target."""
    y = np.asarray(y, dtype=np.float64)
    lo, hi = float(y.min()), float(y.max())
    y01 = ((y - lo) / (hi - lo)).astype(np.float32)
    grid = []
    for i in range(1, n_grid + 1):
        e = i / n_grid
        grid.append(e if norm == NORM_MAX else e * e)
    grid = np.array(grid, dtype=np.float32)
    _, le = count(y01, m, tau, norm, w, grid)
    M = num_pairs(num_vectors(len(y01), m, tau), w)
    rr = [int(c) / M for c in le]
    eps_out, rr_out, err = [], [], []
    for t in targets:
        best = 0
        for i in range(1, len(rr)):
            if abs(rr[i] - t) < abs(rr[best] - t):
                best = i
        eps_out.append(grid[best])
        rr_out.append(rr[best])
        err.append(abs(rr[best] - t))
    return (np.array(eps_out, dtype=np.float32), np.array(rr_out, dtype=np.float64),
            np.array(err, dtype=np.float64))


def num_threads():
    return int(_load().orc_num_threads())
