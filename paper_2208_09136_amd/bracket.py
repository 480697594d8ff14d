"""Threshold-bracket network: training set, training, calibration and
evaluation.

The network (66 -> 128 -> 128 -> 20, GELU) maps the distance sketch of a
series (a 64-bin histogram of 4096 sampled keys around their median, plus
log2 N / 16 and m / 4) to the offsets t_r = (bits(eps_r) - bits(scale)) / 2^23
of its exact thresholds eps_r, i.e. approximately log2(eps_r / scale).  The
library turns the prediction into one key window per series
[scale * 2^(t_r - d_r), scale * 2^(t_r + d_r)] (union over r); exact selection
inside that window takes two counting passes instead of three, and a series
whose threshold falls outside it is selected again by the plain three-pass
radix refinement, so every threshold stays the exact order statistic.  This
is an extension of the method; the paper selects thresholds by recurrence
rate (Methodology section) but predicts nothing.

Everything numerical runs in the library: sketches (rqa_sketch_batch), exact
targets (rqa_batch with plain selection), training (rqa_mlp_train_step: the
library's forward, backward and Adam kernels) and the windowed selection.
This module only moves arrays, standardises inputs and targets on the host
(folded into the first and last layers afterwards), and keeps score.
"""
import json
import math
import time

import numpy as np

from . import rqa

SKETCH_SEED = 0   # series s of a call uses stream seed + s, as selection does


def _torch():
    import torch
    return torch


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def targets(eps, scale):
    """t_r = (bits(eps_r) - scale) / 2^23 for eps (S, K) float32 and scale (S,) uint32."""
    bits = np.ascontiguousarray(eps, dtype=np.float32).view(np.uint32).astype(np.int64)
    return ((bits - scale.astype(np.int64)[:, None]) / 8388608.0).astype(np.float64)


def examples(ctx, concat, offsets, params, rr, chunk=2048, seed=SKETCH_SEED, log=None):
    """(features (S, 66) float32, targets (S, K) float64, scale (S,) uint32)
    of S series back to back in host array `concat`: features from the
    sketch, targets from exact plain selection.  Works through the series in
    chunks so device memory stays bounded."""
    torch = _torch()
    offsets = np.asarray(offsets, dtype=np.uint64)
    S = len(offsets) - 1
    rr = np.asarray(rr, dtype=np.float64)
    feats = np.zeros((S, rqa.SKETCH_FEATURES), np.float32)
    tgts = np.zeros((S, rr.shape[1]), np.float64)
    scales = np.zeros(S, np.uint32)
    for a in range(0, S, chunk):
        b = min(S, a + chunk)
        lo, hi = int(offsets[a]), int(offsets[b])
        y = _dev(concat[lo:hi])
        offs = offsets[a:b + 1] - offsets[a]
        f, sc = ctx.sketch_batch(y, offs, params[a:b], seed)
        res = ctx.batch(y, offs, params[a:b], rr[a:b])
        feats[a:b], scales[a:b] = f, sc
        tgts[a:b] = targets(res["eps"], sc)
        del y
        torch.cuda.synchronize()
        if log:
            log(f"examples {b}/{S}")
    return feats, tgts, scales


class Standardiser:
    """Per-column affine maps x -> (x - mu) / sd of inputs and targets; the
    trained network on standardised data is folded back into one that takes
    raw features and returns raw offsets."""

    def __init__(self, X, T, floor=1e-3):
        self.mx = X.mean(0)
        self.sx = np.maximum(X.std(0), floor)
        self.mt = T.mean(0)
        self.st = np.maximum(T.std(0), floor)

    def x(self, X):
        return (X - self.mx) / self.sx

    def t(self, T):
        return (T - self.mt) / self.st

    def fold(self, theta):
        """Parameters of the network f'(x) = mt + st * f((x - mx) / sx)."""
        IN, H, OUT = rqa.MLP_INPUTS, 128, rqa.MLP_OUTPUTS
        th = np.asarray(theta, dtype=np.float64).copy()
        o_b1 = IN * H
        o_W3 = o_b1 + H + H * H + H
        o_b3 = o_W3 + H * OUT
        W1 = th[:o_b1].reshape(IN, H)
        b1 = th[o_b1:o_b1 + H]
        W1f = W1 / self.sx[:, None]
        b1f = b1 - (self.mx / self.sx) @ W1
        W3 = th[o_W3:o_b3].reshape(H, OUT)
        b3 = th[o_b3:o_b3 + OUT]
        th[:o_b1] = W1f.ravel()
        th[o_b1:o_b1 + H] = b1f
        th[o_W3:o_b3] = (W3 * self.st[None, :]).ravel()
        th[o_b3:o_b3 + OUT] = b3 * self.st + self.mt
        return th.astype(np.float32)


def fit(ctx, X, T, epochs=40, batch=256, lr=2e-3, seed=1, log=None):
    """Train on (X, T) with the library's kernels (Adam, cosine-decayed
    learning rate); leaves the folded network in the context and returns
    (params float32, loss per epoch)."""
    torch = _torch()
    std = Standardiser(X, T)
    Xs = std.x(X).astype(np.float32)
    Ts = std.t(T).astype(np.float32)
    n = len(Xs)
    rng = np.random.default_rng(seed)
    ctx.mlp_init(seed)
    steps = epochs * max(1, n // batch)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        xd, td = _dev(Xs[perm]), _dev(Ts[perm])
        tot = 0.0
        nb = max(1, n // batch)
        for i in range(nb):
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / steps))
            tot += ctx.mlp_train_step(xd[i * batch:(i + 1) * batch], td[i * batch:(i + 1) * batch], cur)
            step += 1
        hist.append(tot / nb)
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep} loss {hist[-1]:.5f}")
        del xd, td
    theta = std.fold(ctx.mlp_get_params())
    ctx.mlp_set_params(theta)
    torch.cuda.synchronize()
    return theta, hist


def predict(ctx, X):
    torch = _torch()
    xd = _dev(X)
    yd = torch.zeros((len(X), rqa.MLP_OUTPUTS), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(xd, yd)
    return yd.cpu().numpy().astype(np.float64)


def calibrate(ctx, X, T, quantile=0.999, margin=1.25, floor=1.0 / 256):
    """Half-widths d_r = margin * quantile of |prediction - target| over a
    validation set (at least `floor`); sets them in the context."""
    err = np.abs(predict(ctx, X) - T)
    delta = np.maximum(margin * np.quantile(err, quantile, axis=0), floor).astype(np.float32)
    ctx.mlp_set_bracket(delta)
    return delta, err


def _timed(fn, repeats):
    torch = _torch()
    best = float("inf")
    out = None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return out, best


def evaluate(ctx, concat, offsets, params, rr, repeats=3):
    """Plain, network-window and sample-window selection (each followed by
    the sweep) on one batch: results must agree exactly; returns timings,
    passes per series and miss rates."""
    y = _dev(concat) if isinstance(concat, np.ndarray) else concat
    offsets = np.asarray(offsets, dtype=np.uint64)
    S = len(offsets) - 1
    rr = np.asarray(rr, dtype=np.float64)
    out = {"series": S}
    ref = None
    ctx.set_timing(True)
    for name, flags in (("plain", rqa.RQA_SEL_PLAIN), ("network", rqa.RQA_SEL_LEARNED),
                        ("sample", rqa.RQA_SEL_SAMPLE)):
        ctx.batch(y, offsets, params, rr, flags=flags)        # warm-up
        res, secs = _timed(lambda: ctx.batch(y, offsets, params, rr, flags=flags), repeats)
        st = ctx.selection_stats()
        ph = ctx.phase_times()
        if ref is None:
            ref = res
        exact = all(np.array_equal(res[k], ref[k]) for k in ("eps", "count", "det", "det_mean"))
        fb = st["series_fallback"]
        out[name] = {"seconds": secs, "exact": bool(exact), "series_fallback": fb,
                     "targets_missed": st["targets_missed"],
                     "passes_per_series": 3.0 if flags == rqa.RQA_SEL_PLAIN else 2.0 + 3.0 * fb / S,
                     "selection_passes_ms": ph["select_pass1"] + ph["select_pass2"] + ph["select_pass3"],
                     "sweep_ms": ph["sweep"], "other_ms": ph["other"]}
    ctx.set_timing(False)
    for name in ("network", "sample"):
        out[name]["speedup_vs_plain"] = out["plain"]["seconds"] / out[name]["seconds"]
        out[name]["selection_speedup_vs_plain"] = (out["plain"]["selection_passes_ms"]
                                                   / out[name]["selection_passes_ms"])
        out[name]["miss_rate"] = out[name]["series_fallback"] / S
        out[name]["passes_saved_per_series"] = 3.0 - out[name]["passes_per_series"]
    return out


def window_widths(ctx, feats, scales, delta):
    """log2 width of each series' network window (hi / lo of the key window)."""
    pred = predict(ctx, feats)
    lo = (pred - delta[None, :]).min(1)
    hi = (pred + delta[None, :]).max(1)
    return hi - lo


def save(path, theta, delta, meta):
    np.savez(path, params=np.asarray(theta, np.float32), delta=np.asarray(delta, np.float32),
             meta=np.array(json.dumps(meta)))


def load(ctx, path):
    """Load trained parameters and half-widths into the context; returns meta."""
    z = np.load(path, allow_pickle=False)
    ctx.mlp_set_params(z["params"])
    ctx.mlp_set_bracket(z["delta"])
    return json.loads(str(z["meta"]))


def main(argv=None):
    import argparse
    import torch
    import synth

    ap = argparse.ArgumentParser(description="train, calibrate and evaluate the threshold-bracket network")
    ap.add_argument("--train", type=int, default=50_000, help="training series (one example each)")
    ap.add_argument("--val", type=int, default=5_000, help="validation series (calibration)")
    ap.add_argument("--test", type=int, default=200, help="held-out evaluation series")
    ap.add_argument("--n-lo", type=int, default=1_000)
    ap.add_argument("--n-hi", type=int, default=100_000)
    ap.add_argument("--n-test", type=int, default=50_000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--out", default="bracket_params.npz")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[bracket {time.strftime('%H:%M:%S')}] {msg}", flush=True)

    ctx = rqa.Context(0, torch.cuda.current_stream())
    K = len(synth.RR_20)
    report = {"args": vars(a)}

    def make(count, seed, lo, hi, m):
        t0 = time.perf_counter()
        c, o, p, sy, sn = synth.bracket_set(count, seed, lo, hi, m=m)
        log(f"generated {count} series ({o[-1] / 1e6:.1f} M samples) in {time.perf_counter() - t0:.1f} s")
        return c, o, p, np.tile(np.array(synth.RR_20), (count, 1))

    tr = make(a.train, a.seed, a.n_lo, a.n_hi, None)
    t0 = time.perf_counter()
    Xtr, Ttr, _ = examples(ctx, *tr, log=log)
    report["train_examples_seconds"] = time.perf_counter() - t0
    va = make(a.val, a.seed + 1, a.n_lo, a.n_hi, None)
    Xva, Tva, _ = examples(ctx, *va, log=log)
    t0 = time.perf_counter()
    theta, hist = fit(ctx, Xtr, Ttr, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    report["train_seconds"] = time.perf_counter() - t0
    report["loss_first_last"] = [hist[0], hist[-1]]
    delta, err = calibrate(ctx, Xva, Tva)
    report["val_rmse"] = float(np.sqrt(np.mean((predict(ctx, Xva) - Tva) ** 2)))
    report["delta"] = [float(d) for d in delta]
    log(f"validation rmse {report['val_rmse']:.4f}, half-widths {delta.min():.3f}..{delta.max():.3f}")

    te = make(a.test, a.seed + 2, a.n_test, a.n_test, 3)
    Xte, Tte, Ste = examples(ctx, *te)
    report["test_rmse"] = float(np.sqrt(np.mean((predict(ctx, Xte) - Tte) ** 2)))
    w = window_widths(ctx, Xte, Ste, delta)
    report["test_window_log2_width_median"] = float(np.median(w))
    ev = evaluate(ctx, *te)
    report["evaluation"] = ev
    log(json.dumps(ev))
    save(a.out, theta, delta, {"val_rmse": report["val_rmse"], "train": a.train, "seed": a.seed,
                              "sketch_seed": SKETCH_SEED})
    if a.json:
        with open(a.json, "w") as f:
            json.dump(report, f, indent=1)
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
