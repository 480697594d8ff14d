"""Evaluation harnesses of the paper, on top of librqa.

Host logic only: every pair of every series is evaluated by the library's
kernels through the binding.

* Sorting rate S (Methodology section, Eq. 5): an ensemble of 10 series of
  increasing SNR per realisation is ordered by a measure (the averaged DET
  over RR* = 1..99 %, or DET at one RR); S compares the order with the true
  SNR order, 100 % for a perfect sort and 0 % for the reversed one.
* Grid-threshold variant (Averaged RQA section, a commented-out paragraph):
  the series is rescaled to [0, 1], RR is computed at 400 fixed thresholds
  and each target RR takes the grid threshold whose RR is closest; its RR
  error is compared with exact selection's.

Readings where the paper is silent: the measure is sorted ascending with a
stable sort (equal values keep the SNR order), a NaN DET sorts last; grid
thresholds are i / 400 for i = 1..400 in distance units (squared for the
Euclidean key), ties in |RR - target| go to the smaller threshold.
"""
import numpy as np

from . import rqa

RR_STAR = tuple(k / 100.0 for k in range(1, 100))   # 1 %, 2 %, ..., 99 %
GRID = 400


def sorting_rate(measure):
    """S in percent for measure[i][j] = the measure of realisation i's series
    of SNR index j (ascending SNR): 100 (worst - departure) / worst, with
    departure = sum over realisations of sum_j |x_j - y_j| (x_j the position
    of series j in the ascending order of the measure, y_j = j) and worst
    the same sum for the reversed order."""
    m = np.asarray(measure, dtype=np.float64)
    if m.ndim != 2 or m.shape[1] < 2:
        raise ValueError("measure must be (realisations, series >= 2)")
    R, n = m.shape
    y = np.arange(1, n + 1, dtype=np.int64)
    worst = R * int(np.abs(y[::-1] - y).sum())
    dep = 0
    for i in range(R):
        order = np.argsort(m[i], kind="stable")
        x = np.empty(n, dtype=np.int64)
        x[order] = y
        dep += int(np.abs(x - y).sum())
    return 100.0 * (worst - dep) / worst


def ensemble_measures(ctx, ensemble, params, rr=RR_STAR):
    """DET at every target of rr for each series of ensemble (a list over
    realisations of lists over SNRs of float32 host series), in one
    rqa_batch call.  Returns (det_avg, det_first): the averaged DET over the
    targets and DET at the first target, each (realisations, SNRs)."""
    import torch
    R, n = len(ensemble), len(ensemble[0])
    flat = [y for row in ensemble for y in row]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in flat])]).astype(np.uint64)
    dev = torch.from_numpy(np.concatenate(flat).astype(np.float32)).to("cuda:0")
    rr_all = np.tile(np.asarray(rr, dtype=np.float64), (len(flat), 1))
    out = ctx.batch(dev, offs, [params] * len(flat), rr_all)
    det = out["det"].reshape(R, n, len(rr))
    avg = np.array([[rqa.rqa_averaged_det(det[i, j])[-1] for j in range(n)] for i in range(R)])
    return avg, det[:, :, 0].copy()


def rescale01(y):
    """(y - min) / (max - min) in float64, returned as float32 (the paper's
    transformation of every series into [0, 1])."""
    y = np.asarray(y, dtype=np.float64)
    lo, hi = float(y.min()), float(y.max())
    if hi <= lo:
        raise ValueError("constant series")
    return ((y - lo) / (hi - lo)).astype(np.float32)


def grid_thresholds(norm, n_grid=GRID):
    """The fixed grid in key units: i / n_grid (i = 1..n_grid) for the
    maximum norm, its square for the squared-Euclidean key."""
    e = np.arange(1, n_grid + 1, dtype=np.float64) / n_grid
    return (e if norm == 0 else e * e).astype(np.float32)


def grid_rr(ctx, series_dev, params, eps, chunk=100):
    """RR at every threshold of eps (rqa_det_curve in chunks)."""
    out = np.empty(len(eps), dtype=np.float64)
    for a in range(0, len(eps), chunk):
        out[a:a + chunk] = ctx.det_curve(series_dev, params, eps[a:a + chunk])["rr"]
    return out


def grid_select(rr_grid, eps, targets):
    """Per target the grid threshold whose RR is closest (first on ties):
    (eps_sel, rr_sel, |rr_sel - target|)."""
    rr_grid = np.asarray(rr_grid, dtype=np.float64)
    idx = np.array([int(np.argmin(np.abs(rr_grid - t))) for t in targets], dtype=np.int64)
    rr_sel = rr_grid[idx]
    return np.asarray(eps)[idx], rr_sel, np.abs(rr_sel - np.asarray(targets, dtype=np.float64))


def grid_vs_exact(ctx, y, params, targets=RR_STAR, n_grid=GRID):
    """RR errors (fractions) of the grid variant and of exact selection on
    the [0, 1]-rescaled series y (host float32)."""
    import torch
    y01 = rescale01(y)
    dev = torch.from_numpy(y01).to("cuda:0")
    eps = grid_thresholds(params[2], n_grid)
    _, _, err_grid = grid_select(grid_rr(ctx, dev, params, eps), eps, targets)
    exact = ctx.run(dev, params, targets)
    err_exact = np.abs(exact["rr"] - np.asarray(targets, dtype=np.float64))
    return err_grid, err_exact


def main():
    """Full sorting-rate table and grid-variant errors (lengths 10^2..10^5)."""
    import argparse
    import json
    import os
    import sys
    import time
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--lengths", default="100,1000,10000,100000")
    ap.add_argument("--realisations", type=int, default=10)
    ap.add_argument("--grid-series", type=int, default=2, help="realisations per cell for the grid variant")
    args = ap.parse_args()
    lengths = [int(v) for v in args.lengths.split(",")]
    ctx = rqa.Context(0, torch.cuda.current_stream())
    rows = []
    gerr, eerr = [], []
    t0 = time.perf_counter()
    for system in synth.SYSTEMS:
        m, tau = synth.paper_embedding(system)
        params = (m, tau, 0, 1, 2)
        for level in synth.SNR_LEVELS:
            for n in lengths:
                ens = synth.paper_ensemble(system, n, level, args.realisations)
                avg, first = ensemble_measures(ctx, ens, params)
                rows.append({"system": system, "level": level, "n": n,
                             "S_det_avg_99": sorting_rate(avg), "S_det_1": sorting_rate(first)})
                print(json.dumps(rows[-1]), flush=True)
                for r in range(min(args.grid_series, args.realisations)):
                    for y in ens[r]:
                        g, e = grid_vs_exact(ctx, y, params)
                        gerr.append(g)
                        eerr.append(e)
    gerr, eerr = np.concatenate(gerr), np.concatenate(eerr)
    print(json.dumps({"grid_rr_error_pct": {"mean": 100 * float(gerr.mean()), "max": 100 * float(gerr.max()),
                                            "targets": int(gerr.size)},
                      "exact_rr_error_pct": {"mean": 100 * float(eerr.mean()), "max": 100 * float(eerr.max())},
                      "seconds": time.perf_counter() - t0}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
