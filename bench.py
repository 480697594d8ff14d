#!/usr/bin/env python3
"""Benchmark of the averaged-RQA hot path on one MI355X.

A step is one whole pass of the path over the large workload: exact
threshold selection for K = 20 target recurrence rates (two radix counting
passes, the last bits resolved by the line sweep) and the line sweep giving
RR, DET and the averaged DET, for both large series (Lorenz-x + 0 dB noise
and logistic r=4 + -10 dB noise, N = 10^5, m = 3, tau = 5, Euclidean norm,
Theiler window 1, l_min = 2), as one rqa_batch call with plain selection.
Inputs are resident in device memory before the timed region.

value = pairs x thresholds per second over the timed steps, where pairs are
the M = (Nv-1) Nv / 2 upper-triangle pairs each series has.

Also reported (outside the timed steps): the same step with the sketch
window and the trained network's window, the 600-series batched ensemble
(series/s, batched against one call per series), the network on 200
held-out series, per-phase device times from HIP events on the library's
stream, the roofline of the dominant kernel (with counter-derived traffic
and VALU rate when the stored counters match the sources) and the CPU
oracle timed on a bounded sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "recurrence cells x thresholds/s at N=1e5, K=20 (+ batched series/s), % VALU peak"
K = 20
# VALU peak of MI355X in lane-ops/s: the FP32 vector peak of 157.3 TFLOP/s
# counts an FMA as two, i.e. 256 CUs x 128 lanes x 2.4 GHz one-op lane slots.
VALU_PEAK = 157.3e12 / 2
# Algorithmic VALU lane-ops of one key for (norm, m): the m subtractions, the
# m |.| or squares and the m-1 max or add steps.
def key_ops(norm, m):
    return 3 * m - 1


def cells_of(case):
    nv = len(case["y"]) - (case["m"] - 1) * case["tau"]
    a = nv - case["theiler"]
    return a * (a + 1) // 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true", help="skip the 600-series ensemble")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=15_000,
                    help="prefix length of the Lorenz series the oracle is timed on")
    ap.add_argument("--tune-file", default=None,
                    help="load launch shapes from this file if it exists, else tune and save them there")
    ap.add_argument("--no-bracket", action="store_true", help="skip the learned-bracket evaluation")
    ap.add_argument("--no-hist", action="store_true", help="skip the full line-length histogram")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the plain step only (no windowed selection, K = 99 or histogram lines)")
    ap.add_argument("--bracket-file", default=os.path.join(ROOT, "paper_2208_09136_amd", "bracket_params.npz"),
                    help="trained bracket network (written by paper_2208_09136_amd.bracket)")
    ap.add_argument("--bracket-series", type=int, default=200)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def sources_digest():
    """SHA-256 over the device sources, to tell whether stored counters still
    describe the kernels being run."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2208_09136_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


COUNTERS = os.path.join(ROOT, "profiles", "counters_n1e5_k20.json")


def stored_counters():
    """Per-launch hardware counters of the timed kernels (rocprofv3 --pmc,
    summarised in profiles/), or None when absent or taken on other sources."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    return c if c.get("sources_sha256") == sources_digest() else None


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the path shards by diagonal "
                                   "bands across GPUs in design only", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2208_09136_amd import rqa

    cases = synth.config_large()
    prm = [(c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"]) for c in cases]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    dev = torch.device("cuda:0")
    concat = torch.from_numpy(np.concatenate(ys)).to(dev)
    rr = np.stack([c["rr"] for c in cases])
    cells = [cells_of(c) for c in cases]
    cell_thr = sum(cells) * K

    stream = torch.cuda.current_stream()
    ctx = rqa.Context(0, stream)
    # launch shapes from the library's autotuner (timed trials on this workload;
    # shapes never change results)
    t_tune = time.perf_counter()
    if args.tune_file and os.path.exists(args.tune_file):
        ctx.tune_load(args.tune_file)
        tuned_chunk = None
    else:
        tuned_chunk = ctx.autotune_batch(concat, offs, prm, rr)
        if args.tune_file:
            ctx.tune_save(args.tune_file)
    t_tune = time.perf_counter() - t_tune
    ctx.set_timing(True)

    ref = None
    for _ in range(args.warmup):
        ref = ctx.batch(concat, offs, prm, rr)
    torch.cuda.synchronize()
    phases = np.zeros(len(rqa.PHASES))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.batch(concat, offs, prm, rr)
        phases += np.array([ctx.phase_times()[p] for p in rqa.PHASES])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if ref is not None:
        assert np.array_equal(ref["det_mean"], out["det_mean"]), "results changed between steps"
    sec = (t1 - t0) / args.steps
    value = cell_thr / sec
    ph = dict(zip(rqa.PHASES, (phases / args.steps).tolist()))

    # roofline of the dominant kernel: the phase with the largest device time;
    # one launch per phase per step.  Algorithmic lane-ops per pair: the key
    # (3m - 1), then per counting pass 6 (bucket, table lookup, count) and for
    # the line sweep 2 per threshold (one comparison, one run-length update)
    # plus the 6 of the last radix pass it takes over.
    kops = key_ops(1, 3)
    per_launch_ops = {
        "select_pass1": sum(cells) * (kops + 6),
        "select_pass2": sum(cells) * (kops + 6),
        "sweep": sum(cells) * (kops + 6 + 2 * K),
    }
    dom = max(per_launch_ops, key=lambda p: ph[p])
    achieved = per_launch_ops[dom] / (ph[dom] * 1e-3)
    step_ops = sum(per_launch_ops.values())
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
                "algorithmic_ops_per_launch": per_launch_ops[dom], "launch_ms": ph[dom]}
    counters = stored_counters()
    if counters and dom in counters.get("kernels", {}):
        kc = counters["kernels"][dom]
        # HBM bytes per launch from FETCH_SIZE + WRITE_SIZE, each scaled by
        # the factor a plain copy of known size gave for that counter
        if kc.get("fetch_bytes") is not None and kc.get("write_bytes") is not None:
            roofline["traffic"] = kc["fetch_bytes"] + kc["write_bytes"]
            roofline["traffic_unit"] = "bytes/launch"
        if kc.get("valu_insts") is not None:
            # executed VALU instructions x 64 lanes against the same peak
            roofline["valu_lane_ops_measured"] = kc["valu_insts"] * 64
            roofline["valu_busy_frac"] = kc["valu_insts"] * 64 / (ph[dom] * 1e-3) / VALU_PEAK

    # the same step with windowed selection (sketch-sample window, and the
    # trained network's window when present): identical results, fewer passes
    windows = {}
    from paper_2208_09136_amd import bracket
    have_net = not args.no_bracket and os.path.exists(args.bracket_file)
    if have_net:
        bracket.load(ctx, args.bracket_file)
    for name, flags in (("sample", rqa.RQA_SEL_SAMPLE), ("network", rqa.RQA_SEL_LEARNED)):
        if args.no_extras or (name == "network" and not have_net):
            continue
        got = ctx.batch(concat, offs, prm, rr, flags=flags)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            got = ctx.batch(concat, offs, prm, rr, flags=flags)
        torch.cuda.synchronize()
        wsec = (time.perf_counter() - t0) / args.steps
        st = ctx.selection_stats()
        wph = ctx.phase_times()
        windows[name] = {"ms_per_step": wsec * 1e3, "value": cell_thr / wsec, "full_passes": st["full_passes"],
                         "phases_ms": wph,
                         "series_fallback": st["series_fallback"],
                         "identical": bool(all(np.array_equal(got[k], out[k]) for k in ("eps", "count", "det"))),
                         "speedup_vs_plain": sec / wsec}

    k99 = None if args.no_extras else bench_k99(ctx, torch, rqa, concat, offs, prm, len(cases), sum(cells),
                                                 args.steps)
    full_hist = None if (args.no_hist or args.no_extras) else bench_hist(ctx, torch, concat, offs, prm, out["eps"],
                                                                          args.steps)
    sorting = None if args.no_extras else bench_sorting(ctx)

    result = {
        "metric": METRIC, "value": value, "unit": "cell-thresholds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2 series x N=1e5 (Lorenz-x 0 dB, logistic r=4 -10 dB), m=3, tau=5, "
                               "Euclidean, Theiler 1, l_min 2, K=20 RR 0.01..0.20; exact selection + DET",
                   "pairs_per_series": cells, "K": K, "global_batch": len(cases), "seq_len": 100_000,
                   "parallelism": "single-gpu"},
        "phases_ms": ph,
        "autotune": {"chunk_tiles": tuned_chunk, "seconds": t_tune},
        "valu_peak_frac": step_ops / sec / VALU_PEAK,
        "roofline": roofline,
        "windowed_selection": windows,
        "k99": k99,
        "full_histogram": full_hist,
        "sorting_rate": sorting,
        "det_mean": out["det_mean"].tolist(),
    }

    if not args.no_batch:
        result["batched"] = bench_batch(ctx, torch, rqa)

    if not args.no_bracket:
        result["learned_bracket"] = bench_bracket(ctx, torch, args)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(cases[0], args.cpu_sample)

    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = n

    ctx.close()
    print(json.dumps(result), flush=True)


def bench_k99(ctx, torch, rqa, concat, offs, prm, nseries, cells, steps):
    """The paper's RR set 1..99 % on the bench series (averaged-DET curve over RR*)."""
    rr99 = np.tile(np.array([k / 100.0 for k in range(1, 100)]), (nseries, 1))
    got99 = ctx.batch(concat, offs, prm, rr99)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        got99 = ctx.batch(concat, offs, prm, rr99)
    torch.cuda.synchronize()
    sec99 = (time.perf_counter() - t0) / steps
    ph99 = ctx.phase_times()
    # the same with the sketch-sample window (identical results)
    win = ctx.batch(concat, offs, prm, rr99, flags=rqa.RQA_SEL_SAMPLE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        win = ctx.batch(concat, offs, prm, rr99, flags=rqa.RQA_SEL_SAMPLE)
    torch.cuda.synchronize()
    secw = (time.perf_counter() - t0) / steps
    return {"ms_per_step": sec99 * 1e3, "value": cells * 99 / sec99, "unit": "cell-thresholds/s",
            "phases_ms": ph99,
            "sample_window_ms_per_step": secw * 1e3,
            "sample_window_identical": bool(all(np.array_equal(win[k], got99[k]) for k in ("eps", "count", "det"))),
            "averaged_det_curve_end": [float(rqa.rqa_averaged_det(d)[-1]) for d in got99["det"]]}


def bench_sorting(ctx, lengths=(100, 1000, 10_000), grid_realisations=1):
    """Sorting rate S (Eq. 5) of the paper's ensemble (sine of 25 cycles,
    logistic r = 3.679, Lorenz-x; linear SNR levels 0.1, 1, 10; 10 SNRs x 10
    realisations per cell; maximum norm, m = 1 or m = 3 / tau = 3 for
    Lorenz) ordered by the averaged DET over RR* = 1..99 % and by DET at
    RR = 1 %, and the grid-threshold variant's RR error against exact
    selection on one realisation per cell."""
    from paper_2208_09136_amd import harness
    t0 = time.perf_counter()
    table, gerr, eerr = [], [], []
    gpu = 0.0
    for system in synth.SYSTEMS:
        m, tau = synth.paper_embedding(system)
        params = (m, tau, 0, 1, 2)
        for level in synth.SNR_LEVELS:
            for n in lengths:
                ens = synth.paper_ensemble(system, n, level)
                t1 = time.perf_counter()
                avg, first = harness.ensemble_measures(ctx, ens, params)
                gpu += time.perf_counter() - t1
                table.append({"system": system, "snr_level": level, "n": n,
                              "S_det_avg_99_pct": harness.sorting_rate(avg),
                              "S_det_1_pct": harness.sorting_rate(first)})
                for r in range(grid_realisations):
                    for y in ens[r]:
                        g, e = harness.grid_vs_exact(ctx, y, params)
                        gerr.append(g)
                        eerr.append(e)
    gerr, eerr = np.concatenate(gerr), np.concatenate(eerr)
    wins = sum(1 for row in table if row["S_det_avg_99_pct"] > row["S_det_1_pct"])
    ties = sum(1 for row in table if row["S_det_avg_99_pct"] == row["S_det_1_pct"])
    return {"workload": f"{len(table)} cells x 100 series, lengths {list(lengths)}, K = 99 per series",
            "table": table, "cells_avg_better": wins, "cells_equal": ties,
            "batch_seconds": gpu, "seconds": time.perf_counter() - t0,
            "grid_variant": {"targets": int(gerr.size),
                             "grid_rr_error_pct": {"mean": 100 * float(gerr.mean()), "max": 100 * float(gerr.max())},
                             "exact_rr_error_pct": {"mean": 100 * float(eerr.mean()),
                                                    "max": 100 * float(eerr.max())}}}


def bench_hist(ctx, torch, concat, offs, prm, eps, steps):
    """Full diagonal line-length histogram P_r(l) (every length, hist_len =
    nv + 1) at each series' selected thresholds: device time of the histogram
    pass (segment pass + border join), and the identity sum_l l P_r(l) = C_r
    against the sweep's counts."""
    rows = []
    for i, p in enumerate(prm):
        y = concat[int(offs[i]):int(offs[i + 1])]
        nv = int(offs[i + 1] - offs[i]) - (p[0] - 1) * p[1]
        got = ctx.det_curve(y, p, eps[i], hist_len=nv + 1)
        torch.cuda.synchronize()
        hms = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            got = ctx.det_curve(y, p, eps[i], hist_len=nv + 1)
            hms += ctx.phase_times()["histogram"]
        wsec = (time.perf_counter() - t0) / steps
        h = got["hist"].astype(np.int64)
        lens = np.arange(h.shape[1], dtype=np.int64)
        nz = np.nonzero(h.sum(axis=0))[0]
        from paper_2208_09136_amd import rqa
        L, lmax = rqa.rqa_line_measures(got["hist"], p[4])
        rows.append({"histogram_ms": hms / steps, "call_ms": wsec * 1e3,
                     "longest_line": int(nz.max()) if len(nz) else 0,
                     "L_mean_over_thresholds": float(rqa.rqa_averaged_det(L)[-1]),
                     "Lmax_mean_over_thresholds": float(lmax.astype(np.float64).mean()),
                     "sum_l_P_equals_C": bool(np.array_equal((h * lens).sum(axis=1).astype(np.uint64),
                                                             got["count"]))})
    return {"workload": "each bench series at its 20 selected thresholds, every length kept",
            "series": rows}


def bench_batch(ctx, torch, rqa, reps=3):
    """The 600-series ensemble (3 systems x 10 SNRs x 20 realisations, lengths
    log-uniform in [100, 2e4]) in one rqa_batch call, against one rqa_run call
    per series on the same GPU."""
    cases = synth.config_batch()
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    concat = torch.from_numpy(np.concatenate(ys)).to("cuda:0")
    prm = [(c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"]) for c in cases]
    rr = np.stack([c["rr"] for c in cases])
    cells = sum(cells_of(c) for c in cases)
    t_tune = time.perf_counter()
    chunk = ctx.autotune_batch(concat, offs, prm, rr)
    t_tune = time.perf_counter() - t_tune
    ctx.batch(concat, offs, prm, rr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = ctx.batch(concat, offs, prm, rr)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    singles = [torch.from_numpy(y).to("cuda:0") for y in ys]
    for s in range(3):
        ctx.run(singles[s], prm[s], rr[s])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    for s in range(len(cases)):
        o = ctx.run(singles[s], prm[s], rr[s])
        same &= bool(np.array_equal(o["det"], out["det"][s]))
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    return {"series": len(cases), "pairs": int(cells), "ms": tb * 1e3, "series_per_s": len(cases) / tb,
            "cell_thresholds_per_s": cells * K / tb, "single_calls_ms": ts * 1e3,
            "single_series_per_s": len(cases) / ts, "batched_over_single": ts / tb,
            "equal_to_single": same, "autotune_chunk_tiles": chunk, "autotune_seconds": t_tune}


def bench_bracket(ctx, torch, args):
    """Held-out evaluation of the threshold-bracket network: 200 series at
    N = 5e4 (three systems, SNR ~ U[-25, 20] dB, m = 3, tau = 5, Euclidean,
    K = 20) in one rqa_batch call with plain selection, with the network's
    window and with the sketch-sample window; results must be identical."""
    from paper_2208_09136_amd import bracket
    if not os.path.exists(args.bracket_file):
        return {"skipped": "no trained network at " + os.path.relpath(args.bracket_file, ROOT)}
    meta = bracket.load(ctx, args.bracket_file)
    n = 50_000
    c, o, p, _, _ = synth.bracket_set(args.bracket_series, 13, n, n, m=3)
    rr = np.tile(np.array(synth.RR_20), (args.bracket_series, 1))
    ev = bracket.evaluate(ctx, torch.from_numpy(c).to("cuda:0"), o, p, rr)
    pairs = args.bracket_series * ((n - 10 - 1) * (n - 10) // 2)
    for name in ("plain", "network", "sample"):
        ev[name]["cell_thresholds_per_s"] = pairs * K / ev[name]["seconds"]
    ev["workload"] = (f"{args.bracket_series} held-out series x N={n} (sine, logistic, Lorenz-x; "
                      "SNR U[-25,20] dB), m=3, tau=5, Euclidean, K=20; select + sweep")
    ev["network"]["trained_on"] = meta.get("train")
    return ev


def cpu_baseline(case, n_sample):
    """The CPU oracle (plain C, OpenMP over diagonals) on a prefix of the Lorenz
    series with the same parameters: exact selection (sort path) and the
    per-threshold run-length pass."""
    import oracle
    y = case["y"][:n_sample]
    sub = dict(case, y=y)
    t0 = time.perf_counter()
    oracle.run(y, case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"], case["rr"])
    dt = time.perf_counter() - t0
    cells = cells_of(sub)
    return {"value": cells * K / dt, "unit": "cell-thresholds/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": dt,
            "sample": f"first {n_sample} samples of the Lorenz-x 0 dB series, m=3, tau=5, Euclidean, "
                      f"K=20: {cells} pairs, selection + lines"}


if __name__ == "__main__":
    main()
