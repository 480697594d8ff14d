#!/usr/bin/env python3
"""Benchmark of the averaged-RQA hot path on one MI355X.

A step is one whole pass of the path over the large workload: exact
threshold selection for K = 20 target recurrence rates and the line sweep
giving RR, DET and the averaged DET, for both large series (Lorenz-x + 0 dB
noise and logistic r=4 + -10 dB noise, N = 10^5, m = 3, tau = 5, Euclidean
norm, Theiler window 1, l_min = 2), as one rqa_batch call with the library's
default selection (at this size the sample window: one counting pass over
the pairs inside a key window, the last bits resolved by the line sweep, a
plain radix fallback for any target outside the window).  Inputs are
resident in device memory before the timed region.

value = pairs x thresholds per second over the timed steps, where pairs are
the M = (Nv-1) Nv / 2 upper-triangle pairs each series has.

Also reported (outside the timed steps): the same step with plain radix
selection and with the trained network's window, the 600-series batched ensemble
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
# VALU peak of MI355X in lane-ops/s from its unit counts and clock: the FP32
# vector peak of 157.3 TFLOP/s counts an FMA as two flops, i.e. 256 CUs x 128
# one-op lane slots per clock x 2.4 GHz.  The library's issue-rate probe
# measures what the chip sustains (rqa_valu_rate) and is reported beside it.
VALU_PEAK = 157.3e12 / 2
# Work of a per-threshold implementation of the method: about 2 + key/K VALU
# ops per pair and threshold (a compare and a run update per threshold, the
# key shared) --
# 48 per pair at K = 20 with the Euclidean m = 3 key (8 ops).  The range
# sweep does O(1) work per pair whatever K is, so this count over time is a
# ratio to peak, not a fraction of it.
PER_THRESHOLD_OPS_PER_PAIR = 2 * K + 8
# Lower bound of this algorithm's VALU work per pair (lane-ops), per kernel,
# Euclidean m = 3: the key needs one new difference, its square and m - 1 = 2
# adds per cell (the walker reuses each difference m times), 4 ops; then
#   counting pass 1: the bucket index                                   +1
#   counting pass 2: bucket index, slot test, sub-bucket index          +3
#   window pass 1:   offset from the window start, range test, bin      +3
#   range sweep:     rank (bucket index, boundary compare, add),
#                    line rank (min, max), histogram address            +6
# The LDS read or atomic each kernel needs per pair is not VALU work.
KEY_OPS = 4
LOWER_BOUND_OPS = {"select_pass1": KEY_OPS + 1, "select_pass2": KEY_OPS + 3, "window_pass1": KEY_OPS + 3,
                   "sweep": KEY_OPS + 6}


def valu_roofline(ph, pairs, step_sec, probe, windowed):
    """Roofline of the dominant kernel and VALU fractions of the step.

    ph: phase -> device ms per step (HIP events on the library stream; one
    launch per phase); pairs: pairs per launch; probe: measured issue rates
    (lane-ops/s) of a double-rate (v_add_u32) and a half-rate (v_max_u32)
    instruction, and of the add with a scalar-register operand, which gfx950
    issues at the half rate.  `achieved` counts the algorithm's lower-bound VALU work
    (LOWER_BOUND_OPS) per launch over the launch time; measured instruction
    counts (SQ_INSTS_VALU x 64) come from the stored counter profile while
    it matches the device sources."""
    names = {"select_pass1": "window_pass1" if windowed else "select_pass1", "select_pass2": "select_pass2",
             "sweep": "sweep"}
    phases = [p for p in ("select_pass1", "select_pass2", "sweep") if ph.get(p, 0.0) > 0.0]
    alg = {p: pairs * LOWER_BOUND_OPS[names[p]] for p in phases}
    dom = max(phases, key=lambda p: ph[p])
    t = ph[dom] * 1e-3
    achieved = alg[dom] / t
    roof = {"bound": "alu", "kernel": names[dom], "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
            "algorithmic_ops_per_pair": LOWER_BOUND_OPS[names[dom]], "pairs_per_launch": pairs,
            "launch_ms": ph[dom], "measured_peak": probe["v_add_u32"] / 1e12,
            "measured_peak_half_rate": probe["v_max_u32"] / 1e12,
            "measured_add_with_sgpr_operand": probe["v_add_u32_sgpr"] / 1e12 if "v_add_u32_sgpr" in probe else None,
            "per_threshold_count_ratio": pairs * PER_THRESHOLD_OPS_PER_PAIR / t / VALU_PEAK if names[dom] == "sweep" else None}
    step = {"algorithmic": sum(alg.values()) / step_sec / VALU_PEAK,
            "per_phase_algorithmic": {names[p]: alg[p] / (ph[p] * 1e-3) / VALU_PEAK for p in phases},
            "issue": None, "per_phase_issue": None}
    counters = stored_counters(windowed)
    if counters:
        kcs = counters.get("kernels", {})
        kc = kcs.get(names[dom])
        if kc and kc.get("fetch_bytes") is not None and kc.get("write_bytes") is not None:
            # HBM bytes per launch from FETCH_SIZE + WRITE_SIZE, each scaled by
            # the factor a plain copy of known size gave for that counter
            roof["traffic"] = kc["fetch_bytes"] + kc["write_bytes"]
            roof["traffic_unit"] = "bytes/launch"
        if all(kcs.get(names[p], {}).get("valu_insts") is not None for p in phases):
            # executed VALU instructions x 64 lanes over the live launch time,
            # against the measured double-rate issue peak
            vi = {p: kcs[names[p]]["valu_insts"] for p in phases}
            issue = {p: vi[p] * 64 / (ph[p] * 1e-3) / probe["v_add_u32"] for p in phases}
            step["per_phase_issue"] = {names[p]: v for p, v in issue.items()}
            step["issue"] = sum(vi[p] * 64 for p in phases) / step_sec / probe["v_add_u32"]
            roof["issue_frac"] = issue[dom]
            roof["valu_insts_per_pair"] = vi[dom] * 64 / pairs
    return roof, step


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
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of the CPU oracle on the 600-series ensemble (series started within it)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time the CPU oracle on the configurations only (no GPU) and print it")
    ap.add_argument("--tune-file", default=None,
                    help="load launch shapes from this file if it exists, else tune and save them there")
    ap.add_argument("--no-bracket", action="store_true", help="skip the learned-bracket evaluation")
    ap.add_argument("--no-hist", action="store_true", help="skip the full line-length histogram")
    ap.add_argument("--select", choices=("auto", "plain", "sample"), default="auto",
                    help="selection method of the timed step (auto: the library's default)")
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


def stored_counters(windowed):
    """Per-launch hardware counters of the timed kernels (rocprofv3 --pmc of
    the step with window or plain selection, summarised in profiles/ by
    paper_2208_09136_amd.profsum), or None when absent or taken on other
    sources."""
    path = os.path.join(ROOT, "profiles", f"counters_n1e5_k20_{'window' if windowed else 'plain'}.json")
    try:
        with open(path) as f:
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

    if args.cpu_only:
        print(json.dumps({"cpu_baseline": cpu_baseline(args.cpu_budget)}), flush=True)
        return

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

    # the step: the library's default selection (RQA_SEL_AUTO: the sample
    # window at this size, exact, with the plain fallback)
    step_flags = {"auto": rqa.RQA_SEL_AUTO, "plain": rqa.RQA_SEL_PLAIN, "sample": rqa.RQA_SEL_SAMPLE}[args.select]
    ref = None
    for _ in range(args.warmup):
        ref = ctx.batch(concat, offs, prm, rr, flags=step_flags)
    torch.cuda.synchronize()
    phases = np.zeros(len(rqa.PHASES))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.batch(concat, offs, prm, rr, flags=step_flags)
        phases += np.array([ctx.phase_times()[p] for p in rqa.PHASES])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if ref is not None:
        assert np.array_equal(ref["det_mean"], out["det_mean"]), "results changed between steps"
    step_stats = ctx.selection_stats()
    windowed = step_stats["full_passes"] != 3
    sec = (t1 - t0) / args.steps
    value = cell_thr / sec
    ph = dict(zip(rqa.PHASES, (phases / args.steps).tolist()))

    # roofline of the dominant kernel (the phase with the largest device time;
    # one launch per phase per step) and the step's fraction of VALU peak
    probe = {k: rqa.rqa_valu_rate(ctx.ctx, k)[0] for k in ("v_add_u32", "v_max_u32", "v_add_u32_sgpr")}
    roofline, step_frac = valu_roofline(ph, sum(cells), sec, probe, windowed=windowed)

    # the same step with each selection method: identical results, different
    # numbers of passes over the pairs (plain radix: three; sample or network
    # window: two)
    methods = {}
    from paper_2208_09136_amd import bracket
    have_net = not args.no_bracket and os.path.exists(args.bracket_file)
    if have_net:
        bracket.load(ctx, args.bracket_file)
    for name, flags in (("plain", rqa.RQA_SEL_PLAIN), ("sample", rqa.RQA_SEL_SAMPLE),
                        ("network", rqa.RQA_SEL_LEARNED)):
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
        methods[name] = {"ms_per_step": wsec * 1e3, "value": cell_thr / wsec, "full_passes": st["full_passes"],
                         "phases_ms": wph,
                         "series_fallback": st["series_fallback"],
                         "identical": bool(all(np.array_equal(got[k], out[k]) for k in ("eps", "count", "det"))),
                         "step_over_this": wsec / sec}

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
        "valu_peak_frac": step_frac["algorithmic"],
        "valu_peak": step_frac,
        "roofline": roofline,
        "selection": {"method": "sample window" if windowed else "plain radix",
                      "full_passes": step_stats["full_passes"], "series_fallback": step_stats["series_fallback"]},
        "selection_methods": methods,
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
        result["cpu_baseline"] = cpu_baseline(args.cpu_budget)

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
    # the same with plain radix selection (identical results)
    pl = ctx.batch(concat, offs, prm, rr99, flags=rqa.RQA_SEL_PLAIN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pl = ctx.batch(concat, offs, prm, rr99, flags=rqa.RQA_SEL_PLAIN)
    torch.cuda.synchronize()
    secp = (time.perf_counter() - t0) / steps
    return {"ms_per_step": sec99 * 1e3, "value": cells * 99 / sec99, "unit": "cell-thresholds/s",
            "phases_ms": ph99,
            "plain_ms_per_step": secp * 1e3,
            "plain_identical": bool(all(np.array_equal(pl[k], got99[k]) for k in ("eps", "count", "det"))),
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
    # the paper's RR set 1..99 %: selection, DET and the histogram at all 99
    # thresholds of both series in one call (four histogram passes)
    rr99 = np.tile(np.arange(1, 100) / 100.0, (len(prm), 1))
    nvs = [int(offs[i + 1] - offs[i]) - (p[0] - 1) * p[1] for i, p in enumerate(prm)]
    hl = max(nvs) + 1
    got = ctx.batch_hist(concat, offs, prm, rr99, hl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = ctx.batch_hist(concat, offs, prm, rr99, hl)
    call = time.perf_counter() - t0
    hms = ctx.phase_times()["histogram"]
    from paper_2208_09136_amd import rqa
    lens = np.arange(hl, dtype=np.int64)
    k99 = {"ms_per_call": call * 1e3, "histogram_ms": hms, "series": []}
    for s_ in range(len(prm)):
        h = got["hist"][s_].astype(np.int64)
        L, lmax = rqa.rqa_line_measures(got["hist"][s_], prm[s_][4])
        k99["series"].append({
            "sum_l_P_equals_C": bool(np.array_equal((h * lens).sum(axis=1).astype(np.uint64), got["count"][s_])),
            "averaged_det_99": float(rqa.rqa_averaged_det(got["det"][s_])[-1]),
            "averaged_L_99": float(rqa.rqa_averaged_det(L)[-1]),
            "averaged_Lmax_99": float(rqa.rqa_averaged_det(lmax.astype(np.float64))[-1])})
    return {"workload": "each bench series at its 20 selected thresholds, every length kept",
            "series": rows,
            "k99_one_call": dict(k99, workload="both bench series, RR 1..99 %: selection + DET + P(l) at every "
                                               "threshold, one rqa_batch_hist call")}


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
    pl = ctx.batch(concat, offs, prm, rr, flags=rqa.RQA_SEL_PLAIN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pl = ctx.batch(concat, offs, prm, rr, flags=rqa.RQA_SEL_PLAIN)
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
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
            "equal_to_single": same, "plain_selection_ms": tp * 1e3,
            "plain_identical": bool(all(np.array_equal(pl[k], out[k]) for k in ("eps", "count", "det"))),
            "autotune_chunk_tiles": chunk, "autotune_seconds": t_tune}


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


def cpu_model():
    """CPU model string of the host (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Host threads this process may use (the scheduler's affinity set)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_case(case, method=0):
    import oracle
    oracle.run(case["y"], case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"], case["rr"],
               method=method)
    return cells_of(case)


def time_oracle(cases, workers, budget=None, method=0):
    """Wall time of the oracle's whole path (selection + lines) on `cases`,
    independent series running concurrently on `workers` host threads (each
    call's line passes also use OpenMP).  With a budget in seconds, series
    are started in the given order until the budget is spent; those started
    are finished and counted.  Returns (series done, pairs done, seconds)."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    done, pairs = 0, 0
    with cf.ThreadPoolExecutor(workers) as ex:
        futs = []
        it = iter(cases)
        for c in it:
            futs.append(ex.submit(oracle_case, c, method))
            if len(futs) >= workers:
                break
        pending = set(futs)
        while pending:
            fin, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
            for f in fin:
                pairs += f.result()
                done += 1
            if budget is None or time.perf_counter() - t0 < budget:
                for _ in range(len(fin)):
                    c = next(it, None)
                    if c is not None:
                        pending.add(ex.submit(oracle_case, c, method))
    return done, pairs, time.perf_counter() - t0


def cpu_baseline(budget, workers=None):
    """The CPU oracle as it stands (plain C, qsort selection up to 2e8 pairs
    and a 31-step bisection above, one run-length pass per threshold, OpenMP
    over diagonals) on every configuration, independent series running
    concurrently on all host threads:
      * the 10 seeds of the N = 10^3 logistic configuration;
      * all 15 series of the N = 10^4 configuration;
      * the 600-series ensemble: series in a seeded random order until the
        budget is spent, with the whole ensemble's time projected from the
        rate (pairs of the whole ensemble / pairs per second);
      * the N = 10^5 bench series: the method the oracle takes at that size
        (bisection) on the first 15,000 samples of both series, projected to
        the full size linearly in the pairs (every step of that path is a
        pass over all pairs).  This is `value`, in the bench's unit."""
    nthreads = host_threads()
    workers = workers or nthreads
    out = {"unit": "cell-thresholds/s", "cores": nthreads, "kind": "oracle", "cpu_model": cpu_model(),
           "omp_num_threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or None}
    rows = {}
    small = [synth.config_small(s) for s in range(10)]
    n, pairs, sec = time_oracle(small, workers)
    rows["n1e3_logistic_10_seeds"] = {"series": n, "pairs": pairs, "seconds": sec, "value": pairs * K / sec}
    medium = synth.config_medium()
    n, pairs, sec = time_oracle(medium, workers)
    rows["n1e4_15_series"] = {"series": n, "pairs": pairs, "seconds": sec, "value": pairs * K / sec,
                              "series_per_s": n / sec}
    ens = synth.config_batch()
    order = np.random.default_rng(11).permutation(len(ens))
    total_pairs = sum(cells_of(c) for c in ens)
    n, pairs, sec = time_oracle([ens[i] for i in order], workers, budget=budget)
    rate = pairs / sec
    rows["ensemble_600"] = {"series": n, "pairs": pairs, "seconds": sec, "value": pairs * K / sec,
                            "series_per_s": n / sec, "ensemble_pairs": total_pairs,
                            "projected_ensemble_seconds": total_pairs / rate,
                            "sample": f"{n} of 600 series in a seeded random order, started within {budget} s"}
    large = synth.config_large()
    pre = [dict(c, y=c["y"][:15_000]) for c in large]
    n, pairs, sec = time_oracle(pre, workers, method=2)
    full = sum(cells_of(c) for c in large)
    rows["n1e5_bench_series"] = {"series": n, "pairs": pairs, "seconds": sec, "value": pairs * K / sec,
                                 "method": "bisection", "full_pairs": full,
                                 "projected_seconds_full_size": sec * full / pairs}
    out["value"] = rows["n1e5_bench_series"]["value"]
    out["seconds"] = sum(r["seconds"] for r in rows.values())
    out["sample"] = ("bench series (N = 1e5, m = 3, tau = 5, Euclidean, K = 20): their first 15,000 samples, "
                     "bisection selection + lines, both series at once; the other configurations below")
    out["configs"] = rows
    return out


if __name__ == "__main__":
    main()
