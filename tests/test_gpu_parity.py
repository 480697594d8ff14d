"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results (thresholds as bit patterns, ranks, counts) must match
bit for bit; RR, DET and the averaged DET are ratios of those integers
computed in double on both sides, so they must match exactly too."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handbuilt_plots.json")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2208_09136_amd import rqa
    c = rqa.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


def dev(y):
    import torch
    return torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to("cuda:0")


def prm(case):
    return (case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"])


def assert_run_equal(got, want, label=""):
    assert np.array_equal(got["eps"].view(np.uint32), want["eps"].view(np.uint32)), f"{label} eps"
    assert np.array_equal(got["k"], want["k"]), f"{label} k"
    assert np.array_equal(got["count"], want["count"]), f"{label} count"
    assert np.array_equal(got["rr"], want["rr"]), f"{label} rr"
    assert np.array_equal(got["det"], want["det"], equal_nan=True), f"{label} det"
    assert got["det_mean"] == want["det_mean"] or (np.isnan(got["det_mean"]) and np.isnan(want["det_mean"])), label


def oracle_run(case, rr=None):
    rr = case["rr"] if rr is None else rr
    return oracle.run(case["y"], case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"], rr)


def check_case(ctx, case, rr=None):
    print(f"[parity] {case['name']} n={len(case['y'])} params={prm(case)}", flush=True)
    rr = case["rr"] if rr is None else rr
    got = ctx.run(dev(case["y"]), prm(case), rr)
    want = oracle_run(case, rr)
    assert_run_equal(got, want, case["name"])
    return got


# ---------------------------------------------------------------- workloads
@pytest.mark.parametrize("seed", range(10))
def test_small_logistic_max_norm(ctx, seed):
    """Logistic r=4 + 10 dB noise, N=1000, m=1, max norm, K=20."""
    check_case(ctx, synth.config_small(seed))


@pytest.mark.parametrize("idx", range(15))
def test_medium_systems_reduced_length(ctx, idx):
    """The 15 series of the N=10^4 configuration, at N=2500 so the oracle's
    sort path stays fast."""
    check_case(ctx, synth.config_medium(n=2500)[idx])


@pytest.mark.parametrize("idx", range(15))
def test_medium_systems_full_length(ctx, idx):
    """Every series of the N=10^4 configuration at full length: sine,
    logistic and Lorenz at SNR 20, 10, 0, -10, -20 dB (Euclidean; m=3, tau=5
    for Lorenz, m=1 otherwise), K=20, against the oracle's sort path."""
    check_case(ctx, synth.config_medium()[idx])


def test_large_bench_batch(ctx):
    """The bench step: both N = 10^5 series (m = 3, tau = 5, Euclidean, K = 20,
    4,998,950,055 pairs each) in one rqa_batch call.  The oracle cannot sort
    5e9 keys in a test, so every threshold is pinned through properties that
    hold at any size: the order-statistic bracket #{key < eps_r} < k_r <=
    #{key <= eps_r} = count_r, and RR and DET at that threshold recomputed
    by the oracle's plain per-threshold run-length pass, for all 20 targets
    of both series."""
    import torch
    cases = synth.config_large()
    prm_ = [prm(c) for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(c["y"]) for c in cases])]).astype(np.uint64)
    concat = torch.from_numpy(np.concatenate([c["y"] for c in cases])).to("cuda:0")
    rr = np.stack([c["rr"] for c in cases])
    print("[parity] bench batch 2 x N=1e5", flush=True)
    got = ctx.batch(concat, offs, prm_, rr)
    M = oracle.num_pairs(oracle.num_vectors(100_000, 3, 5), 1)
    assert M == 4998950055
    for s, targets in ((0, list(range(20))), (1, list(range(20)))):
        c = cases[s]
        eps = got["eps"][s][targets]
        print(f"[parity] {c['name']} oracle counts at {len(targets)} thresholds", flush=True)
        lt, le = oracle.count(c["y"], 3, 5, 1, 1, eps)
        for i, r in enumerate(targets):
            k = oracle.rank(c["rr"][r], M)
            assert lt[i] < k <= le[i]
            assert le[i] == got["count"][s][r]
        nv = oracle.num_vectors(100_000, 3, 5)
        print(f"[parity] {c['name']} oracle lines and histograms at {len(targets)} thresholds", flush=True)
        lin = oracle.lines(c["y"], 3, 5, 1, 1, 2, eps, hist_len=nv + 1)
        assert np.array_equal(lin["count"], got["count"][s][targets])
        assert np.array_equal(lin["rr"], got["rr"][s][targets])
        assert np.array_equal(lin["det"], got["det"][s][targets])
        # the full line-length histogram at the selected thresholds, every
        # length kept, element by element (Eq. 4's P(l) at full size)
        print(f"[parity] {c['name']} GPU histograms at {len(targets)} thresholds", flush=True)
        full = ctx.det_curve(dev(c["y"]), prm(c), eps, hist_len=nv + 1)
        assert full["hist"].shape == lin["hist"].shape
        assert np.array_equal(full["hist"], lin["hist"])
        assert np.array_equal(full["count"], lin["count"])
        assert np.array_equal(full["det"], lin["det"])
    # the averaged DET is the left-to-right mean of the 20 DET values
    for s in range(2):
        assert got["det_mean"][s] == sum(got["det"][s].tolist()) / 20


def test_ensemble_slice_one_batch(ctx):
    """A seeded 60-series slice of the 600-series ensemble (both embedding
    groups: m = 1 for sine and logistic, m = 3 / tau = 5 for Lorenz, and the
    ensemble's longest series) selected and swept in one rqa_batch call,
    every series against the oracle's whole path."""
    import concurrent.futures as cf
    import torch
    cases = synth.config_batch()
    lengths = np.array([len(c["y"]) for c in cases])
    rng = np.random.default_rng(2024)
    pick = set(rng.choice(len(cases), 59, replace=False).tolist())
    pick.add(int(np.argmax(lengths)))
    while len(pick) < 60:
        pick.add(int(rng.integers(len(cases))))
    sel = [cases[i] for i in sorted(pick)]
    assert {c["m"] for c in sel} == {1, 3}
    assert max(len(c["y"]) for c in sel) == lengths.max()
    offs = np.concatenate([[0], np.cumsum([len(c["y"]) for c in sel])]).astype(np.uint64)
    concat = torch.from_numpy(np.concatenate([c["y"] for c in sel])).to("cuda:0")
    rr = np.stack([c["rr"] for c in sel])
    print(f"[parity] ensemble slice: 60 series, longest {lengths.max()}", flush=True)
    got = ctx.batch(concat, offs, [prm(c) for c in sel], rr)
    with cf.ThreadPoolExecutor(8) as ex:
        wants = list(ex.map(oracle_run, sel))
    for s_, (c, want) in enumerate(zip(sel, wants)):
        one = {key: got[key][s_] for key in ("eps", "count", "rr", "det")}
        one["k"] = want["k"]
        one["det_mean"] = got["det_mean"][s_]
        assert_run_equal(one, want, c["name"])


# ---------------------------------------------------------------- golden plots
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("case", golden()["cases"], ids=lambda c: c["name"])
def test_handbuilt_plots(ctx, case):
    y = np.array(case["y"], dtype=np.float32)
    out = ctx.det_curve(dev(y), (case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"]),
                        [case["eps"]])
    assert int(out["count"][0]) == case["count"]
    assert out["rr"][0] == case["count"] / case["M"]
    assert out["det"][0] == case["det_num"] / case["count"]


def test_handbuilt_ranks(ctx):
    g = golden()["ranks"]
    y = np.array(g["y"], dtype=np.float32)
    rr = [c["rr"] for c in g["cases"]]
    eps, k, cnt = ctx.select_thresholds(dev(y), (g["m"], g["tau"], g["norm"], g["theiler"], 2), rr)
    for i, c in enumerate(g["cases"]):
        assert int(k[i]) == c["k"] and float(eps[i]) == c["eps"] and int(cnt[i]) == c["count"]


# ---------------------------------------------------------------- parameters and edges
@pytest.mark.parametrize("m,tau,norm,w,lmin", [
    (1, 1, 0, 1, 2), (1, 1, 1, 1, 2), (3, 5, 1, 1, 2), (3, 5, 0, 1, 2), (2, 3, 1, 1, 2),
    (4, 2, 0, 3, 2), (3, 3, 1, 7, 3), (1, 1, 0, 1, 1), (3, 5, 1, 1, 1), (2, 1, 1, 2, 5),
    (1, 1, 1, 1, 16), (5, 1, 0, 1, 4), (3, 5, 1, 40, 2)])
def test_parameter_grid(ctx, m, tau, norm, w, lmin):
    y = synth.series("lorenz", 1500, 5.0, (7, m, tau, w))
    case = {"name": f"grid_m{m}_tau{tau}_n{norm}_w{w}_l{lmin}", "y": y, "m": m, "tau": tau, "norm": norm,
            "theiler": w, "lmin": lmin, "rr": np.array([0.003, 0.01, 0.05, 0.2, 0.5, 0.9])}
    check_case(ctx, case)


@pytest.mark.parametrize("shape", [(64, 1), (128, 3), (192, 2), (64, 4096), (4096, 1)])
@pytest.mark.parametrize("n", [70, 130, 1000, 1023, 3001])
def test_segment_and_chunk_shapes(ctx, shape, n):
    """Ragged bands, segment halos and chunk boundaries: every launch shape
    gives the oracle's result (a race canary as well)."""
    ctx.set_shape(*shape)
    try:
        y = synth.series("logistic", n, 0.0, (8, n, 0, 0))
        case = {"name": f"shape{shape}_n{n}", "y": y, "m": 2, "tau": 2, "norm": 1, "theiler": 1, "lmin": 2,
                "rr": np.array(synth.RR_20)}
        check_case(ctx, case)
    finally:
        ctx.set_shape(0, 0)


@pytest.mark.parametrize("grid", [1, 7, 4096])
def test_more_workgroups_than_chunks(ctx, grid):
    """Regression: persistent workgroups whose first ticket is already past
    the end of the work queue must exit cleanly (they once dereferenced the
    descriptor of a non-existent chunk).  grid=4096 on a one-chunk series makes
    almost every workgroup start on a drained queue."""
    ctx.set_grid(grid)
    try:
        check_case(ctx, synth.config_small(7))
        case = synth.config_medium(n=3000)[12]
        check_case(ctx, case)
    finally:
        ctx.set_grid(0)


def test_autotuned_shapes_keep_results(ctx, tmp_path):
    """The autotuner only changes launch shapes: results after tuning (single
    and batched), and after a save/load round trip of the table, equal the
    oracle's / the untuned run's."""
    case = synth.config_medium(n=3000)[12]
    before = ctx.run(dev(case["y"]), prm(case), case["rr"])
    seg, chunk = ctx.autotune(dev(case["y"]), prm(case), case["rr"])
    assert seg % 64 == 0 and 64 <= seg <= 4096 and chunk in (2, 8, 32)
    assert_run_equal(ctx.run(dev(case["y"]), prm(case), case["rr"]), before, "tuned")
    cases = synth.config_batch(realisations=1)[1::3][:10]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    concat = dev(np.concatenate(ys))
    rr = np.stack([c["rr"] for c in cases])
    plain = ctx.batch(concat, offs, [prm(c) for c in cases], rr)
    ctx.autotune_batch(concat, offs, [prm(c) for c in cases], rr)
    path = str(tmp_path / "tune.json")
    ctx.tune_save(path)
    ctx.tune_load(path)
    tuned = ctx.batch(concat, offs, [prm(c) for c in cases], rr)
    for key in ("eps", "count", "det", "det_mean"):
        assert np.array_equal(tuned[key], plain[key]), key
    assert_run_equal(ctx.run(dev(cases[0]["y"]), prm(cases[0]), cases[0]["rr"]), oracle_run(cases[0]), "tuned batch")


def test_unsorted_and_repeated_targets(ctx):
    case = synth.config_small(4)
    rr = np.array([0.2, 0.01, 0.05, 0.05, 1.0, 0.013, 0.2, 1e-9])
    check_case(ctx, case, rr)


def test_single_target_and_full_rate(ctx):
    case = synth.config_small(5)
    check_case(ctx, case, np.array([1.0]))
    check_case(ctx, case, np.array([0.5]))


def test_periodic_series_ties(ctx):
    for n, P in [(600, 7), (1000, 37)]:
        y = synth.periodic_integer(n, P)
        Z = sum(n - d for d in range(P, n, P))
        M = oracle.num_pairs(n, 1)
        rr = np.array([Z / M * 0.3, Z / M * 0.9, 0.1, 0.5])
        case = {"name": f"periodic_{n}_{P}", "y": y, "m": 1, "tau": 1, "norm": 0, "theiler": 1, "lmin": 2,
                "rr": rr}
        got = check_case(ctx, case)
        assert got["eps"][0] == 0.0 and got["eps"][1] == 0.0


def test_pass3_prefix_table_overflow(ctx):
    # keys of this series are multiples of 3; the thresholds 3, 6, 12, 24 and
    # 48 have equal mantissas, so their 21-bit prefixes share the low bits and
    # fall in one set of the pass-3 prefix table: more than the set holds, so
    # the series takes the slot-table lookups.  Each target sits in the middle
    # of its threshold's run of equal keys.
    y = synth.periodic_integer(900, 23, seed=3)
    i, j = np.triu_indices(len(y), 1)
    keys = np.sort(np.abs(y[i] - y[j]).astype(np.float32))
    vals = np.array([3, 6, 12, 24, 48], np.float32)
    assert len({int(v.view(np.uint32)) >> 10 & 4095 for v in vals}) == 1
    rr = np.array([(np.searchsorted(keys, v, "left") + np.searchsorted(keys, v, "right")) / 2 / len(keys)
                   for v in vals])
    p = (1, 1, 0, 1, 2)
    print("[parity] pass-3 prefix set overflow", flush=True)
    got = ctx.select_thresholds(dev(y), p, rr)[0]
    want = oracle.select(y, 1, 1, 0, 1, rr)[0]
    assert np.array_equal(np.asarray(got, np.float32).view(np.uint32), np.asarray(want, np.float32).view(np.uint32))
    assert np.array_equal(np.asarray(got, np.float32), vals)
    # two of them (a set holds two) and a non-integer series take the table
    got = ctx.select_thresholds(dev(y), p, rr[:2])[0]
    assert np.array_equal(np.asarray(got, np.float32), vals[:2])
    case = synth.config_small(3)
    rr2 = np.linspace(0.01, 0.3, 12)
    got = ctx.select_thresholds(dev(case["y"]), prm(case), rr2)[0]
    want = oracle.select(case["y"], case["m"], case["tau"], case["norm"], case["theiler"], rr2)[0]
    assert np.array_equal(np.asarray(got, np.float32).view(np.uint32), np.asarray(want, np.float32).view(np.uint32))


def test_constant_series(ctx):
    y = np.full(300, 2.5, dtype=np.float32)
    case = {"name": "constant", "y": y, "m": 3, "tau": 2, "norm": 1, "theiler": 1, "lmin": 2,
            "rr": np.array([0.01, 0.5, 1.0])}
    got = check_case(ctx, case)
    assert np.all(got["eps"] == 0.0)


def test_minimal_series(ctx):
    # nv - w = 1: exactly one pair
    y = np.array([0.0, 1.0, 3.0, 7.0], dtype=np.float32)
    case = {"name": "minimal", "y": y, "m": 2, "tau": 2, "norm": 1, "theiler": 1, "lmin": 2,
            "rr": np.array([0.5, 1.0])}
    got = check_case(ctx, case)
    assert np.all(got["count"] == 1)


def test_close_thresholds_share_buckets(ctx):
    """Thresholds one ulp apart land in one bucket of the rank table and take
    the slow comparison path."""
    case = synth.config_small(6)
    base = oracle.select(case["y"], 1, 1, 0, 1, [0.05])[0][0]
    eps = [base]
    for _ in range(6):
        eps.append(np.nextafter(eps[-1], np.float32(np.inf), dtype=np.float32))
    eps += [np.float32(base * 3), np.float32(0.0), np.float32(np.inf), np.float32(base * 0.5)]
    eps = np.array(eps, dtype=np.float32)
    got = ctx.det_curve(dev(case["y"]), prm(case), eps)
    want = oracle.lines(case["y"], 1, 1, 0, 1, 2, eps)
    assert np.array_equal(got["count"], want["count"])
    assert np.array_equal(got["det"], want["det"], equal_nan=True)
    assert np.array_equal(got["rr"], want["rr"])


def test_det_curve_matches_selected(ctx):
    case = synth.config_medium(n=2000)[13]
    got = ctx.run(dev(case["y"]), prm(case), case["rr"])
    dc = ctx.det_curve(dev(case["y"]), prm(case), got["eps"])
    assert np.array_equal(dc["count"], got["count"])
    assert np.array_equal(dc["det"], got["det"])
    eps, k, cnt = ctx.select_thresholds(dev(case["y"]), prm(case), case["rr"])
    assert np.array_equal(eps, got["eps"]) and np.array_equal(cnt, got["count"])


def test_batch_equals_single(ctx):
    cases = synth.config_batch(realisations=1)[::2][:12]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    concat = dev(np.concatenate(ys))
    rr = np.stack([c["rr"] for c in cases])
    out = ctx.batch(concat, offs, [prm(c) for c in cases], rr)
    for s, c in enumerate(cases):
        single = ctx.run(dev(c["y"]), prm(c), c["rr"])
        assert np.array_equal(out["eps"][s].view(np.uint32), single["eps"].view(np.uint32))
        assert np.array_equal(out["count"][s], single["count"])
        assert np.array_equal(out["det"][s], single["det"])
        assert out["det_mean"][s] == single["det_mean"]
    for s in (0, 5, 11):
        assert_run_equal({**ctx.run(dev(cases[s]["y"]), prm(cases[s]), cases[s]["rr"])},
                         oracle_run(cases[s]), cases[s]["name"])


# ---------------------------------------------------------------- errors
def test_error_paths(ctx):
    from paper_2208_09136_amd.rqa import RqaError
    y = synth.config_small(0)["y"]
    good = (1, 1, 0, 1, 2)
    bad = y.copy()
    bad[500] = np.nan
    with pytest.raises(RqaError) as e:
        ctx.run(dev(bad), good, [0.1])
    assert e.value.name == "RQA_ERR_NONFINITE"
    bad[500] = np.inf
    with pytest.raises(RqaError) as e:
        ctx.det_curve(dev(bad), good, [0.1])
    assert e.value.name == "RQA_ERR_NONFINITE"
    with pytest.raises(RqaError) as e:
        ctx.run(dev(y[:5]), (3, 2, 0, 1, 2), [0.1])
    assert e.value.name == "RQA_ERR_TOO_SHORT"
    for p in [(0, 1, 0, 1, 2), (1, 0, 0, 1, 2), (1, 1, 2, 1, 2), (1, 1, 0, 0, 2), (1, 1, 0, 1, 0)]:
        with pytest.raises(RqaError) as e:
            ctx.run(dev(y), p, [0.1])
        assert e.value.name == "RQA_ERR_INVALID_ARG"
    with pytest.raises(RqaError) as e:
        ctx.run(dev(y), (1, 1, 0, 1, 17), [0.1])
    assert e.value.name == "RQA_ERR_UNSUPPORTED"
    for rr in ([], [0.0], [1.5], [float("nan")], [0.1] * 129):
        with pytest.raises(RqaError) as e:
            ctx.run(dev(y), good, rr)
        assert e.value.name == "RQA_ERR_INVALID_ARG"
    for eps in ([float("nan")], [-1.0]):
        with pytest.raises(RqaError) as e:
            ctx.det_curve(dev(y), good, eps)
        assert e.value.name == "RQA_ERR_INVALID_ARG"
    with pytest.raises(RqaError) as e:
        ctx.run(dev(y), good, [0.1], flags=2)
    assert e.value.name == "RQA_ERR_UNSUPPORTED"
    # the context still works after errors
    check_case(ctx, synth.config_small(0))


# ---------------------------------------------------------------- sketch
def test_sketch_matches_oracle(ctx):
    from oracle import sketch
    cases = [synth.config_small(0), synth.config_medium(n=2000)[12], synth.config_medium(n=3000)[3]]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    feats, scale = ctx.sketch_batch(dev(np.concatenate(ys)), offs, [prm(c) for c in cases], seed=777)
    for s, c in enumerate(cases):
        f, sc = sketch.sketch(c["y"], c["m"], c["tau"], c["norm"], c["theiler"], seed=777 + s)
        assert int(scale[s]) == sc
        assert np.array_equal(feats[s], f)


def test_sketch_sample_sorted_equals_oracle(ctx):
    # the sample the sample window takes its order statistics from: every
    # sampled key, sorted, bit for bit the oracle's (ties included)
    from oracle import sketch
    cases = [synth.config_small(0), synth.config_medium(n=2000)[12], synth.config_medium(n=3000)[3],
             {"y": np.round(synth.series("logistic", 1500, 5.0, (3, 1, 2, 3)), 1).astype(np.float32),
              "m": 1, "tau": 1, "norm": 0, "theiler": 1, "lmin": 2}]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    got = ctx.sketch_sample(dev(np.concatenate(ys)), offs, [prm(c) for c in cases], seed=4242)
    for s, c in enumerate(cases):
        keys = sketch.sample_keys(c["y"], c["m"], c["tau"], c["norm"], c["theiler"], 4242 + s)
        want = np.sort(np.asarray(keys, np.float32).view(np.uint32))
        assert np.array_equal(got[s], want), s


@pytest.mark.parametrize("m,tau,norm,w,lmin", [
    (1, 1, 0, 1, 2), (3, 5, 1, 1, 2), (3, 3, 0, 2, 2), (2, 3, 1, 1, 2), (3, 5, 1, 1, 3),
    (1, 1, 1, 1, 7), (3, 5, 0, 5, 16), (1, 1, 0, 1, 1)])
def test_selection_lines_equal_sweep(ctx, m, tau, norm, w, lmin):
    # D counted by line values inside the radix selection equals D from the
    # separate line sweep at the same thresholds (two independent device
    # algorithms), on a series long enough for interior walker tiles
    y = synth.series("logistic", 5000, 0.0, (9, m, tau, lmin))
    p = (m, tau, norm, w, lmin)
    rr = np.array([0.001, 0.01, 0.02, 0.05, 0.1, 0.13, 0.2, 0.35])
    print(f"[lines] m={m} tau={tau} norm={norm} w={w} lmin={lmin}", flush=True)
    got = ctx.run(dev(y), p, rr)
    dc = ctx.det_curve(dev(y), p, got["eps"])
    assert np.array_equal(dc["count"], got["count"])
    assert np.array_equal(dc["det"], got["det"], equal_nan=True)
    assert dc["det_mean"] == got["det_mean"] or (np.isnan(dc["det_mean"]) and np.isnan(got["det_mean"]))


# ---------------------------------------------------------------- paper-scale RR set
RR_99 = np.array([k / 100.0 for k in range(1, 100)])


@pytest.mark.parametrize("system,m,tau,norm", [("logistic", 1, 1, 0), ("lorenz", 3, 5, 1), ("sine", 1, 1, 1)])
def test_paper_rr_set_k99(ctx, system, m, tau, norm):
    # the paper's RR set 1..99 %: exact thresholds, RR and DET for all 99
    # targets equal the oracle, and the averaged-DET curve over RR* equals the
    # running means of the oracle's DET values
    y = synth.series(system, 3000, 0.0, (10, m, tau, norm))
    case = {"name": f"k99_{system}", "y": y, "m": m, "tau": tau, "norm": norm, "theiler": 1, "lmin": 2,
            "rr": RR_99}
    got = check_case(ctx, case)
    want = oracle_run(case)
    from paper_2208_09136_amd import rqa
    curve = rqa.rqa_averaged_det(got["det"])
    s, ref = 0.0, []
    for r, d in enumerate(want["det"]):
        s += d
        ref.append(s / (r + 1))
    assert np.array_equal(curve, np.array(ref))
    assert curve[-1] == got["det_mean"]
    win = ctx.run(dev(y), prm(case), RR_99, flags=4)
    assert np.array_equal(win["eps"], got["eps"]) and np.array_equal(win["det"], got["det"])


@pytest.mark.parametrize("K", [21, 39, 40, 41, 64, 65, 80])
def test_path_switch_by_k(ctx, K):
    # the library switches between the range sweep and complete selection
    # plus the threshold sweep by K and selection method; every side of each
    # switch gives the oracle's thresholds, RR and DET
    y = synth.series("lorenz", 2500, 5.0, (11, K, 0, 0))
    rr = np.array([0.003 + 0.6 * k / K for k in range(K)])
    case = {"name": f"switch_k{K}", "y": y, "m": 3, "tau": 5, "norm": 1, "theiler": 1, "lmin": 2, "rr": rr}
    print(f"[parity] {case['name']}", flush=True)
    got = check_case(ctx, case)
    for flags in (4, 1):
        if flags == 1:
            from paper_2208_09136_amd import bracket
            import os
            path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                "paper_2208_09136_amd", "bracket_params.npz")
            bracket.load(ctx, path)
        win = ctx.run(dev(y), prm(case), rr, flags=flags)
        for key in ("eps", "count", "rr", "det", "det_mean"):
            assert np.array_equal(win[key], got[key]), (flags, key)


def test_maximum_k(ctx):
    # the largest target count a call takes, unsorted, with repeated rates and
    # both extremes, in one call and in a batch of two series, with plain and
    # sample-window selection: the scan and set-up kernels sort and number
    # the targets one thread each, here at their largest size
    from paper_2208_09136_amd import rqa
    K = rqa.RQA_MAX_K
    rng = np.random.default_rng(128)
    extra = [0.05, 0.05, 0.3, 0.3, 1e-9, 1.0, 0.002, 0.7]
    rr = rng.permutation(np.concatenate([np.linspace(0.002, 0.7, K - len(extra)), extra]))
    assert len(rr) == K
    cases = [{"name": f"maxk_{name}", "y": synth.series(name, n, 5.0, (21, i, 0, 0)), "m": 3, "tau": 5,
              "norm": 1, "theiler": 1, "lmin": 2, "rr": rr}
             for i, (name, n) in enumerate([("lorenz", 2000), ("logistic", 1500)])]
    wants = [oracle_run(c) for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(c["y"]) for c in cases])]).astype(np.uint64)
    concat = dev(np.concatenate([c["y"] for c in cases]))
    for flags in (rqa.RQA_SEL_PLAIN, rqa.RQA_SEL_SAMPLE):
        print(f"[parity] maxk K={K} flags={flags}", flush=True)
        assert_run_equal(ctx.run(dev(cases[0]["y"]), prm(cases[0]), rr, flags=flags), wants[0], f"single {flags}")
        out = ctx.batch(concat, offs, [prm(c) for c in cases], np.stack([rr, rr]), flags=flags)
        for s, want in enumerate(wants):
            label = f"batch {flags} series {s}"
            assert np.array_equal(out["eps"][s].view(np.uint32), want["eps"].view(np.uint32)), label
            assert np.array_equal(out["count"][s], want["count"]), label
            assert np.array_equal(out["rr"][s], want["rr"]), label
            assert np.array_equal(out["det"][s], want["det"], equal_nan=True), label
            assert out["det_mean"][s] == want["det_mean"] or np.isnan(want["det_mean"]), label
