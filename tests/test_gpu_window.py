"""Windowed selection (sample-quantile, caller-given and network windows):
thresholds identical to the plain radix selection whatever the window, with
fallback when a target lies outside it."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SAMPLE, WINDOW, LEARNED = 4, 8, 1


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


def prm(c):
    return (c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"])


CASES = [synth.config_small(3), synth.config_medium(n=3000)[12], synth.config_medium(n=2500)[2],
         synth.config_medium(n=2500)[6]]


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_sample_window_is_exact(ctx, idx):
    c = CASES[idx]
    print(f"[window] {c['name']}", flush=True)
    plain = ctx.run(dev(c["y"]), prm(c), c["rr"])
    got = ctx.run(dev(c["y"]), prm(c), c["rr"], flags=SAMPLE)
    st = ctx.selection_stats()
    for key in ("eps", "k", "count", "det"):
        assert np.array_equal(got[key], plain[key]), key
    assert st["full_passes"] in (2, 5)
    if st["series_fallback"] == 0:
        assert st["full_passes"] == 2 and st["targets_missed"] == 0
    want = oracle.select(c["y"], c["m"], c["tau"], c["norm"], c["theiler"], c["rr"])
    assert np.array_equal(got["eps"].view(np.uint32), want[0].view(np.uint32))


def test_given_window_hit_miss_and_too_wide(ctx):
    c = CASES[1]
    y = dev(c["y"])
    plain_eps, plain_k, plain_cnt = ctx.select_thresholds(y, prm(c), c["rr"])
    lo, hi = float(plain_eps.min()) * 0.97, float(plain_eps.max()) * 1.03
    cases = [((lo, hi), 0), ((float(plain_eps.max()) * 2, float(plain_eps.max()) * 4), 1),
             ((0.0, float("inf")), 1), ((float(plain_eps[7]), float(plain_eps[7])), 1)]
    for (a, b), fallback in cases:
        ctx.set_window(a, b)
        eps, k, cnt = ctx.select_thresholds(y, prm(c), c["rr"], flags=WINDOW)
        st = ctx.selection_stats()
        assert np.array_equal(eps.view(np.uint32), plain_eps.view(np.uint32)), (a, b)
        assert np.array_equal(cnt, plain_cnt) and np.array_equal(k, plain_k)
        assert st["series_fallback"] == fallback, (a, b, st)
        assert st["full_passes"] == (5 if fallback else 2)


def test_window_single_point_resolves_its_target(ctx):
    c = CASES[0]
    y = dev(c["y"])
    plain_eps, _, plain_cnt = ctx.select_thresholds(y, prm(c), c["rr"])
    e = float(plain_eps[10])
    ctx.set_window(e, e)
    eps, _, cnt = ctx.select_thresholds(y, prm(c), c["rr"], flags=WINDOW)
    st = ctx.selection_stats()
    assert np.array_equal(eps, plain_eps) and np.array_equal(cnt, plain_cnt)
    # targets whose threshold equals e were resolved inside the one-value window
    assert st["targets_missed"] == int(np.sum(plain_eps != plain_eps[10]))


def test_network_window_falls_back_when_untrained(ctx):
    c = CASES[2]
    y = dev(c["y"])
    ctx.mlp_init(3)
    ctx.mlp_set_bracket(np.full(20, 50.0, np.float32))   # window wider than the float range
    got = ctx.run(y, prm(c), c["rr"], flags=LEARNED)
    st = ctx.selection_stats()
    plain = ctx.run(y, prm(c), c["rr"])
    assert np.array_equal(got["eps"], plain["eps"]) and np.array_equal(got["det"], plain["det"])
    assert st["series_fallback"] == 1


def test_batch_sample_window_equals_plain(ctx):
    cases = synth.config_batch(realisations=1)[::3][:10]
    ys = [c["y"] for c in cases]
    offs = np.concatenate([[0], np.cumsum([len(y) for y in ys])]).astype(np.uint64)
    concat = dev(np.concatenate(ys))
    rr = np.stack([c["rr"] for c in cases])
    plain = ctx.batch(concat, offs, [prm(c) for c in cases], rr)
    got = ctx.batch(concat, offs, [prm(c) for c in cases], rr, flags=SAMPLE)
    for key in ("eps", "count", "det", "det_mean"):
        assert np.array_equal(got[key], plain[key]), key


@pytest.mark.parametrize("lmin", [1, 2, 3, 6])
@pytest.mark.parametrize("m,tau,norm", [(1, 1, 0), (3, 5, 1), (2, 3, 1)])
def test_window_lines_match_plain_and_sweep(ctx, lmin, m, tau, norm):
    # line values refined inside the window give the same D as the plain
    # three-pass refinement and as the separate sweep at the same thresholds
    y = synth.series("lorenz", 2500, 3.0, (8, m, tau, lmin))
    p = (m, tau, norm, 1, lmin)
    rr = np.array(synth.RR_20)
    print(f"[window-lines] m={m} tau={tau} norm={norm} lmin={lmin}", flush=True)
    plain = ctx.run(dev(y), p, rr)
    for flags in (SAMPLE, WINDOW):
        if flags == WINDOW:
            ctx.set_window(float(plain["eps"].min()) * 0.9, float(plain["eps"].max()) * 1.1)
        got = ctx.run(dev(y), p, rr, flags=flags)
        st = ctx.selection_stats()
        for key in ("eps", "count", "det", "det_mean"):
            assert np.array_equal(got[key], plain[key]), (flags, key)
        if flags == WINDOW:
            assert st["series_fallback"] == 0 and st["full_passes"] == 2
    dc = ctx.det_curve(dev(y), p, plain["eps"])
    assert np.array_equal(dc["count"], plain["count"]) and np.array_equal(dc["det"], plain["det"])


def test_nonfinite_series_rejected_in_every_selection_mode(ctx):
    from paper_2208_09136_amd.rqa import RqaError
    c = CASES[0]
    bad = c["y"].copy()
    bad[321] = np.nan
    ctx.set_window(0.0, 1.0)
    for flags in (0, SAMPLE, WINDOW):
        print(f"[window-nan] flags={flags}", flush=True)
        with pytest.raises(RqaError) as e:
            ctx.run(dev(bad), prm(c), c["rr"], flags=flags)
        assert e.value.name == "RQA_ERR_NONFINITE"
    # the context still works afterwards
    got = ctx.run(dev(c["y"]), prm(c), c["rr"], flags=SAMPLE)
    assert np.array_equal(got["eps"], ctx.run(dev(c["y"]), prm(c), c["rr"])["eps"])


def test_automatic_method_by_call_size(ctx):
    """RQA_SEL_AUTO (flags 0) takes the plain radix passes for small calls and
    the sample window from 2^29 pairs on; the results equal the plain
    method's either way."""
    from paper_2208_09136_amd import rqa
    small = CASES[1]
    ctx.run(dev(small["y"]), prm(small), small["rr"])
    assert ctx.selection_stats()["full_passes"] == 3
    # N = 32,800, m = 1: 537,903,600 pairs >= 2^29
    y = synth.series("logistic", 32_800, 0.0, (8, 9, 9, 9))
    p = (1, 1, 1, 1, 2)
    print("[window] automatic method, N = 32800", flush=True)
    auto = ctx.run(dev(y), p, synth.RR_20)
    st = ctx.selection_stats()
    assert st["full_passes"] in (2, 5)
    plain = ctx.run(dev(y), p, synth.RR_20, flags=rqa.RQA_SEL_PLAIN)
    assert ctx.selection_stats()["full_passes"] == 3
    for key in ("eps", "k", "count", "det"):
        assert np.array_equal(auto[key], plain[key]), key
