"""Full diagonal line-length histogram P_r(l) (the histogram behind Eq. 4):
element-by-element equal to the oracle's at every threshold, for every kernel
variant, with ties, repeated, zero and infinite thresholds, lumped and
unlumped tails, and at the full N = 10^5 size through the identities
sum_l l P(l) = C and sum_{l >= lmin} l P(l) = D of the sweep."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FULL_HIST = 2


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


def nv_of(n, m, tau):
    return n - (m - 1) * tau


def eps_set(y, m, tau, norm, w, rr):
    return oracle.select(y, m, tau, norm, w, rr)[0]


def case(name, y, m, tau, norm, w, lmin, eps):
    return dict(name=name, y=np.asarray(y, np.float32), m=m, tau=tau, norm=norm, w=w, lmin=lmin,
                eps=np.asarray(eps, np.float32))


def cases():
    out = []
    rr = np.linspace(0.01, 0.2, 20)
    # m = 1 (logistic, max norm)
    c = synth.config_small(5)
    out.append(case("logistic_m1_max", c["y"], 1, 1, 0, 1, 2, eps_set(c["y"], 1, 1, 0, 1, rr)))
    # long lines: lightly noisy sine, Euclidean, m = 1
    y = synth.series("sine", 3000, 20.0, (7, 0, 0, 1))
    out.append(case("sine_m1_euclid", y, 1, 1, 1, 1, 2, eps_set(y, 1, 1, 1, 1, rr)))
    # m = 3, tau = 5, Theiler window 5, lmin 3, repeated / zero / infinite thresholds
    y = synth.series("lorenz", 2500, 10.0, (7, 1, 0, 2))
    e = eps_set(y, 3, 5, 1, 5, rr[::2])
    e = np.concatenate([e, e[:3], [0.0, np.inf]]).astype(np.float32)
    out.append(case("lorenz_m3t5_w5_dups", y, 3, 5, 1, 5, 3, e))
    # m = 3, tau = 3 and the generic walker (m = 2, tau = 7), ragged lengths
    y = synth.series("logistic", 1733, 0.0, (7, 2, 0, 3))
    out.append(case("logistic_m3t3_max", y, 3, 3, 0, 1, 2, eps_set(y, 3, 3, 0, 1, rr)))
    y = synth.series("lorenz", 1701, -10.0, (7, 3, 0, 4))
    out.append(case("lorenz_m2t7_w3", y, 2, 7, 1, 3, 4, eps_set(y, 2, 7, 1, 3, rr[::3])))
    # integer series: many keys equal to the thresholds
    y = synth.periodic_integer(1200, 17, seed=3)
    out.append(case("periodic_ties", y, 2, 1, 0, 1, 2, np.array([0, 1, 2, 3, 5, 8], np.float32)))
    # 32 distinct thresholds, the most one call takes
    c = synth.config_small(6)
    out.append(case("logistic_k32", c["y"], 1, 1, 1, 2, 2,
                    eps_set(c["y"], 1, 1, 1, 2, np.linspace(0.005, 0.6, 32))))
    return out


CASES = cases()


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_histogram_equals_oracle(ctx, idx):
    c = CASES[idx]
    p = (c["m"], c["tau"], c["norm"], c["w"], c["lmin"])
    nv = nv_of(len(c["y"]), c["m"], c["tau"])
    y = dev(c["y"])
    plain = ctx.det_curve(y, p, c["eps"])
    for hl in (nv + 1, 16, 2, 1):
        print(f"[hist] {c['name']} hist_len={hl}", flush=True)
        got = ctx.det_curve(y, p, c["eps"], hist_len=hl)
        want = oracle.lines(c["y"], c["m"], c["tau"], c["norm"], c["w"], c["lmin"], c["eps"], hist_len=hl)
        assert got["hist"].shape == (len(c["eps"]), hl)
        assert np.array_equal(got["hist"], want["hist"]), hl
        from paper_2208_09136_amd import rqa
        gl, gm = rqa.rqa_line_measures(got["hist"], c["lmin"])
        wl, wm = oracle.line_measures(want["hist"], c["lmin"])
        assert np.array_equal(gl, wl, equal_nan=True) and np.array_equal(gm, wm)
        # the other outputs do not change with the histogram
        for key in ("count", "rr"):
            assert np.array_equal(got[key], plain[key]), key
        assert np.array_equal(got["det"], plain["det"], equal_nan=True)
    # identities of the unlumped histogram
    h = ctx.det_curve(y, p, c["eps"], hist_len=nv + 1)["hist"].astype(np.int64)
    l = np.arange(nv + 1, dtype=np.int64)
    assert np.array_equal((h * l).sum(axis=1).astype(np.uint64), plain["count"])
    D = (h[:, c["lmin"]:] * l[c["lmin"]:]).sum(axis=1)
    for r in range(len(c["eps"])):
        if plain["count"][r]:
            assert D[r] == round(plain["det"][r] * float(plain["count"][r]))
        else:
            assert D[r] == 0


def test_infinite_threshold_closed_form(ctx):
    # at eps = +inf every diagonal j - i = d (theiler <= d < nv) is one line of nv - d pairs
    y = synth.series("logistic", 900, 10.0, (7, 4, 0, 5))
    m, tau, w = 2, 3, 4
    nv = nv_of(len(y), m, tau)
    got = ctx.det_curve(dev(y), (m, tau, 1, w, 2), [np.inf], hist_len=nv + 2)["hist"][0]
    want = np.zeros(nv + 2, np.uint64)
    want[1:nv - w + 1] = 1
    assert np.array_equal(got, want)
    # at eps below every key there is no line
    got = ctx.det_curve(dev(y + np.arange(len(y), dtype=np.float32) * 10), (m, tau, 1, w, 2), [0.0],
                        hist_len=50)["hist"][0]
    assert not got.any()


def test_launch_shape_does_not_change_histogram(ctx):
    c = CASES[2]
    p = (c["m"], c["tau"], c["norm"], c["w"], c["lmin"])
    y = dev(c["y"])
    ref = oracle.lines(c["y"], c["m"], c["tau"], c["norm"], c["w"], c["lmin"], c["eps"], hist_len=300)["hist"]
    try:
        for g in (1, 3, 17):
            ctx.set_grid(g)
            assert np.array_equal(ctx.det_curve(y, p, c["eps"], hist_len=300)["hist"], ref), g
        ctx.set_grid(0)
        # segments from one tile wide to longer than every diagonal
        for seg in (64, 128, 192, 640, 4096):
            ctx.set_shape(segment=seg)
            assert np.array_equal(ctx.det_curve(y, p, c["eps"], hist_len=300)["hist"], ref), seg
    finally:
        ctx.set_grid(0)
        ctx.set_shape()


def test_histogram_limits(ctx):
    from paper_2208_09136_amd.rqa import RqaError
    c = synth.config_small(1)
    y = dev(c["y"])
    p = (1, 1, 0, 1, 2)
    e33 = eps_set(c["y"], 1, 1, 0, 1, np.linspace(0.01, 0.5, 33))
    assert len(np.unique(e33)) == 33
    # 33 distinct thresholds: one more than a histogram pass takes, so two
    # passes in the call
    got = ctx.det_curve(y, p, e33, hist_len=10)
    want = oracle.lines(c["y"], 1, 1, 0, 1, 2, e33, hist_len=10)
    assert np.array_equal(got["hist"], want["hist"])
    # 33 thresholds with 32 distinct values
    e = np.concatenate([e33[:32], e33[:1]])
    got = ctx.det_curve(y, p, e, hist_len=10)
    want = oracle.lines(c["y"], 1, 1, 0, 1, 2, e, hist_len=10)
    assert np.array_equal(got["hist"], want["hist"])
    # flag without an output buffer
    with pytest.raises(RqaError) as e:
        ctx.det_curve(y, p, e33[:3], flags=FULL_HIST)
    assert e.value.name == "RQA_ERR_INVALID_ARG"
    bad = c["y"].copy()
    bad[10] = np.nan
    with pytest.raises(RqaError) as e:
        ctx.det_curve(dev(bad), p, e33[:3], hist_len=10)
    assert e.value.name == "RQA_ERR_NONFINITE"
    # the context still works afterwards
    got = ctx.det_curve(y, p, e33[:3], hist_len=10)
    assert np.array_equal(got["hist"], oracle.lines(c["y"], 1, 1, 0, 1, 2, e33[:3], hist_len=10)["hist"])


def test_full_size_identities(ctx):
    # N = 10^5, m = 3, tau = 5, Euclidean: the workload's size, checked through
    # sum_l l P(l) = C and sum_{l >= lmin} l P(l) = D from the sweep
    c = synth.config_large(which="lorenz")[0]
    p = (c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"])
    y = dev(c["y"])
    eps = ctx.select_thresholds(y, p, c["rr"])[0]
    nv = nv_of(len(c["y"]), c["m"], c["tau"])
    print(f"[hist] {c['name']} full size", flush=True)
    got = ctx.det_curve(y, p, eps, hist_len=nv + 1)
    h = got["hist"].astype(np.int64)
    l = np.arange(nv + 1, dtype=np.int64)
    assert np.array_equal((h * l).sum(axis=1).astype(np.uint64), got["count"])
    D = (h[:, c["lmin"]:] * l[c["lmin"]:]).sum(axis=1)
    assert np.array_equal(D, np.round(got["det"] * got["count"].astype(np.float64)).astype(np.int64))
    assert (h[:, 0] == 0).all() and (h >= 0).all()


@pytest.mark.parametrize("name", ["sine_m1_euclid", "lorenz_m3t5_w5_dups"])
def test_paper_rr_set_in_one_call(ctx, name):
    """The paper's RR set 1..99 % (four histogram passes in one call), every
    row element by element against the oracle, unlumped and lumped."""
    c = next(x for x in CASES if x["name"] == name)
    p = (c["m"], c["tau"], c["norm"], c["w"], c["lmin"])
    nv = nv_of(len(c["y"]), c["m"], c["tau"])
    eps = eps_set(c["y"], c["m"], c["tau"], c["norm"], c["w"], np.arange(1, 100) / 100.0)
    assert len(np.unique(eps)) > 90
    y = dev(c["y"])
    for hl in (nv + 1, 7):
        print(f"[hist] {name} K=99 hist_len={hl}", flush=True)
        got = ctx.det_curve(y, p, eps, hist_len=hl)
        want = oracle.lines(c["y"], c["m"], c["tau"], c["norm"], c["w"], c["lmin"], eps, hist_len=hl)
        assert np.array_equal(got["hist"], want["hist"]), hl
        assert np.array_equal(got["count"], want["count"])


def batch_of(cases_):
    import torch
    offs = np.concatenate([[0], np.cumsum([len(c["y"]) for c in cases_])]).astype(np.uint64)
    concat = torch.from_numpy(np.concatenate([c["y"] for c in cases_])).to("cuda:0")
    prm = [(c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"]) for c in cases_]
    return concat, offs, prm


@pytest.mark.parametrize("K", [20, 99])
def test_batch_hist_equals_oracle(ctx, K):
    """The whole path plus the histogram at the selected thresholds in one
    call, for a slice of the ensemble (both embedding groups): thresholds,
    counts, DET and every histogram entry against the oracle's run."""
    import concurrent.futures as cf
    ens = synth.config_batch(realisations=1)
    short = [c for c in ens if len(c["y"]) <= 3000]
    sel = [c for c in short if c["m"] == 1][::3] + [c for c in short if c["m"] == 3][::2]
    assert {c["m"] for c in sel} == {1, 3} and len(sel) >= 8
    rr = np.tile(np.arange(1, K + 1) / 100.0, (len(sel), 1))
    concat, offs, prm = batch_of(sel)
    hl = max(len(c["y"]) for c in sel) + 1
    print(f"[hist] batch_hist {len(sel)} series K={K} hist_len={hl}", flush=True)
    got = ctx.batch_hist(concat, offs, prm, rr, hl)
    plain = ctx.batch(concat, offs, prm, rr)
    for key in ("eps", "count", "det", "det_mean"):
        assert np.array_equal(got[key], plain[key], equal_nan=True), key

    def want(i):
        c = sel[i]
        return oracle.run(c["y"], c["m"], c["tau"], c["norm"], c["theiler"], c["lmin"], rr[i], hist_len=hl)

    with cf.ThreadPoolExecutor(8) as ex:
        wants = list(ex.map(want, range(len(sel))))
    for i, w in enumerate(wants):
        assert np.array_equal(got["eps"][i].view(np.uint32), w["eps"].view(np.uint32)), i
        assert np.array_equal(got["count"][i], w["count"]), i
        assert np.array_equal(got["hist"][i], w["hist"]), i


def test_batch_hist_full_size_k99(ctx):
    """Both N = 10^5 bench series at the paper's 99 targets in one call: the
    averaged L and L_max curves come from its rows.  Every row satisfies
    sum_l l P(l) = C and sum_{l >= lmin} l P(l) = D; three rows per series,
    one from each of three histogram passes, equal the oracle's element by
    element."""
    from paper_2208_09136_amd import rqa
    cases_ = synth.config_large()
    concat, offs, prm = batch_of(cases_)
    rr = np.tile(np.arange(1, 100) / 100.0, (2, 1))
    nv = nv_of(100_000, 3, 5)
    print("[hist] batch_hist 2 x N=1e5 K=99", flush=True)
    got = ctx.batch_hist(concat, offs, prm, rr, nv + 1)
    ref = ctx.batch(concat, offs, prm, rr)
    for key in ("eps", "count", "det"):
        assert np.array_equal(got[key], ref[key]), key
    l = np.arange(nv + 1, dtype=np.int64)
    for s, c in enumerate(cases_):
        h = got["hist"][s].astype(np.int64)
        assert np.array_equal((h * l).sum(axis=1).astype(np.uint64), got["count"][s])
        D = (h[:, 2:] * l[2:]).sum(axis=1)
        assert np.array_equal(D, np.round(got["det"][s] * got["count"][s].astype(np.float64)).astype(np.int64))
        L, lmax = rqa.rqa_line_measures(got["hist"][s], 2)
        assert np.isfinite(rqa.rqa_averaged_det(L)).all() and (lmax >= 2).all()
        rows = [4, 50, 97]
        print(f"[hist] {c['name']} oracle rows {rows}", flush=True)
        want = oracle.lines(c["y"], 3, 5, 1, 1, 2, got["eps"][s][rows], hist_len=nv + 1)
        assert np.array_equal(got["hist"][s][rows], want["hist"])
