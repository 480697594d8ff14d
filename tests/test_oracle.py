"""Pins for the CPU oracle: checks against hand-derived plots, brute force in
numpy, closed forms and invariants.  None of these re-types the oracle's own
code; each would catch a dropped term, a wrong sign or index, or a transposed
operand in it.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handbuilt_plots.json")


# ---------------------------------------------------------------- brute force
def np_vectors(y, m, tau):
    """Delay vectors as an (Nv, m) float32 array; column k is y[i + (m-1-k)tau]."""
    y = np.asarray(y, dtype=np.float32)
    nv = len(y) - (m - 1) * tau
    return np.stack([y[(m - 1 - k) * tau:(m - 1 - k) * tau + nv] for k in range(m)], axis=1)


def np_key_matrix(y, m, tau, norm):
    """Full Nv x Nv key matrix, float32 elementwise (IEEE, no contraction)."""
    v = np_vectors(y, m, tau)
    nv = v.shape[0]
    acc = np.zeros((nv, nv), dtype=np.float32)
    for k in range(m):
        d = (v[:, k][:, None] - v[:, k][None, :]).astype(np.float32)
        if norm == 0:
            acc = np.maximum(acc, np.abs(d))
        else:
            sq = (d * d).astype(np.float32)
            acc = sq if k == 0 else (acc + sq).astype(np.float32)
    return acc


def np_keys_diag_major(y, m, tau, norm, w):
    K = np_key_matrix(y, m, tau, norm)
    nv = K.shape[0]
    return np.concatenate([np.diagonal(K, offset=d) for d in range(w, nv)]).astype(np.float32)


def np_line_hist(y, m, tau, norm, w, eps):
    """P(l) from the explicit boolean matrix: run lengths on each upper diagonal."""
    R = np_key_matrix(y, m, tau, norm) <= np.float32(eps)
    nv = R.shape[0]
    P = {}
    for d in range(w, nv):
        diag = np.concatenate([[False], np.diagonal(R, offset=d), [False]]).astype(np.int8)
        edges = np.diff(diag)
        starts = np.flatnonzero(edges == 1)
        ends = np.flatnonzero(edges == -1)
        for s, e in zip(starts, ends):
            P[e - s] = P.get(e - s, 0) + 1
    return P


def rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ golden fixtures
def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("case", load_golden()["cases"], ids=lambda c: c["name"])
def test_handbuilt_plots(case):
    y = np.array(case["y"], dtype=np.float32)
    nv = oracle.num_vectors(len(y), case["m"], case["tau"])
    assert oracle.num_pairs(nv, case["theiler"]) == case["M"]
    hl = nv + 1
    out = oracle.lines(y, case["m"], case["tau"], case["norm"], case["theiler"], case["lmin"],
                       [case["eps"]], hist_len=hl)
    want = np.zeros(hl, dtype=np.uint64)
    for l, c in case["P"].items():
        want[int(l)] = c
    np.testing.assert_array_equal(out["hist"][0], want)
    assert int(out["count"][0]) == case["count"]
    assert out["rr"][0] == case["count"] / case["M"]
    assert out["det"][0] == case["det_num"] / case["count"]


@pytest.mark.parametrize("rc", load_golden()["ranks"]["cases"], ids=lambda c: str(c["rr"]))
def test_handbuilt_ranks(rc):
    g = load_golden()["ranks"]
    y = np.array(g["y"], dtype=np.float32)
    eps, k, c = oracle.select(y, g["m"], g["tau"], g["norm"], g["theiler"], [rc["rr"]], method=1)
    assert int(k[0]) == rc["k"] and float(eps[0]) == rc["eps"] and int(c[0]) == rc["count"]
    eps2, k2, c2 = oracle.select(y, g["m"], g["tau"], g["norm"], g["theiler"], [rc["rr"]], method=2)
    assert eps2[0] == eps[0] and k2[0] == k[0] and c2[0] == c[0]


# ---------------------------------------------------------------------- keys
@pytest.mark.parametrize("m,tau,norm", [(1, 1, 0), (1, 1, 1), (3, 5, 1), (3, 5, 0), (2, 3, 1),
                                        (4, 2, 1), (3, 1, 0)])
def test_keys_match_numpy_brute_force(m, tau, norm):
    for seed, n in [(0, 40), (1, 64), (2, 300)]:
        y = rng(seed).standard_normal(n).astype(np.float32)
        got = oracle.keys(y, m, tau, norm, 1)
        want = np_keys_diag_major(y, m, tau, norm, 1)
        assert got.view(np.uint32).tolist() == want.view(np.uint32).tolist()


def test_key_single_pair_definition():
    # Component k of vector i is y[i + (m-1-k) tau] (k = 0 the newest sample);
    # the squared Euclidean key folds left from k = 0.  With d0 = 1 and
    # d1 = d2 = 2^-12 the left fold gives (1 + 2^-24) + 2^-24 = 1 (two ties to
    # even), while the reversed fold would give 1 + 2^-23.
    y = np.zeros(10, dtype=np.float32)
    y[4] = 1.0             # i=0, k=0 -> y[4]; j=1, k=0 -> y[5] = 0
    y[2] = 2.0 ** -12      # k=1 -> y[2] vs y[3]
    y[0] = 2.0 ** -12      # k=2 -> y[0] vs y[1]
    k = oracle.key(y, 3, 2, 1, 0, 1)
    assert k == np.float32(1.0)
    assert np.float32(1.0) + np.float32(2.0 ** -23) != k
    # swapping which sample is newest changes the key: component 0 would be
    # y[0] - y[1] = 2^-12 and the fold 2^-24 + 2^-24 + 1 = 1 + 2^-23
    y3 = np.zeros(10, dtype=np.float32)
    y3[0] = 1.0
    y3[2] = 2.0 ** -12
    y3[4] = 2.0 ** -12
    assert oracle.key(y3, 3, 2, 1, 0, 1) == np.float32(1.0) + np.float32(2.0 ** -23)
    # the max norm is order-free
    assert oracle.key(y, 3, 2, 0, 0, 1) == np.float32(1.0)


def test_key_scaling_and_negation_invariance():
    y = rng(5).standard_normal(200).astype(np.float32)
    for m, tau in [(1, 1), (3, 5)]:
        for norm, power in [(0, 1), (1, 2)]:
            base = oracle.keys(y, m, tau, norm, 1)
            for j in (-3, 2, 7):
                scaled = oracle.keys(y * np.float32(2.0 ** j), m, tau, norm, 1)
                np.testing.assert_array_equal(scaled, base * np.float32(2.0 ** (power * j)))
            np.testing.assert_array_equal(oracle.keys(-y, m, tau, norm, 1), base)


# ---------------------------------------------------------------------- ranks
def test_rank_closed_forms():
    assert oracle.rank(0.07, 100) == 7
    assert oracle.rank(0.01, 499500) == 4995
    assert oracle.rank(0.2, 499500) == 99900
    assert oracle.rank(0.5, 7) == 4            # ceil(3.5)
    assert oracle.rank(1.0, 4998950055) == 4998950055
    assert oracle.rank(1e-12, 1000) == 1       # clamped to 1
    assert oracle.rank(0.03, 4998950055) == 149968502     # ceil(149968501.65)
    assert oracle.rank(0.0, 10) == 0 and oracle.rank(1.5, 10) == 0 and oracle.rank(float("nan"), 10) == 0


def test_rank_quantisation_integer_products():
    # 0.07 * 100 in binary64 is 7.000000000000001; the 1e-9 quantised target
    # makes rr * M an exact integer whenever it is one in decimal.
    for M in (100, 1000, 123400, 10 ** 10):
        for pct in range(1, 100):
            assert oracle.rank(pct / 100.0, M) == -(-pct * M // 100)


def test_pair_counts():
    assert oracle.num_vectors(100000, 3, 5) == 99990
    assert oracle.num_pairs(99990, 1) == 4998950055
    assert oracle.num_pairs(1000, 1) == 499500
    assert oracle.num_pairs(10, 10) == 0 and oracle.num_pairs(10, 9) == 1
    assert oracle.num_vectors(10, 4, 3) == 1 and oracle.num_vectors(9, 4, 3) == 0


# ------------------------------------------------------------------ selection
@pytest.mark.parametrize("m,tau,norm,w", [(1, 1, 0, 1), (3, 5, 1, 1), (2, 2, 0, 3), (1, 1, 1, 5)])
def test_select_matches_sorted_brute_force(m, tau, norm, w):
    rr = np.array([0.001, 0.01, 0.05, 0.1, 0.2, 0.37, 0.5, 0.99, 1.0])
    for seed, n in [(0, 64), (1, 500)]:
        y = rng(seed).standard_normal(n).astype(np.float32)
        keys = np.sort(np_keys_diag_major(y, m, tau, norm, w))
        M = len(keys)
        eps, k, c = oracle.select(y, m, tau, norm, w, rr, method=1)
        for r in range(len(rr)):
            q = int(round(rr[r] * 1e9))
            kr = max(1, min(M, -(-q * M // 10 ** 9)))
            assert int(k[r]) == kr
            assert eps[r] == keys[kr - 1]
            assert int(c[r]) == int(np.sum(keys <= eps[r]))


def test_select_bisection_equals_sort():
    rr = np.array(synth.RR_20)
    for seed, (n, m, tau, norm) in enumerate([(700, 1, 1, 0), (900, 3, 5, 1), (1500, 2, 4, 1)]):
        y = synth.series(synth.SYSTEMS[seed % 3], n, 0.0, (9, seed, 0, 0))
        a = oracle.select(y, m, tau, norm, 1, rr, method=1)
        b = oracle.select(y, m, tau, norm, 1, rr, method=2)
        for x, z in zip(a, b):
            np.testing.assert_array_equal(x, z)


def test_order_statistic_invariant():
    y = synth.config_small(3)["y"]
    rr = np.array(synth.RR_20)
    eps, k, c = oracle.select(y, 1, 1, 0, 1, rr)
    lt, le = oracle.count(y, 1, 1, 0, 1, eps)
    assert np.all(lt < k) and np.all(k <= le)
    np.testing.assert_array_equal(le, c)
    # eps is increasing with rr and attains the target rate
    assert np.all(np.diff(eps) >= 0)
    M = oracle.num_pairs(1000, 1)
    assert np.all(c / M >= rr - 1e-12)


@pytest.mark.parametrize("m,tau,norm,w,kind", [(1, 1, 0, 1, "integer"), (1, 1, 1, 1, "integer"),
                                               (3, 5, 1, 1, "normal"), (2, 3, 0, 2, "normal"),
                                               (3, 2, 1, 3, "integer")])
def test_count_strict_and_inclusive_match_numpy(m, tau, norm, w, kind):
    """#{key < v} and #{key <= v} (the two sides of the order-statistic
    bracket #{key < eps} < k <= #{key <= eps} that pins a threshold at any
    size) against numpy counts over the brute-force key list: values equal
    to keys (ties: integer series make many equal keys), values between
    consecutive distinct keys, 0, +inf and values outside the key range."""
    r = rng(31 + m + w)
    n = 900
    if kind == "integer":
        y = r.integers(0, 12, n).astype(np.float32)
    else:
        y = r.standard_normal(n).astype(np.float32)
    keys = np_keys_diag_major(y, m, tau, norm, w)
    u = np.unique(keys)
    if kind == "integer":
        assert len(u) < len(keys) // 100             # many ties
    pick = u[r.choice(len(u), 12, replace=False)]
    between = [np.nextafter(u[i], u[i + 1]) for i in r.choice(len(u) - 1, 8, replace=False)]
    vals = np.concatenate([pick, np.array(between, dtype=np.float32), u[:1], u[-1:],
                           np.array([0.0, np.inf, u[-1] * 2 + 1, np.float32(1e-30)], dtype=np.float32)])
    lt, le = oracle.count(y, m, tau, norm, w, vals)
    want_lt = np.array([np.sum(keys < v) for v in vals], dtype=np.uint64)
    want_le = np.array([np.sum(keys <= v) for v in vals], dtype=np.uint64)
    np.testing.assert_array_equal(lt, want_lt)
    np.testing.assert_array_equal(le, want_le)
    # at a key value the two counts differ by its multiplicity (> 1 for ties)
    mult = le[:12] - lt[:12]
    assert np.all(mult >= 1)
    if kind == "integer":
        assert np.all(mult > 1)
    assert lt[-4] == 0 and le[-3] == len(keys)       # v = 0 (no key below 0), v = +inf


def test_select_ties_all_equal():
    y = np.full(50, 3.25, dtype=np.float32)
    eps, k, c = oracle.select(y, 2, 3, 1, 1, [0.01, 0.5, 1.0])
    assert np.all(eps == 0.0)
    M = oracle.num_pairs(oracle.num_vectors(50, 2, 3), 1)
    assert np.all(c == M)


# ---------------------------------------------------------------------- lines
@pytest.mark.parametrize("m,tau,norm,w,lmin", [(1, 1, 0, 1, 2), (3, 5, 1, 1, 2), (2, 3, 0, 2, 3),
                                               (1, 1, 1, 1, 1), (3, 2, 1, 4, 4)])
def test_lines_match_numpy_run_lengths(m, tau, norm, w, lmin):
    y = rng(11).standard_normal(180).astype(np.float32)
    keys = np.sort(np_keys_diag_major(y, m, tau, norm, w))
    eps = [keys[len(keys) // 50], keys[len(keys) // 7], keys[len(keys) // 3]]
    nv = oracle.num_vectors(len(y), m, tau)
    out = oracle.lines(y, m, tau, norm, w, lmin, eps, hist_len=nv + 1)
    M = oracle.num_pairs(nv, w)
    for r, e in enumerate(eps):
        P = np_line_hist(y, m, tau, norm, w, e)
        want = np.zeros(nv + 1, dtype=np.uint64)
        for l, c in P.items():
            want[l] = c
        np.testing.assert_array_equal(out["hist"][r], want)
        C = sum(l * c for l, c in P.items())
        assert int(out["count"][r]) == C == int(np.sum(keys <= e))
        assert out["rr"][r] == C / M
        assert out["det"][r] == sum(l * c for l, c in P.items() if l >= lmin) / C


def test_periodic_closed_form():
    # y_t = c_{t mod P} with distinct levels: the zero keys are exactly the
    # diagonals d = P, 2P, ...; for k_r <= Z the threshold is 0 and every
    # recurrence lies on a full-length diagonal line.
    for n, P in [(400, 7), (1000, 37), (333, 10)]:
        y = synth.periodic_integer(n, P)
        nv = n
        Z = sum(nv - d for d in range(P, nv, P))
        M = oracle.num_pairs(nv, 1)
        rr = [Z / M * f for f in (0.1, 0.5, 0.999)]
        eps, k, c = oracle.select(y, 1, 1, 0, 1, rr)
        assert np.all(eps == 0.0) and np.all(c == Z)
        out = oracle.lines(y, 1, 1, 0, 1, 2, eps)
        want = sum(nv - d for d in range(P, nv, P) if nv - d >= 2) / Z
        assert np.all(out["det"] == want)
        assert np.all(out["rr"] == Z / M)


def test_lmin_one_gives_det_one():
    y = synth.config_small(1)["y"]
    eps, _, _ = oracle.select(y, 1, 1, 0, 1, synth.RR_20)
    out = oracle.lines(y, 1, 1, 0, 1, 1, eps)
    assert np.all(out["det"] == 1.0)


def test_single_recurrence_det_zero():
    y = rng(3).permutation(200).astype(np.float32) * np.float32(1.5) + rng(4).random(200).astype(np.float32)
    keys = np_keys_diag_major(y, 1, 1, 0, 1)
    assert np.sum(keys == keys.min()) == 1
    eps, k, c = oracle.select(y, 1, 1, 0, 1, [1e-9])
    assert k[0] == 1 and c[0] == 1 and eps[0] == keys.min()
    out = oracle.lines(y, 1, 1, 0, 1, 2, eps)
    assert out["count"][0] == 1 and out["det"][0] == 0.0


def test_time_reversal_and_negation():
    y = synth.series("lorenz", 400, 10.0, (9, 9, 9, 9))
    eps, _, _ = oracle.select(y, 3, 2, 0, 1, [0.02, 0.1, 0.3])
    a = oracle.lines(y, 3, 2, 0, 1, 2, eps, hist_len=50)
    b = oracle.lines(y[::-1].copy(), 3, 2, 0, 1, 2, eps, hist_len=50)
    c = oracle.lines(-y, 3, 2, 0, 1, 2, eps, hist_len=50)
    for o in (b, c):
        np.testing.assert_array_equal(o["hist"], a["hist"])
        np.testing.assert_array_equal(o["det"], a["det"])


def test_det_mean_is_plain_average():
    case = synth.config_small(2)
    out = oracle.run(case["y"], 1, 1, 0, 1, 2, case["rr"])
    s = 0.0
    for d in out["det"]:
        s += d
    assert out["det_mean"] == s / len(out["det"])
    assert np.all(out["count"] == out["count_select"])


def test_uniform_noise_statistics():
    # i.i.d. U(0,1), m = 1, max norm: P(|a-b| <= e) = 2e - e^2 and, with
    # neighbouring cells on a diagonal independent, DET ~ 1 - (1-p)^2.
    y = rng(21).random(1500).astype(np.float32)
    eps = np.array([0.02, 0.05, 0.1], dtype=np.float32)
    out = oracle.lines(y, 1, 1, 0, 1, 2, eps)
    p = 2 * eps.astype(np.float64) - eps.astype(np.float64) ** 2
    assert np.all(np.abs(out["rr"] - p) < 0.01)
    assert np.all(np.abs(out["det"] - (1 - (1 - p) ** 2)) < 0.02)


def test_error_paths():
    y = np.arange(10, dtype=np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.select(y, 4, 3, 0, 1, [0.1])
    assert e.value.status == oracle.ERR_TOO_SHORT
    bad = y.copy()
    bad[3] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.select(bad, 1, 1, 0, 1, [0.1])
    assert e.value.status == oracle.ERR_NONFINITE
    with pytest.raises(oracle.OracleError) as e:
        oracle.select(y, 1, 1, 0, 0, [0.1])
    assert e.value.status == oracle.ERR_INVALID
    with pytest.raises(oracle.OracleError) as e:
        oracle.select(y, 1, 1, 0, 1, [0.0])
    assert e.value.status == oracle.ERR_INVALID


# ------------------------------------------------------- L and L_max from P(l)
def np_line_lengths(y, m, tau, norm, w, eps):
    """Every diagonal line's length, from the explicit boolean matrix."""
    R = np_key_matrix(y, m, tau, norm) <= np.float32(eps)
    out = []
    for d in range(w, R.shape[0]):
        diag = np.concatenate([[False], np.diagonal(R, offset=d), [False]]).astype(np.int8)
        edges = np.diff(diag)
        out += (np.flatnonzero(edges == -1) - np.flatnonzero(edges == 1)).tolist()
    return out


def test_line_measures_literal_example():
    # P = (0, 3, 0, 2, 0, 1): lines 1,1,1,3,3,5
    h = np.array([[0, 3, 0, 2, 0, 1], [0, 4, 0, 0, 0, 0], [0] * 6], dtype=np.uint64)
    L, lmax = oracle.line_measures(h, 2)
    assert L[0] == 11 / 3 and lmax[0] == 5
    assert math.isnan(L[1]) and lmax[1] == 1
    assert math.isnan(L[2]) and lmax[2] == 0
    L1, _ = oracle.line_measures(h, 1)
    assert L1[0] == 14 / 6 and L1[1] == 1.0


@pytest.mark.parametrize("m,tau,norm,w,lmin", [(1, 1, 0, 1, 2), (3, 5, 1, 1, 2), (2, 3, 0, 2, 3)])
def test_line_measures_brute_force(m, tau, norm, w, lmin):
    # mean length of the lines of at least lmin, and the longest line, taken
    # directly from the run lengths of the boolean matrix
    y = rng(12).standard_normal(150).astype(np.float32)
    keys = np.sort(np_keys_diag_major(y, m, tau, norm, w))
    eps = [keys[len(keys) // 40], keys[len(keys) // 5], keys[len(keys) // 2]]
    nv = oracle.num_vectors(len(y), m, tau)
    out = oracle.lines(y, m, tau, norm, w, lmin, eps, hist_len=nv + 1)
    L, lmax = oracle.line_measures(out["hist"], lmin)
    for r, e in enumerate(eps):
        ls = np_line_lengths(y, m, tau, norm, w, e)
        long_ = [l for l in ls if l >= lmin]
        assert lmax[r] == max(ls)
        if long_:
            assert L[r] == pytest.approx(sum(long_) / len(long_), rel=1e-15)
        else:
            assert math.isnan(L[r])


def test_line_measures_periodic_closed_form():
    # y_t = c_{t mod P}: at eps = 0 the lines are the whole diagonals d = P, 2P, ...
    for n, P in [(400, 7), (333, 10)]:
        y = synth.periodic_integer(n, P)
        out = oracle.lines(y, 1, 1, 0, 1, 2, [0.0], hist_len=n + 1)
        L, lmax = oracle.line_measures(out["hist"], 2)
        lens = [n - d for d in range(P, n, P) if n - d >= 2]
        assert lmax[0] == n - P
        assert L[0] == pytest.approx(sum(lens) / len(lens), rel=1e-15)


# ------------------------------------------------------- sorting rate (Eq. 5)
def test_sorting_rate_closed_forms():
    perfect = [list(range(10)) for _ in range(10)]
    assert oracle.sorting_rate(perfect) == 100.0
    reversed_ = [list(range(10, 0, -1)) for _ in range(10)]
    assert oracle.sorting_rate(reversed_) == 0.0
    # the worst-case total is 500 for ten realisations of ten series: one
    # swapped neighbour pair in one realisation departs by 2
    one_swap = [list(range(10)) for _ in range(10)]
    one_swap[4][3], one_swap[4][4] = one_swap[4][4], one_swap[4][3]
    assert oracle.sorting_rate(one_swap) == 100.0 * (500 - 2) / 500
    # equal values keep the SNR order; NaN sorts after every number
    assert oracle.sorting_rate([[0.5] * 10]) == 100.0
    nan_first = [[float("nan")] + list(range(1, 10))]
    # series 1 moves to position 10, series j (j >= 2) to j - 1: departure 9 + 9
    assert oracle.sorting_rate(nan_first) == 100.0 * (50 - 18) / 50


def test_grid_select_brute_force():
    # RR at each grid threshold from the explicit key matrix of the rescaled
    # series, then the closest grid RR per target by a plain scan
    y = rng(21).standard_normal(70).astype(np.float32)
    for m, tau, norm in ((1, 1, 0), (3, 3, 0), (2, 2, 1)):
        y64 = y.astype(np.float64)
        y01 = ((y64 - y64.min()) / (y64.max() - y64.min())).astype(np.float32)
        K = np_key_matrix(y01, m, tau, norm)
        nv = K.shape[0]
        upper = K[np.triu_indices(nv, 1)]
        n_grid = 50
        grid = np.array([(i / n_grid) if norm == 0 else (i / n_grid) ** 2 for i in range(1, n_grid + 1)],
                        dtype=np.float32)
        rr = np.array([np.sum(upper <= g) for g in grid]) / upper.size
        targets = [0.01, 0.1, 0.37, 0.9]
        eps, got_rr, err = oracle.grid_select(y, m, tau, norm, 1, targets, n_grid=n_grid)
        for t, e, r, d in zip(targets, eps, got_rr, err):
            best = min(range(n_grid), key=lambda i: (abs(rr[i] - t), i))
            assert e == grid[best] and r == rr[best] and d == abs(rr[best] - t)
