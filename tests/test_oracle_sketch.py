"""Pins for the sketch oracle (CPU only)."""
import json
import os

import numpy as np

import oracle
import synth
from oracle import sketch


def test_splitmix64_published_sequence():
    # SplitMix64 from state 0: the first three outputs of the reference
    # generator (Steele, Lea and Flood; Vigna's constants).
    assert sketch.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert sketch.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert sketch.splitmix64(0, 2) == 0x06C45D188009454F


def test_pair_index_is_diagonal_major_enumeration():
    for nv, w in [(10, 1), (17, 3), (33, 32)]:
        L0 = nv - w
        pairs = [(t, t + d) for d in range(w, nv) for t in range(nv - d)]
        assert len(pairs) == oracle.num_pairs(nv, w)
        for p, want in enumerate(pairs):
            assert sketch.pair_of(p, L0, w) == want


def test_sketch_invariants():
    case = synth.config_small(0)
    f, scale = sketch.sketch(case["y"], 1, 1, 0, 1, seed=12345)
    assert f.dtype == np.float32 and f.shape == (66,)
    assert abs(float(f[:64].sum()) - 1.0) < 1e-6
    keys = np.sort(sketch.sample_keys(case["y"], 1, 1, 0, 1, 12345).view(np.uint32))
    assert keys[2047] == scale
    # half of the samples lie at or below the median bucket boundary
    assert float(f[:33].sum()) >= 0.5
    assert f[64] == np.float32(np.log2(1000) / 16) and f[65] == np.float32(0.25)
    # sampled keys are keys of real pairs
    allk = np.sort(oracle.keys(case["y"], 1, 1, 0, 1))
    assert np.all(np.isin(keys.view(np.float32), allk))


def test_target_offsets_sign_and_scale():
    scale = int(np.float32(1.0).view(np.uint32))
    t = sketch.target_offsets([2.0, 0.5, 1.0], scale)
    np.testing.assert_array_equal(t, np.array([1.0, -1.0, 0.0], np.float32))


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sketch_bins.json")


def test_sketch_binning_hand_derived():
    """Bins, scale and features of a hand-built key multiset: each value's
    bin is derived by hand from its bit pattern in the fixture, chosen so
    that a shift of 20 instead of 21, an offset of 31 instead of 32, a
    rounding toward zero instead of a floor, the other median or a wrong
    clamp each change some bin."""
    with open(GOLDEN) as f:
        g = json.load(f)
    keys = []
    for e in g["keys"]:
        v = np.float32(float(e["value"]))
        assert int(v.view(np.uint32)) == int(e["bits"], 16), e
        keys += [v] * e["count"]
    keys = np.array(keys, dtype=np.float32)
    np.random.default_rng(0).shuffle(keys)          # the sample comes in pair order
    f, scale = sketch.features_from_keys(keys, g["n"], g["m"])
    assert scale == int(g["scale"], 16)
    want = np.zeros(64, dtype=np.float32)
    for b, c in g["bins"].items():
        want[int(b)] = np.float32(c / 4096)
    np.testing.assert_array_equal(f[:64], want)
    assert f[64] == np.float32(g["feature_64"]) and f[65] == np.float32(g["feature_65"])
    for e in g["keys"]:
        assert sketch.bin_of(int(e["bits"], 16), scale) in [int(b) for b in g["bins"]]
