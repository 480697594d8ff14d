"""Host-side pieces of the threshold-bracket training: the many-series
generator and the folding of input/target standardisation into the network."""
import numpy as np

import oracle.mlp as omlp
import synth
from paper_2208_09136_amd import bracket


def test_many_series_generator_matches_single_series_generators():
    # one series per system: the vectorised iteration must reproduce the
    # scalar recursions exactly (same draws, same float64 arithmetic)
    for many, one in ((synth._logistic_many, synth.logistic), (synth._lorenz_many, synth.lorenz_x)):
        a = many(np.array([2500]), synth.rng_for(9, 1))[0]
        b = one(2500, synth.rng_for(9, 1))
        assert np.array_equal(a, b)


def test_many_series_uneven_lengths_keep_their_own_trajectories():
    # a series' samples do not depend on the lengths of the others in its group
    a = synth._logistic_many(np.array([50, 400, 120]), synth.rng_for(4))
    x0 = synth.rng_for(4).uniform(0.1, 0.9, size=3)
    for s, n in enumerate((50, 400, 120)):
        x = x0[s]
        for _ in range(1000):
            x = 4.0 * x * (1.0 - x)
        ref = np.empty(n)
        for i in range(n):
            ref[i] = x
            x = 4.0 * x * (1.0 - x)
        assert np.array_equal(a[s], ref)


def test_bracket_set_deterministic_and_shaped():
    c1, o1, p1, s1, q1 = synth.bracket_set(40, 5, 1000, 3000)
    c2, o2, p2, s2, q2 = synth.bracket_set(40, 5, 1000, 3000)
    assert np.array_equal(c1, c2) and np.array_equal(o1, o2) and p1 == p2
    lens = np.diff(o1.astype(np.int64))
    assert lens.min() >= 1000 and lens.max() <= 3000 and c1.dtype == np.float32
    assert set(s1) <= set(synth.SYSTEMS) and np.all((q1 >= -25) & (q1 <= 20))
    assert all(p[0] in (1, 3) and p[1] == (5 if p[0] == 3 else 1) and p[2] == synth.NORM_EUCLID for p in p1)
    c3, o3, p3, *_ = synth.bracket_set(10, 6, 2000, 2000, m=3)
    assert np.all(np.diff(o3.astype(np.int64)) == 2000) and all(p[0] == 3 for p in p3)


def test_standardiser_fold_equals_standardised_network():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(50, omlp.IN)) * rng.uniform(0.01, 3.0, size=omlp.IN) + rng.normal(size=omlp.IN)
    T = rng.normal(size=(50, omlp.OUT)) * 2.0 - 4.0
    std = bracket.Standardiser(X, T)
    theta = omlp.init(7)
    theta[omlp.PARAMS - omlp.OUT:] = rng.normal(size=omlp.OUT)   # nonzero output bias
    want = std.mt + std.st * omlp.forward(theta, std.x(X))[0]
    got = omlp.forward(std.fold(theta).astype(np.float64), X)[0]
    assert np.allclose(got, want, rtol=1e-5, atol=1e-5 * np.abs(want).max())


def test_targets_are_bit_offsets():
    eps = np.array([[1.0, 2.0, 0.5]], np.float32)
    scale = np.array([np.float32(1.0).view(np.uint32)], np.uint32)
    assert np.array_equal(bracket.targets(eps, scale), [[0.0, 1.0, -1.0]])

