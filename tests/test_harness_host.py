"""Host logic of the evaluation harnesses (sorting rate of Eq. 5, grid
thresholds), against the oracle and hand-computed values."""
import numpy as np
import pytest


def test_harness_sorting_rate_equals_oracle():
    # host logic of the sorting-rate harness against the oracle's plain loops,
    # with ties and NaN
    import oracle
    from paper_2208_09136_amd import harness
    g = np.random.default_rng(5)
    for trial in range(50):
        R, n = int(g.integers(1, 12)), int(g.integers(2, 12))
        m = g.integers(0, 4, size=(R, n)).astype(np.float64)   # many ties
        if trial % 3 == 0:
            m[g.random(size=(R, n)) < 0.2] = np.nan
        assert harness.sorting_rate(m) == oracle.sorting_rate(m.tolist())
    with pytest.raises(ValueError):
        harness.sorting_rate([[1.0]])


def test_harness_grid_thresholds_and_selection():
    from paper_2208_09136_amd import harness
    e = harness.grid_thresholds(0, 400)
    assert e.dtype == np.float32 and e[0] == np.float32(1 / 400) and e[-1] == 1.0 and e.size == 400
    e2 = harness.grid_thresholds(1, 4)
    assert e2.tolist() == [np.float32(0.0625), np.float32(0.25), np.float32(0.5625), 1.0]
    eps, rr, err = harness.grid_select([0.1, 0.2, 0.3, 0.3], [1, 2, 3, 4], [0.0, 0.15, 0.26, 0.31])
    assert eps.tolist() == [1, 1, 3, 3] and rr.tolist() == [0.1, 0.1, 0.3, 0.3]
    y = harness.rescale01(np.array([2.0, 4.0, 3.0]))
    assert y.tolist() == [0.0, 1.0, 0.5]
