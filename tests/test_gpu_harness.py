"""Evaluation harnesses on the GPU: the sorting-rate ensemble's DET values
and sorting rates equal the oracle's, and the grid-threshold variant picks
the same thresholds as the oracle's grid selection."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2208_09136_amd import rqa
    c = rqa.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


@pytest.mark.parametrize("system,n,level", [("sine", 100, "10"), ("logistic", 300, "1"), ("lorenz", 250, "0.1")])
def test_sorting_rate_equals_oracle(ctx, system, n, level):
    from paper_2208_09136_amd import harness
    print(f"[harness] sorting {system} n={n} level={level}", flush=True)
    m, tau = synth.paper_embedding(system)
    params = (m, tau, 0, 1, 2)
    ens = synth.paper_ensemble(system, n, level, realisations=3, seed=4)
    avg, first = harness.ensemble_measures(ctx, ens, params)
    want_avg = np.zeros_like(avg)
    want_first = np.zeros_like(first)
    for i, row in enumerate(ens):
        for j, y in enumerate(row):
            o = oracle.run(y, m, tau, 0, 1, 2, list(harness.RR_STAR))
            want_avg[i, j] = o["det_mean"]
            want_first[i, j] = o["det"][0]
    assert np.array_equal(avg, want_avg, equal_nan=True)
    assert np.array_equal(first, want_first, equal_nan=True)
    assert harness.sorting_rate(avg) == oracle.sorting_rate(want_avg.tolist())
    assert harness.sorting_rate(first) == oracle.sorting_rate(want_first.tolist())


@pytest.mark.parametrize("system,n,norm", [("logistic", 400, 0), ("lorenz", 350, 0), ("sine", 300, 1)])
def test_grid_variant_equals_oracle(ctx, system, n, norm):
    import torch
    from paper_2208_09136_amd import harness
    print(f"[harness] grid {system} n={n} norm={norm}", flush=True)
    m, tau = synth.paper_embedding(system)
    params = (m, tau, norm, 1, 2)
    y = synth.paper_ensemble(system, n, "1", realisations=1, seed=5)[0][6]
    eps = harness.grid_thresholds(norm)
    dev = torch.from_numpy(harness.rescale01(y)).to("cuda:0")
    got = harness.grid_select(harness.grid_rr(ctx, dev, params, eps), eps, harness.RR_STAR)
    want = oracle.grid_select(y, m, tau, norm, 1, list(harness.RR_STAR))
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    err_grid, _ = harness.grid_vs_exact(ctx, y, params)
    assert np.array_equal(err_grid, want[2])
