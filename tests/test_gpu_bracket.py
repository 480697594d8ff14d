"""The threshold-bracket network end to end on the GPU: trained by the
library's own kernels on examples the exact selector generates, it must cut
the full passes of threshold selection (three for plain radix refinement,
two inside a hit window) while every result stays identical to plain
selection, and an untrained network must fall back every time."""
import numpy as np
import pytest

import synth
from paper_2208_09136_amd import bracket, rqa

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    c = rqa.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


def _set(count, seed, lo, hi, m=None):
    c, o, p, _, _ = synth.bracket_set(count, seed, lo, hi, m=m)
    return c, o, p, np.tile(np.array(synth.RR_20), (count, 1))


@pytest.fixture(scope="module")
def trained(ctx):
    print("[bracket] building training set", flush=True)
    tr = _set(1500, 101, 1000, 8000)
    Xtr, Ttr, _ = bracket.examples(ctx, *tr)
    va = _set(400, 102, 1000, 8000)
    Xva, Tva, _ = bracket.examples(ctx, *va)
    print("[bracket] training", flush=True)
    theta, hist = bracket.fit(ctx, Xtr, Ttr, epochs=40, batch=128, lr=2e-3, seed=5)
    delta, _ = bracket.calibrate(ctx, Xva, Tva)
    return theta, hist, delta, (Xva, Tva)


def test_training_reduces_loss_and_beats_constant_predictor(ctx, trained):
    theta, hist, delta, (Xva, Tva) = trained
    assert hist[-1] < 0.2 * hist[0]
    pred = bracket.predict(ctx, Xva)
    rmse = np.sqrt(np.mean((pred - Tva) ** 2))
    const = np.sqrt(np.mean((Tva - Tva.mean(0)) ** 2))
    assert rmse < 0.5 * const, (rmse, const)
    assert np.all(delta > 0) and np.all(np.isfinite(delta))


def test_trained_window_saves_passes_and_stays_exact(ctx, trained):
    te = _set(60, 103, 6000, 6000, m=3)
    ev = bracket.evaluate(ctx, *te, repeats=1)
    print(ev, flush=True)
    assert ev["network"]["exact"] and ev["sample"]["exact"]
    assert ev["network"]["miss_rate"] <= 0.1
    assert ev["network"]["passes_per_series"] < 2.4 < ev["plain"]["passes_per_series"]


def test_untrained_network_falls_back_and_stays_exact(ctx, trained):
    theta = trained[0]
    te = _set(20, 104, 3000, 3000, m=3)
    ctx.mlp_init(77)
    ctx.mlp_set_bracket(np.full(20, 1.0 / 256, np.float32))
    try:
        ev = bracket.evaluate(ctx, *te, repeats=1)
        assert ev["network"]["exact"]
        assert ev["network"]["miss_rate"] >= 0.9
        assert ev["network"]["passes_per_series"] >= 4.7
    finally:
        ctx.mlp_set_params(theta)
        ctx.mlp_set_bracket(trained[2])


def test_committed_network_saves_a_pass_on_held_out_series(ctx):
    # the shipped parameters (trained on 50,000 seeded series) bracket every
    # target of fresh held-out series: two passes, results identical to plain
    import os
    path = os.path.join(os.path.dirname(bracket.__file__), "bracket_params.npz")
    meta = bracket.load(ctx, path)
    assert meta["train"] == 50000
    te = _set(40, 907, 20000, 20000, m=3)
    ev = bracket.evaluate(ctx, *te, repeats=1)
    print(ev, flush=True)
    assert ev["network"]["exact"]
    assert ev["network"]["miss_rate"] <= 0.05
    assert ev["network"]["passes_per_series"] <= 2.15
