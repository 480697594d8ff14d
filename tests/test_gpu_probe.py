"""The VALU issue-rate probe (rqa_valu_rate), the measured denominator of the
bench line's VALU fractions: every kind runs and gives a finite rate, and an
unknown kind is an argument error.  The rates themselves are measurements
(reported by bench.py), not asserted here beyond their order of magnitude."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2208_09136_amd import rqa
    c = rqa.Context(0, torch.cuda.current_stream())
    yield c
    c.close()


def test_every_probe_kind_runs(ctx):
    from paper_2208_09136_amd import rqa
    rates = {}
    for name in rqa.VALU_PROBES:
        print(f"[probe] {name}", flush=True)
        rate, ms = ctx.valu_rate(name)
        assert math.isfinite(rate) and ms > 0.0
        # between 1 and 1000 T lane-operations per second on any recent GPU
        assert 1e12 < rate < 1e15, (name, rate)
        rates[name] = rate
    print({k: round(v / 1e12, 1) for k, v in rates.items()}, flush=True)


def test_unknown_probe_kind_is_rejected(ctx):
    from paper_2208_09136_amd import rqa
    with pytest.raises(rqa.RqaError) as e:
        ctx.valu_rate(4)
    assert e.value.name == "RQA_ERR_INVALID_ARG"
