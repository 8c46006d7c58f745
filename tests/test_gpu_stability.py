"""The Re_max sweep's stability verdicts (the paper's Discussion section and its
Re_max figure) against the FP64 oracle: every lid speed of the scan at cavity
sides 50 and 100, run in FP64 on the GPU as one batch of LBMTau1 cavities, must be
flagged stable or unstable exactly as the oracle flags it, at the same 100-step
check.  The oracle's verdicts are in tests/golden/stability_verdicts.json, written
by tests/golden/make_stability_verdicts.py from the oracle alone."""
import json
import os
import sys

import pytest

from paper_1912_09327_amd import stability as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stability_verdicts.json")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _golden(L):
    return json.load(open(GOLDEN))["sides"][str(L)]


@pytest.mark.parametrize("L", [50, 100])
def test_batched_fp64_verdicts_equal_the_oracle(L):
    ref = _golden(L)
    speeds = S.lid_speeds(0.1, 1.6, 1.05)
    assert len(speeds) == len(ref)
    for u, r in zip(speeds, ref):
        assert u == pytest.approx(r["u0"], rel=1e-14)
        assert S.horizon(L, u) >= r["steps"] or r["unstable"]
    _say(f"[stability] L={L}: {len(speeds)} FP64 cavities as one batch")
    got = S.scan_batched(L, speeds, prec="f64")
    for (u, bad, steps), r in zip(got, ref):
        assert (bad, steps) == (r["unstable"], r["steps"]), (L, u, bad, steps, r)
    re_gpu = S.re_max_from_scan(L, 1.0, [(u, bad) for u, bad, _ in got])
    re_ref = S.re_max_from_scan(L, 1.0, [(r["u0"], r["unstable"]) for r in ref])
    _say(f"[stability] L={L}: Re_max {re_gpu:.1f} on the GPU, {re_ref:.1f} from the oracle")
    assert re_gpu == pytest.approx(re_ref, rel=1e-14)


def test_population_runner_fp64_verdicts_equal_the_oracle():
    """The stored-population runner at tau = 1 (one grid after another, stopping at the
    first unstable speed) reaches the same verdicts on the side-50 scan."""
    L = 50
    ref = _golden(L)
    got = S.scan_populations(L, 1.0, S.lid_speeds(0.1, 1.6, 1.05), prec="f64")
    assert len(got) == next(i for i, r in enumerate(ref) if r["unstable"]) + 1
    for (u, bad, steps), r in zip(got, ref):
        assert (bad, steps) == (r["unstable"], r["steps"]), (u, bad, steps, r)
