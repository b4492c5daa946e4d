"""The FP32 probability bars (helpers.fp32_bars) can fail on the observables
they are meant to pin: a planted error of a few percent in P_+1 or P_flip of a
stored 512^2 oracle result is caught, rounding-level differences are not."""
import json
import os

import numpy as np
import pytest

from helpers import check_fp32_probabilities, fp32_bars

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def ref_obs(name="mid_w2"):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        rec = json.load(f)
    return np.array(rec["observables"]), rec["workload"]["obs"]["n_max"], rec["steps"]


def test_bars_are_below_the_diffracted_and_flip_probabilities():
    ref, n_max, steps = ref_obs()
    nb = 2 * n_max + 1
    bars = fp32_bars(ref, n_max, steps)
    p1, flip = 1 + n_max + 1, 1 + 3 * nb
    assert bars[p1] < 0.05 * ref[p1]      # P_+1 = 1.4e-5
    assert bars[flip] < 0.05 * ref[flip]  # P_flip = 9.0e-7
    assert np.all(bars <= 1e-4)


@pytest.mark.parametrize("which,rel", [("P_+1", 0.05), ("P_flip", 0.05)])
def test_planted_error_fails(which, rel):
    ref, n_max, steps = ref_obs()
    nb = 2 * n_max + 1
    k = 1 + n_max + 1 if which == "P_+1" else 1 + 3 * nb
    got = ref.copy()
    got[k] *= 1 + rel
    with pytest.raises(AssertionError):
        check_fp32_probabilities(got, ref, n_max, steps, "planted")


def test_rounding_level_difference_passes():
    ref, n_max, steps = ref_obs()
    got = ref * (1 + 1e-7) + 1e-12
    check_fp32_probabilities(got, ref, n_max, steps, "rounding")
