"""What the trained learned guess gains over the method without it (held-out seeds).

The committed models were trained on perturbation seeds 0..199 at 8x (default) and 4x the
explicit step; seeds 1000+ are held out.  Every stage converges to ||R|| <= 1e-10 ||R(0)||.
At 4x the learned run needs fewer Newton iterations; at 8x, where the plain extrapolated
iterate often tangles the stage mesh (non-finite residual, the solve restarts from zero), the
learned iterate is used at every step and starts from a far smaller residual.  The
zero-output control carries the same inference and judging overhead and must not beat plain.
"""
import os

import numpy as np
import pytest

import paper_2609_16424_amd as ilh

pytestmark = pytest.mark.gpu


def _eval(path, seeds, steps):
    L = ilh.learned
    z = np.load(path)
    scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
    opts = L.model_newton_options(z)
    state = {k: z[k] for k in ("widths", "master", "mu", "sd", "osc")}
    return L.evaluate(112, 48, 3, seeds, steps, float(z["cfl_factor"]), opts, state, scales)


@pytest.mark.skipif(not os.path.exists(ilh.learned.MODEL_4X), reason="no trained model committed")
def test_trained_guess_reduces_newton_iterations_4x():
    res = _eval(ilh.learned.MODEL_4X, [1003, 1007], 12)
    plain, learned, zero = res["plain"], res["learned"], res["zero"]
    assert plain["steps"] == learned["steps"] == 12 * 2
    assert learned["newton_per_step"] < plain["newton_per_step"] - 0.5
    assert learned["median_initial_residual_ratio"] < 0.5 * plain["median_initial_residual_ratio"]
    assert zero["newton_per_step"] >= plain["newton_per_step"] - 0.2


@pytest.mark.skipif(not os.path.exists(ilh.learned.DEFAULT_MODEL), reason="no trained model committed")
def test_trained_guess_8x():
    res = _eval(ilh.learned.DEFAULT_MODEL, [1003, 1007], 12)
    plain, learned, zero = res["plain"], res["learned"], res["zero"]
    assert learned["steps"] == 12 * 2
    assert learned["learned_used"] == learned["steps"]
    assert learned["newton_per_step"] <= plain["newton_per_step"]
    assert learned["median_initial_residual_ratio"] < 0.1 * plain["median_initial_residual_ratio"]
    assert zero["newton_per_step"] >= plain["newton_per_step"] - 0.2
