"""What the trained learned guess gains over the method without it (held-out seeds).

The committed model was trained on perturbation seeds 0..199; seeds 1000+ are held out.
Both runs converge every stage to ||R|| <= 1e-10 ||R(0)||; the learned run must need fewer
Newton iterations and start from a smaller residual.  The zero-output control carries the
same inference and judging overhead and must not beat plain.
"""
import os

import numpy as np
import pytest

import paper_2609_16424_amd as ilh

pytestmark = pytest.mark.gpu


@pytest.mark.skipif(not os.path.exists(ilh.learned.DEFAULT_MODEL), reason="no trained model committed")
def test_trained_guess_reduces_newton_iterations():
    L = ilh.learned
    z = np.load(L.DEFAULT_MODEL)
    scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=30, gmres_maxit=150)
    state = {k: z[k] for k in ("widths", "master", "mu", "sd", "osc")}
    res = L.evaluate(112, 48, 3, [1003, 1007], 12, float(z["cfl_factor"]), opts, state, scales)
    plain, learned, zero = res["plain"], res["learned"], res["zero"]
    assert plain["steps"] == learned["steps"] == 12 * 2
    assert learned["newton_per_step"] < plain["newton_per_step"] - 0.5
    assert learned["median_initial_residual_ratio"] < 0.5 * plain["median_initial_residual_ratio"]
    assert zero["newton_per_step"] >= plain["newton_per_step"] - 0.2
