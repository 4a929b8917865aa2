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
    # over matched steps the learned iterate saves Krylov work against both plain iterates (the
    # bench leg measures 1.37x / 1.26x in s/step over 5 seeds x 30 steps)
    for other in ("plain", "plain_fallback"):
        m = res["learned_vs_" + other]
        assert m["matched_steps"] == 24
        assert m["gmres_learned"] < 0.9 * m["gmres_" + other], (other, m)


@pytest.mark.skipif(not os.path.exists(ilh.learned.DEFAULT_MODEL), reason="no trained model committed")
def test_trained_guess_8x():
    """At 8x the learned iterate is used at every step and carries the run through every step (on
    this held-out seed the plain run fails after step 21 with Newton not converging, and the
    plain iterate with the previous-rate fallback earlier still)."""
    res = _eval(ilh.learned.DEFAULT_MODEL, [1003], 24)
    plain, learned, zero = res["plain"], res["learned"], res["zero"]
    assert learned["steps"] == 24
    assert learned["steps"] >= plain["steps"] and learned["steps"] >= res["plain_fallback"]["steps"]
    assert learned["learned_used"] == learned["steps"]
    assert zero["steps"] <= learned["steps"]
    # over the steps both complete, the learned iterate needs no more Newton iterations than the
    # plain one (its s/step there is about plain's: the bench leg measures 0.92x over 129 matched
    # steps at 8x, so at this step size its gain is that it keeps every held-out run going)
    m = res["learned_vs_plain"]
    assert m["newton_learned"] <= m["newton_plain"] + 0.2, m


@pytest.mark.skipif(not os.path.exists(ilh.learned.DEFAULT_MODEL), reason="no trained model committed")
def test_fused_guess_infer_matches_composed_calls():
    """ilh_guess_infer (features, MLP, assembly, judge in one call) equals the same steps called
    one by one, on a triple-point state a few steps in."""
    import torch
    L = ilh.learned
    z = np.load(L.DEFAULT_MODEL)
    scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
    h = L.make_triple(112, 48, 3, seed=1001)
    u = h.init_state()
    dt = float(z["cfl_factor"]) * h.dt_estimate(u, 0.5)
    opts = L.model_newton_options(z)
    hist = []
    for _ in range(3):
        k, _ = h.implicit_step(u, dt, guess=h.plain_guess(u, hist, 0.5 * dt), opts=opts)
        hist = (hist + [k])[-2:]
    mlp = L.GuessMLP(h, [int(w) for w in z["widths"]])
    mlp.load_state({k: z[k] for k in ("widths", "master")})
    lg = L.LearnedGuess(h, mlp, scales, norm={k: z[k] for k in ("mu", "sd", "osc")})
    tau = 0.5 * dt
    kf, used = lg.guess(u, hist, tau)
    base = h.plain_guess(u, hist, tau)
    kl = lg.predict(u, base, tau)
    nl = float(torch.linalg.norm(h.residual(kl, u, tau)))
    nb = float(torch.linalg.norm(h.residual(base, u, tau)))
    expect_learned = np.isfinite(nl) and (nl < nb or not np.isfinite(nb))
    assert used == expect_learned
    ref = kl if expect_learned else base
    assert float(torch.linalg.norm(kf - ref)) <= 1e-12 * float(torch.linalg.norm(ref))
