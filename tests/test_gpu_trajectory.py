"""Multi-step parity: implicit midpoint trajectories on the GPU against the oracle.

Newton solutions are unique only up to the nonlinear tolerance, so states are compared
with a bound proportional to it (1e-10 relative residual -> 1e-8 relative state).
"""
import numpy as np
import pytest
import torch

import paper_2609_16424_amd as ilh
from gpu_common import make_pair, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [64, 32])
def test_c1_trajectory_matches_oracle(prec):
    from oracle import krylov
    O, G = make_pair("tg2d", (8, 8), 2)
    u0 = O.init_state()
    states, _, ostats = krylov.run_midpoint(O, u0, 0.01, 10)
    u = to_dev(u0)
    hist = []
    opts = ilh.newton_options(tol=1e-10, jvp_prec=prec)
    for n in range(10):
        g = G.plain_guess(u, hist)
        k, st = G.implicit_step(u, 0.01, guess=g, opts=opts)
        assert st["status"] == 0 and st["res_final"] <= 1e-10 * st["res0"]
        hist = (hist + [k])[-2:]
        assert rel(to_np(u), states[n + 1]) <= 1e-8, (n, rel(to_np(u), states[n + 1]))
    # energy drift of the GPU run equals the oracle's (both are source-driven only)
    Eg = sum(G.energy(u))
    Eo = sum(O.energy(states[-1]))
    assert abs(Eg - Eo) <= 1e-10 * abs(Eo)


def test_stage_failure_paths():
    O, G = make_pair("tg2d", (4, 4), 2)
    u = to_dev(O.init_state())
    # Newton limited to zero iterations cannot converge from a zero guess
    opts = ilh.newton_options(tol=1e-10, max_newton=0)
    k, st = G.implicit_step(u.clone(), 0.01, opts=opts, raise_on_fail=False)
    assert st["status"] == ilh._lib.ILH_ENOCONV
    # a huge time step tangles the mesh: the line search gives up
    opts = ilh.newton_options(tol=1e-10, max_halvings=0, max_newton=5)
    uu = u.clone()
    k, st = G.implicit_step(uu, 50.0, opts=opts, raise_on_fail=False)
    assert st["status"] in (ilh._lib.ILH_ETANGLED, ilh._lib.ILH_ENOCONV)
    assert torch.equal(uu, u)  # state untouched on failure
