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


@pytest.mark.parametrize("n", [(2, 2, 2), (5, 3, 2)])
def test_3d_trajectory_matches_oracle(n):
    """3D Taylor-Green Q2Q1: implicit midpoint steps with the 3D strip residual, whose det J of
    the stage positions feeds the line search, match the oracle's (one and two partial strips)."""
    from oracle import krylov
    O, G = make_pair("tg3d", n, 2)
    u0 = O.init_state()
    states, _, _ = krylov.run_midpoint(O, u0, 0.01, 2)
    u = to_dev(u0)
    hist = []
    opts = ilh.newton_options(tol=1e-10, jvp_prec=64)
    for i in range(2):
        g = G.plain_guess(u, hist)
        k, st = G.implicit_step(u, 0.01, guess=g, opts=opts)
        assert st["status"] == 0 and st["halvings"] == 0
        hist = (hist + [k])[-2:]
        assert rel(to_np(u), states[i + 1]) <= 1e-8, (i, rel(to_np(u), states[i + 1]))


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


def test_line_search_tangling_decision_matches_oracle():
    """At dt = 2 on the 4x4 Q2 Taylor-Green mesh the full first Newton step of the oracle tangles
    the stage mesh (no halving allowed: ETANGLED) and halving lets it go on.  The GPU line search,
    whose det J comes out of the strip residual kernel, takes the same decisions: ETANGLED
    without halvings, and at least one halving in its first iteration with them."""
    from oracle import krylov
    O, G = make_pair("tg2d", (4, 4), 2)
    u0 = O.init_state()
    with pytest.raises(krylov.NewtonFailure) as e:
        krylov.implicit_midpoint_step(O, u0, 2.0, np.zeros_like(u0), krylov.NewtonOptions(max_halvings=0))
    assert e.value.kind == "ETANGLED"
    dmid = O.min_detj(u0)  # the initial mesh is untangled
    assert dmid > 0.0
    u = to_dev(u0)
    opts = ilh.newton_options(tol=1e-10, max_halvings=0, ls_residual=0)
    k, st = G.implicit_step(u.clone(), 2.0, opts=opts, raise_on_fail=False)
    assert st["status"] == ilh._lib.ILH_ETANGLED
    assert st["newton"] == 0
    opts = ilh.newton_options(tol=1e-10, max_halvings=10, max_newton=1, ls_residual=0)
    k, st = G.implicit_step(u.clone(), 2.0, opts=opts, raise_on_fail=False)
    assert st["status"] == ilh._lib.ILH_ENOCONV  # one Newton iteration allowed, taken with a halving
    assert st["newton"] == 1 and st["halvings"] >= 1


@pytest.mark.parametrize("cgs2", [1, 0])
def test_speculative_arnoldi_step_does_no_counted_work(cgs2):
    """The host enqueues an Arnoldi step before it reads the residual estimate of the column before;
    the step after the one that ends a solve reads that step's end flag on the device and returns
    at once.  With cycles that never restart, the Jacobian actions counted are then exactly the
    GMRES iterations with both passes in the step (cgs2 = 1), and one more per solve with the
    second pass lagged (the step that finishes the last column applies J to the next vector), and
    the trajectory still matches the oracle's."""
    from oracle import krylov
    O, G = make_pair("tg2d", (8, 8), 2)
    u0 = O.init_state()
    states, _, _ = krylov.run_midpoint(O, u0, 0.01, 3)
    u = to_dev(u0)
    hist = []
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32, restart=64, cgs2=cgs2)
    for n in range(3):
        g = G.plain_guess(u, hist)
        k, st = G.implicit_step(u, 0.01, guess=g, opts=opts)
        assert st["status"] == 0
        assert st["jvp_calls"] == st["gmres"] + (0 if cgs2 else st["newton"]), st
        hist = (hist + [k])[-2:]
        assert rel(to_np(u), states[n + 1]) <= 1e-8


@pytest.mark.parametrize("cgs2", [1, 0])
def test_iteration_limit_enqueues_no_extra_step(cgs2):
    """When the iteration limit (not convergence) ends every FGMRES solve, the host knows in advance
    which step is the last one and enqueues none after it (with the second pass lagged, a closing
    step that finishes the last column without a Jacobian action): the Jacobian actions counted
    equal the GMRES iterations (restart 64: no restart actions), for both precisions of the action."""
    O, G = make_pair("tg2d", (8, 8), 2)
    u = to_dev(O.init_state())
    for prec in (32, 64):
        opts = ilh.newton_options(tol=1e-10, jvp_prec=prec, restart=64, gmres_maxit=3, gmres_rtol=1e-14,
                                  max_newton=8, cgs2=cgs2)
        k, st = G.implicit_step(u.clone(), 0.01, opts=opts, raise_on_fail=False)
        assert st["newton"] >= 2
        assert st["gmres"] >= 6 and st["gmres"] % 3 == 0, st
        assert st["jvp_calls"] == st["gmres"], st


def test_graph_replay_with_changing_dt():
    """Graph replay (graphs = 1) against the kernel-by-kernel path when the time step grows from step
    to step, so that later solves need more Arnoldi steps than the first one and capture new steps
    in later cycles: the captured actions read tau from the device, so the trajectories agree."""
    states, gm = {}, {}
    for graphs in (0, 1):
        G = ilh.Hydro("tg2d", (24, 20), 3)
        u = G.init_state()
        dt0 = G.dt_estimate(u, 0.5)
        opts = ilh.newton_options(graphs=graphs, tol=1e-10, jvp_prec=32)
        hist, traj, its = [], [], []
        for n in range(5):
            dt = (1.0 + 1.5 * n) * dt0
            g = G.plain_guess(u, hist, 0.5 * dt)
            k, st = G.implicit_step(u, dt, guess=g, opts=opts)
            assert st["status"] == 0
            hist = (hist + [k])[-2:]
            traj.append(to_np(u))
            its.append(st["gmres"] / max(1, st["newton"]))
        states[graphs], gm[graphs] = traj, its
    assert max(gm[1][1:]) > gm[1][0]  # later solves took longer Krylov cycles
    for a, b in zip(states[0], states[1]):
        assert rel(a, b) <= 1e-9


@pytest.mark.parametrize("case", ["tg2d", "triple"])
def test_graph_replay_matches_eager_launches(case):
    """Arnoldi steps replayed as captured HIP graphs give the trajectory of the kernel-by-kernel
    path (graphs = 0) over many steps, each graph replayed many times with eager work between."""
    if case == "tg2d":
        mk = lambda: ilh.Hydro("tg2d", (24, 20), 3)
        opts_kw = dict(tol=1e-10, jvp_prec=32)
        fac = 4.0
    else:
        from paper_2609_16424_amd import learned as L
        mk = lambda: L.make_triple(28, 12, 3)
        opts_kw = dict(tol=1e-10, jvp_prec=32, prec_probe=2, prec_lag=1)
        fac = 2.0
    states = {}
    for graphs in (0, 1):
        G = mk()
        u = G.init_state()
        dt = fac * G.dt_estimate(u, 0.5)
        opts = ilh.newton_options(graphs=graphs, **opts_kw)
        hist, traj = [], []
        for _ in range(6):
            g = G.plain_guess(u, hist, 0.5 * dt)
            k, st = G.implicit_step(u, dt, guess=g, opts=opts)
            assert st["status"] == 0
            hist = (hist + [k])[-2:]
            traj.append(to_np(u))
        states[graphs] = traj
    for a, b in zip(states[0], states[1]):
        assert rel(a, b) <= 1e-9


@pytest.mark.parametrize("restart,graphs", [(3, 0), (1, 0), (3, 1)])
def test_short_restart_cycles_match_oracle(restart, graphs):
    """FGMRES restarted every `restart` Arnoldi steps (many cycles per Newton iteration, each
    with its own residual-estimate tag) reaches the oracle's trajectory to the Newton tolerance."""
    from oracle import krylov
    O, G = make_pair("tg2d", (8, 8), 2)
    u0 = O.init_state()
    states, _, _ = krylov.run_midpoint(O, u0, 0.01, 4)
    u = to_dev(u0)
    hist = []
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32, restart=restart, gmres_maxit=400, graphs=graphs)
    for n in range(4):
        g = G.plain_guess(u, hist)
        k, st = G.implicit_step(u, 0.01, guess=g, opts=opts)
        assert st["status"] == 0 and st["res_final"] <= 1e-10 * st["res0"]
        assert st["gmres"] > restart  # more than one cycle per step
        hist = (hist + [k])[-2:]
        assert rel(to_np(u), states[n + 1]) <= 1e-8, (n, rel(to_np(u), states[n + 1]))
