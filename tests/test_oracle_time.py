"""Pins of the oracle's implicit midpoint step and of the whole scheme (CPU only).

* the exact energy identity of implicit midpoint, derived from eqs. (v_semi), (e_semi):
  E(u+) - E(u) = dt (w_v^T R_v + 1^T R_e + 1^T b) for any stage iterate k;
* second order in time (dt-halving self-convergence);
* the paper's Taylor-Green table: step counts of the explicit estimate and L1 errors
  (tests/golden/tg_table_q2q1_sd2.txt).
"""
import math
import os

import numpy as np
import pytest

from oracle import krylov
from oracle.hydro import Hydro, ViscosityOptions

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tg_table_q2q1_sd2.txt")


def _table():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        h, n, cfl, err, steps = line.split()
        rows.append((int(n), float(cfl), float(err), int(steps)))
    return rows


def _run_to(H, tf, cfl):
    u = H.init_state()
    dt0 = H.dt_estimate(u, cfl)
    t, hist, steps = 0.0, [], 0
    while t < tf - 1e-12:
        dt = min(dt0, tf - t)
        g = krylov.plain_guess(H, u, hist)
        u, k = krylov.implicit_midpoint_step(H, u, dt, g)
        hist.append(k)
        t += dt
        steps += 1
    return u, steps


@pytest.mark.parametrize("visc", [False, True])
def test_midpoint_energy_identity(visc):
    """dE = dt [sum_{free} w_v R_v + sum_{constrained} w_v (M_V k_v + F 1) + 1^T R_e + 1^T b].

    Follows from u+ = u + dt k, w = (u + u+)/2, the residual definition and the force
    transpose identity v^T (F 1) = 1^T (F^T v); it holds for any iterate k.
    """
    H = Hydro("tg2d", (8, 8), 2) if not visc else Hydro("triple", (14, 6), 2,
                                                          visc=ViscosityOptions(on=True))
    u = H.init_state()
    dt = 0.01
    rng = np.random.default_rng(0)
    cons = H.cons
    for it in range(2):
        g = krylov.plain_guess(H, u, [])
        st = {}
        un, k = krylov.implicit_midpoint_step(H, u, dt, g, None, st)
        assert st["hist"][-1] <= 1e-10
        for kk in (k, k + 1e-3 * rng.standard_normal(k.size)):
            w = u + 0.5 * dt * kk
            r = H.residual(kk, u, 0.5 * dt)
            _, rv, re = H.split(r)
            wx, wv, _ = H.split(w)
            F1, _ = H.force(w)
            Mk = H.mass_v(H.split(kk)[1])
            dE = sum(H.energy(u + dt * kk)) - sum(H.energy(u))
            pred = dt * (wv[~cons] @ rv[~cons] + wv[cons] @ (Mk[cons] + F1[cons])
                         + re.sum() + H.energy_source(wx).sum())
            assert abs(dE - pred) <= 1e-13 * sum(H.energy(u)), (dE, pred)
        u = un


def test_midpoint_second_order_in_time():
    H = Hydro("tg2d", (3, 3), 2)
    u0 = H.init_state()
    finals = []
    for steps in (2, 4, 8):
        states, _, _ = krylov.run_midpoint(H, u0, 0.1 / steps, steps)
        finals.append(states[-1])
    e1 = np.linalg.norm(finals[0] - finals[1])
    e2 = np.linalg.norm(finals[1] - finals[2])
    assert 3.6 < e1 / e2 < 4.4, e1 / e2


def test_tg_step_counts_from_explicit_estimate():
    """The paper's step counts at FS-CFL 0.5 and 8 equal ceil(t_f / dt_est) on an n x n mesh."""
    for n, cfl, err, steps in _table():
        H = Hydro("tg2d", (n, n), 2)
        pred = math.ceil(0.5 / H.dt_estimate(H.init_state(), cfl) - 1e-9)
        if cfl == 2.0:
            assert abs(pred - steps) <= 1  # the paper's run may enlarge dt by 5 % per step
        else:
            assert pred == steps, (n, cfl, pred, steps)


@pytest.mark.parametrize("n,cfl,tol", [(4, 0.5, 0.01), (4, 2.0, 0.02), (8, 0.5, 0.01), (8, 2.0, 0.02)])
def test_tg_l1_error_matches_paper_table(n, cfl, tol):
    ref = [r for r in _table() if r[0] == n and r[1] == cfl][0]
    H = Hydro("tg2d", (n, n), 2)
    u, steps = _run_to(H, 0.5, cfl)
    assert steps == ref[3]
    err = H.l1_velocity_error(u)
    assert abs(err - ref[2]) <= tol * ref[2], (err, ref[2])
