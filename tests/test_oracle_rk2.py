"""Pins of the oracle's explicit RK2-average step (the RK2 reference of Sec. 4).

* total energy: with the averaged velocity in the full step the change of
  E = 1/2 v^T M_V v + 1^T M_E e is exactly zero without an energy source (walls, any state);
* second order in time (dt-halving self-convergence);
* the paper's Taylor-Green table, Q2Q1 + RK2 columns: the L1 velocity errors at the printed
  step counts (tests/golden/tg_table_rk2.txt).
"""
import os

import numpy as np
import pytest

import seeded_inputs as si
from oracle.hydro import Hydro, ViscosityOptions
from oracle.krylov import rk2avg_step

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tg_table_rk2.txt")


def _table():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        _, n, err, steps = line.split()
        rows.append((int(n), float(err), int(steps)))
    return rows


@pytest.mark.parametrize("name,n,k,visc", [("tg2d", (3, 3), 2, None), ("triple", (7, 3), 2, "formula"),
                                           ("triple", (4, 2), 3, "const")])
def test_rk2avg_conserves_total_energy(name, n, k, visc):
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=0.05)
    H = Hydro(name, n, k, visc=vo, source=False)
    h = float(np.min(H.mesh.h)) / k
    u = si.perturb_state(H.init_state(), 9, H.nh1, 0.02 * h, 0.3, 0.2)
    u[H.nh1:2 * H.nh1] = np.where(H.cons, 0.0, u[H.nh1:2 * H.nh1])  # walls hold v.n = 0
    e0 = sum(H.energy(u))
    u1 = rk2avg_step(H, u, 0.2 * H.dt_estimate(u, 0.5))
    assert abs(sum(H.energy(u1)) - e0) <= 1e-13 * abs(e0)
    assert np.linalg.norm(u1 - u) > 1e-6 * np.linalg.norm(u)  # the step did something


def test_rk2avg_second_order_in_time():
    H = Hydro("tg2d", (3, 3), 2)
    u0 = H.init_state()

    def run(m):
        u = u0.copy()
        for _ in range(m):
            u = rk2avg_step(H, u, 0.1 / m)
        return u

    ref = run(64)
    e1 = np.linalg.norm(run(8) - ref)
    e2 = np.linalg.norm(run(16) - ref)
    assert 3.5 < e1 / e2 < 4.6


@pytest.mark.parametrize("n", [4, 8])
def test_tg_l1_error_matches_paper_rk2_column(n):
    row = [r for r in _table() if r[0] == n][0]
    _, err_ref, steps = row
    H = Hydro("tg2d", (n, n), 2)
    u = H.init_state()
    for _ in range(steps):
        u = rk2avg_step(H, u, 0.5 / steps)
    assert abs(H.l1_velocity_error(u) / err_ref - 1.0) <= 0.02
