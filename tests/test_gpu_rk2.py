"""GPU explicit RK2-average step (the RK2 reference of Sec. 4) against the oracle, the paper's
Taylor-Green RK2 column, and exact energy conservation on the Sedov blast (Sec. 4.2)."""
import os

import numpy as np
import pytest
import torch

from gpu_common import make_pair, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tg_table_rk2.txt")


def _sedov_pair(n, k):
    import paper_2609_16424_amd as ilh
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    O = OHydro("sedov", (n, n), k, visc=ViscosityOptions(on=True, mode="formula", h_coarse=1.0 / k))
    return O, ilh.make_sedov(n, k)


@pytest.mark.parametrize("case", ["tg2d", "triple", "sedov"])
def test_rk2avg_matches_oracle(case):
    from oracle.krylov import rk2avg_step
    if case == "tg2d":
        O, G = make_pair("tg2d", (5, 4), 2)
    elif case == "triple":
        O, G = make_pair("triple", (7, 3), 3, "formula")
    else:
        O, G = _sedov_pair(6, 2)
    u = O.init_state()
    ug = to_dev(u)
    for _ in range(3):
        dt = 0.3 * O.dt_estimate(u, 1.0)
        u = rk2avg_step(O, u, dt)
        G.rk2avg_step(ug, dt)
        assert rel(to_np(ug), u) <= 1e-11


@pytest.mark.parametrize("n", [4, 8])
def test_rk2_tg_table_on_gpu(n):
    """The table's 4x4 and 8x8 rows at their printed step counts.  The 16x16 and 32x32 rows are
    not reproducible with equal steps and no damping: RK2's amplification factor exceeds 1 on
    the imaginary axis, and the inviscid run grows high-frequency modes over 135 steps (the
    oracle does the same)."""
    import paper_2609_16424_amd as ilh
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    err_ref, steps = [(float(r[2]), int(r[3])) for r in rows if int(r[1]) == n][0]
    H = ilh.Hydro("tg2d", (n, n), 2)
    u = H.init_state()
    for _ in range(steps):
        H.rk2avg_step(u, 0.5 / steps)
    assert abs(H.l1_error(u) / err_ref - 1.0) <= 0.02


def test_rk2_sedov_energy_conserved():
    import paper_2609_16424_amd as ilh
    H = ilh.make_sedov(16, 2)
    u = H.init_state()
    e0 = sum(H.energy(u))
    for _ in range(60):
        H.rk2avg_step(u, 0.5 * H.dt_estimate(u, 1.0))
    ke, ie = H.energy(u)
    assert abs(ke + ie - e0) <= 1e-12 * e0
    assert ke > 1e-3  # the blast has started to move


def test_rk2_rejected_in_3d():
    from paper_2609_16424_amd import IlhError
    O, G = make_pair("tg3d", (2, 2, 2), 2)
    with pytest.raises(IlhError):
        G.rk2avg_step(to_dev(O.init_state()), 0.01)
