"""Curved initial meshes (node positions given per node) and boxes with faces that are not
walls, against the oracle on the same inputs.  These set-ups run on the generic element kernels,
which form det J0 and m_q per quadrature point; every operator of the stage solve is compared
entry by entry (per block, both the 2-norm ratio and the max-entry bound)."""
import numpy as np
import pytest
import torch

import paper_2609_16424_amd as ilh
import seeded_inputs as si
from gpu_common import blocks_close, maxrel, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

BOXES = {"tg2d": ((0, 0), (1, 1)), "tg3d": ((0, 0, 0), (1, 1, 1)), "triple": ((0, 0), (7, 3))}
CASES = [
    ("tg2d", (5, 4), 3, None, 0, 0.08),       # curved, walls everywhere, TG source
    ("tg2d", (4, 3), 2, None, 0b0110, 0.0),   # Cartesian, no walls on x = hi and y = lo
    ("triple", (7, 3), 3, "formula", 0b1000, 0.06),  # curved, viscosity, no wall on y = hi
    ("tg3d", (3, 2, 3), 2, "formula", 0b010001, 0.05),  # curved 3D, viscosity, two free faces
]


def _pair(problem, n, k, visc, free, amp):
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    from oracle.mesh import BoxMesh
    lo, hi = BOXES[problem]
    m = BoxMesh(len(n), n, lo, hi, k)
    x0 = si.curved_positions(m.x0, lo, hi, amp) if amp > 0 else None
    hc = 1.0 / k if problem == "triple" else None
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", h_coarse=hc)
    O = OHydro(problem, n, k, visc=vo, x0=x0, free_faces=free)
    G = ilh.Hydro(problem, n, k, visc=visc is not None, dscale_mode=visc or "const", h_coarse=hc or 0.0,
                  tg_source=O.use_source, x0=x0, free_faces=free)
    return O, G


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c[0] + "-" + str(c[4]) for c in CASES])
def pair(request):
    return _pair(*CASES[request.param])


def test_initial_state_and_masses(pair):
    O, G = pair
    u = to_np(G.init_state())
    uo = O.init_state()
    assert blocks_close(u, uo, O.nh1, 1e-12) <= 1.0
    b = si.block_direction(7, O.nh1, O.nl2)[2 * O.nh1:]
    assert maxrel(to_np(G.mass_e_inv(to_dev(b))), O.mass_e_inv(b)) <= 1e-12
    bv = si.zero_rows(si.block_direction(8, O.nh1, O.nl2)[:O.nh1], O.cons)
    xv, _, _ = G.mass_v_solve(to_dev(bv), rtol=1e-14, maxit=2000)
    assert maxrel(to_np(xv), O.mass_v_solve(bv)) <= 1e-11
    ke, ie = G.energy(to_dev(uo))
    keo, ieo = O.energy(uo)
    assert abs(ke - keo) <= 1e-12 * max(abs(keo), 1e-300) + 1e-300 and abs(ie - ieo) <= 1e-12 * abs(ieo)
    dt = G.dt_estimate(to_dev(uo), 0.5)
    assert abs(dt - O.dt_estimate(uo, 0.5)) <= 1e-12 * dt


def test_residual_and_jacobian_actions(pair):
    from oracle.krylov import jvp_cs
    O, G = pair
    u = si.perturb_state(O.init_state(), 21, O.nh1, 0.002, 0.05, 0.05)
    k = 0.1 * si.block_direction(22, O.nh1, O.nl2, 0.01, 1.0, 1.0)
    dk = si.block_direction(23, O.nh1, O.nl2, 0.01, 1.0, 1.0)
    tau = 0.5 * O.dt_estimate(u, 2.0)
    r = to_np(G.residual(to_dev(k), to_dev(u), tau))
    assert blocks_close(r, O.residual(k, u, tau), O.nh1, 1e-12) <= 1.0
    jo = jvp_cs(lambda q: O.residual(q, u, tau), k, dk)
    j64 = to_np(G.jvp(to_dev(k), to_dev(u), tau, to_dev(dk), 64))
    j32 = to_np(G.jvp(to_dev(k), to_dev(u), tau, to_dev(dk, torch.float32), 32))
    assert blocks_close(j64, jo, O.nh1, 1e-12) <= 1.0
    assert blocks_close(j32, jo, O.nh1, 1e-5) <= 1.0
    # the transpose action is built for the structured kernels only
    with pytest.raises(ilh.IlhError):
        G.vjp(to_dev(k), to_dev(u), tau, to_dev(dk), 64)


def test_curved_trajectory_matches_oracle():
    """Three implicit midpoint steps on the curved Taylor-Green mesh, FP32 Jacobian actions."""
    from oracle import krylov
    O, G = _pair("tg2d", (5, 4), 3, None, 0, 0.08)
    u0 = O.init_state()
    dt = 2.0 * O.dt_estimate(u0, 0.5)
    states, _, _ = krylov.run_midpoint(O, u0, dt, 3)
    u = to_dev(u0)
    hist = []
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32)
    for i in range(3):
        g = G.plain_guess(u, hist)
        kk, st = G.implicit_step(u, dt, guess=g, opts=opts)
        assert st["status"] == 0
        hist = (hist + [kk])[-2:]
        assert rel(to_np(u), states[i + 1]) <= 1e-8, (i, rel(to_np(u), states[i + 1]))
