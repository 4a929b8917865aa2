"""Parity at the benchmark configurations' full sizes, in the launch configuration that
bench.py times (linearize + FP32 Jacobian action through the register-resident kernel).

C2 (2D TG 128x128 Q3Q2) and C4 (triple point 112x48 Q3Q2, viscosity) are compared with the
oracle directly.  C3 (3D TG 32^3 Q2Q1 on a displaced mesh) is checked on sampled outputs the
oracle evaluates element by element, against central finite differences of FP64 residuals
(eps = 1e-7, seeded random directions), and through identities that hold at any size.
"""
import numpy as np
import pytest
import torch

import paper_2609_16424_amd as ilh
import seeded_inputs as si
from gpu_common import close, elements_of_dof, jvp_local, rel, to_dev, to_np, random_state, random_dir

pytestmark = pytest.mark.gpu


def _pair(problem, n, k, visc=None, **kw):
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", h_coarse=kw.pop("h_coarse", None))
    O = OHydro(problem, n, k, visc=vo)
    G = ilh.Hydro(problem, n, k, visc=visc is not None, dscale_mode=visc or "const",
                  h_coarse=vo.h_coarse or 0.0, tg_source=O.use_source)
    return O, G


@pytest.mark.parametrize("case", ["C2", "C4"])
def test_full_size_residual_and_jvp(case):
    from oracle.krylov import jvp_cs
    if case == "C2":
        O, G = _pair("tg2d", (128, 128), 3)
    else:
        O, G = _pair("triple", (112, 48), 3, visc="formula", h_coarse=1.0 / 3.0)
    u0 = O.init_state()
    h = 1.0 / (O.k * max(O.mesh.n))
    u = si.perturb_state(u0, 11, O.nh1, 0.05 * h, 0.05, 0.02)
    tau = 0.5 * O.dt_estimate(u, 2.0)
    k = si.block_direction(12, O.nh1, O.nl2, 0.1 * h, 0.1, 0.1)
    dk = si.block_direction(13, O.nh1, O.nl2, h, 1.0, 1.0)
    r = to_np(G.residual(to_dev(k), to_dev(u), tau))
    assert close(r, O.residual(k, u, tau), 1e-12, O.nh1)
    jo = jvp_cs(lambda q: O.residual(q, u, tau), k, dk)
    G.linearize(to_dev(k), to_dev(u), tau)
    j32 = to_np(G.jvp_lin(to_dev(dk, torch.float32), 32))
    j64 = to_np(G.jvp_lin(to_dev(dk), 64))
    assert close(j32, jo, 1e-5, O.nh1), rel(j32, jo)
    assert close(j64, jo, 1e-12, O.nh1), rel(j64, jo)


@pytest.fixture(scope="module", params=[None, "formula"])
def c3(request):
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    visc = request.param
    vo = ViscosityOptions(on=visc is not None, mode="formula")
    O = OHydro("tg3d", (32, 32, 32), 2, visc=vo)
    G = ilh.Hydro("tg3d", (32, 32, 32), 2, visc=visc is not None, dscale_mode="formula")
    u0 = O.init_state()
    w = si.displace_positions(u0, O.nh1, 0.05)  # x = x0 + 0.05 v_TG(x0)
    return O, G, w


def test_c3_sampled_outputs_match_oracle(c3):
    O, G, w = c3
    f1, ftv = G.force(to_dev(w))
    f1, ftv = to_np(f1), to_np(ftv)
    rng = np.random.default_rng(0)
    m = O.mesh
    els = np.sort(rng.choice(m.Ne, 40, replace=False))
    _, otv = O.force(w, elements=els)
    assert close(ftv.reshape(m.Ne, -1)[els], otv, 1e-12)
    # F 1 at sampled nodes: evaluate exactly the elements that contain them
    nodes = rng.choice(m.N, 12, replace=False)
    adj = np.unique(np.nonzero(np.isin(m.conn, nodes))[0])
    of1, _ = O.force(w, elements=adj)
    idx = np.concatenate([c * m.N + nodes for c in range(3)])
    assert close(f1[idx], of1[idx], 1e-12)


@pytest.mark.parametrize("prec,tol", [(64, 1e-6), (32, 1e-5)])
def test_c3_jvp_matches_central_fd(c3, prec, tol):
    O, G, w = c3
    dev = to_dev(w)
    tau = 0.5 * G.dt_estimate(dev, 8.0)
    h = 1.0 / 64
    for seed in range(3):
        dk = si.block_direction(100 + seed, O.nh1, O.nl2, sx=h, sv=0.1, se=0.1)
        dk = si.zero_rows(dk, np.concatenate([np.zeros(O.nh1, bool), O.mesh.constrained.ravel(),
                                              np.zeros(O.nl2, bool)]))
        k = torch.zeros_like(dev)
        eps = 1e-7
        dkd = to_dev(dk)
        rp = G.residual(k + eps * dkd, dev, tau)
        rm = G.residual(k - eps * dkd, dev, tau)
        fd = to_np((rp - rm) / (2 * eps))
        dt = torch.float64 if prec == 64 else torch.float32
        j = to_np(G.jvp(k, dev, tau, to_dev(dk, dt), prec))
        assert rel(j, fd) <= tol, (seed, rel(j, fd))


def test_c3_identities(c3):
    O, G, w = c3
    f1, ftv = G.force(to_dev(w))
    f1 = to_np(f1).reshape(3, -1)
    v = w[O.nh1:2 * O.nh1]
    assert np.abs(f1.sum(1)).max() <= 1e-12 * np.abs(f1).sum()
    assert abs(v @ f1.ravel() - to_np(ftv).sum()) <= 1e-12 * np.abs(v * f1.ravel()).sum()


def test_autograd_forward_mode_matches_fd():
    """ForceFn.jvp (hand-written tangent) against central differences of the forward."""
    O, G = _pair("tg3d", (6, 5, 4), 2)
    w = si.displace_positions(O.init_state(), O.nh1, 0.05)
    dw = si.block_direction(5, O.nh1, O.nl2, 1 / 12, 0.1, 0.1)
    wd, dwd = to_dev(w), to_dev(dw)
    (f1, ftv), (df1, dftv) = torch.func.jvp(lambda x: ilh.ForceFn.apply(G, x), (wd,), (dwd,))
    eps = 1e-7
    p1, ptv = G.force(wd + eps * dwd)
    m1, mtv = G.force(wd - eps * dwd)
    assert rel(to_np(df1), to_np((p1 - m1) / (2 * eps))) <= 1e-6
    assert rel(to_np(dftv), to_np((ptv - mtv) / (2 * eps))) <= 1e-6


def test_autograd_dual_residual_matches_oracle():
    """ResidualFn under torch.autograd.forward_ad equals the oracle's complex-step J dk."""
    O, G = _pair("tg2d", (7, 5), 3)
    from oracle.krylov import jvp_cs
    u, k, dk = random_state(O, 11), 0.1 * random_dir(O, 12), random_dir(O, 13)
    tau = 2e-3
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        kd = fwAD.make_dual(to_dev(k), to_dev(dk))
        r = ilh.ResidualFn.apply(G, kd, to_dev(u), tau)
        val, tan = fwAD.unpack_dual(r)
    assert close(to_np(val), O.residual(k, u, tau), 1e-12)
    assert close(to_np(tan), jvp_cs(lambda q: O.residual(q, u, tau), k, dk), 1e-12)


def _sample_dofs(O, seed, strip_cols):
    """Seeded block degrees of freedom: x and v components at random nodes, at nodes on the
    columns where two strips of the lane map meet, on the walls, and energy dofs."""
    rng = np.random.default_rng(seed)
    m, nh1 = O.mesh, O.nh1
    nodes = list(rng.choice(m.N, 10, replace=False))
    J = rng.integers(1, m.ng[1] - 1, len(strip_cols))
    nodes += [int(I + m.ng[0] * j) for I, j in zip(strip_cols, J)]   # strip seams
    nodes += [0, m.ng[0] - 1, int(m.ng[0] * (m.ng[1] // 2))]          # corners, a wall node
    dofs = []
    for nd in nodes:
        c = int(rng.integers(0, O.dim))
        dofs += [c * m.N + nd, nh1 + c * m.N + nd]
    dofs += list(2 * nh1 + rng.choice(O.nl2, 8, replace=False))
    return np.array(sorted(set(int(d) for d in dofs)))


def test_c2_transpose_action_sampled_entries():
    """C2 (2D TG 128x128 Q3Q2) transpose action J^T y at full size, entry by entry at sampled
    degrees of freedom: (J^T y)_j = <y, J e_j>, the column J e_j from the oracle's complex step
    over the elements that hold j (exact: no other row depends on k_j)."""
    O, G = _pair("tg2d", (128, 128), 3)
    u0 = O.init_state()
    h = 1.0 / (O.k * 128)
    u = si.perturb_state(u0, 11, O.nh1, 0.05 * h, 0.05, 0.02)
    tau = 0.5 * O.dt_estimate(u, 2.0)
    k = si.block_direction(12, O.nh1, O.nl2, 0.1 * h, 0.1, 0.1)
    y = si.block_direction(14, O.nh1, O.nl2, 1.0, 1.0, 1.0)
    G.linearize(to_dev(k), to_dev(u), tau)
    g64 = to_np(G.vjp_lin(to_dev(y), 64))
    g32 = to_np(G.vjp_lin(to_dev(y, torch.float32), 32))
    dofs = _sample_dofs(O, 15, strip_cols=[30, 60, 90, 120, 300, 330])  # 10 elements (30 nodes) per strip
    ref = np.empty(len(dofs))
    for i, j in enumerate(dofs):
        ej = np.zeros(O.nblock)
        ej[j] = 1.0
        ref[i] = float(y @ jvp_local(O, k, u, tau, ej, elements_of_dof(O, j)))
    assert close(g64[dofs], ref, 1e-12), np.abs(g64[dofs] - ref).max() / np.abs(ref).max()
    assert close(g32[dofs], ref, 1e-5), np.abs(g32[dofs] - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 1e-5)])
def test_c3_jvp_sampled_rows_match_oracle(c3, prec, tol):
    """C3 (3D TG 32^3 Q2Q1, displaced mesh) Jacobian action at full size against the oracle's
    complex step at sampled rows (the force over the elements reaching those rows only)."""
    O, G, w = c3
    dev = to_dev(w)
    tau = 0.5 * G.dt_estimate(dev, 8.0)
    k = np.zeros(O.nblock)
    dk = si.block_direction(100, O.nh1, O.nl2, sx=1.0 / 64, sv=0.1, se=0.1)
    dt = torch.float64 if prec == 64 else torch.float32
    j = to_np(G.jvp(to_dev(k), dev, tau, to_dev(dk, dt), prec))
    rng = np.random.default_rng(101)
    m = O.mesh
    nodes = list(rng.choice(m.N, 12, replace=False)) + [int(8 + m.ng[0] * (5 + m.ng[1] * 7))]  # a strip seam
    rows = []
    for nd in nodes:
        for c in range(3):
            rows += [c * m.N + nd, O.nh1 + c * m.N + nd]
    rows += list(2 * O.nh1 + rng.choice(O.nl2, 10, replace=False))
    rows = np.array(sorted(set(int(r) for r in rows)))
    adj = np.unique(np.concatenate([elements_of_dof(O, r) for r in rows]))
    ref = jvp_local(O, k, w, tau, dk, adj)[rows]
    assert close(j[rows], ref, tol), np.abs(j[rows] - ref).max() / np.abs(ref).max()
