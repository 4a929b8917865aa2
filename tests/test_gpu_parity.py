"""GPU parity of every single-call entry point against the CPU oracle.

Inputs are seeded (seeded_inputs) perturbations of the oracle's initial state; each
output vector is compared with ||gpu - oracle|| / ||oracle|| against the bounds
1e-12 (FP64 kernels) and 1e-5 (FP32 Jacobian actions).  Meshes are chosen so that the
last work-group of every element kernel is partial (ragged tail).
"""
import numpy as np
import pytest
import torch

from gpu_common import close, make_pair, maxrel, random_dir, random_state, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [
    ("tg2d", (8, 8), 2, None),
    ("tg2d", (13, 11), 3, None),
    ("tg2d", (6, 5), 1, None),
    ("tg2d", (5, 4), 4, None),
    ("triple", (14, 6), 3, "const"),
    ("triple", (9, 5), 2, "formula"),
    ("tg3d", (5, 3, 4), 2, None),
    ("tg3d", (3, 2, 2), 2, "formula"),
    ("tg3d", (3, 3, 2), 1, None),
    ("tg3d", (2, 2, 1), 3, "const"),
]
IDS = ["%s-%s-k%d-%s" % (p, "x".join(map(str, n)), k, v) for p, n, k, v in CASES]

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def pair(request):
    p, n, k, v = request.param
    O, G = make_pair(p, n, k, v, width=0.05 if v == "const" else 1e-3)
    return O, G


def test_init_state(pair):
    O, G = pair
    u = to_np(G.init_state())
    uo = O.init_state()
    assert rel(u, uo) <= 1e-13
    # entry-wise at the FP64 bound: the projection of e0 goes through M_E^-1, whose Bernstein
    # blocks at k = 4 (3D: k = 3) are conditioned ~1e3, so single entries carry ~1e-13
    assert close(u, uo, 1e-12, O.nh1), maxrel(u, uo)


def test_force(pair):
    O, G = pair
    w = random_state(O, 1)
    f1, ftv = G.force(to_dev(w))
    o1, otv = O.force(w)
    assert close(to_np(f1), o1, FP64_TOL)
    assert close(to_np(ftv), otv, FP64_TOL)


def test_residual(pair):
    O, G = pair
    u = random_state(O, 2)
    k = 0.1 * random_dir(O, 3)
    tau = 0.003
    r = to_np(G.residual(to_dev(k), to_dev(u), tau))
    ro = O.residual(k, u, tau)
    assert close(r, ro, FP64_TOL, O.nh1)


@pytest.mark.parametrize("prec,tol", [(64, FP64_TOL), (32, FP32_TOL)])
def test_jvp(pair, prec, tol):
    from oracle.krylov import jvp_cs
    O, G = pair
    u = random_state(O, 4)
    k = 0.1 * random_dir(O, 5)
    dk = random_dir(O, 6)
    tau = 0.004
    dt = torch.float64 if prec == 64 else torch.float32
    j = to_np(G.jvp(to_dev(k), to_dev(u), tau, to_dev(dk, dt), prec))
    jo = jvp_cs(lambda q: O.residual(q, u, tau), k, dk)
    assert close(j, jo, tol, O.nh1), rel(j, jo)
    # block-wise too: the x, v and e rows separately
    for a, b in ((0, O.nh1), (O.nh1, 2 * O.nh1), (2 * O.nh1, O.nblock)):
        assert close(j[a:b], jo[a:b], 10 * tol)


@pytest.mark.parametrize("prec,tol", [(64, FP64_TOL), (32, FP32_TOL)])
def test_force_jvp(pair, prec, tol):
    from oracle.krylov import jvp_cs
    O, G = pair
    w = random_state(O, 7)
    dw = random_dir(O, 8)
    dt = torch.float64 if prec == 64 else torch.float32
    d1, dtv = G.force_jvp(to_dev(w), to_dev(dw, dt), prec)
    o1 = jvp_cs(lambda q: O.force(q)[0], w, dw)
    otv = jvp_cs(lambda q: O.force(q)[1], w, dw)
    assert close(to_np(d1), o1, tol)
    assert close(to_np(dtv), otv, tol)


def test_mass_operators(pair):
    O, G = pair
    rng = np.random.default_rng(9)
    x = rng.standard_normal(O.nh1)
    assert close(to_np(G.mass_v_apply(to_dev(x))), O.mass_v(x), 1e-13)
    e = rng.standard_normal(O.nl2)
    assert close(to_np(G.mass_e_inv(to_dev(e))), O.mass_e_inv(e), 1e-13)
    b = O.mass_v(x)
    sol, its, rr = G.mass_v_solve(to_dev(b), 1e-13, 1000)
    assert rr <= 1e-13
    assert close(to_np(sol), O.mass_v_solve(b), 1e-11)


def test_diagnostics(pair):
    O, G = pair
    u = random_state(O, 10, amp=0.01)
    du = to_dev(u)
    ke, ie = G.energy(du)
    ko, io = O.energy(u)
    assert abs(ke - ko) <= 1e-13 * abs(ko) and abs(ie - io) <= 1e-13 * abs(io)
    assert abs(G.min_detj(du) - O.min_detj(u)) <= 1e-13 * abs(O.min_detj(u))
    assert abs(G.dt_estimate(du, 0.5) - O.dt_estimate(u, 0.5)) <= 1e-12 * O.dt_estimate(u, 0.5)
    if O.prob.exact_v is not None:
        assert abs(G.l1_error(du) - O.l1_velocity_error(u)) <= 1e-12 * O.l1_velocity_error(u)


def test_rate(pair):
    O, G = pair
    u = random_state(O, 11, amp=0.01)
    f = to_np(G.rate(to_dev(u)))
    assert close(f, O.rate(u), 1e-11)


def test_zero_direction_gives_zero():
    O, G = make_pair("tg2d", (4, 3), 3)
    u = to_dev(O.init_state())
    k = torch.zeros_like(u)
    z = G.jvp(k, u, 0.01, torch.zeros_like(u), 64)
    assert float(z.abs().max()) == 0.0


@pytest.mark.parametrize("prec,tol", [(64, 1e-13), (32, 5e-6)])
@pytest.mark.parametrize("prob,n,k,visc", [("tg2d", (23, 7), 3, None), ("tg2d", (17, 4), 2, None),
                                           ("triple", (21, 9), 3, "const"), ("triple", (33, 5), 2, "formula"),
                                           ("tg2d", (12, 11), 3, "formula"), ("tg3d", (9, 5, 4), 2, None),
                                           ("tg3d", (6, 4, 3), 2, "formula")])
def test_jvp_variants_agree(prob, n, k, visc, prec, tol):
    """Linearised (0), generic (1) and register-resident recompute (2) Jacobian-action kernels
    (variant 2 is the generic kernel in 3D)."""
    O, G = make_pair(prob, n, k, visc)
    u = random_state(O, 21)
    kk = 0.1 * random_dir(O, 22)
    dk = random_dir(O, 23)
    dt = torch.float64 if prec == 64 else torch.float32
    G.linearize(to_dev(kk), to_dev(u), 0.003)
    out = []
    for v in (0, 1, 2):
        assert G.lib.ilh_set_kernel_variant(G.ctx, v) == 0
        out.append(to_np(G.jvp_lin(to_dev(dk, dt), prec)))
    G.lib.ilh_set_kernel_variant(G.ctx, 0)
    assert close(out[0], out[1], tol)
    assert close(out[2], out[1], tol)


@pytest.mark.parametrize("prob,n,k,visc", [("tg2d", (23, 7), 3, None), ("triple", (21, 9), 3, "const"),
                                           ("triple", (33, 5), 2, "formula"), ("tg2d", (12, 11), 3, "formula"),
                                           ("tg2d", (10, 1), 3, None)])
def test_apply_rows_match_oracle(prob, n, k, visc):
    """The linearised apply with one or two waves per strip (FP32) walking R element rows (partial
    last walk, partial last strip) against the oracle's complex-step Jacobian action, FP64 and
    FP32."""
    from oracle.krylov import jvp_cs
    O, G = make_pair(prob, n, k, visc)
    u = random_state(O, 51)
    kk = 0.1 * random_dir(O, 52)
    dk = random_dir(O, 53)
    tau = 0.003
    ref = jvp_cs(lambda q: O.residual(q, u, tau), kk, dk)
    G.linearize(to_dev(kk), to_dev(u), tau)
    for W in (1, 2):
        G.set_apply_waves(W)
        for R in (1, 2, 3, 4, 8):
            G.set_apply_rows(R)
            a64 = to_np(G.jvp_lin(to_dev(dk), 64))
            a32 = to_np(G.jvp_lin(to_dev(dk, torch.float32), 32))
            assert close(a64, ref, 1e-12), (W, R)
            assert close(a32, ref, 1e-5), (W, R)
    G.set_apply_rows(0)
    G.set_apply_waves(0)
    from paper_2609_16424_amd import IlhError
    with pytest.raises(IlhError):
        G.set_apply_rows(-1)
    for bad in (-1, 3):
        with pytest.raises(IlhError):
            G.set_apply_waves(bad)


def test_linearised_coefficients_follow_the_point():
    """Stored tangent coefficients are re-evaluated after each linearisation, per precision."""
    from oracle.krylov import jvp_cs
    O, G = make_pair("triple", (14, 6), 3, "formula")
    u = random_state(O, 31)
    dk = random_dir(O, 32)
    tau = 0.002
    ks = [0.1 * random_dir(O, 33), 0.1 * random_dir(O, 34)]
    for kk in ks + ks[:1]:
        G.linearize(to_dev(kk), to_dev(u), tau)
        a64 = to_np(G.jvp_lin(to_dev(dk), 64))
        a32 = to_np(G.jvp_lin(to_dev(dk, torch.float32), 32))
        b64 = to_np(G.jvp_lin(to_dev(dk), 64))
        ref = jvp_cs(lambda q: O.residual(q, u, tau), kk, dk)
        assert close(a64, ref, 1e-12)
        assert close(b64, a64, 1e-15)  # same coefficients; atomic summation order may differ
        assert close(a32, ref, 1e-5)


@pytest.mark.parametrize("n,k", [((130, 330), 3), ((64, 1040), 2)])
def test_linearised_large_mesh(n, k):
    """Linearised kernels on meshes of several thousand waves against the generic kernel, FP64
    and FP32, block by block, at a randomly perturbed state."""
    import paper_2609_16424_amd as ilh
    G = ilh.Hydro("tg2d", n, k)
    u = G.init_state()
    rng = np.random.default_rng(41)
    h = 1.0 / (k * max(n))
    pert = np.concatenate([0.03 * h * rng.standard_normal(G.nh1), 0.3 * rng.standard_normal(G.nh1),
                           0.2 * rng.standard_normal(G.nl2)])
    u = u + torch.from_numpy(pert).to(u.device)
    kk = torch.from_numpy(0.1 * np.concatenate([h * rng.standard_normal(G.nh1), rng.standard_normal(G.nh1 + G.nl2)])).to(u.device)
    dk = torch.from_numpy(np.concatenate([h * rng.standard_normal(G.nh1), rng.standard_normal(G.nh1 + G.nl2)])).to(u.device)
    G.linearize(kk, u, 0.002)
    # FP64 at the oracle-parity bound: the velocity rows sum element contributions with some
    # cancellation at this perturbation, so the two kernels' rounding differs by up to ~3e-13
    for prec, tol in ((64, 1e-12), (32, 5e-6)):
        d = dk if prec == 64 else dk.float()
        G.set_kernel_variant("generic")
        b = G.jvp_lin(d, prec).double()
        G.set_kernel_variant("lin")
        # by mesh size, then forced walks of 1, 4 and 8 element rows; one and two waves per strip
        for R, W in ((0, 0), (1, 1), (4, 1), (8, 1), (1, 2), (4, 2)):
            G.set_apply_rows(R)
            G.set_apply_waves(W)
            a = G.jvp_lin(d, prec).double()
            for lo, hi in ((0, G.nh1), (G.nh1, 2 * G.nh1), (2 * G.nh1, G.nblock)):
                err = float(torch.linalg.norm(a[lo:hi] - b[lo:hi]) / torch.linalg.norm(b[lo:hi]))
                assert err <= tol, (prec, R, W, lo, err)
        G.set_apply_rows(0)
        G.set_apply_waves(0)


@pytest.mark.parametrize("prob,n,k,visc", [("tg2d", (23, 7), 3, None), ("tg2d", (9, 1), 3, None),
                                           ("tg2d", (33, 5), 2, None), ("triple", (21, 9), 3, None),
                                           ("triple", (17, 4), 2, None), ("uniform", (12, 3), 3, None),
                                           ("tg2d", (1, 1), 3, None), ("tg2d", (2, 2), 2, None),
                                           ("uniform", (1, 5), 2, None), ("triple", (21, 9), 3, "formula"),
                                           ("triple", (13, 5), 2, "const"), ("tg3d", (5, 3, 4), 2, None),
                                           ("tg3d", (9, 2, 3), 2, "formula"), ("tg3d", (1, 1, 1), 2, None),
                                           ("tg3d", (4, 1, 2), 2, "const")])
def test_strip_residual_matches_oracle_and_generic(prob, n, k, visc):
    """The strip residual kernels (2D k = 2, 3; 3D Q2Q1) against the oracle and against the
    generic element kernel (kernel variant 1): partial strips, one-row meshes, per-element gamma
    and rho (triple point), with and without the TG source and the artificial viscosity."""
    import paper_2609_16424_amd as ilh
    O, G = make_pair(prob, n, k, visc, width=0.05 if visc == "const" else 1e-3)
    u = random_state(O, 61)
    kk = 0.1 * random_dir(O, 62)
    tau = 0.004
    ro = O.residual(kk, u, tau)
    r_strip = to_np(G.residual(to_dev(kk), to_dev(u), tau))
    G.set_kernel_variant("generic")
    r_gen = to_np(G.residual(to_dev(kk), to_dev(u), tau))
    G.set_kernel_variant("lin")
    assert close(r_strip, ro, FP64_TOL)
    assert close(r_gen, ro, FP64_TOL)
    assert close(r_strip, r_gen, FP64_TOL)


@pytest.mark.parametrize("n,k", [((130, 330), 3), ((64, 1040), 2), ((40, 24, 16), 2)])
def test_strip_residual_large_mesh(n, k):
    """Strip and generic residual kernels agree block by block on meshes of several thousand
    waves at a randomly perturbed state."""
    import paper_2609_16424_amd as ilh
    G = ilh.Hydro("tg2d" if len(n) == 2 else "tg3d", n, k)
    u = G.init_state()
    rng = np.random.default_rng(43)
    h = 1.0 / (k * max(n))
    pert = np.concatenate([0.03 * h * rng.standard_normal(G.nh1), 0.3 * rng.standard_normal(G.nh1),
                           0.2 * rng.standard_normal(G.nl2)])
    u = u + torch.from_numpy(pert).to(u.device)
    kk = torch.from_numpy(0.1 * np.concatenate([h * rng.standard_normal(G.nh1),
                                                rng.standard_normal(G.nh1 + G.nl2)])).to(u.device)
    a = G.residual(kk, u, 0.002)
    G.set_kernel_variant("generic")
    b = G.residual(kk, u, 0.002)
    G.set_kernel_variant("lin")
    for lo, hi in ((0, G.nh1), (G.nh1, 2 * G.nh1), (2 * G.nh1, G.nblock)):
        err = float(torch.linalg.norm(a[lo:hi] - b[lo:hi]) / torch.linalg.norm(b[lo:hi]))
        assert err <= 1e-12, (lo, err)
