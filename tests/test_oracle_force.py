"""Pins of the oracle's force operator, masses and pointwise physics (CPU only).

Each check is a closed form, an identity of the semi-discrete equations, or an
invariance, derived from the paper's definitions (eq. matrices, v_semi, e_semi,
energy_regularization, visc_* equations) independently of the oracle's code.
"""
import numpy as np
import pytest

from oracle.hydro import EPS_E, Hydro, ViscosityOptions, e_plus, tg2d_energy_source


def _lagrange_integrals(nodes):
    """Exact integrals over [0,1] of the Lagrange polynomials through ``nodes`` (via np.poly)."""
    out = []
    for b, tb in enumerate(nodes):
        others = [t for m, t in enumerate(nodes) if m != b]
        c = np.poly(others) / np.prod([tb - t for t in others])
        ci = np.polyint(c)
        out.append(np.polyval(ci, 1.0) - np.polyval(ci, 0.0))
    return np.array(out)


def _random_state(H, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    u = H.init_state()
    x, v, e = H.split(u)
    h = float(np.min(H.mesh.h)) / H.k
    x = x + amp * h * rng.standard_normal(x.size)
    v = v + 0.3 * rng.standard_normal(v.size)
    e = e * (1 + 0.2 * rng.standard_normal(e.size))
    return np.concatenate([x, v, e])


@pytest.mark.parametrize("dim,k,n", [(2, 2, (3, 2)), (2, 3, (2, 2)), (3, 2, (2, 1, 2))])
def test_uniform_pressure_boundary_closed_form(dim, k, n):
    H = Hydro("uniform", n, k)
    u = H.init_state()
    F1, Ftv = H.force(u)
    assert np.abs(Ftv).max() < 1e-14
    p = 0.4 * 1.0 * e_plus(np.array(2.5))
    # (F 1)_{n,c} = -p * oint w_n n_c ds; faces normal to c only
    m = H.mesh
    I1 = _lagrange_integrals(H.T["gll"])
    F1 = F1.reshape(dim, m.N)
    for c in range(dim):
        expect = np.zeros(m.N)
        gi = m.node_grid_index
        for node in range(m.N):
            side = 0
            if gi[c, node] == 0:
                side = -1
            elif gi[c, node] == m.ng[c] - 1:
                side = 1
            if side == 0:
                continue
            val = 1.0
            for a in range(dim):
                if a == c:
                    continue
                I = gi[a, node]
                loc, el = I % k, I // k
                tot = 0.0
                if loc == 0:  # element vertex line: shared by left/right elements
                    if el > 0:
                        tot += m.h[a] * I1[k]
                    if el < m.n[a]:
                        tot += m.h[a] * I1[0]
                else:
                    tot = m.h[a] * I1[loc]
                val *= tot
            expect[node] = -p * side * val
        assert np.allclose(F1[c], expect, atol=1e-14, rtol=0), (c, np.abs(F1[c] - expect).max())


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
def test_affine_velocity_energy_closed_form(dim, k):
    H = Hydro("uniform", (2,) * dim, k)
    u = H.init_state()
    x, v, e = H.split(u)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((dim, dim))
    X = x.reshape(dim, -1)
    v = (A @ X).ravel()
    F1, Ftv = H.force(np.concatenate([x, v, e]))
    p = 0.4 * e_plus(np.array(2.5))
    vol_e = np.prod(H.mesh.h)
    expect = -p * np.trace(A) * vol_e / k ** dim  # int phi_j = |Omega_e| / k^d for Bernstein
    assert np.allclose(Ftv, expect, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("prob,dim,k,visc", [("tg2d", 2, 2, None), ("tg2d", 2, 3, "const"),
                                             ("triple", 2, 2, "formula"), ("tg3d", 3, 2, "const")])
def test_momentum_and_force_transpose_identities(prob, dim, k, visc):
    n = {"tg2d": (3, 4), "triple": (7, 3), "tg3d": (2, 2, 2)}[prob]
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=0.05)
    H = Hydro(prob, n, k, visc=vo)
    w = _random_state(H, 7)
    F1, Ftv = H.force(w)
    _, v, _ = H.split(w)
    scale = np.abs(F1).max()
    # momentum: sum_n (F 1)_{n,c} = 0 (partition of unity of the H1 basis)
    assert np.abs(F1.reshape(dim, -1).sum(1)).max() < 1e-13 * scale * F1.size
    # force transpose identity: v^T (F 1) = 1^T (F^T v)
    assert abs(v @ F1 - Ftv.sum()) < 1e-12 * np.abs(v * F1).sum()
    # translation and Galilean invariance
    x, v2, e = H.split(w)
    c = np.repeat(rng_vec := np.random.default_rng(1).standard_normal(dim), H.mesh.N)
    F1t, Ftvt = H.force(np.concatenate([x + c, v2, e]))
    assert np.allclose(F1t, F1, rtol=0, atol=1e-12 * scale)
    F1g, Ftvg = H.force(np.concatenate([x, v2 + c, e]))
    assert np.allclose(F1g, F1, rtol=0, atol=1e-12 * scale)
    assert np.allclose(Ftvg, Ftv, rtol=0, atol=1e-11 * np.abs(Ftv).max())


def test_masses_totals_and_inverse():
    H = Hydro("tg2d", (4, 4), 3)
    one = np.ones(H.mesh.N)
    assert abs(one @ (H.Ms @ one) - 1.0) < 1e-13
    assert abs(np.sum(H.mass_e(np.ones(H.nl2))) - 1.0) < 1e-13
    Ht = Hydro("triple", (14, 6), 2)
    assert abs(Ht.total_mass() - 13.125) < 1e-12
    assert abs(np.sum(Ht.mass_e(np.ones(Ht.nl2))) - 13.125) < 1e-12
    e = np.random.default_rng(0).standard_normal(H.nl2)
    assert np.allclose(H.mass_e_inv(H.mass_e(e)), e, atol=1e-12)


def test_tg_source_closed_form():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (2, 50))
    s = tg2d_energy_source(x, 5.0 / 3.0)
    closed = 3 * np.pi / 8 * (np.cos(3 * np.pi * x[0]) * np.cos(np.pi * x[1])
                              - np.cos(np.pi * x[0]) * np.cos(3 * np.pi * x[1]))
    assert np.allclose(s, closed, atol=1e-14)


def test_energy_regularization_constants():
    # e+(0) = eps/2 (stated in the paper); e+ -> e for e >> eps; e+ -> eps^2/(4|e|) for e << -eps
    assert e_plus(np.array(0.0)) == pytest.approx(EPS_E / 2, rel=1e-15)
    assert e_plus(np.array(3.0)) == pytest.approx(3.0, rel=1e-15)
    assert e_plus(np.array(-2.0)) == pytest.approx(EPS_E ** 2 / 8, rel=1e-10)


def test_viscosity_special_values():
    """mu at div v = 0 uses |0|_s = delta_scale and psi(0) = psi0; limits under strong
    compression / expansion reduce to rho h (q2 |dv| + q1 c_s) and rho h q2 dv."""
    for a, expect_fn in [
        (0.0, lambda rho, h, cs, dv, w: rho * h * (1.0 * w + 0.5 * cs * 0.5)),
        (-400.0, lambda rho, h, cs, dv, w: rho * h * (abs(dv) + 0.5 * cs)),
        (400.0, lambda rho, h, cs, dv, w: rho * h * dv),
    ]:
        vo = ViscosityOptions(on=True, mode="const", width=1e-3)
        H = Hydro("uniform", (2, 2), 2, visc=vo)
        u = H.init_state()
        x, v, e = H.split(u)
        v = (a * x.reshape(2, -1)).ravel()
        pw = H.pointwise(np.concatenate([x, v, e]))
        h = vo.h0
        dv = h * 2 * a
        rho = 1.0
        cs = np.sqrt(1.4 * 0.4 * e_plus(np.array(2.5)))
        assert np.allclose(pw["mu"], expect_fn(rho, h, cs, dv, vo.width), rtol=1e-6, atol=0)


def test_affine_viscous_stress_is_uniform():
    vo = ViscosityOptions(on=True, mode="formula")
    H = Hydro("uniform", (3, 3), 2, visc=vo)
    u = H.init_state()
    x, v, e = H.split(u)
    A = np.array([[-0.7, 0.2], [0.4, -0.1]])
    v = (A @ x.reshape(2, -1)).ravel()
    F1, Ftv = H.force(np.concatenate([x, v, e]))
    m = H.mesh
    interior = ~(m.constrained[0] | m.constrained[1])
    assert np.abs(F1.reshape(2, -1)[:, interior]).max() < 1e-13
    ratio = Ftv / (np.prod(m.h) / 4.0)  # int phi_j = |Omega_e| / k^2
    assert np.allclose(ratio, ratio[0], rtol=1e-12)


@pytest.mark.parametrize("dim,k,visc", [(2, 2, False), (2, 3, True), (3, 2, True), (3, 1, False)])
def test_affinely_deformed_mesh_closed_form(dim, k, visc):
    """x = B x0 (det B != 1), v = A x with non-symmetric A, constant e.

    The stress is uniform: rho = rho0 / det B (strong mass conservation), p = (g-1) rho e+,
    grad v = A.  In the strong-expansion limit (div v >> delta_scale) the smoothed
    viscosity reduces to mu = rho h q2 delta_v with h = h0 (det B)^(1/d), delta_v = h tr A.
    Then interior (F 1) = 0 and (F^T v)_j = (sigma : A) * |det B| |Omega_e| / k^d.
    """
    vo = ViscosityOptions(on=visc, mode="const", width=1e-3)
    H = Hydro("uniform", (2,) * dim, k, visc=vo)
    u = H.init_state()
    x, v, e = H.split(u)
    rng = np.random.default_rng(11)
    B = np.eye(dim) + 0.25 * rng.standard_normal((dim, dim))
    detB = np.linalg.det(B)
    assert detB > 0.3
    A = 0.5 * rng.standard_normal((dim, dim))
    A += (400.0 - np.trace(A)) / dim * np.eye(dim)  # strong expansion, tr A = 400
    X = B @ x.reshape(dim, -1)
    V = A @ X
    w = np.concatenate([X.ravel(), V.ravel(), e])
    F1, Ftv = H.force(w)
    m = H.mesh
    ep = e_plus(np.array(2.5))
    rho = 1.0 / detB
    p = 0.4 * rho * ep
    sigma = -p * np.eye(dim)
    if visc:
        h = vo.h0 * detB ** (1.0 / dim)
        mu = rho * h * 1.0 * (h * np.trace(A))
        sigma = sigma + mu * 0.5 * (A + A.T)
    expect = np.sum(sigma * A) * detB * np.prod(m.h) / k ** dim
    assert np.allclose(Ftv, expect, rtol=1e-9), (Ftv[:3], expect)
    interior = np.ones(m.N, dtype=bool)
    for c in range(dim):
        interior &= ~m.constrained[c]
    if interior.any():
        assert np.abs(F1.reshape(dim, -1)[:, interior]).max() < 1e-10 * np.abs(F1).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
@pytest.mark.parametrize("m", [1.0, -1.0, 2.0, -2.0])
def test_viscosity_formula_scale_closed_form(dim, k, m):
    """The paper's smoothing scale delta_scale = 2 (h / h_coarse) c_s (eq. visc_imp_scale) and the
    switch psi = (1 + tanh((-delta_v - s) / (2 delta_scale))) / 2 (eq. visc_imp_switch, s = 0 at
    psi0 = 1/2), pinned through the work of the force on an affinely compressed or expanded gas.

    x = B x0 (diagonal B, det B != 1), v = a x, constant e: then rho = 1 / det B, h = h0 (det B)^(1/d),
    grad v = a I and delta_v = h d a.  The velocity scale is chosen as a = m delta_scale / (h d), so
    that delta_v = m delta_scale and the smoothed quantities take the values
        |delta_v|_s = delta_scale sqrt(1 + m^2),   psi = (1 + tanh(-m / 2)) / 2,
    and mu = rho h (q2 |delta_v|_s + q1 c_s psi).  The stress is (-p + mu a) I, so
    (F^T v)_j = (-p + mu a) d a det B |Omega_e| / k^d.  h_coarse differs from h0, so the ratio
    h / h_coarse matters; a factor 2 dropped from delta_scale or from the tanh width moves psi and
    |delta_v|_s away from these values.
    """
    hc = 0.6 * (1.0 / 2) / k  # h_coarse != h0 = 1 / (2 k) on the 2^d mesh of the unit box
    vo = ViscosityOptions(on=True, mode="formula", h_coarse=hc)
    H = Hydro("uniform", (2,) * dim, k, visc=vo)
    u = H.init_state()
    x, _, e = H.split(u)
    Bd = np.array([1.2, 0.9, 1.1][:dim])
    detB = float(np.prod(Bd))
    X = Bd[:, None] * x.reshape(dim, -1)
    ep = 0.5 * (2.5 + np.sqrt(2.5 ** 2 + EPS_E ** 2))
    gam = 1.4
    rho = 1.0 / detB
    p = (gam - 1.0) * rho * ep
    cs = np.sqrt(gam * (gam - 1.0) * ep)
    h0 = (1.0 / 2 ** dim) ** (1.0 / dim) / k
    h = h0 * detB ** (1.0 / dim)
    dscale = 2.0 * (h / hc) * cs
    a = m * dscale / (h * dim)
    V = a * X
    F1, Ftv = H.force(np.concatenate([X.ravel(), V.ravel(), e]))
    mu = rho * h * (1.0 * dscale * np.sqrt(1.0 + m * m) + 0.5 * cs * 0.5 * (1.0 + np.tanh(-m / 2.0)))
    expect = (-p + mu * a) * dim * a * detB * (0.5 ** dim) / k ** dim
    assert np.allclose(Ftv, expect, rtol=1e-12, atol=0), (Ftv[:2], expect)
    # the viscous part is a sizeable share of the work, so the check sees mu
    assert abs(mu * a) > 0.05 * p
