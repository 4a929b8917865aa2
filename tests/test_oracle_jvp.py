"""Pins of the oracle's Jacobian actions (CPU only).

The complex-step derivative is checked against central finite differences, against
brute-force dense Jacobians on tiny meshes, against the exact structure of the stage
Jacobian at tau = 0 (the mass matrices, computed here from exact 1D integrals), and
against the derivative of the force-transpose identity.
"""
import math

import numpy as np
import pytest

from oracle.hydro import Hydro, ViscosityOptions
from oracle.krylov import dense_jacobian, jvp_cs, jvp_fd


def _state(H, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    u = H.init_state()
    x, v, e = H.split(u)
    h = float(np.min(H.mesh.h)) / H.k
    return np.concatenate([x + amp * h * rng.standard_normal(x.size),
                           v + 0.3 * rng.standard_normal(v.size),
                           e * (1 + 0.2 * rng.standard_normal(e.size))])


def _dir(H, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(H.nblock)
    h = float(np.min(H.mesh.h)) / H.k
    d[:H.nh1] *= h
    return d


CASES = [("tg2d", (3, 2), 2, None), ("tg2d", (2, 2), 3, "const"),
         ("triple", (7, 3), 2, "formula"), ("tg3d", (2, 1, 2), 2, "formula")]


@pytest.mark.parametrize("prob,n,k,visc", CASES)
def test_complex_step_matches_central_fd(prob, n, k, visc):
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=0.05)
    H = Hydro(prob, n, k, visc=vo)
    u = _state(H, 1)
    kk = 0.1 * _dir(H, 2) / max(1e-3, float(np.min(H.mesh.h)))
    dk = _dir(H, 3)
    tau = 0.004
    R = lambda q: H.residual(q, u, tau)
    a = jvp_cs(R, kk, dk)
    b = jvp_fd(R, kk, dk, 1e-7)
    assert np.linalg.norm(a - b) <= 2e-7 * np.linalg.norm(a)


@pytest.mark.parametrize("prob,n,k,visc", [("tg2d", (1, 1), 2, "const"), ("tg2d", (2, 2), 1, None),
                                           ("tg3d", (1, 1, 1), 1, "formula")])
def test_dense_jacobian_brute_force(prob, n, k, visc):
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=0.05)
    H = Hydro(prob, n, k, visc=vo)
    u = _state(H, 4)
    kk = 0.05 * _dir(H, 5)
    tau = 0.01
    R = lambda q: H.residual(q, u, tau)
    Jd = dense_jacobian(R, kk)
    nb = H.nblock
    # brute force: every column by central differences
    for j in range(nb):
        ej = np.zeros(nb)
        ej[j] = 1.0
        col = jvp_fd(R, kk, ej, 1e-6)
        assert np.allclose(Jd[:, j], col, rtol=1e-5, atol=1e-7 * (1 + np.abs(col).max()))
    # J applied to a direction equals the complex-step action (linearity)
    dk = _dir(H, 6)
    assert np.allclose(Jd @ dk, jvp_cs(R, kk, dk), rtol=1e-12, atol=1e-14)
    # x rows: d R_x / d k = [I, -tau I, 0]
    a = H.nh1
    assert np.allclose(Jd[:a, :a], np.eye(a), atol=1e-15)
    assert np.allclose(Jd[:a, a:2 * a], -tau * np.eye(a), atol=1e-15)
    assert np.allclose(Jd[:a, 2 * a:], 0, atol=1e-15)


def _lagr_mass_1d(nodes):
    P = []
    for b, tb in enumerate(nodes):
        others = [t for m, t in enumerate(nodes) if m != b]
        P.append(np.poly(others) / np.prod([tb - t for t in others]))
    M = np.zeros((len(nodes), len(nodes)))
    for i in range(len(nodes)):
        for j in range(len(nodes)):
            c = np.polyint(np.polymul(P[i], P[j]))
            M[i, j] = np.polyval(c, 1.0) - np.polyval(c, 0.0)
    return M


def _bern_mass_1d(n):
    return np.array([[math.comb(n, i) * math.comb(n, j) / ((2 * n + 1) * math.comb(2 * n, i + j))
                      for j in range(n + 1)] for i in range(n + 1)])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_stage_jacobian_at_tau0_is_block_mass(k):
    H = Hydro("tg2d", (2, 2), k)
    u = H.init_state()
    R = lambda q: H.residual(q, u, 0.0)
    Jd = dense_jacobian(R, np.zeros(H.nblock))
    m = H.mesh
    # assembled scalar mass from exact 1D Lagrange integrals (affine elements, rho = 1)
    M1 = _lagr_mass_1d(H.T["gll"])
    Me = np.prod(m.h) * np.kron(M1, M1)  # local order: first direction fastest
    Ms = np.zeros((m.N, m.N))
    for e in range(m.Ne):
        idx = m.conn[e]
        Ms[np.ix_(idx, idx)] += Me
    a, b = H.nh1, 2 * H.nh1
    Jvv = Jd[a:b, a:b]
    cons = m.constrained.ravel()
    expect = np.kron(np.eye(2), Ms)
    expect[cons] = np.eye(H.nh1)[cons]
    assert np.allclose(Jvv, expect, atol=1e-15)
    assert np.allclose(Jd[a:b, :a], 0, atol=1e-15) and np.allclose(Jd[a:b, b:], 0, atol=1e-15)
    B1 = _bern_mass_1d(k - 1)
    MEe = np.prod(m.h) * np.kron(B1, B1)
    expect_e = np.kron(np.eye(m.Ne), MEe)
    assert np.allclose(Jd[b:, b:], expect_e, atol=1e-15)


@pytest.mark.parametrize("visc", [None, "formula"])
def test_tangent_of_force_transpose_identity(visc):
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const")
    H = Hydro("triple", (7, 3), 2, visc=vo)
    w = _state(H, 8)
    dw = _dir(H, 9)
    F1, Ftv = H.force(w)
    dF1 = jvp_cs(lambda q: H.force(q)[0], w, dw)
    dFtv = jvp_cs(lambda q: H.force(q)[1], w, dw)
    _, v, _ = H.split(w)
    _, dv, _ = H.split(dw)
    lhs = dv @ F1 + v @ dF1
    rhs = dFtv.sum()
    assert abs(lhs - rhs) <= 1e-11 * (np.abs(dv * F1).sum() + np.abs(v * dF1).sum())
