"""Pins of the oracle on curved initial meshes (positions given per node, Sec. 2.1: the mesh is a
field of the kinematic space) and on boxes with faces that are not walls (CPU only).

The curved meshes come from an interior displacement that keeps every boundary node in place,
so the domain is still the box: its mass, the boundary integrals of a uniform pressure and the
projection of a constant energy are the box's, whatever the interior curvature.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.hydro import Hydro, e_plus
from oracle.krylov import jvp_cs
from oracle.mesh import BoxMesh


def _curved(problem, n, k, amp=0.08, **kw):
    dims = {"tg2d": 2, "tg3d": 3, "uniform": len(n), "triple": 2}
    boxes = {"tg2d": ((0, 0), (1, 1)), "tg3d": ((0, 0, 0), (1, 1, 1)), "triple": ((0, 0), (7, 3)),
             "uniform": ((0,) * len(n), (1,) * len(n))}
    lo, hi = boxes[problem]
    m = BoxMesh(dims[problem], n, lo, hi, k)
    x0 = si.curved_positions(m.x0, lo, hi, amp)
    return Hydro(problem, n, k, x0=x0, **kw), x0


@pytest.mark.parametrize("problem,n,k", [("tg2d", (3, 4), 3), ("tg3d", (2, 3, 2), 2), ("triple", (7, 3), 2)])
def test_curved_mesh_keeps_the_box_mass(problem, n, k):
    H, x0 = _curved(problem, n, k)
    u = H.init_state()
    assert np.abs(H.split(u)[0] - x0.ravel()).max() == 0.0
    # the map is curved: det J0 varies inside the elements
    assert np.ptp(H.detJ0) > 0.05 * np.mean(H.detJ0)
    # the domain is still the box: its volume is exact (det J0 is a polynomial the quadrature
    # integrates exactly); with rho0 = 1 so is the mass; the triple point's elements carry their
    # density with them, so its mass is sum_e rho0_e |Omega_e|
    vol = {"tg2d": 1.0, "tg3d": 1.0, "triple": 21.0}[problem]
    assert abs(float(np.einsum("q,eq->", H.T["qw"], H.detJ0)) - vol) <= 1e-13 * vol
    mass = float(np.sum(H.rho0_e * np.einsum("q,eq->e", H.T["qw"], H.detJ0)))
    if problem != "triple":
        assert abs(mass - 1.0) <= 1e-13
    assert abs(H.total_mass() - mass) <= 1e-13 * mass
    one_h1 = np.ones(H.mesh.N)
    assert abs(one_h1 @ (H.Ms @ one_h1) - mass) <= 1e-12 * mass
    assert abs(np.sum(H.mass_e(np.ones(H.nl2))) - mass) <= 1e-12 * mass


@pytest.mark.parametrize("dim,k,n", [(2, 2, (3, 2)), (2, 3, (2, 3)), (3, 2, (2, 2, 2))])
def test_curved_uniform_pressure(dim, k, n):
    """Uniform gas at rest on a curved mesh: no interior force (the divergence theorem per node),
    the boundary forces of the straight box faces, no work, and e0 projected exactly."""
    H, _ = _curved("uniform", n, k, amp=0.06)
    Hb = Hydro("uniform", n, k)
    u = H.init_state()
    assert np.abs(H.split(u)[2] - 2.5).max() <= 1e-13
    F1, Ftv = H.force(u)
    F1b, _ = Hb.force(Hb.init_state())
    assert np.abs(Ftv).max() <= 1e-14
    # interior nodes carry no force; boundary nodes the same as on the Cartesian mesh
    assert np.abs(F1 - F1b).max() <= 1e-13 * np.abs(F1b).max()
    interior = np.ones(H.mesh.N, bool)
    for c in range(dim):
        gi = H.mesh.node_grid_index[c]
        interior &= (gi > 0) & (gi < H.mesh.ng[c] - 1)
    assert np.abs(F1.reshape(dim, -1)[:, interior]).max() <= 1e-13


def test_curved_energy_identity_and_jacobian():
    """The exact midpoint energy identity and complex step vs central FD hold on a curved mesh."""
    H, _ = _curved("tg2d", (3, 3), 2)
    u = si.perturb_state(H.init_state(), 3, H.nh1, 0.002, 0.05, 0.02)
    k = 0.2 * si.block_direction(4, H.nh1, H.nl2, 0.01, 1.0, 1.0)
    dt = 0.01
    tau = dt / 2
    r = H.residual(k, u, tau)
    w = u + tau * k
    _, wv, _ = H.split(w)
    _, Rv, Re = H.split(r)
    kx, kv, ke = H.split(k)
    cons = H.cons
    E0 = sum(H.energy(u))
    E1 = sum(H.energy(u + dt * k))
    F1, _ = H.force(w)
    Rv_true = np.where(cons, H.mass_v(kv) + F1, Rv)
    ident = dt * (wv @ Rv_true + np.sum(Re) + np.sum(H.energy_source(H.split(w)[0])))
    assert abs((E1 - E0) - ident) <= 1e-13 * max(1.0, abs(E0))
    dk = si.block_direction(5, H.nh1, H.nl2, 0.01, 1.0, 1.0)
    jc = jvp_cs(lambda q: H.residual(q, u, tau), k, dk)
    eps = 1e-7
    fd = (H.residual(k + eps * dk, u, tau) - H.residual(k - eps * dk, u, tau)) / (2 * eps)
    assert np.linalg.norm(jc - fd) <= 2e-7 * np.linalg.norm(jc)


@pytest.mark.parametrize("face", [0, 1, 2, 3])
def test_free_face_accelerates_outward(face):
    """Uniform gas at rest with one face that is not a wall: the explicit rate pushes that face's
    nodes outward (along its normal), and every wall keeps v.n = 0."""
    H = Hydro("uniform", (3, 2), 2, free_faces=1 << face)
    u = H.init_state()
    a = H.split(H.rate(u))[1].reshape(2, -1)
    m = H.mesh
    c, side = face // 2, face % 2
    gi = m.node_grid_index[c]
    on_face = gi == (0 if side == 0 else m.ng[c] - 1)
    normal = -1.0 if side == 0 else 1.0
    assert np.all(normal * a[c][on_face] > 1e-3)
    # walls: the normal component vanishes on every other face
    for cc in range(2):
        for ss in range(2):
            if (cc, ss) == (c, side):
                continue
            g = m.node_grid_index[cc]
            f = g == (0 if ss == 0 else m.ng[cc] - 1)
            assert np.abs(a[cc][f]).max() == 0.0
    # the constrained rows are exactly the wall rows
    assert m.constrained.sum() == Hydro("uniform", (3, 2), 2).mesh.constrained.sum() - on_face.sum()
