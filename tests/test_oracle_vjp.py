"""Pins of the oracle's transpose Jacobian action (compressed complex-step columns).

The transpose of the Jacobian action (Sec. 3.4: transpose actions share the gather-apply-
scatter structure) has no closed form here; it is pinned to its definition, the transpose of
the dense complex-step Jacobian, on meshes small enough for n columns but large enough that
each colour class holds several columns, and by the adjoint identity <y, J dk> = <J^T y, dk>
against the independent complex-step Jacobian action on a mesh of several hundred unknowns.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.hydro import Hydro, ViscosityOptions
from oracle.krylov import dense_jacobian, jvp_cs, vjp_colored


def _setup(name, n, k, visc):
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=0.05)
    O = Hydro(name, n, k, visc=vo)
    h = float(np.min(O.mesh.h)) / k
    u = si.perturb_state(O.init_state(), 3, O.nh1, 0.03 * h, 0.3, 0.2)
    kk = 0.1 * si.block_direction(4, O.nh1, O.nl2, sx=h, sv=1.0, se=1.0)
    y = si.block_direction(5, O.nh1, O.nl2, sx=1.0, sv=1.0, se=1.0)
    return O, u, kk, y, h


@pytest.mark.parametrize("name,n,k,visc", [("tg2d", (4, 3), 1, None), ("tg2d", (4, 3), 2, None),
                                           ("triple", (4, 2), 2, "const"), ("triple", (3, 2), 3, "formula"),
                                           ("tg3d", (3, 2, 2), 1, None)])
def test_vjp_equals_dense_transpose(name, n, k, visc):
    O, u, kk, y, _ = _setup(name, n, k, visc)
    fun = lambda q: O.residual(q, u, 0.01)
    a = vjp_colored(O, fun, kk, y)
    b = dense_jacobian(fun, kk).T @ y
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(b)


@pytest.mark.parametrize("name,n,k,visc", [("tg2d", (18, 2), 2, None), ("triple", (7, 3), 2, "formula")])
def test_vjp_adjoint_identity(name, n, k, visc):
    O, u, kk, y, h = _setup(name, n, k, visc)
    fun = lambda q: O.residual(q, u, 0.01)
    a = vjp_colored(O, fun, kk, y)
    for s in (6, 7, 8):
        dk = si.block_direction(s, O.nh1, O.nl2, sx=h, sv=1.0, se=1.0)
        lhs = y @ jvp_cs(fun, kk, dk)
        assert abs(lhs - a @ dk) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("prob,n,k", [("tg2d", (5, 4), 3), ("tg3d", (3, 2, 2), 2)])
def test_local_complex_step_rows_and_columns(prob, n, k):
    """The full-size sampled checks evaluate the complex step on the elements that reach the
    sampled rows (or hold the sampled column's dof) only: on a small mesh those rows equal the
    whole-mesh complex step, and <y, J e_j> equals the coloured transpose action's entry j."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from gpu_common import elements_of_dof, jvp_local
    from oracle.hydro import Hydro
    from oracle.krylov import jvp_cs, vjp_colored
    import seeded_inputs as si
    O = Hydro(prob, n, k)
    h = float(np.min(O.mesh.h)) / k
    u = si.perturb_state(O.init_state(), 1, O.nh1, 0.03 * h, 0.3, 0.2)
    kk = 0.1 * si.block_direction(2, O.nh1, O.nl2, h, 1.0, 1.0)
    dk = si.block_direction(3, O.nh1, O.nl2, h, 1.0, 1.0)
    y = si.block_direction(4, O.nh1, O.nl2)
    tau = 0.003
    full = jvp_cs(lambda q: O.residual(q, u, tau), kk, dk)
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(O.nblock, 10, replace=False))
    adj = np.unique(np.concatenate([elements_of_dof(O, r) for r in rows]))
    assert len(adj) < O.mesh.Ne
    loc = jvp_local(O, kk, u, tau, dk, adj)
    assert np.abs(loc[rows] - full[rows]).max() <= 1e-13 * np.abs(full).max()
    if O.dim == 3:
        return  # the coloured transpose of the 3D oracle is pinned elsewhere (and slow)
    vt = vjp_colored(O, lambda q: O.residual(q, u, tau), kk, y)
    for j in rows:
        ej = np.zeros(O.nblock)
        ej[j] = 1.0
        val = float(y @ jvp_local(O, kk, u, tau, ej, elements_of_dof(O, j)))
        assert abs(val - vt[j]) <= 1e-12 * np.abs(vt).max()
