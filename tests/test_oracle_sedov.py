"""Pins of the oracle's Sedov problem and exact self-similar solution (Sec. 4.2).

* the similarity profiles conserve mass: the shocked region holds exactly the ambient mass it
  swept (nu int_0^1 R eta^(nu-1) deta = 1), planar, cylindrical and spherical;
* the spherical gamma = 1.4 blast gives Taylor's constant r_s = 1.033 (E t^2 / rho0)^(1/5);
* the initial state deposits total energy 0.25 in the element at the origin, mass 1.
"""
import numpy as np
import pytest

from oracle import sedov
from oracle.hydro import Hydro, ViscosityOptions


@pytest.mark.parametrize("gamma,nu", [(1.4, 1), (1.4, 2), (1.4, 3), (5.0 / 3.0, 2)])
def test_similarity_solution_conserves_mass(gamma, nu):
    assert abs(sedov.mass_fraction(gamma, nu) - 1.0) <= 1e-8


def test_spherical_constant():
    xi0 = sedov.alpha(1.4, 3) ** (-1.0 / 5.0)
    assert abs(xi0 - 1.033) <= 1e-3


def test_shock_state_and_radius():
    eta, R, U, P = sedov.profiles(1.4, 2)
    assert abs(R[0] - 6.0) < 1e-12 and abs(U[0] - 2.0 / 2.4) < 1e-12
    assert np.all(np.diff(R) < 0)  # density falls monotonically behind the shock
    r = sedov.shock_radius(0.8, 1.0)
    assert 0.85 < r < 0.95


def test_initial_state():
    H = Hydro("sedov", (6, 6), 2, visc=ViscosityOptions(on=True, mode="formula", h_coarse=0.5))
    u = H.init_state()
    ke, ie = H.energy(u)
    assert ke == 0.0 and abs(ie - 0.25) < 1e-14
    assert abs(H.total_mass() - 1.0) < 1e-14
