"""Exact self-similar Sedov blast wave in a uniform ideal gas (oracle; test infrastructure only).

Used as the reference of the 2D Sedov test (Sec. 4.2: the shock position should converge to
the exact Sedov solution).  Written from the similarity form of the Euler equations, not from
a tabulation: with r_s(t) = (E t^2 / (alpha rho0))^(1/(nu+2)) (nu = 1, 2, 3 for planar,
cylindrical, spherical), delta = 2/(nu+2), D = dr_s/dt = delta r_s / t and eta = r / r_s,
    u = D eta U(eta),  rho = rho0 R(eta),  p = rho0 D^2 P(eta),
mass, momentum and entropy (p rho^-gamma constant along particle paths) give
    eta (U - 1) R' + eta R U'                 = -nu R U
    eta^2 (U - 1) U' + P' / R                 = eta U (1 - U) - (delta - 1)/delta eta U
    eta (U - 1) (P'/P - gamma R'/R)           = -(2 delta - 2) / delta,
integrated from the strong-shock (Rankine-Hugoniot) state at eta = 1,
    R = (gamma + 1)/(gamma - 1),  U = P = 2/(gamma + 1),
towards eta = 0.  The energy E = sigma_nu int (rho u^2/2 + p/(gamma-1)) r^(nu-1) dr then fixes
alpha = sigma_nu delta^2 int_0^1 (R eta^2 U^2 / 2 + P/(gamma-1)) eta^(nu-1) deta,
sigma_nu = 2, 2 pi, 4 pi.
"""
import numpy as np
from scipy.integrate import quad, solve_ivp


def _rhs(eta, y, gamma, nu):
    R, U, P = y
    delta = 2.0 / (nu + 2.0)
    # linear system A [R', U', P'] = b
    A = np.array([[eta * (U - 1.0), eta * R, 0.0],
                  [0.0, eta * eta * (U - 1.0), 1.0 / R],
                  [-gamma * eta * (U - 1.0) / R, 0.0, eta * (U - 1.0) / P]])
    b = np.array([-nu * R * U,
                  eta * U * (1.0 - U) - (delta - 1.0) / delta * eta * U,
                  -(2.0 * delta - 2.0) / delta])
    return np.linalg.solve(A, b)


def profiles(gamma=1.4, nu=2, eta_min=1e-4, npts=2000):
    """(eta, R, U, P) from the shock (eta = 1) inwards to eta_min."""
    y0 = [(gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0), 2.0 / (gamma + 1.0)]
    etas = np.linspace(1.0, eta_min, npts)
    sol = solve_ivp(_rhs, (1.0, eta_min), y0, args=(gamma, nu), t_eval=etas, rtol=1e-11, atol=1e-13,
                    method="LSODA")
    assert sol.success, sol.message
    return sol.t, sol.y[0], sol.y[1], sol.y[2]


def alpha(gamma=1.4, nu=2):
    """alpha(gamma, nu) of r_s = (E t^2 / (alpha rho0))^(1/(nu+2))."""
    delta = 2.0 / (nu + 2.0)
    sigma = {1: 2.0, 2: 2.0 * np.pi, 3: 4.0 * np.pi}[nu]
    y0 = [(gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0), 2.0 / (gamma + 1.0)]
    sol = solve_ivp(_rhs, (1.0, 1e-6), y0, args=(gamma, nu), dense_output=True, rtol=1e-11, atol=1e-13,
                    method="LSODA")
    assert sol.success, sol.message

    def integrand(eta):
        R, U, P = sol.sol(eta)
        return (0.5 * R * eta * eta * U * U + P / (gamma - 1.0)) * eta ** (nu - 1)

    val, _ = quad(integrand, 1e-6, 1.0, limit=200, epsabs=1e-13, epsrel=1e-11)
    return sigma * delta * delta * val


def mass_fraction(gamma=1.4, nu=2):
    """nu int_0^1 R eta^(nu-1) deta: the mass inside the shock over rho0 times its volume (= 1)."""
    y0 = [(gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0), 2.0 / (gamma + 1.0)]
    sol = solve_ivp(_rhs, (1.0, 1e-6), y0, args=(gamma, nu), dense_output=True, rtol=1e-11, atol=1e-13,
                    method="LSODA")
    val, _ = quad(lambda eta: sol.sol(eta)[0] * eta ** (nu - 1), 1e-6, 1.0, limit=200)
    return nu * val


def shock_radius(t, energy, rho0=1.0, gamma=1.4, nu=2):
    return (energy * t * t / (alpha(gamma, nu) * rho0)) ** (1.0 / (nu + 2.0))
