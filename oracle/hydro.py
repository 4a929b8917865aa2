"""Semi-discrete Lagrangian hydrodynamics, written out from the paper (oracle; test infrastructure only).

Everything here is FP64 (or complex128 when a complex-step derivative is taken) and is
written with dense per-element matrices: the element force matrix F_e is formed
explicitly and then applied to the vector of ones and to the velocity, exactly as in
eq. (matrices) and eq. (v_semi)/(e_semi).  No sum factorisation, fusion or reordering.

Block vectors are [x | v | e]; x and v are component-major ([d][N_nodes]) H1 vectors,
e is the element-major L2 vector.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import tensor_tables
from .mesh import BoxMesh

EPS_E = 1.0e-6  # energy regularisation width, eq. (energy_regularization)


# ----------------------------------------------------------------------------------------
# Problem definitions (initial data).  These are the paper's benchmark set-ups as read in
# the design notes; the oracle keeps its own copy, independent of the GPU library.
# ----------------------------------------------------------------------------------------

def tg2d_velocity(x):
    """2D Taylor-Green velocity (sin pi x cos pi y, -cos pi x sin pi y) on [0,1]^2."""
    return np.stack([np.sin(np.pi * x[0]) * np.cos(np.pi * x[1]),
                     -np.cos(np.pi * x[0]) * np.sin(np.pi * x[1])])


def tg2d_pressure(x, rho=1.0):
    """p = rho/4 (cos 2 pi x + cos 2 pi y) + 1."""
    return rho / 4.0 * (np.cos(2 * np.pi * x[0]) + np.cos(2 * np.pi * x[1])) + 1.0


def tg2d_pressure_gradient(x, rho=1.0):
    return np.stack([-rho * np.pi / 2.0 * np.sin(2 * np.pi * x[0]),
                     -rho * np.pi / 2.0 * np.sin(2 * np.pi * x[1])])


def tg2d_energy_source(x, gamma):
    """Specific-energy source s = v . grad e for the steady TG state (rho = 1).

    With e = p / ((gamma-1) rho) and div v = 0, the energy equation rho de/dt = sigma:grad v
    + rho s is steady only with s = v . grad e.  Written as the dot product of the
    velocity with the energy gradient (no closed-form simplification here; the test-suite
    checks it against the closed form separately).
    """
    v = tg2d_velocity(x)
    gp = tg2d_pressure_gradient(x)
    return (v[0] * gp[0] + v[1] * gp[1]) / (gamma - 1.0)


def tg3d_velocity(x):
    """3D Taylor-Green velocity on the unit box."""
    return np.stack([np.sin(np.pi * x[0]) * np.cos(np.pi * x[1]) * np.cos(np.pi * x[2]),
                     -np.cos(np.pi * x[0]) * np.sin(np.pi * x[1]) * np.cos(np.pi * x[2]),
                     np.zeros_like(x[0])])


def tg3d_pressure(x):
    return 1.0 + (np.cos(2 * np.pi * x[0]) + np.cos(2 * np.pi * x[1])) * (np.cos(2 * np.pi * x[2]) + 2.0) / 16.0


TRIPLE_STATES = {  # region: (rho, p, gamma)
    "left": (1.0, 1.0, 1.5),
    "bottom": (1.0, 0.1, 1.4),
    "top": (0.125, 0.1, 1.5),
}


def triple_region(xc):
    """Region of an element centre: x<1 left; x>1, y<1.5 bottom; x>1, y>1.5 top."""
    if xc[0] < 1.0:
        return "left"
    return "bottom" if xc[1] < 1.5 else "top"


class Problem:
    """Container for an analytic problem: box, per-element rho0/gamma, initial fields."""

    def __init__(self, name, dim, lo, hi, rho0_elem, gamma_elem, v0, e0, source=None,
                 exact_v=None):
        self.name, self.dim, self.lo, self.hi = name, dim, lo, hi
        self.rho0_elem, self.gamma_elem = rho0_elem, gamma_elem
        self.v0, self.e0, self.source, self.exact_v = v0, e0, source, exact_v


def make_problem(name, mesh, perturb=None):
    """Build a Problem for ``name`` in {'tg2d', 'tg3d', 'triple', 'sedov', 'uniform'} on ``mesh``.

    ``perturb`` (triple point only) = dict(scale={'left':(sr,sp),...}, shift=dx) multiplies
    the per-region rho and p and shifts the region interfaces; used for the learned-guess
    training runs.
    """
    Ne = mesh.Ne
    if name == "tg2d":
        gam = 5.0 / 3.0
        return Problem(name, 2, (0, 0), (1, 1), np.ones(Ne), np.full(Ne, gam),
                       v0=tg2d_velocity,
                       e0=lambda x, e_idx: tg2d_pressure(x) / ((gam - 1.0) * 1.0),
                       source=lambda x: tg2d_energy_source(x, gam),
                       exact_v=tg2d_velocity)
    if name == "tg3d":
        gam = 5.0 / 3.0
        return Problem(name, 3, (0, 0, 0), (1, 1, 1), np.ones(Ne), np.full(Ne, gam),
                       v0=tg3d_velocity,
                       e0=lambda x, e_idx: tg3d_pressure(x) / ((gam - 1.0) * 1.0))
    if name == "triple":
        xc = mesh.element_centers()
        rho = np.zeros(Ne)
        gam = np.zeros(Ne)
        pe = np.zeros(Ne)
        shift = 0.0 if perturb is None else perturb.get("shift", 0.0)
        scale = {} if perturb is None else perturb.get("scale", {})
        for e in range(Ne):
            c = xc[:, e].copy()
            c[0] -= shift
            c[1] -= shift
            reg = triple_region(c)
            r, p, g = TRIPLE_STATES[reg]
            sr, spp = scale.get(reg, (1.0, 1.0))
            rho[e], pe[e], gam[e] = r * sr, p * spp, g
        e0v = pe / ((gam - 1.0) * rho)
        return Problem(name, 2, (0, 0), (7, 3), rho, gam,
                       v0=lambda x: np.zeros_like(x),
                       e0=lambda x, e_idx: e0v[e_idx])
    if name == "sedov":
        # Sec. 4.2: unit square, walls, gamma 1.4, rho 1, v 0; the delta-like energy source at
        # the origin is read as all of the deposited energy 0.25 in the element at the origin
        # (constant specific energy there, zero elsewhere)
        e0v = np.zeros(Ne)
        e0v[0] = 0.25 / (1.0 * float(np.prod(mesh.h)))
        return Problem(name, 2, (0, 0), (1, 1), np.ones(Ne), np.full(Ne, 1.4),
                       v0=lambda x: np.zeros_like(x),
                       e0=lambda x, e_idx: e0v[e_idx])
    if name == "uniform":
        d = mesh.dim
        return Problem(name, d, tuple(mesh.lo), tuple(mesh.hi), np.ones(Ne), np.full(Ne, 1.4),
                       v0=lambda x: np.zeros_like(x),
                       e0=lambda x, e_idx: np.full(np.shape(x)[1:], 2.5))
    raise ValueError(name)


# ----------------------------------------------------------------------------------------
# Pointwise physics
# ----------------------------------------------------------------------------------------

def e_plus(e):
    """Smooth positive part e+ = (e + sqrt(e^2 + eps^2))/2, eq. (energy_regularization).

    For e < 0 the algebraically identical form eps^2 / (2 (sqrt(e^2+eps^2) - e)) avoids
    cancellation.  The branch is chosen on the real part so the function stays analytic
    for complex-step differentiation.
    """
    r = np.sqrt(e * e + EPS_E * EPS_E)
    pos = 0.5 * (e + r)
    neg = EPS_E * EPS_E / (2.0 * (r - e))
    return np.where(np.real(e) >= 0.0, pos, neg)


class ViscosityOptions:
    """Smoothed artificial viscosity mu_imp, eqs. (visc_mu_imp)-(visc_imp_scale).

    mode 'const': delta_scale = width (C4 reads "smoothing width 1e-3" this way);
    mode 'formula': delta_scale = 2 (h / h_coarse) c_s.
    """

    def __init__(self, on=False, q1=0.5, q2=1.0, psi0=0.5, mode="const", width=1e-3,
                 h0=None, h_coarse=None):
        self.on, self.q1, self.q2, self.psi0 = on, q1, q2, psi0
        self.mode, self.width, self.h0, self.h_coarse = mode, width, h0, h_coarse


# ----------------------------------------------------------------------------------------
# Discretisation
# ----------------------------------------------------------------------------------------

class Hydro:
    """Q_k Q_{k-1} Lagrangian hydrodynamics on a Cartesian box (paper Sec. 2.1, 2.2)."""

    def __init__(self, problem_name, n, k, visc=None, source=True, perturb=None, nq1d=None, x0=None,
                 free_faces=0):
        """x0 (optional, [dim][N]): initial node positions of a curved initial mesh, the positions
        being a field of the kinematic space (Sec. 2.1); free_faces: box faces without walls."""
        dims = {"tg2d": 2, "tg3d": 3, "triple": 2, "sedov": 2, "uniform": len(n)}
        dim = dims[problem_name]
        boxes = {"tg2d": ((0, 0), (1, 1)), "tg3d": ((0, 0, 0), (1, 1, 1)),
                 "triple": ((0, 0), (7, 3)), "sedov": ((0, 0), (1, 1)), "uniform": ((0,) * dim, (1,) * dim)}
        lo, hi = boxes[problem_name]
        self.mesh = m = BoxMesh(dim, n, lo, hi, k, free_faces)
        if x0 is not None:
            m.x0 = np.array(x0, dtype=np.float64).reshape(dim, m.N)
        self.prob = make_problem(problem_name, m, perturb)
        self.dim, self.k = dim, k
        self.T = tensor_tables(dim, k, nq1d)
        self.Q = len(self.T["qw"])
        self.visc = visc if visc is not None else ViscosityOptions(on=False)
        if self.visc.h0 is None:
            vol = float(np.prod(m.hi - m.lo))
            if x0 is not None:  # |Omega_0| of the curved mesh: the integral of det J0
                X0 = m.x0[:, m.conn]
                vol = float(np.einsum("q,eq->", self.T["qw"],
                                      np.linalg.det(np.einsum("cen,qna->eqca", X0, self.T["dW"]))))
            self.visc.h0 = (vol / m.Ne) ** (1.0 / dim) / k
        if self.visc.h_coarse is None:
            self.visc.h_coarse = self.visc.h0
        self.use_source = source and (self.prob.source is not None)
        self.gamma_e = self.prob.gamma_elem
        self.rho0_e = self.prob.rho0_elem
        # initial geometry at quadrature points
        X0 = m.x0[:, m.conn]  # (d, Ne, Nh)
        J0 = np.einsum("cen,qna->eqca", X0, self.T["dW"])
        self.detJ0 = np.linalg.det(J0)  # (Ne, Q)
        self.x0q = np.einsum("cen,qn->ceq", X0, self.T["W"])
        # quadrature-point mass m_q = rho0 detJ0 w_q (strong mass conservation)
        self.mq = self.rho0_e[:, None] * self.detJ0 * self.T["qw"][None, :]
        self._build_masses()

    # ---- sizes / layout ----
    @property
    def nh1(self):
        return self.dim * self.mesh.N

    @property
    def nl2(self):
        return self.mesh.Ne * self.mesh.Nl

    @property
    def nblock(self):
        return 2 * self.nh1 + self.nl2

    def split(self, u):
        a, b = self.nh1, 2 * self.nh1
        return u[:a], u[a:b], u[b:]

    # ---- masses ----
    def _build_masses(self):
        T = self.T
        # L2 mass blocks and their inverses (block diagonal: L2 is discontinuous)
        self.MEb = np.einsum("eq,qi,qj->eij", self.mq, T["Phi"], T["Phi"])
        self.MEinv = np.linalg.inv(self.MEb)
        self.cons = self.mesh.constrained.ravel()  # (d*N,)
        self._Ms = None
        self._Mhat_lu = None

    @property
    def Ms(self):
        """Scalar H1 mass M_s(i,j) = sum_e sum_q m_q w_i w_j, eq. (matrices) (built on first use)."""
        if self._Ms is None:
            m, T = self.mesh, self.T
            Me = np.einsum("eq,qi,qj->eij", self.mq, T["W"], T["W"])
            rows = np.repeat(m.conn, m.Nh, axis=1).ravel()
            cols = np.tile(m.conn, (1, m.Nh)).ravel()
            self._Ms = sp.csr_matrix((Me.ravel(), (rows, cols)), shape=(m.N, m.N))
        return self._Ms

    def _mhat_lu(self):
        """LU factors of the BC-eliminated scalar masses (identity on constrained DOFs)."""
        if self._Mhat_lu is None:
            m = self.mesh
            self._Mhat_lu = []
            for c in range(self.dim):
                free = ~m.constrained[c]
                P = sp.diags(free.astype(float))
                Mhat = P @ self.Ms @ P + sp.diags((~free).astype(float))
                self._Mhat_lu.append(spla.splu(Mhat.tocsc()))
        return self._Mhat_lu

    def mass_v(self, v):
        """M_V v with M_V = I_d (x) M_s (no boundary conditions)."""
        d, N = self.dim, self.mesh.N
        vv = v.reshape(d, N)
        return np.concatenate([self.Ms @ vv[c] for c in range(d)])

    def mass_v_solve(self, b):
        """Solve Mhat x = b, Mhat = P_u M_V P_u + P_c (constrained rows/cols -> identity)."""
        d, N = self.dim, self.mesh.N
        bb = b.reshape(d, N)
        out = []
        lus = self._mhat_lu()
        for c in range(d):
            lu = lus[c]
            if np.iscomplexobj(bb):
                out.append(lu.solve(bb[c].real) + 1j * lu.solve(bb[c].imag))
            else:
                out.append(lu.solve(bb[c]))
        return np.concatenate(out)

    def mass_v_diag(self):
        """Diagonal of M_V with ones on constrained DOFs (the Jacobi preconditioner)."""
        dg = np.tile(self.Ms.diagonal(), self.dim)
        dg[self.cons] = 1.0
        return dg

    def mass_e(self, e):
        Ee = e.reshape(self.mesh.Ne, self.mesh.Nl)
        return np.einsum("eij,ej->ei", self.MEb, Ee).ravel()

    def mass_e_inv(self, e):
        Ee = e.reshape(self.mesh.Ne, self.mesh.Nl)
        return np.einsum("eij,ej->ei", self.MEinv, Ee).ravel()

    # ---- fields at quadrature points ----
    def _gather(self, x):
        d, N = self.dim, self.mesh.N
        return x.reshape(d, N)[:, self.mesh.conn]  # (d, Ne, Nh)

    def geometry(self, wx, elements=None):
        X = self._gather(wx)
        if elements is not None:
            X = X[:, elements]
        J = np.einsum("cen,qna->eqca", X, self.T["dW"])
        return J, np.linalg.det(J)

    def min_detj(self, w):
        _, detJ = self.geometry(self.split(w)[0])
        return float(np.min(np.real(detJ)))

    # ---- the force operator ----
    def pointwise(self, w, elements=None):
        """Quadrature-point state: J, detJ, J^-1, rho, e+, p, c_s, grad v, sigma, mu.

        ``elements`` restricts the evaluation to a subset of elements (same arithmetic).
        """
        wx, wv, we = self.split(w)
        d, T, m = self.dim, self.T, self.mesh
        sel = slice(None) if elements is None else elements
        J, detJ = self.geometry(wx, elements)
        Jinv = np.linalg.inv(J)
        detJ0 = self.detJ0[sel]
        rho = self.rho0_e[sel, None] * detJ0 / detJ
        E = we.reshape(m.Ne, m.Nl)[sel]
        eq = np.einsum("ej,qj->eq", E, T["Phi"])
        ep = e_plus(eq)
        g = self.gamma_e[sel, None]
        p = (g - 1.0) * rho * ep
        cs = np.sqrt(g * (g - 1.0) * ep)
        V = self._gather(wv)[:, sel]
        gradv = np.einsum("cen,qnb,eqba->eqca", V, T["dW"], Jinv)  # d v_c / d x_a
        I = np.eye(d)
        sigma = -p[..., None, None] * I
        mu = np.zeros_like(p)
        if self.visc.on:
            vo = self.visc
            h = vo.h0 * (detJ / detJ0) ** (1.0 / d)                          # eq. visc_imp_h
            dv = h * np.trace(gradv, axis1=-2, axis2=-1)                     # eq. visc_imp_dv
            if vo.mode == "const":
                dsc = vo.width * np.ones_like(h)
            else:
                dsc = 2.0 * (h / vo.h_coarse) * cs                           # eq. visc_imp_scale
            absd = np.sqrt(dv * dv + dsc * dsc)                              # eq. visc_imp_abs
            s = 2.0 * dsc * np.arctanh(1.0 - 2.0 * vo.psi0)
            psi = 0.5 + 0.5 * np.tanh((-dv - s) / (2.0 * dsc))               # eq. visc_imp_switch
            mu = rho * h * (vo.q2 * absd + vo.q1 * cs * psi)                  # eq. visc_mu_imp
            eps = 0.5 * (gradv + np.swapaxes(gradv, -1, -2))                 # eq. visc_stress
            sigma = sigma + mu[..., None, None] * eps
        return dict(J=J, detJ=detJ, Jinv=Jinv, rho=rho, ep=ep, p=p, cs=cs, gradv=gradv,
                    sigma=sigma, mu=mu)

    def force_matrix(self, w, elements=None):
        """Element force matrices F_e[e, c, n, j] = int_{Omega_e(t)} (sigma : grad w_{n,c}) phi_j.

        The integral is the reference quadrature sum_q w_q |J_q| (...); the physical
        gradient of the H1 basis function w_n e_c is e_c (x) J^{-T} grad_xi w_n.
        ``elements`` restricts the evaluation to a subset of elements.
        """
        pw = self.pointwise(w, elements)
        T = self.T
        gw = np.einsum("qnb,eqba->eqna", T["dW"], pw["Jinv"])  # physical grad of w_n
        return np.einsum("q,eq,eqca,eqna,qj->ecnj", T["qw"], pw["detJ"], pw["sigma"], gw, T["Phi"])

    def force(self, w, elements=None):
        """(F 1, F^T v): the two actions of the force matrix used in eqs. (v_semi), (e_semi).

        F 1 is an H1 vector (component-major, no boundary conditions), F^T v an L2 vector;
        v is the velocity block of the same state w.  With ``elements`` only those elements
        contribute (F 1 is then exact at nodes whose elements are all listed, and F^T v is
        returned for the listed elements only, shape [len(elements), Nl]).
        """
        Fe = self.force_matrix(w, elements)
        m = self.mesh
        sel = np.arange(m.Ne) if elements is None else np.asarray(elements)
        F1e = Fe.sum(axis=-1)  # (ne, d, Nh)
        F1 = np.zeros((self.dim, m.N), dtype=Fe.dtype)
        for c in range(self.dim):
            np.add.at(F1[c], m.conn[sel], F1e[:, c, :])
        V = self._gather(self.split(w)[1])[:, sel]
        Ftv = np.einsum("ecnj,cen->ej", Fe, V)
        if elements is not None:
            return F1.ravel(), Ftv
        return F1.ravel(), Ftv.ravel()

    def force_transpose(self, w, vt):
        """F(w)^T vt: the force matrix of state w applied to another velocity field vt (H1)."""
        Fe = self.force_matrix(w)
        Vt = self._gather(vt)
        return np.einsum("ecnj,cen->ej", Fe, Vt).ravel()

    def energy_source(self, wx):
        """TG energy source b_j = sum_q m_q s(x_q) phi_j at the current positions x_q."""
        if not self.use_source:
            return np.zeros(self.nl2, dtype=wx.dtype)
        X = self._gather(wx)
        xq = np.einsum("cen,qn->ceq", X, self.T["W"])
        s = self.prob.source(xq)
        return np.einsum("eq,eq,qj->ej", self.mq, s, self.T["Phi"]).ravel()

    # ---- stage residual (eq. nonlinear_system) ----
    def residual(self, k, u, tau):
        """R(k; tau, u) at the stage state w = u + tau k.

        R_x = k_x - w_v,   R_v = M_V k_v + F(w) 1 (constrained rows: R_v = k_v),
        R_e = M_E k_e - F(w)^T w_v - b(w_x).
        """
        w = u + tau * k
        kx, kv, ke = self.split(k)
        wx, wv, we = self.split(w)
        F1, Ftv = self.force(w)
        Rx = kx - wv
        Rv = self.mass_v(kv) + F1
        Rv = np.where(self.cons, kv, Rv)
        Re = self.mass_e(ke) - Ftv - self.energy_source(wx)
        return np.concatenate([Rx, Rv, Re])

    def rate(self, u):
        """Explicit rate f(u) = [v; -Mhat^-1 P_u F 1; M_E^-1 (F^T v + b)] (plain initial guess)."""
        ux, uv, ue = self.split(u)
        F1, Ftv = self.force(u)
        F1 = np.where(self.cons, 0.0, F1)
        return np.concatenate([uv, -self.mass_v_solve(F1),
                               self.mass_e_inv(Ftv + self.energy_source(ux))])

    # ---- initial state and diagnostics ----
    def init_state(self):
        """x0 = mesh nodes; v0 = nodal interpolation; e0 = rho-weighted L2 projection."""
        m, T = self.mesh, self.T
        x = m.x0.copy()
        v = self.prob.v0(m.x0)
        v = np.where(m.constrained, 0.0, v)
        eidx = np.repeat(np.arange(m.Ne)[:, None], self.Q, axis=1)
        e0q = self.prob.e0(self.x0q, eidx)
        rhs = np.einsum("eq,eq,qj->ej", self.mq, e0q, T["Phi"])
        e = np.einsum("eij,ej->ei", self.MEinv, rhs)
        return np.concatenate([x.ravel(), v.ravel(), e.ravel()])

    def energy(self, u):
        """Kinetic 1/2 v^T M_V v and internal 1^T M_E e energies."""
        _, uv, ue = self.split(u)
        ke = 0.5 * float(np.dot(uv, self.mass_v(uv)))
        ie = float(np.sum(self.mass_e(ue)))
        return ke, ie

    def total_mass(self):
        return float(np.sum(self.mq))

    def l1_velocity_error(self, u):
        """int_{Omega(t)} |v_h - v_exact(x)|_2 dx on the current mesh (TG only).

        The pointwise error is the Euclidean length of the velocity error vector; with this
        reading the oracle reproduces the L1 errors of the paper's Taylor-Green table.
        """
        ux, uv, _ = self.split(u)
        J, detJ = self.geometry(ux)
        xq = np.einsum("cen,qn->ceq", self._gather(ux), self.T["W"])
        vq = np.einsum("cen,qn->ceq", self._gather(uv), self.T["W"])
        ve = self.prob.exact_v(xq)
        err = np.sqrt(np.sum((vq - ve) ** 2, axis=0))
        return float(np.einsum("q,eq,eq->", self.T["qw"], detJ, err))

    def dt_estimate(self, u, cfl):
        """Explicit time-step estimate: cfl * min_q h_min / (c_s + 2.5 mu / (rho h_min)).

        h_min = smallest singular value of the reference-to-physical Jacobian divided by
        the kinematic order k.  This is the reading used for the "k x explicit CFL" time
        steps of the benchmark configurations.
        """
        pw = self.pointwise(u)
        sv = np.linalg.svd(pw["J"], compute_uv=False)
        hmin = sv[..., -1] / self.k
        inv_dt = pw["cs"] / hmin + 2.5 * pw["mu"] / (pw["rho"] * hmin * hmin)
        return float(cfl / np.max(inv_dt))
