"""Derivatives and solvers of the implicit stage (oracle; test infrastructure only).

* Jacobian actions by the complex step: J dk = Im R(k + i h dk) / h.  Every operation in
  the residual is analytic (polynomials, division, sqrt, tanh, real powers), so this is
  the exact directional derivative up to rounding; it replaces the paper's automatic
  differentiation of the quadrature-point kernel (eq. pa_jac_action).  The oracle holds
  no hand-written tangent.
* Transpose actions J^T y from complex-step columns, compressed by a colouring of the
  columns that reach disjoint rows (vjp_colored).
* The explicit RK2-average step that Sec. 4 uses as its RK2 reference (rk2avg_step).
* Jacobi preconditioned CG (Sec. 2.2 mass solves), restarted flexible GMRES and inexact
  Newton with a backtracking line search that rejects steps producing a non-positive
  Jacobian determinant (Sec. 3.5, eq. newton_linear).
* The implicit midpoint rule: k = f(u + dt/2 k), u+ = u + dt k, and the singly diagonally
  implicit Runge-Kutta steps SD3 / SD4 of Sec. 4 (each implicit stage is one solve of the
  same stage residual with tau = gamma dt).
"""
import numpy as np

CS_H = 1.0e-30


def jvp_cs(fun, x, dx, h=CS_H):
    """Directional derivative of ``fun`` at x along dx by the complex step."""
    return np.imag(fun(x + 1j * h * dx)) / h


def jvp_fd(fun, x, dx, eps=1.0e-7):
    """Central finite difference (fun(x + eps dx) - fun(x - eps dx)) / (2 eps)."""
    return (fun(x + eps * dx) - fun(x - eps * dx)) / (2.0 * eps)


def dense_jacobian(fun, x):
    """Dense Jacobian by complex-step columns (brute force; tiny problems only)."""
    n = x.size
    cols = []
    for j in range(n):
        ej = np.zeros(n)
        ej[j] = 1.0
        cols.append(jvp_cs(fun, x, ej))
    return np.stack(cols, axis=1)


def pcg(apply, b, diag, rtol=1e-12, maxit=1000):
    """Jacobi-preconditioned conjugate gradients on an SPD operator."""
    x = np.zeros_like(b)
    r = b.copy()
    z = r / diag
    p = z.copy()
    rz = np.dot(r, z)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    it = 0
    while it < maxit:
        if np.linalg.norm(r) <= rtol * nb:
            break
        Ap = apply(p)
        alpha = rz / np.dot(p, Ap)
        x += alpha * p
        r -= alpha * Ap
        z = r / diag
        rz_new = np.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, np.linalg.norm(r) / nb


def fgmres(apply, b, precond, restart=30, rtol=1e-6, maxit=60, x0=None):
    """Right-preconditioned restarted flexible GMRES (Arnoldi with modified Gram-Schmidt).

    Returns (x, iterations, final relative residual estimate).
    """
    n = b.size
    x = np.zeros(n) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    total = 0
    rel = 1.0
    while total < maxit:
        r = b - apply(x) if total > 0 or x0 is not None else b.copy()
        beta = np.linalg.norm(r)
        rel = beta / nb
        if rel <= rtol:
            break
        m = min(restart, maxit - total)
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        cs = np.zeros(m)
        sn = np.zeros(m)
        j_end = 0
        for j in range(m):
            Z[j] = precond(V[j])
            wv = apply(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(wv, V[i])
                wv = wv - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(wv)
            if H[j + 1, j] > 0:
                V[j + 1] = wv / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            rel = abs(g[j + 1]) / nb
            if rel <= rtol or total >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + Z[:j_end].T @ y
        if rel <= rtol:
            break
    return x, total, rel


class NewtonOptions:
    def __init__(self, tol=1e-10, max_newton=30, restart=30, gmres_rtol=1e-6,
                 gmres_maxit=60, max_halvings=10):
        self.tol, self.max_newton = tol, max_newton
        self.restart, self.gmres_rtol, self.gmres_maxit = restart, gmres_rtol, gmres_maxit
        self.max_halvings = max_halvings


class NewtonFailure(RuntimeError):
    def __init__(self, kind, msg):
        super().__init__(msg)
        self.kind = kind


def block_preconditioner(hyd):
    """P^-1 = diag(I, Mhat_V^-1, M_E^-1): the mass-only block preconditioner (exact solves)."""
    def apply(r):
        rx, rv, re = hyd.split(r)
        return np.concatenate([rx, hyd.mass_v_solve(rv), hyd.mass_e_inv(re)])
    return apply


def newton_stage(hyd, u, tau, k0, opts=None, stats=None):
    """Solve R(k; tau, u) = 0 by inexact Newton-FGMRES with the detJ line search.

    Converged when ||R(k)|| <= tol ||R(0; tau, u)||.
    """
    opts = opts or NewtonOptions()
    R = lambda k: hyd.residual(k, u, tau)
    r0 = np.linalg.norm(R(np.zeros_like(u)))
    prec = block_preconditioner(hyd)
    k = k0.copy()
    hist = []
    gm_total = 0
    for it in range(opts.max_newton + 1):
        r = R(k)
        nr = np.linalg.norm(r)
        hist.append(nr / r0)
        if nr <= opts.tol * r0:
            break
        if it == opts.max_newton:
            raise NewtonFailure("ENOCONV", "Newton did not converge")
        J = lambda dk, k=k: jvp_cs(R, k, dk)
        dk, its, _ = fgmres(J, -r, prec, opts.restart, opts.gmres_rtol, opts.gmres_maxit)
        gm_total += its
        alpha = 1.0
        for _ in range(opts.max_halvings + 1):
            if hyd.min_detj(u + tau * (k + alpha * dk)) > 0.0:
                break
            alpha *= 0.5
        else:
            raise NewtonFailure("ETANGLED", "line search could not keep detJ > 0")
        k = k + alpha * dk
    if stats is not None:
        stats.update(newton=len(hist) - 1, gmres=gm_total, hist=hist)
    return k


def implicit_midpoint_step(hyd, u, dt, k_guess, opts=None, stats=None):
    """One implicit midpoint step: k = f(u + dt/2 k), returns (u + dt k, k)."""
    k = newton_stage(hyd, u, 0.5 * dt, k_guess, opts, stats)
    return u + dt * k, k


def plain_guess(hyd, u, history):
    """Plain initial iterate: explicit rate at the first step, then k_{n-1}, then 2 k_{n-1} - k_{n-2}."""
    if len(history) == 0:
        return hyd.rate(u)
    if len(history) == 1:
        return history[-1].copy()
    return 2.0 * history[-1] - history[-2]


def run_midpoint(hyd, u0, dt, steps, opts=None):
    """Run ``steps`` implicit midpoint steps from u0 with the plain guess; returns states and stats."""
    u = u0.copy()
    hist_k, states, allstats = [], [u.copy()], []
    for _ in range(steps):
        st = {}
        g = plain_guess(hyd, u, hist_k)
        u, k = implicit_midpoint_step(hyd, u, dt, g, opts, st)
        hist_k.append(k)
        states.append(u.copy())
        allstats.append(st)
    return states, hist_k, allstats


# ---- SDIRK steps (Sec. 4: SD2 = implicit midpoint, SD3, SD4) ------------------------------

def sdirk_tableau(scheme):
    """Butcher tableau (A, b) of the singly diagonally implicit schemes named in Sec. 4.

    sd2: implicit midpoint, one stage with gamma = 1/2.
    sd3: three-stage, third-order, L-stable SDIRK of Alexander (1977): gamma is the root in
         (1/6, 1/2) of gamma^3 - 3 gamma^2 + 3/2 gamma - 1/6 = 0, c2 = (1 + gamma)/2, and the
         last row (stiffly accurate) b1 = -(6 gamma^2 - 16 gamma + 1)/4,
         b2 = (6 gamma^2 - 20 gamma + 5)/4, b3 = gamma.
    sd4: three-stage, fourth-order SDIRK of Crouzeix (1975): gamma = 1/2 + cos(pi/18)/sqrt(3),
         c = (gamma, 1/2, 1 - gamma), a21 = 1/2 - gamma, a31 = 2 gamma, a32 = 1 - 4 gamma,
         b1 = b3 = 1/(6 (1 - 2 gamma)^2), b2 = 1 - 2 b1.
    """
    if scheme == "sd2":
        return np.array([[0.5]]), np.array([1.0])
    if scheme == "sd3":
        roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
        g = float([r.real for r in roots if abs(r.imag) < 1e-12 and 1.0 / 6.0 < r.real < 0.5][0])
        c2 = 0.5 * (1.0 + g)
        b1 = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0
        b2 = (6.0 * g * g - 20.0 * g + 5.0) / 4.0
        A = np.array([[g, 0.0, 0.0], [c2 - g, g, 0.0], [b1, b2, g]])
        return A, np.array([b1, b2, g])
    if scheme == "sd4":
        g = 0.5 + np.cos(np.pi / 18.0) / np.sqrt(3.0)
        b1 = 1.0 / (6.0 * (1.0 - 2.0 * g) ** 2)
        A = np.array([[g, 0.0, 0.0], [0.5 - g, g, 0.0], [2.0 * g, 1.0 - 4.0 * g, g]])
        return A, np.array([b1, 1.0 - 2.0 * b1, b1])
    raise ValueError(scheme)


def sdirk_step(hyd, u, dt, scheme, k_guess=None, opts=None, stats=None):
    """One SDIRK step: stage i solves k_i = f(u + dt sum_{j<i} a_ij k_j + dt a_ii k_i), i.e.
    R(k_i; a_ii dt, u + dt sum_{j<i} a_ij k_j) = 0; then u+ = u + dt sum_i b_i k_i.

    Newton starts stage 1 from k_guess (None: the explicit rate at u) and stage i > 1 from
    k_{i-1}.  Returns (u+, [k_1, ...])."""
    A, b = sdirk_tableau(scheme)
    ks = []
    for i in range(len(b)):
        ubase = u + dt * sum(A[i, j] * ks[j] for j in range(i)) if i else u.copy()
        if i:
            g0 = ks[-1]
        else:
            g0 = hyd.rate(u) if k_guess is None else k_guess
        st = {} if stats is not None else None
        k = newton_stage(hyd, ubase, A[i, i] * dt, g0, opts, st)
        if stats is not None:
            for key, v in st.items():
                if isinstance(v, (int, float)):
                    stats[key] = stats.get(key, 0) + v
        ks.append(k)
    return u + dt * sum(bi * ki for bi, ki in zip(b, ks)), ks


# ---- Newton-based step-size control (Sec. 4, "Implicit time step control") ------------------

def adaptive_run(hyd, u0, tf, fscfl, scheme="sd2", opts=None, max_reject=60, zero_guess=False):
    """Integrate to tf with the paper's step control: the first step is fscfl times the explicit
    estimate; after a step whose stages needed at most one Newton iteration each the next step
    grows by 5 %; two or three keep it; a step needing four or more in some stage (or failing)
    is rejected and repeated with 85 % of its size.  Newton iterations are counted as updates
    (the maximum over the stages).  Stage 1 of every step starts from the explicit rate (first
    step) or the last stage rate of the previous step; with zero_guess every stage solve starts
    from k = 0 instead (the paper's solver defaults of Sec. 3.5 leave the initial iterate to the
    Newton solver, read here as its default zero iterate).  Returns (u, accepted steps, rejected)."""
    u = u0.copy()
    dt = hyd.dt_estimate(u, fscfl)
    t, steps, rejected, kg = 0.0, 0, 0, None
    while t < tf - 1e-12:
        dtt = min(dt, tf - t)
        g = np.zeros_like(u) if zero_guess else (hyd.rate(u) if kg is None else kg)
        st = {}
        try:
            A, b = sdirk_tableau(scheme)
            ks, nmax = [], 0
            for i in range(len(b)):
                ubase = u + dtt * sum(A[i, j] * ks[j] for j in range(i)) if i else u
                sti = {}
                k0 = np.zeros_like(u) if zero_guess else (ks[-1] if i else g)
                ks.append(newton_stage(hyd, ubase, A[i, i] * dtt, k0, opts, sti))
                nmax = max(nmax, sti["newton"])
            ok = nmax < 4
        except NewtonFailure:
            ok = False
        if not ok:
            rejected += 1
            if rejected > max_reject:
                raise NewtonFailure("ENOCONV", "step size control: too many rejections")
            dt = 0.85 * dtt
            continue
        u = u + dtt * sum(bi * ki for bi, ki in zip(b, ks))
        kg = ks[-1]
        t += dtt
        steps += 1
        dt = 1.05 * dtt if nmax <= 1 else dtt
    return u, steps, rejected


def vjp_colored(hyd, fun, x, y, h=CS_H):
    """Transpose action J^T y of the Jacobian of ``fun`` (the stage residual of ``hyd``) at x.

    The Jacobian of the partial-assembly residual couples a column only to the rows of the
    elements that hold it (eq. pa_jac_action and its transpose): H1 node p reaches the H1 rows
    of nodes within k grid steps of p in every direction and the L2 rows of the elements whose
    node box contains p; an L2 degree of freedom of element e reaches the H1 rows of e's nodes
    and e's own L2 rows.  Columns whose node indices agree modulo 2k+1 (H1), or whose element
    indices agree modulo 3 with the same local index (L2), reach disjoint sets of rows, so one
    complex-step Jacobian action along their sum returns each of their columns intact
    (Curtis-Powell-Reid compression).  Entry j of J^T y is then the sum over j's rows of
    (J e_class)_i y_i.  Exact to rounding, like the columns it is built from.
    """
    m = hyd.mesh
    d, k, N = hyd.dim, m.k, m.N
    ng = np.array(m.ng)
    ne = np.array(m.n)
    P = 2 * k + 1
    nh = hyd.nh1
    stride = np.cumprod([1] + list(ng[:-1]))
    qg = m.node_grid_index                    # (d, N): grid coordinates of every node
    eg = m.elem_index                         # (d, Ne): element coordinates
    # every block row: H1 rows (x, then v; component-major) carry a node, L2 rows an element
    h1_node = np.tile(np.arange(N), 2 * d)    # node of H1 row r
    l2_elem = np.repeat(np.arange(m.Ne), m.Nl)
    out = np.zeros(x.size)
    y_h1, y_l2 = y[:2 * nh], y[2 * nh:]

    def accumulate(g, col_h1, col_l2):
        """Add g_i y_i to the column associated with each row (-1: row reached by none)."""
        g_h1, g_l2 = g[:2 * nh], g[2 * nh:]
        assert np.all(g_h1[col_h1 < 0] == 0.0) and np.all(g_l2[col_l2 < 0] == 0.0)
        sel = col_h1 >= 0
        np.add.at(out, col_h1[sel], g_h1[sel] * y_h1[sel])
        sel = col_l2 >= 0
        np.add.at(out, col_l2[sel], g_l2[sel] * y_l2[sel])

    # H1 columns: field f (0 = x, 1 = v), component c, node residues o modulo P
    for f in range(2):
        for c in range(d):
            for o in np.ndindex(*([P] * d)):
                o = np.array(o)
                members = np.all(qg % P == o[:, None], axis=0)
                if not members.any():
                    continue
                base = (f * d + c) * N
                dx = np.zeros(x.size)
                dx[base + np.nonzero(members)[0]] = 1.0
                g = jvp_cs(fun, x, dx, h)
                # H1 rows: the class member nearest to the row's node in every direction
                q = qg[:, h1_node]
                p = o[:, None] + P * np.round((q - o[:, None]) / P).astype(np.int64)
                ok = np.all((np.abs(q - p) <= k) & (p >= 0) & (p < ng[:, None]), axis=0)
                col_h1 = np.where(ok, base + (p * stride[:, None]).sum(axis=0), -1)
                # L2 rows: the class member inside the row element's node box
                lo = k * eg[:, l2_elem]
                p = lo + (o[:, None] - lo) % P
                ok = np.all((p - lo <= k) & (p < ng[:, None]), axis=0)
                col_l2 = np.where(ok, base + (p * stride[:, None]).sum(axis=0), -1)
                accumulate(g, col_h1, col_l2)
    # L2 columns: local index l, element residues o modulo 3
    for l in range(m.Nl):
        for o in np.ndindex(*([3] * d)):
            o = np.array(o)
            members = np.all(eg % 3 == o[:, None], axis=0)
            if not members.any():
                continue
            dx = np.zeros(x.size)
            dx[2 * nh + np.nonzero(members)[0] * m.Nl + l] = 1.0
            g = jvp_cs(fun, x, dx, h)
            # H1 rows: along each direction the elements holding the node are
            # floor(q/k) and, on an element boundary, the one before; one of them is in the class
            q = qg[:, h1_node]
            e_hi = np.minimum(q // k, ne[:, None] - 1)
            e_lo = np.maximum((q + k - 1) // k - 1, 0)
            e_pick = np.where(e_hi % 3 == o[:, None], e_hi, np.where(e_lo % 3 == o[:, None], e_lo, -1))
            ok = np.all((e_pick >= 0) & (k * e_pick <= q) & (q <= k * e_pick + k), axis=0)
            estr = np.cumprod([1] + list(ne[:-1]))
            e_col = (np.where(e_pick >= 0, e_pick, 0) * estr[:, None]).sum(axis=0)
            col_h1 = np.where(ok, 2 * nh + e_col * m.Nl + l, -1)
            # L2 rows: only the element's own
            ok = np.all(eg[:, l2_elem] % 3 == o[:, None], axis=0)
            col_l2 = np.where(ok, 2 * nh + l2_elem * m.Nl + l, -1)
            accumulate(g, col_h1, col_l2)
    return out


def rk2avg_step(hyd, u, dt):
    """One explicit step of the RK2-average scheme (Sec. 4 names it RK2 and defines it by
    reference to Dobrev et al. 2012, Sec. 7.1; restated here from that published method).

    For dv/dt = -M_V^-1 F 1, de/dt = M_E^-1 (F^T v + b), dx/dt = v:
      half step:  v_h = v + dt/2 a(u),  e_h = e + dt/2 M_E^-1 (F(u)^T v_h + b(x)),
                  x_h = x + dt/2 v_h;
      full step:  v+ = v + dt a(u_h),  vbar = (v + v+)/2,
                  e+ = e + dt M_E^-1 (F(u_h)^T vbar + b(x_h)),  x+ = x + dt vbar,
    where a(w) = -Mhat^-1 P_u F(w) 1 (wall rows held at zero).  Using the averaged velocity in
    the full step makes the total energy change exactly dt 1^T b(x_h).
    """
    x, v, e = hyd.split(u)

    def accel(w):
        F1, _ = hyd.force(w)
        return -hyd.mass_v_solve(np.where(hyd.cons, 0.0, F1))

    def erate(w, vt):
        return hyd.mass_e_inv(hyd.force_transpose(w, vt) + hyd.energy_source(hyd.split(w)[0]))

    vh = v + 0.5 * dt * accel(u)
    eh = e + 0.5 * dt * erate(u, vh)
    xh = x + 0.5 * dt * vh
    uh = np.concatenate([xh, vh, eh])
    v1 = v + dt * accel(uh)
    vb = 0.5 * (v + v1)
    e1 = e + dt * erate(uh, vb)
    x1 = x + dt * vb
    return np.concatenate([x1, v1, e1])
