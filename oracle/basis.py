"""1D bases and quadrature on the reference interval [0, 1] (oracle; test infrastructure only).

The paper uses the mixed space Q_k Q_{k-1}: a continuous degree-k space for position and
velocity and a discontinuous degree-(k-1) space for the specific internal energy
(Sec. 2.1, "Compressible Euler equations and FE discretization").  It does not name the
bases or the quadrature rule; the readings taken here are

* H1: Lagrange polynomials through the k+1 Gauss-Lobatto-Legendre (GLL) points;
* L2: Bernstein polynomials of degree k-1 (a positive partition of unity);
* quadrature: Gauss-Legendre with 2k points per direction (exact to degree 4k-1).
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(k):
    """The k+1 Gauss-Lobatto-Legendre points mapped to [0, 1] (k >= 1).

    Interior points are the roots of P_k' (derivative of the Legendre polynomial),
    polished by Newton's method in extended arithmetic-free FP64.
    """
    if k < 1:
        raise ValueError("k >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    dc = npleg.legder(c)
    ddc = npleg.legder(dc)
    r = np.sort(npleg.legroots(dc).real)
    for _ in range(5):
        r = r - npleg.legval(r, dc) / npleg.legval(r, ddc)
    z = np.concatenate([[-1.0], r, [1.0]])
    return 0.5 * (z + 1.0)


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0, 1]; weights sum to 1."""
    z, w = npleg.leggauss(n)
    return 0.5 * (z + 1.0), 0.5 * w


def lagrange(nodes, t):
    """Values and first derivatives of the Lagrange polynomials through ``nodes``.

    Returns (V, D) with V[p, a] = l_a(t_p), D[p, a] = l_a'(t_p).  Written as the plain
    product formula and its product-rule derivative; works for complex ``t``.
    """
    nodes = np.asarray(nodes, dtype=float)
    t = np.asarray(t)
    n = len(nodes)
    V = np.zeros((t.size, n), dtype=np.result_type(t, float))
    D = np.zeros_like(V)
    for a in range(n):
        den = 1.0
        for b in range(n):
            if b != a:
                den *= nodes[a] - nodes[b]
        for p, tp in enumerate(t.ravel()):
            num = 1.0
            for b in range(n):
                if b != a:
                    num *= tp - nodes[b]
            V[p, a] = num / den
            s = 0.0
            for m in range(n):
                if m == a:
                    continue
                prod = 1.0
                for b in range(n):
                    if b != a and b != m:
                        prod *= tp - nodes[b]
                s += prod
            D[p, a] = s / den
    return V, D


def bernstein(deg, t):
    """Bernstein polynomials of degree ``deg`` on [0, 1]: B[p, j] = C(deg, j) t^j (1-t)^(deg-j)."""
    t = np.asarray(t)
    B = np.zeros((t.size, deg + 1), dtype=np.result_type(t, float))
    for j in range(deg + 1):
        B[:, j] = math.comb(deg, j) * t.ravel() ** j * (1.0 - t.ravel()) ** (deg - j)
    return B


def tensor_tables(dim, k, nq1d=None):
    """Element basis tables at the tensor quadrature points of the reference cube [0,1]^dim.

    Returns a dict with
      qpts  [Q, dim]     reference coordinates of the quadrature points,
      qw    [Q]          reference weights (sum 1),
      W     [Q, Nh]      H1 basis values  w_n(xi_q),
      dW    [Q, Nh, dim] H1 reference gradients d w_n / d xi_a,
      Phi   [Q, Nl]      L2 basis values  phi_j(xi_q),
    with lexicographic ordering (first reference direction fastest) for quadrature
    points, H1 nodes and L2 basis functions alike.  The tables are dense products of the
    1D tables; no sum factorisation is used here.
    """
    if nq1d is None:
        nq1d = 2 * k
    xg, wg = gauss_legendre(nq1d)
    nodes = gll_points(k)
    V1, D1 = lagrange(nodes, xg)
    L1 = bernstein(k - 1, xg)
    nh1, nl1 = k + 1, k
    grids_q = np.array(np.meshgrid(*([np.arange(nq1d)] * dim), indexing="ij")).reshape(dim, -1)
    # lexicographic, first direction fastest: index = i0 + n*i1 + n^2*i2
    def lex(n):
        idx = np.array(np.meshgrid(*([np.arange(n)] * dim), indexing="ij")).reshape(dim, -1)
        order = np.lexsort(idx)  # last row is the primary key -> first direction fastest
        return idx[:, order]
    iq = lex(nq1d)
    ih = lex(nh1)
    il = lex(nl1)
    Q, Nh, Nl = iq.shape[1], ih.shape[1], il.shape[1]
    qpts = np.stack([xg[iq[a]] for a in range(dim)], axis=1)
    qw = np.prod(np.stack([wg[iq[a]] for a in range(dim)], axis=1), axis=1)
    W = np.ones((Q, Nh))
    dW = np.ones((Q, Nh, dim))
    Phi = np.ones((Q, Nl))
    for a in range(dim):
        va = V1[np.ix_(iq[a], ih[a])]
        da = D1[np.ix_(iq[a], ih[a])]
        W *= va
        for b in range(dim):
            dW[:, :, b] *= da if b == a else va
        Phi *= L1[np.ix_(iq[a], il[a])]
    del grids_q
    return dict(qpts=qpts, qw=qw, W=W, dW=dW, Phi=Phi, nq1d=nq1d, k=k, dim=dim,
                gll=nodes, ih=ih, il=il, iq=iq)
