"""Cartesian box meshes with a lexicographic high-order node grid (oracle; test infrastructure only).

Element e = ex + nx*ey (+ nx*ny*ez).  Global H1 node (I, J[, K]) on the (k*nx+1) x ... grid
has index I + (k*nx+1)*(J + (k*ny+1)*K).  Element-local H1 node (a, b[, c]) is global
(k*ex+a, k*ey+b[, k*ez+c]).  L2 degrees of freedom are element-major.
The partial-assembly decomposition of the paper (eq. decompose) maps T- to E-vectors by
the element restriction G; here G is the index table ``conn``.
"""
import numpy as np

from .basis import gll_points


class BoxMesh:
    def __init__(self, dim, n, lo, hi, k, free_faces=0):
        """free_faces: bit 2a set = no wall (v . n = 0 not imposed) on the face x_a = lo_a,
        bit 2a+1 = likewise on x_a = hi_a."""
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.lo = np.array(lo[:dim], dtype=float)
        self.hi = np.array(hi[:dim], dtype=float)
        self.k = int(k)
        self.h = (self.hi - self.lo) / np.array(self.n)
        self.ng = tuple(self.k * m + 1 for m in self.n)  # node grid extents
        self.N = int(np.prod(self.ng))
        self.Ne = int(np.prod(self.n))
        self.Nh = (self.k + 1) ** dim
        self.Nl = self.k ** dim
        gll = gll_points(self.k)
        # node coordinates along each direction
        coords = []
        for a in range(dim):
            I = np.arange(self.ng[a])
            ex = np.minimum(I // self.k, self.n[a] - 1)
            loc = I - self.k * ex
            coords.append(self.lo[a] + self.h[a] * (ex + gll[loc]))
        grid = np.meshgrid(*coords, indexing="ij")  # grid[a][I, J, K]
        # flatten with first index fastest
        self.x0 = np.stack([g.transpose(*range(dim)[::-1]).ravel() for g in grid])  # (dim, N)
        gidx = np.array(np.meshgrid(*[np.arange(m) for m in self.ng], indexing="ij"))
        self.node_grid_index = np.stack([g.transpose(*range(dim)[::-1]).ravel() for g in gidx])
        # element -> node map
        eidx = np.array(np.meshgrid(*[np.arange(m) for m in self.n], indexing="ij"))
        eidx = np.stack([g.transpose(*range(dim)[::-1]).ravel() for g in eidx])  # (dim, Ne)
        lidx = np.array(np.meshgrid(*([np.arange(self.k + 1)] * dim), indexing="ij"))
        lidx = np.stack([g.transpose(*range(dim)[::-1]).ravel() for g in lidx])  # (dim, Nh)
        conn = np.zeros((self.Ne, self.Nh), dtype=np.int64)
        stride = 1
        for a in range(dim):
            conn += (self.k * eidx[a][:, None] + lidx[a][None, :]) * stride
            stride *= self.ng[a]
        self.conn = conn
        self.elem_index = eidx
        # wall boundary: component c of node n is constrained when the node lies on a wall
        # face normal to direction c (v . n = 0 on every box face not listed in free_faces)
        cons = np.zeros((dim, self.N), dtype=bool)
        for c in range(dim):
            gi = self.node_grid_index[c]
            wall_lo = not (free_faces >> (2 * c)) & 1
            wall_hi = not (free_faces >> (2 * c + 1)) & 1
            cons[c] = ((gi == 0) & wall_lo) | ((gi == self.ng[c] - 1) & wall_hi)
        self.constrained = cons  # (dim, N)

    def element_centers(self):
        return self.lo[:, None] + self.h[:, None] * (self.elem_index + 0.5)
