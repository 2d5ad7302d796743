"""Structured box meshes for the oracle (test infrastructure).

Sec. 3 of the paper decomposes the domain into hexahedra (quadrilaterals in
2D) K with skeleton E = E^I (interior faces) u E^B (boundary faces).  The
workloads here are logically Cartesian boxes: cells are numbered
lexicographically with x fastest; each cell is the image of [0,1]^d under the
multilinear (Q1) map through its 2^d vertices.  A periodic direction wraps
the neighbour index; a non-periodic direction produces boundary faces.
"""
import numpy as np


class BoxMesh:
    def __init__(self, dim, n_cells, lo, hi, periodic, vertex_map=None):
        """``vertex_map(X) -> X'`` displaces the (N_vertices, dim) grid points.

        The map is applied to vertices only (Q1 geometry), so every cell stays
        a multilinear image of the reference cell.
        """
        self.dim = int(dim)
        self.n_cells = tuple(int(v) for v in n_cells[:dim])
        self.lo = np.asarray(lo[:dim], dtype=np.float64)
        self.hi = np.asarray(hi[:dim], dtype=np.float64)
        self.periodic = tuple(bool(v) for v in periodic[:dim])
        self.N = int(np.prod(self.n_cells))
        axes = [np.linspace(self.lo[a], self.hi[a], self.n_cells[a] + 1)
                for a in range(self.dim)]
        # vertex grid, x fastest
        grids = np.meshgrid(*axes[::-1], indexing="ij")
        V = np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)
        if vertex_map is not None:
            V = np.asarray(vertex_map(V.copy()), dtype=np.float64)
        self.vertices = V
        self.affine = vertex_map is None

    # -- indexing ---------------------------------------------------------
    def cell_ijk(self, c):
        out = []
        for a in range(self.dim):
            out.append(c % self.n_cells[a])
            c //= self.n_cells[a]
        return out

    def cell_index(self, ijk):
        c = 0
        stride = 1
        for a in range(self.dim):
            c += ijk[a] * stride
            stride *= self.n_cells[a]
        return c

    def neighbor(self, c, direction, side):
        """Cell across face (direction, side) of cell c, or None on E^B.

        side 0 is the face at reference coordinate 0 along ``direction``,
        side 1 the face at reference coordinate 1.
        """
        ijk = self.cell_ijk(c)
        ijk[direction] += 1 if side == 1 else -1
        n = self.n_cells[direction]
        if ijk[direction] < 0 or ijk[direction] >= n:
            if not self.periodic[direction]:
                return None
            ijk[direction] %= n
        return self.cell_index(ijk)

    def cell_vertices(self, c):
        """(2^dim, dim) vertex coordinates, vertex index v = vx + 2 vy + 4 vz.

        The vertex grid has n+1 points per direction, so cells next to a
        periodic wrap keep their own unwrapped shape.
        """
        ijk = self.cell_ijk(c)
        nv = [self.n_cells[a] + 1 for a in range(self.dim)]
        out = np.zeros((2 ** self.dim, self.dim))
        for v in range(2 ** self.dim):
            idx = 0
            stride = 1
            for a in range(self.dim):
                bit = (v >> a) & 1
                idx += (ijk[a] + bit) * stride
                stride *= nv[a]
            out[v] = self.vertices[idx]
        return out

    def volume(self):
        return float(np.prod(self.hi - self.lo))
