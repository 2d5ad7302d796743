"""Adaptive quadrilateral meshes with hanging nodes (oracle; test infrastructure).

TEST INFRASTRUCTURE ONLY.  Sec. 4 of the paper repeats the lid-driven cavity
with adaptive meshes: in every cell K the refinement indicator

    eta_K = diam(K)^2 ||omega||^2_K      (omega the vorticity of u)

ranks the cells, the 10 % with the largest indicator are refined and the
30 % with the smallest coarsened, with a smallest and a largest admissible
element size; the remeshing is repeated every 1000 steps (and every 50
steps while the largest velocity change of one step exceeds 1e-2).  The
resulting meshes are non-conforming: a face of a cell can meet two cells of
half its size (a hanging node in the middle of the face).

This module holds, in 2D:

* ``QuadForest`` - a quadtree over every cell of a base box grid, leaves
  2:1 balanced across faces, refined and coarsened by one level per call;
* ``AdaptiveDisc`` - the pressure mass matrix and the SIP form a_p of Sec. 3
  on such a mesh, and the velocity mass, SIP (eq. bilin_diff, Dirichlet
  walls) and Lax-Friedrichs advection (eq. trilinear) forms, with the face
  integrals of a face shared by one coarse and two fine cells taken on each
  fine face; the indicator eta_K;
* ``mark`` - the fixed-fraction marking with the size limits;
* ``transfer`` - velocity and pressure fields from one mesh to the adapted
  one (refinement: exact interpolation of the parent polynomial; coarsening:
  the L2 projection onto the parent).

Readings (the paper names the strategy, not these details):

* Meshes are 2:1 balanced across faces, the usual constraint of such
  quadtree meshes: a face carries at most one hanging node.
* Cell order: by base tree (x fastest), then by the Morton index (x bit
  below y bit) of the cell's lower-left corner at the finest level.
* On a face between a coarse cell and two fine ones every face integral is
  the sum over the two fine faces, each with the Gauss rule of the fine
  cell, the coarse traces evaluated at those points (exact: the integrands
  are polynomials of degree 2 n_p - 2 on each fine face).
* SIP penalty on a face: the average of the two cells' k^2 |Gamma_K|/|K|
  (pressure) or (k+1)^2 |Gamma_K|/|K| (velocity), |Gamma_K| the cell's own
  full face (the conforming reading; on a rectangle |Gamma_K|/|K| = 1/h_a).
  Pressure faces on the boundary carry no term (homogeneous Neumann), as on
  the conforming meshes; velocity boundary faces the Dirichlet terms of the
  conforming oracle.
* The Lax-Friedrichs speed on a coarse-fine face is taken pointwise at the
  fine faces' Gauss points from the two traces there, as on conforming
  faces.
* diam(K) in eta_K is the cell's diagonal; the size limits H_min, H_max are
  on the edge length, as the paper's H of its uniform meshes.
* Marking: the floor(0.1 N) cells of largest eta (ties: lower cell index
  first) are flagged for refinement unless their children would be smaller
  than H_min; of the remaining cells, the floor(0.3 N) of smallest eta are
  flagged for coarsening unless their parent would be larger than H_max.
  Refinement spreads to coarser face neighbours until the refined mesh is
  balanced; then a family of four leaves is coarsened when all four are
  flagged, none is refined, and no face neighbour would end finer than the
  family's leaves (checked with the final levels, dropping families until
  no more is dropped).
"""
import numpy as np
import scipy.sparse as sp

from .basis import gauss_legendre_01, lagrange_values, lagrange_derivatives, tensor


def morton2(x, y, bits):
    """Interleave the bits of x (even positions) and y (odd positions)."""
    m = 0
    for b in range(bits):
        m |= ((x >> b) & 1) << (2 * b)
        m |= ((y >> b) & 1) << (2 * b + 1)
    return m


class QuadForest:
    """Leaves (level, i, j) of quadtrees rooted at the cells of a box grid.

    A leaf of level l covers [i, i+1] x [j, j+1] in units of the base cell
    size divided by 2^l; i runs over 0 .. n_cells[0] 2^l - 1.
    """

    def __init__(self, n_cells, lo, hi, periodic, max_level, leaves=None):
        self.n_cells = (int(n_cells[0]), int(n_cells[1]))
        self.lo = np.asarray(lo[:2], dtype=np.float64)
        self.hi = np.asarray(hi[:2], dtype=np.float64)
        self.periodic = (bool(periodic[0]), bool(periodic[1]))
        self.max_level = int(max_level)
        self.H = (self.hi - self.lo) / np.asarray(self.n_cells, dtype=np.float64)
        if leaves is None:
            leaves = [(0, i, j) for j in range(self.n_cells[1]) for i in range(self.n_cells[0])]
        self.leaves = sorted((tuple(int(v) for v in c) for c in leaves), key=self._key)
        self.index = {c: n for n, c in enumerate(self.leaves)}
        self.N = len(self.leaves)
        self.dim = 2

    def _key(self, c):
        l, i, j = c
        L = self.max_level
        tx, ty = i >> l, j >> l
        li, lj = (i - (tx << l)) << (L - l), (j - (ty << l)) << (L - l)
        return (ty * self.n_cells[0] + tx, morton2(li, lj, L))

    # -- geometry ---------------------------------------------------------
    def size(self, c):
        """Edge lengths (h_x, h_y) of leaf number c."""
        l = self.leaves[c][0]
        return self.H / (1 << l)

    def origin(self, c):
        l, i, j = self.leaves[c]
        h = self.H / (1 << l)
        return self.lo + np.array([i, j], dtype=np.float64) * h

    # -- neighbours -------------------------------------------------------
    def _wrap(self, l, i, j):
        n = (self.n_cells[0] << l, self.n_cells[1] << l)
        ij = [i, j]
        for a in range(2):
            if ij[a] < 0 or ij[a] >= n[a]:
                if not self.periodic[a]:
                    return None
                ij[a] %= n[a]
        return (l, ij[0], ij[1])

    def neighbours(self, c, a, s):
        """Leaves across face (direction a, side s) of leaf c.

        Returns ('B',) on the boundary, ('C', nb) for a leaf of the same
        level, ('c', nb, sub) for a coarser leaf (c's face is half ``sub`` of
        nb's face along the tangential direction), ('f', [nb0, nb1]) for two
        finer leaves (tangential halves 0 and 1 of c's face).
        """
        l, i, j = self.leaves[c]
        d = [0, 0]
        d[a] = 1 if s == 1 else -1
        pos = self._wrap(l, i + d[0], j + d[1])
        if pos is None:
            return ("B",)
        if pos in self.index:
            return ("C", self.index[pos])
        if l > 0:
            par = (l - 1, pos[1] >> 1, pos[2] >> 1)
            if par in self.index:
                t = 1 - a
                sub = (pos[1 + t]) & 1
                return ("c", self.index[par], sub)
        # two children of pos adjacent to the face
        kids = []
        for h in (0, 1):
            ch = [2 * pos[1], 2 * pos[2]]
            ch[a] += 0 if s == 1 else 1   # the child column touching c
            ch[1 - a] += h
            key = (l + 1, ch[0], ch[1])
            if key not in self.index:
                raise ValueError("mesh is not 2:1 balanced")
            kids.append(self.index[key])
        return ("f", kids)

    def is_balanced(self):
        for c in range(self.N):
            for a in range(2):
                for s in (0, 1):
                    self.neighbours(c, a, s)
        return True

    # -- adaptation -------------------------------------------------------
    def adapt(self, flags):
        """New forest: flags > 0 refine, < 0 coarsen (families of four
        flagged leaves), then refinement spread until balanced."""
        flags = np.asarray(flags)
        lev = [c[0] for c in self.leaves]
        refine = set(c for c in range(self.N) if flags[c] > 0 and lev[c] < self.max_level)

        def face_leaves(c):
            out = []
            for a in range(2):
                for s in (0, 1):
                    nb = self.neighbours(c, a, s)
                    if nb[0] in ("C", "c"):
                        out.append(nb[1])
                    elif nb[0] == "f":
                        out.extend(nb[1])
            return out

        work = list(refine)
        while work:
            c = work.pop()
            for nb in face_leaves(c):
                if lev[nb] < lev[c] and nb not in refine:
                    refine.add(nb)
                    work.append(nb)
        # families whose four leaves are all flagged for coarsening
        fam = {}
        for c in range(self.N):
            l, i, j = self.leaves[c]
            if l > 0 and flags[c] < 0 and c not in refine:
                fam.setdefault((l - 1, i >> 1, j >> 1), []).append(c)
        fams = {par: kids for par, kids in fam.items() if len(kids) == 4}
        # drop every family one of whose face neighbours would end finer than
        # the family's leaves, with the final levels, until none is dropped
        while True:
            member = {c: par for par, kids in fams.items() for c in kids}

            def final(c):
                return lev[c] + (1 if c in refine else 0) - (1 if c in member else 0)

            drop = [par for par, kids in fams.items()
                    if any(final(nb) > par[0] + 1 for c in kids for nb in face_leaves(c)
                           if member.get(nb) != par)]
            if not drop:
                break
            for par in drop:
                del fams[par]
        coarsen = {c: par for par, kids in fams.items() for c in kids}
        new = []
        seen = set()
        for c in range(self.N):
            l, i, j = self.leaves[c]
            if c in refine:
                for dj in (0, 1):
                    for di in (0, 1):
                        new.append((l + 1, 2 * i + di, 2 * j + dj))
            elif c in coarsen:
                par = coarsen[c]
                if par not in seen:
                    seen.add(par)
                    new.append(par)
            else:
                new.append((l, i, j))
        return QuadForest(self.n_cells, self.lo, self.hi, self.periodic, self.max_level, new)


# ---------------------------------------------------------------------------
def mark(eta, forest, refine_frac=0.1, coarsen_frac=0.3, h_min=0.0, h_max=np.inf):
    """Fixed-fraction marking (Sec. 4): +1 refine, -1 coarsen, 0 keep."""
    eta = np.asarray(eta, dtype=np.float64)
    N = forest.N
    flags = np.zeros(N, dtype=np.int64)
    nr = int(np.floor(refine_frac * N + 1e-12))
    nc = int(np.floor(coarsen_frac * N + 1e-12))
    order = sorted(range(N), key=lambda c: (-eta[c], c))
    top = set(order[:nr])
    for c in order[:nr]:
        if 0.5 * float(np.max(forest.size(c))) >= h_min * (1.0 - 1e-12) \
                and forest.leaves[c][0] < forest.max_level:
            flags[c] = 1
    asc = [c for c in sorted(range(N), key=lambda c: (eta[c], c)) if c not in top]
    for c in asc[:nc]:
        if forest.leaves[c][0] > 0 and 2.0 * float(np.max(forest.size(c))) <= h_max * (1.0 + 1e-12):
            flags[c] = -1
    return flags


# ---------------------------------------------------------------------------
class AdaptiveDisc:
    """Pressure forms (degree k-1, n_p = k Gauss nodes) and the velocity
    indicator (degree k, n = k+1 nodes) on a QuadForest; all cells are
    axis-aligned rectangles, so every map is affine and diagonal."""

    def __init__(self, forest, k, pen_p=1.0, pen_u=1.0, nu=1.0, c=1.0e3):
        self.f = forest
        self.mesh = forest
        self.dim = 2
        self.k = int(k)
        self.pen_p = float(pen_p)
        self.pen_u = float(pen_u)
        self.nu = float(nu)
        self.c = float(c)
        self.n = self.k + 1
        self.n_p = self.k
        self.zu, self.wu = gauss_legendre_01(self.n)
        self.zp, self.wp = gauss_legendre_01(self.n_p)
        self.nbu = self.n ** 2
        self.nbp = self.n_p ** 2
        self.Nc = forest.N
        self.N_p = self.Nc * self.nbp
        self.N_u = 2 * self.Nc * self.nbu
        self.n_scalar = self.Nc * self.nbu

    # tabulation of the 2D Lagrange basis on ``nodes`` at reference points
    # (xr, yr) of a cell of size h: values and physical gradients
    @staticmethod
    def _tab(nodes, xr, yr, h):
        Vx, Vy = lagrange_values(nodes, xr), lagrange_values(nodes, yr)
        Dx, Dy = lagrange_derivatives(nodes, xr), lagrange_derivatives(nodes, yr)
        n = len(nodes)
        idx = np.arange(n * n)
        ix, iy = idx % n, idx // n
        V = Vx[:, ix] * Vy[:, iy]
        G = np.stack([Dx[:, ix] * Vy[:, iy] / h[0], Vx[:, ix] * Dy[:, iy] / h[1]], axis=2)
        return V, G

    def _sigma(self, c, a):
        return self.k ** 2 * self.pen_p / float(self.f.size(c)[a])

    def mass_p(self, cells=None):
        """Pressure mass matrix; with ``cells`` only those cells' rows (as in
        every form taking ``cells``: the other rows may be incomplete)."""
        rows, cols, vals = [], [], []
        for c in (range(self.Nc) if cells is None else cells):
            h = self.f.size(c)
            W = np.kron(self.wp, self.wp) * h[0] * h[1]
            xr = np.tile(self.zp, self.n_p)
            yr = np.repeat(self.zp, self.n_p)
            V, _ = self._tab(self.zp, xr, yr, h)
            blk = V.T @ (W[:, None] * V)
            r0 = c * self.nbp
            rr, cc = np.meshgrid(np.arange(self.nbp) + r0, np.arange(self.nbp) + r0, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.N_p, self.N_p)).tocsr()

    def _face_points(self, c, a, s, sub=None):
        """Reference points on face (a, s) of c at the n_p Gauss points of the
        whole face (sub None) or of its tangential half ``sub``."""
        t = self.zp if sub is None else 0.5 * (sub + self.zp)
        pts = np.zeros((self.n_p, 2))
        pts[:, a] = float(s)
        pts[:, 1 - a] = t
        return pts

    def sip_p(self, cells=None):
        """a_p(psi_j, psi_i): cell terms, then every interior face once, a
        coarse-fine face as two fine faces."""
        nb = self.nbp
        rows, cols, vals = [], [], []

        def add(rc, cc_, blk):
            r0, c0 = rc * nb, cc_ * nb
            rr, cc = np.meshgrid(np.arange(nb) + r0, np.arange(nb) + c0, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())

        xr = np.tile(self.zp, self.n_p)
        yr = np.repeat(self.zp, self.n_p)
        for c in (range(self.Nc) if cells is None else cells):
            h = self.f.size(c)
            W = np.kron(self.wp, self.wp) * h[0] * h[1]
            _, G = self._tab(self.zp, xr, yr, h)
            add(c, c, sum(G[:, :, d].T @ (W[:, None] * G[:, :, d]) for d in range(2)))
        # interior faces once (a coarse-fine face from its fine side); no
        # pressure boundary term
        for a, c, s, other, sub in self._interfaces(cells):
            h = self.f.size(c)
            ho = self.f.size(other)
            pc = self._face_points(c, a, s)
            po = self._face_points(other, a, 1 - s, sub)
            Vc, Gc = self._tab(self.zp, pc[:, 0], pc[:, 1], h)
            Vo, Go = self._tab(self.zp, po[:, 0], po[:, 1], ho)
            dS = self.wp * float(h[1 - a])       # the (smaller or equal) face of c
            nvec = np.zeros(2)
            nvec[a] = 1.0 if s == 1 else -1.0
            C = 0.5 * (self._sigma(c, a) + self._sigma(other, a))
            tabs = [(c, Vc, Gc, nvec), (other, Vo, Go, -nvec)]
            for (ct, Vt, Gt, nt) in tabs:
                for (cs, Vs, Gs, ns) in tabs:
                    avg_trial = 0.5 * np.einsum("qjd,d->qj", Gs, nt)
                    avg_test = 0.5 * np.einsum("qid,d->qi", Gt, ns)
                    nn = float(ns @ nt)
                    blk = (-(Vt * dS[:, None]).T @ avg_trial
                           - (avg_test * dS[:, None]).T @ Vs
                           + (Vt * (C * nn * dS)[:, None]).T @ Vs)
                    add(ct, cs, blk)
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.N_p, self.N_p)).tocsr()

    # ------------------------------------------------------------------
    # velocity forms (one scalar component, degree k, n = k + 1 nodes)
    # ------------------------------------------------------------------
    def _assemble(self, blocks, nb, n):
        rows, cols, vals = [], [], []
        for rc, cc_, blk in blocks:
            rr, cc = np.meshgrid(np.arange(nb) + rc * nb, np.arange(nb) + cc_ * nb, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(blk.ravel())
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n)).tocsr()

    def _cell_tab_u(self, c):
        h = self.f.size(c)
        xr, yr = np.tile(self.zu, self.n), np.repeat(self.zu, self.n)
        V, G = self._tab(self.zu, xr, yr, h)
        return V, G, np.kron(self.wu, self.wu) * h[0] * h[1]

    def _interfaces(self, cells=None):
        """Every interior face once: (a, c, s, other, sub) with c the cell
        whose face (a, s) carries the quadrature (the finer or, on a
        same-level face, the side-0 cell) and sub the half of the other
        cell's face (None when conforming).  With ``cells``: only the faces
        touching those cells."""
        if cells is not None:
            seen = set()
            for c in cells:
                for a in range(2):
                    for s in (0, 1):
                        nbr = self.f.neighbours(c, a, s)
                        if nbr[0] == "C":
                            key = (a, c, 1, nbr[1], None) if s == 1 else (a, nbr[1], 1, c, None)
                        elif nbr[0] == "c":
                            key = (a, c, s, nbr[1], nbr[2])
                        elif nbr[0] == "f":
                            for h, o in enumerate(nbr[1]):
                                key = (a, o, 1 - s, c, h)
                                if key not in seen:
                                    seen.add(key)
                                    yield key
                            continue
                        else:
                            continue
                        if key not in seen:
                            seen.add(key)
                            yield key
            return
        for c in range(self.Nc):
            for a in range(2):
                for s in (0, 1):
                    nbr = self.f.neighbours(c, a, s)
                    if nbr[0] == "C" and s == 1:
                        yield a, c, s, nbr[1], None
                    elif nbr[0] == "c":
                        yield a, c, s, nbr[1], nbr[2]

    def _face_pair_u(self, a, c, s, other, sub):
        h, ho = self.f.size(c), self.f.size(other)
        pc = np.zeros((self.n, 2)); pc[:, a] = float(s); pc[:, 1 - a] = self.zu
        po = np.zeros((self.n, 2)); po[:, a] = float(1 - s)
        po[:, 1 - a] = self.zu if sub is None else 0.5 * (sub + self.zu)
        Vc, Gc = self._tab(self.zu, pc[:, 0], pc[:, 1], h)
        Vo, Go = self._tab(self.zu, po[:, 0], po[:, 1], ho)
        nvec = np.zeros(2); nvec[a] = 1.0 if s == 1 else -1.0
        return Vc, Gc, Vo, Go, nvec, self.wu * float(h[1 - a])

    def _sigma_u(self, c, a):
        return (self.k + 1) ** 2 * self.pen_u / float(self.f.size(c)[a])

    def mass_u(self, cells=None):
        blocks = []
        for c in (range(self.Nc) if cells is None else cells):
            V, _, W = self._cell_tab_u(c)
            blocks.append((c, c, V.T @ (W[:, None] * V)))
        return self._assemble(blocks, self.nbu, self.Nc * self.nbu)

    def sip_u(self, cells=None):
        """The bracket of eq. bilin_diff for one component: interior faces as
        in a_p (penalty (k+1)^2 pen_u |Gamma_K|/|K| averaged), boundary faces
        of a non-periodic direction -grad u.n v - u n.grad v + 2 C u v."""
        blocks = []
        for c in (range(self.Nc) if cells is None else cells):
            V, G, W = self._cell_tab_u(c)
            blocks.append((c, c, sum(G[:, :, d].T @ (W[:, None] * G[:, :, d]) for d in range(2))))
        for a, c, s, other, sub in self._interfaces(cells):
            Vc, Gc, Vo, Go, nvec, dS = self._face_pair_u(a, c, s, other, sub)
            C = 0.5 * (self._sigma_u(c, a) + self._sigma_u(other, a))
            tabs = [(c, Vc, Gc, nvec), (other, Vo, Go, -nvec)]
            for (ct, Vt, Gt, nt) in tabs:
                for (cs, Vs, Gs, ns) in tabs:
                    avg_trial = 0.5 * np.einsum("qjd,d->qj", Gs, nt)
                    avg_test = 0.5 * np.einsum("qid,d->qi", Gt, ns)
                    blk = (-(Vt * dS[:, None]).T @ avg_trial - (avg_test * dS[:, None]).T @ Vs
                           + (Vt * (C * float(ns @ nt) * dS)[:, None]).T @ Vs)
                    blocks.append((ct, cs, blk))
        for c, a, s in self._boundary_faces(cells):
            h = self.f.size(c)
            pc = np.zeros((self.n, 2)); pc[:, a] = float(s); pc[:, 1 - a] = self.zu
            V, G = self._tab(self.zu, pc[:, 0], pc[:, 1], h)
            nvec = np.zeros(2); nvec[a] = 1.0 if s == 1 else -1.0
            dS = self.wu * float(h[1 - a])
            gn = np.einsum("qjd,d->qj", G, nvec)
            C = self._sigma_u(c, a)
            blocks.append((c, c, -(V * dS[:, None]).T @ gn - (gn * dS[:, None]).T @ V
                           + (V * (2.0 * C * dS)[:, None]).T @ V))
        return self._assemble(blocks, self.nbu, self.Nc * self.nbu)

    def _boundary_faces(self, cells=None):
        for c in (range(self.Nc) if cells is None else cells):
            for a in range(2):
                for s in (0, 1):
                    if self.f.neighbours(c, a, s)[0] == "B":
                        yield c, a, s

    def boundary_points(self):
        """Velocity face points of every boundary face: cells in order, faces
        f = 2a + s in order, the n Gauss points along the face."""
        pts = []
        for c, a, s in self._boundary_faces():
            o, h = self.f.origin(c), self.f.size(c)
            x = np.zeros((self.n, 2))
            x[:, a] = o[a] + s * h[a]
            x[:, 1 - a] = o[1 - a] + h[1 - a] * self.zu
            pts.append(x)
        return np.concatenate(pts) if pts else np.zeros((0, 2))

    def _w_cell(self, w, c):
        return w[c * 2 * self.nbu:(c + 1) * 2 * self.nbu].reshape(2, self.nbu)

    def _uD_at(self, uD, b, c, a, s, x):
        """Wall data at the points x of boundary face (c, a, s), the b-th:
        uD an (n_b, 2) array at boundary_points() or uD(c, a, s, x)."""
        if callable(uD):
            return np.asarray(uD(c, a, s, x), dtype=np.float64).reshape(len(x), 2)
        return uD[b * self.n:(b + 1) * self.n]

    def _bnd_face(self, c, a, s):
        h, o = self.f.size(c), self.f.origin(c)
        pc = np.zeros((self.n, 2)); pc[:, a] = float(s); pc[:, 1 - a] = self.zu
        Vu, Gu = self._tab(self.zu, pc[:, 0], pc[:, 1], h)
        Vp, Gp = self._tab(self.zp, pc[:, 0], pc[:, 1], h)
        nvec = np.zeros(2); nvec[a] = 1.0 if s == 1 else -1.0
        x = o[None, :] + pc * h[None, :]
        return Vu, Gu, Vp, Gp, nvec, self.wu * float(h[1 - a]), x

    def _pair_mixed(self, a, c, s, other, sub):
        """Velocity and pressure tabulations of both sides at the velocity
        Gauss points of the face (a, s) of c (the finer side)."""
        h, ho = self.f.size(c), self.f.size(other)
        pc = np.zeros((self.n, 2)); pc[:, a] = float(s); pc[:, 1 - a] = self.zu
        po = np.zeros((self.n, 2)); po[:, a] = float(1 - s)
        po[:, 1 - a] = self.zu if sub is None else 0.5 * (sub + self.zu)
        side_c = self._tab(self.zu, pc[:, 0], pc[:, 1], h) + self._tab(self.zp, pc[:, 0], pc[:, 1], h)
        side_o = self._tab(self.zu, po[:, 0], po[:, 1], ho) + self._tab(self.zp, po[:, 0], po[:, 1], ho)
        nvec = np.zeros(2); nvec[a] = 1.0 if s == 1 else -1.0
        return side_c, side_o, nvec, self.wu * float(h[1 - a])

    def _cell_mixed(self, c):
        h = self.f.size(c)
        xr, yr = np.tile(self.zu, self.n), np.repeat(self.zu, self.n)
        Vu, Gu = self._tab(self.zu, xr, yr, h)
        Vp, Gp = self._tab(self.zp, xr, yr, h)
        return Vu, Gu, Vp, Gp, np.kron(self.wu, self.wu) * h[0] * h[1]

    def faces(self, cells=None):
        """('I', ...) once per interior face or fine half face, ('B', a, c, s)
        per boundary face."""
        for a, c, s, other, sub in self._interfaces():
            yield ("I", a, c, other)
        for c, a, s in self._boundary_faces():
            yield ("B", a, c, s)

    def mass_u_vector(self, cells=None):
        M = self.mass_u()
        out = sp.block_diag([M, M]).tocsr()
        # reorder [component][cell][node] -> [cell][component][node]
        perm = np.arange(self.N_u).reshape(2, self.Nc, self.nbu).transpose(1, 0, 2).reshape(-1)
        return out[perm][:, perm].tocsr()

    def explicit_diffusion(self, cells=None):
        """L0(u, v) = int grad u.grad v - sum_E int {{grad u}}.[[v]], the
        whole skeleton (boundary: the interior trace), one component."""
        blocks = []
        for c in range(self.Nc):
            V, G, W = self._cell_tab_u(c)
            blocks.append((c, c, sum(G[:, :, d].T @ (W[:, None] * G[:, :, d]) for d in range(2))))
        for a, c, s, other, sub in self._interfaces():
            Vc, Gc, Vo, Go, nvec, dS = self._face_pair_u(a, c, s, other, sub)
            tabs = [(c, Vc, Gc, nvec), (other, Vo, Go, -nvec)]
            for (ct, Vt, _, nt) in tabs:
                for (cs, _, Gs, _) in tabs:
                    g = 0.5 * np.einsum("qjd,d->qj", Gs, nt)
                    blocks.append((ct, cs, -(Vt * dS[:, None]).T @ g))
        for c, a, s in self._boundary_faces():
            Vu, Gu, _, _, nvec, dS, _ = self._bnd_face(c, a, s)
            g = np.einsum("qjd,d->qj", Gu, nvec)
            blocks.append((c, c, -(Vu * dS[:, None]).T @ g))
        return self._assemble(blocks, self.nbu, self.Nc * self.nbu)

    def explicit_advection(self, w, cells=None):
        """A0_w(u, v) = int u (w.grad v) - sum_E int {{u w}}.[[v]], no
        upwinding, the whole skeleton, one component."""
        blocks = []
        for c in range(self.Nc):
            V, G, W = self._cell_tab_u(c)
            wq = V @ self._w_cell(w, c).T
            wgv = np.einsum("qd,qid->qi", wq, G)
            blocks.append((c, c, (wgv * W[:, None]).T @ V))
        for a, c, s, other, sub in self._interfaces():
            Vc, _, Vo, _, nvec, dS = self._face_pair_u(a, c, s, other, sub)
            wc = Vc @ self._w_cell(w, c).T
            wo = Vo @ self._w_cell(w, other).T
            tabs = [(c, Vc, nvec, wc), (other, Vo, -nvec, wo)]
            for (ct, Vt, nt, _) in tabs:
                for (cs, Vs, _, ws) in tabs:
                    blocks.append((ct, cs, -(Vt * (0.5 * (ws @ nt) * dS)[:, None]).T @ Vs))
        for c, a, s in self._boundary_faces():
            Vu, _, _, _, nvec, dS, _ = self._bnd_face(c, a, s)
            wq = Vu @ self._w_cell(w, c).T
            blocks.append((c, c, -(Vu * ((wq @ nvec) * dS)[:, None]).T @ Vu))
        return self._assemble(blocks, self.nbu, self.Nc * self.nbu)

    def _mixed(self, blocks, rows_u):
        """Assemble (velocity rows, pressure cols) or the transpose from
        (row cell, col cell, component, block) entries."""
        r, cidx, v = [], [], []
        for (ru, cu, comp, blk) in blocks:
            if rows_u:
                r0 = (ru * 2 + comp) * self.nbu
                c0 = cu * self.nbp
            else:
                r0 = ru * self.nbp
                c0 = (cu * 2 + comp) * self.nbu
            rr, cc = np.meshgrid(np.arange(blk.shape[0]) + r0, np.arange(blk.shape[1]) + c0, indexing="ij")
            r.append(rr.ravel()); cidx.append(cc.ravel()); v.append(blk.ravel())
        shape = (self.N_u, self.N_p) if rows_u else (self.N_p, self.N_u)
        return sp.coo_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(cidx))),
                             shape=shape).tocsr()

    def weak_gradient(self, cells=None):
        """(Gw p)(v) = sum_K int p div v - sum_E int {{p}} [[v]] (eq. rhs1)."""
        blocks = []
        for c in range(self.Nc):
            Vu, Gu, Vp, _, W = self._cell_mixed(c)
            for a in range(2):
                blocks.append((c, c, a, (Gu[:, :, a] * W[:, None]).T @ Vp))
        for a_, c, s, other, sub in self._interfaces():
            (Vuc, _, Vpc, _), (Vuo, _, Vpo, _), nvec, dS = self._pair_mixed(a_, c, s, other, sub)
            tabs = [(c, Vuc, Vpc, nvec), (other, Vuo, Vpo, -nvec)]
            for (ct, Vut, _, nt) in tabs:
                for (cs, _, Vps, _) in tabs:
                    for a in range(2):
                        blocks.append((ct, cs, a, -(Vut * (0.5 * nt[a] * dS)[:, None]).T @ Vps))
        for c, a_, s in self._boundary_faces():
            Vu, _, Vp, _, nvec, dS, _ = self._bnd_face(c, a_, s)
            for a in range(2):
                blocks.append((c, c, a, -(Vu * (nvec[a] * dS)[:, None]).T @ Vp))
        return self._mixed(blocks, True)

    def divergence(self, cells=None):
        """(D u)(q) = sum_K int u.grad q - sum_E int {{u}}.[[q]]."""
        blocks = []
        for c in range(self.Nc):
            Vu, _, _, Gp, W = self._cell_mixed(c)
            for a in range(2):
                blocks.append((c, c, a, (Gp[:, :, a] * W[:, None]).T @ Vu))
        for a_, c, s, other, sub in self._interfaces():
            (Vuc, _, Vpc, _), (Vuo, _, Vpo, _), nvec, dS = self._pair_mixed(a_, c, s, other, sub)
            tabs = [(c, Vuc, Vpc, nvec), (other, Vuo, Vpo, -nvec)]
            for (ct, _, Vpt, nt) in tabs:
                for (cs, Vus, _, _) in tabs:
                    for a in range(2):
                        blocks.append((ct, cs, a, -(Vpt * (0.5 * nt[a] * dS)[:, None]).T @ Vus))
        for c, a_, s in self._boundary_faces():
            Vu, _, Vp, _, nvec, dS, _ = self._bnd_face(c, a_, s)
            for a in range(2):
                blocks.append((c, c, a, -(Vp * (nvec[a] * dS)[:, None]).T @ Vu))
        return self._mixed(blocks, False)

    def projection(self, cells=None):
        """P_ij = sum_K int grad psi_j . phi_i (velocity rows, pressure cols)."""
        blocks = []
        for c in range(self.Nc):
            Vu, _, _, Gp, W = self._cell_mixed(c)
            for a in range(2):
                blocks.append((c, c, a, (Vu * W[:, None]).T @ Gp[:, :, a]))
        return self._mixed(blocks, True)

    def dirichlet_rhs(self, theta, w, uD):
        """Wall-data part of F_u: per component -theta nu int u_D (n.grad v)
        + theta nu int 2 C u_D v - theta int u_D (w.n) v + theta int lambda u_D v."""
        out = np.zeros(self.N_u)
        for b, (c, a, s) in enumerate(self._boundary_faces()):
            Vu, Gu, _, _, nvec, dS, x = self._bnd_face(c, a, s)
            ud = self._uD_at(uD, b, c, a, s, x)
            wq = Vu @ self._w_cell(w, c).T
            wn = wq @ nvec
            lam = np.maximum(np.abs(wn), np.abs((2.0 * ud - wq) @ nvec))
            gn = np.einsum("qid,d->qi", Gu, nvec)
            C = self._sigma_u(c, a)
            for comp in range(2):
                g = ud[:, comp] * dS
                contrib = (-theta * self.nu * (gn.T @ g) + theta * self.nu * 2.0 * C * (Vu.T @ g)
                           - theta * (Vu.T @ (g * wn)) + theta * (Vu.T @ (g * lam)))
                base = (c * 2 + comp) * self.nbu
                out[base:base + self.nbu] += contrib
        return out

    def lf_advection(self, w, uD=None, cells=None):
        """Linearised advection with the local Lax-Friedrichs flux (eq.
        trilinear) for one component, as in the box-mesh oracle:
        -int u (w.grad v) + sum_I int ({{u w}}.[[v]] + lambda/2 [[u]].[[v]])
        + sum_B int lambda u v, lambda = max |w.n| of the two traces at each
        face point (boundary: exterior state 2 u_D - w).  Faces between a
        coarse and two fine cells: the fine faces' Gauss points.  uD: (n_b, 2)
        at boundary_points()."""
        blocks = []
        for c in (range(self.Nc) if cells is None else cells):
            V, G, W = self._cell_tab_u(c)
            wq = V @ self._w_cell(w, c).T
            wgv = np.einsum("qd,qid->qi", wq, G)
            blocks.append((c, c, -(wgv * W[:, None]).T @ V))
        for a, c, s, other, sub in self._interfaces(cells):
            Vc, _, Vo, _, nvec, dS = self._face_pair_u(a, c, s, other, sub)
            wc = Vc @ self._w_cell(w, c).T
            wo = Vo @ self._w_cell(w, other).T
            lam = np.maximum(np.abs(wc @ nvec), np.abs(wo @ nvec))
            tabs = [(c, Vc, nvec, wc), (other, Vo, -nvec, wo)]
            for (ct, Vt, nt, _) in tabs:
                for (cs, Vs, ns, ws) in tabs:
                    coef = 0.5 * (ws @ nt) + 0.5 * lam * float(ns @ nt)
                    blocks.append((ct, cs, (Vt * (coef * dS)[:, None]).T @ Vs))
        bnum = {f: b for b, f in enumerate(self._boundary_faces())} if cells is not None else None
        for b, (c, a, s) in enumerate(self._boundary_faces(cells)):
            if bnum is not None:
                b = bnum[(c, a, s)]
            V, _, _, _, nvec, dS, x = self._bnd_face(c, a, s)
            wq = V @ self._w_cell(w, c).T
            wext = 2.0 * self._uD_at(uD, b, c, a, s, x) - wq
            lam = np.maximum(np.abs(wq @ nvec), np.abs(wext @ nvec))
            blocks.append((c, c, (V * (lam * dS)[:, None]).T @ V))
        return self._assemble(blocks, self.nbu, self.Nc * self.nbu)

    def apply_momentum(self, mc, tnu, th, w, u, uD=None, cells=None):
        """y_c = (mc M + tnu A + th C(w)) u_c for both components of u
        ([cell][component][node]); with ``cells`` valid on those cells only."""
        A = (mc * self.mass_u(cells) + tnu * self.sip_u(cells)
             + th * self.lf_advection(w, uD, cells)).tocsr()
        U = u.reshape(self.Nc, 2, self.nbu)
        out = np.empty_like(U)
        for comp in range(2):
            out[:, comp, :] = (A @ U[:, comp, :].reshape(-1)).reshape(self.Nc, self.nbu)
        return out.reshape(-1)

    def helmholtz_p(self, alpha, cells=None):
        """alpha M^p + K: the stage pressure operator of Sec. 3."""
        return (alpha * self.mass_p(cells) + self.sip_p(cells)).tocsr()

    def indicator(self, u):
        """eta_K = diam(K)^2 ||omega||^2_K, u in [cell][component][node]
        layout, the velocity Gauss rule (exact for omega^2)."""
        eta = np.zeros(self.Nc)
        xr = np.tile(self.zu, self.n)
        yr = np.repeat(self.zu, self.n)
        for c in range(self.Nc):
            h = self.f.size(c)
            W = np.kron(self.wu, self.wu) * h[0] * h[1]
            _, G = self._tab(self.zu, xr, yr, h)
            loc = u[c * 2 * self.nbu:(c + 1) * 2 * self.nbu].reshape(2, self.nbu)
            om = G[:, :, 0] @ loc[1] - G[:, :, 1] @ loc[0]
            eta[c] = float(h[0] ** 2 + h[1] ** 2) * float(np.sum(W * om ** 2))
        return eta

    def node_coords(self, field="u"):
        z = self.zu if field == "u" else self.zp
        n = len(z)
        out = []
        for c in range(self.Nc):
            o, h = self.f.origin(c), self.f.size(c)
            out.append(np.stack([o[0] + h[0] * np.tile(z, n), o[1] + h[1] * np.repeat(z, n)], 1))
        return np.concatenate(out, axis=0)


# ---------------------------------------------------------------------------
def transfer(old, new, vec, n, ncomp):
    """Field on ``old`` (n Gauss nodes per direction, ncomp components per
    cell, [cell][component][node]) moved to ``new`` = old.adapt(...):
    kept cells copy, children interpolate their parent's polynomial, a
    parent is the L2 projection of its four children (per component)."""
    z, w = gauss_legendre_01(n)
    nb = n * n
    W = np.kron(w, w)
    out = np.zeros(new.N * ncomp * nb)
    blk = ncomp * nb
    for c, (l, i, j) in enumerate(new.leaves):
        dst = out[c * blk:(c + 1) * blk].reshape(ncomp, nb)
        if (l, i, j) in old.index:
            o = old.index[(l, i, j)]
            dst[:] = vec[o * blk:(o + 1) * blk].reshape(ncomp, nb)
        elif l > 0 and (l - 1, i >> 1, j >> 1) in old.index:
            o = old.index[(l - 1, i >> 1, j >> 1)]
            src = vec[o * blk:(o + 1) * blk].reshape(ncomp, nb)
            # parent basis at the child's nodes
            P = tensor([lagrange_values(z, 0.5 * ((i & 1) + z)), lagrange_values(z, 0.5 * ((j & 1) + z))])
            dst[:] = src @ P.T
        else:
            # L2 projection: M_parent x = sum over children of int child * phi
            rhs = np.zeros((ncomp, nb))
            for dj in (0, 1):
                for di in (0, 1):
                    o = old.index[(l + 1, 2 * i + di, 2 * j + dj)]
                    src = vec[o * blk:(o + 1) * blk].reshape(ncomp, nb)
                    P = tensor([lagrange_values(z, 0.5 * (di + z)), lagrange_values(z, 0.5 * (dj + z))])
                    # child quadrature weights are W / 4 of the parent's area
                    rhs += (src * (0.25 * W)[None, :]) @ P
            Mp = np.diag(W)   # collocated Gauss basis: the parent mass is diagonal
            dst[:] = np.linalg.solve(Mp, rhs.T).T
    return out
