"""Dense per-cell / per-face tabulation of the paper's DG forms (oracle).

TEST INFRASTRUCTURE ONLY.  Every form of Sec. 3 is written out term by term
with the jump and average operators of Sec. 3 and assembled into a scipy CSR
matrix.  Interior faces are visited once, with both traces, exactly as the
sums over E^I in the paper are written; boundary faces use the boundary
variants of the same sums.

Notation and layout
-------------------
* Reference cell [0,1]^d, Q1 (multilinear) geometry map through the cell's
  vertices; physical gradients are J^{-T} times reference gradients; face
  normals and surface weights follow from Nanson's formula.
* Velocity: Q_k per component, Lagrange at n = k+1 Gauss-Legendre nodes,
  integrated with the n-point Gauss rule (volume) and the n^{d-1}-point rule
  on faces.  Pressure: Q_{k-1}, Lagrange at n_p = k Gauss nodes, integrated
  with the n_p-point rule in the pressure-only forms (mass, a_p).  Mixed
  forms (projection matrix P, weak gradient of the momentum functional,
  divergence functional F_p) use the velocity rule.
* A scalar velocity vector is indexed [cell][node]; a velocity field
  [cell][component][node]; a pressure field [cell][node]; cells and nodes
  lexicographic with x fastest.
* For an interior face visited from cell c at its side-1 face in direction a,
  K^- := c and K^+ := the neighbour; n^- is c's outward normal, n^+ = -n^-.

Readings (where the paper is silent, ambiguous or garbled)
---------------------------------------------------------
* SIP penalties (eq. penconst1 and the pressure analogue): the printed ratio
  diam(Gamma)/diam(K) is dimensionless and cannot make SIP coercive as h->0;
  it is read as face measure over cell measure, |Gamma|/|K| (= 1/h on a
  Cartesian cell), i.e. sigma^u = (k+1)^2 |Gamma|/|K| and
  sigma^p = k^2 |Gamma|/|K| with k the velocity degree.  |Gamma| and |K| are
  computed with the velocity quadrature.  C is the average of the two
  cell values on interior faces and the cell value on boundary faces.
* Local Lax-Friedrichs speed lambda = max(|w^+ . n|, |w^- . n|) is evaluated
  pointwise at each face quadrature point; on a boundary face the exterior
  advecting state is the mirror 2 u_D - w.
* In the explicit functionals (eq. rhs1 and its stage-2 analogue, and F_p),
  the sums "over the whole skeleton E" take the average on a boundary face as
  the interior trace, as the average operator is defined there.
* In the pressure form a_p the superscript on {{grad p^{n+gamma}}} is read
  as the trial function p; the entry A_ij = a(phi_j, phi_j) is read as
  a(phi_j, phi_i).
"""
import numpy as np
import scipy.sparse as sp

from .basis import (gauss_legendre_01, lagrange_values, lagrange_derivatives,
                    tensor, tensor_points, tensor_weights)


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------
def _q1_shape(xi, dim):
    """Multilinear vertex shape functions and their reference gradients."""
    npnt = xi.shape[0]
    nv = 2 ** dim
    N = np.ones((npnt, nv))
    dN = np.ones((npnt, nv, dim))
    for v in range(nv):
        for a in range(dim):
            bit = (v >> a) & 1
            f = xi[:, a] if bit else 1.0 - xi[:, a]
            df = 1.0 if bit else -1.0
            N[:, v] *= f
            for b in range(dim):
                dN[:, v, b] *= df if b == a else f
    return N, dN


def _map(vertices, xi):
    dim = vertices.shape[1]
    N, dN = _q1_shape(xi, dim)
    x = N @ vertices
    # J[q, i, j] = d x_i / d xi_j
    J = np.einsum("vi,qvj->qij", vertices, dN)
    return x, J


class _Tab:
    """Values and physical gradients of one nodal basis at a point set."""

    def __init__(self, V, G):
        self.V = V      # (npnt, nb)
        self.G = G      # (npnt, nb, dim)


# ---------------------------------------------------------------------------
class Discretization:
    """All matrices of Sec. 3 for one mesh, velocity degree k and viscosity.

    Parameters follow the paper's notation: ``k`` velocity degree (pressure
    degree k-1), ``nu`` = 1/Re, ``c`` the artificial sound speed of
    eq. ns_artcomp, ``pen_u``/``pen_p`` multipliers on the SIP penalties
    (1 = the paper's value).
    """

    def __init__(self, mesh, k, nu, c=1.0e3, pen_u=1.0, pen_p=1.0, n_q_adv=None):
        if k < 1:
            raise ValueError("velocity degree k must be >= 1")
        self.mesh = mesh
        self.dim = mesh.dim
        self.k = int(k)
        self.nu = float(nu)
        self.c = float(c)
        self.pen_u = float(pen_u)
        self.pen_p = float(pen_p)
        self.n = self.k + 1
        self.n_p = self.k
        self.zu, self.wu = gauss_legendre_01(self.n)
        self.zp, self.wp = gauss_legendre_01(self.n_p)
        # quadrature of the advection forms (default: the velocity rule)
        self.n_q_adv = self.n if n_q_adv is None else int(n_q_adv)
        self.za, self.wa = gauss_legendre_01(self.n_q_adv)
        self.nbu = self.n ** self.dim
        self.nbp = self.n_p ** self.dim
        self.Nc = mesh.N
        self.n_scalar = self.Nc * self.nbu
        self.N_u = self.dim * self.n_scalar
        self.N_p = self.Nc * self.nbp
        self._cell_cache = {}
        self._face_cache = {}

    # ------------------------------------------------------------------
    # tabulation
    # ------------------------------------------------------------------
    def _basis_tab(self, nodes, xi, JinvT):
        d = self.dim
        Vd = [lagrange_values(nodes, xi[:, a]) for a in range(d)]
        Dd = [lagrange_derivatives(nodes, xi[:, a]) for a in range(d)]
        npnt = xi.shape[0]
        nb = len(nodes) ** d
        # Point-wise tensor product (the points are not necessarily a grid).
        V = np.ones((npnt, nb))
        Gr = np.ones((npnt, nb, d))
        idx = np.arange(nb)
        for a in range(d):
            ia = (idx // (len(nodes) ** a)) % len(nodes)
            V *= Vd[a][:, ia]
            for b in range(d):
                Gr[:, :, b] *= (Dd[a][:, ia] if a == b else Vd[a][:, ia])
        G = np.einsum("qij,qbj->qbi", JinvT, Gr)
        return _Tab(V, G)

    def _rule(self, rule):
        return {"u": (self.zu, self.wu), "p": (self.zp, self.wp),
                "a": (self.za, self.wa)}[rule]

    def cell(self, c, rule="u"):
        """Volume quadrature data of cell c with the velocity ('u') or
        pressure ('p') Gauss rule."""
        key = (c, rule)
        if key in self._cell_cache:
            return self._cell_cache[key]
        d = self.dim
        q, w = self._rule(rule)
        xi = tensor_points([q] * d)
        W = tensor_weights([w] * d)
        x, J = _map(self.mesh.cell_vertices(c), xi)
        det = np.linalg.det(J)
        JinvT = np.transpose(np.linalg.inv(J), (0, 2, 1))
        data = dict(x=x, JxW=W * det, det=det,
                    u=self._basis_tab(self.zu, xi, JinvT),
                    p=self._basis_tab(self.zp, xi, JinvT))
        if len(self._cell_cache) > 4096:
            self._cell_cache.clear()
        self._cell_cache[key] = data
        return data

    def face(self, c, a, s, rule="u"):
        """Face quadrature data of cell c on its face (direction a, side s)."""
        key = (c, a, s, rule)
        if key in self._face_cache:
            return self._face_cache[key]
        d = self.dim
        q, w = self._rule(rule)
        tang = [b for b in range(d) if b != a]
        if d == 1:
            raise ValueError("dim must be 2 or 3")
        tp = tensor_points([q] * (d - 1))
        Wt = tensor_weights([w] * (d - 1))
        xi = np.zeros((tp.shape[0], d))
        xi[:, a] = float(s)
        for j, b in enumerate(tang):
            xi[:, b] = tp[:, j]
        x, J = _map(self.mesh.cell_vertices(c), xi)
        det = np.linalg.det(J)
        JinvT = np.transpose(np.linalg.inv(J), (0, 2, 1))
        nhat = np.zeros(d)
        nhat[a] = 1.0 if s == 1 else -1.0
        m = JinvT @ nhat
        mnorm = np.linalg.norm(m, axis=1)
        data = dict(x=x, n=m / mnorm[:, None], dS=Wt * det * mnorm,
                    u=self._basis_tab(self.zu, xi, JinvT),
                    p=self._basis_tab(self.zp, xi, JinvT))
        if len(self._face_cache) > 8192:
            self._face_cache.clear()
        self._face_cache[key] = data
        return data

    # ------------------------------------------------------------------
    # penalties (eq. penconst1 and its pressure analogue; reading in the
    # module docstring)
    # ------------------------------------------------------------------
    def cell_measure(self, c):
        return float(np.sum(self.cell(c, "u")["JxW"]))

    def face_measure(self, c, a, s):
        return float(np.sum(self.face(c, a, s, "u")["dS"]))

    def _sigma(self, c, a, s, field):
        fac = (self.k + 1) ** 2 * self.pen_u if field == "u" else self.k ** 2 * self.pen_p
        return fac * self.face_measure(c, a, s) / self.cell_measure(c)

    def penalty(self, c, a, s, nb, field):
        """C_u / C_p on the face (a, s) of c; ``nb`` None on a boundary face."""
        sc = self._sigma(c, a, s, field)
        if nb is None:
            return sc
        return 0.5 * (sc + self._sigma(nb, a, 1 - s, field))

    # ------------------------------------------------------------------
    # face iteration
    # ------------------------------------------------------------------
    def faces(self, cells=None):
        """Yield ('I', a, c_minus, c_plus) or ('B', a, c, s) once per face.

        With ``cells`` given, only faces touching those cells are produced.
        """
        mesh = self.mesh
        sel = None if cells is None else set(int(c) for c in cells)
        for c in range(mesh.N):
            for a in range(self.dim):
                nb = mesh.neighbor(c, a, 1)
                if nb is not None:
                    if sel is None or c in sel or nb in sel:
                        yield ("I", a, c, nb)
                else:
                    if sel is None or c in sel:
                        yield ("B", a, c, 1)
                if mesh.neighbor(c, a, 0) is None:
                    if sel is None or c in sel:
                        yield ("B", a, c, 0)

    def _cells(self, cells):
        return range(self.mesh.N) if cells is None else [int(c) for c in cells]

    # ------------------------------------------------------------------
    # sparse accumulation
    # ------------------------------------------------------------------
    class _Acc:
        def __init__(self, shape, row_block, col_block, keep_rows=None):
            self.shape = shape
            self.rb, self.cb = row_block, col_block
            self.keep = None if keep_rows is None else set(int(c) for c in keep_rows)
            self.r, self.c, self.v = [], [], []

        def add(self, rcell, ccell, block, rsub=0, csub=0, rstride=1, cstride=1):
            """Add a dense block for row cell / column cell.

            Rows are rcell*rstride*rb + rsub*rb + i (same for columns), which
            covers the [cell][component][node] layout with rstride = dim.
            """
            if self.keep is not None and rcell not in self.keep:
                return
            nr, nc = block.shape
            r0 = (rcell * rstride + rsub) * self.rb
            c0 = (ccell * cstride + csub) * self.cb
            rr, cc = np.meshgrid(np.arange(nr) + r0, np.arange(nc) + c0, indexing="ij")
            self.r.append(rr.reshape(-1))
            self.c.append(cc.reshape(-1))
            self.v.append(block.reshape(-1))

        def csr(self):
            if not self.r:
                return sp.csr_matrix(self.shape)
            r = np.concatenate(self.r)
            c = np.concatenate(self.c)
            v = np.concatenate(self.v)
            return sp.coo_matrix((v, (r, c)), shape=self.shape).tocsr()

    # ------------------------------------------------------------------
    # field evaluation helpers
    # ------------------------------------------------------------------
    def _vec_cell(self, w, c):
        """Velocity DoFs of cell c as (dim, nbu)."""
        return w[c * self.dim * self.nbu:(c + 1) * self.dim * self.nbu].reshape(self.dim, self.nbu)

    def _eval_vec(self, tabV, w, c):
        """Vector field w evaluated at the points of a tabulation, (npnt, dim)."""
        return tabV @ self._vec_cell(w, c).T

    # ------------------------------------------------------------------
    # scalar velocity forms
    # ------------------------------------------------------------------
    def mass_u(self, cells=None):
        """Scalar velocity mass matrix (eq. mass_matrix, one component)."""
        acc = self._Acc((self.n_scalar, self.n_scalar), self.nbu, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            V = cd["u"].V
            acc.add(c, c, V.T @ (cd["JxW"][:, None] * V))
        return acc.csr()

    def mass_p(self, cells=None):
        """Pressure mass matrix M^p (eq. pressure_mass_matrix)."""
        acc = self._Acc((self.N_p, self.N_p), self.nbp, self.nbp, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "p")
            V = cd["p"].V
            acc.add(c, c, V.T @ (cd["JxW"][:, None] * V))
        return acc.csr()

    def _sip(self, field, cells=None, boundary=True):
        """Symmetric interior penalty form, one scalar component.

        field 'u': the bracket of eq. bilin_diff without the 1/(2Re) or
        a33/Re factor (those are applied by the stepper), boundary terms with
        -grad u.n v - u n.grad v + 2 C_u u v.
        field 'p': the pressure form a_p, interior faces only (homogeneous
        Neumann: no boundary terms).
        """
        nb_ = self.nbu if field == "u" else self.nbp
        n_ = self.n_scalar if field == "u" else self.N_p
        acc = self._Acc((n_, n_), nb_, nb_, cells)
        for c in self._cells(cells):
            cd = self.cell(c, field)
            t = cd[field]
            blk = np.zeros((nb_, nb_))
            for a in range(self.dim):
                blk += t.G[:, :, a].T @ (cd["JxW"][:, None] * t.G[:, :, a])
            acc.add(c, c, blk)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a, cm, cp = f
                fm = self.face(cm, a, 1, field)
                fp = self.face(cp, a, 0, field)
                C = self.penalty(cm, a, 1, cp, field)
                dS = fm["dS"]
                tabs = [(cm, fm[field], fm["n"]), (cp, fp[field], -fm["n"])]
                for (ct, tt, nt) in tabs:          # test side
                    for (cs, ts, ns) in tabs:      # trial side
                        avg_grad_trial_n = 0.5 * np.einsum("qjd,qd->qj", ts.G, nt)
                        avg_grad_test_n = 0.5 * np.einsum("qid,qd->qi", tt.G, ns)
                        nn = np.einsum("qd,qd->q", ns, nt)
                        blk = (-(tt.V * dS[:, None]).T @ avg_grad_trial_n
                               - (avg_grad_test_n * dS[:, None]).T @ ts.V
                               + (tt.V * (C * nn * dS)[:, None]).T @ ts.V)
                        acc.add(ct, cs, blk)
            elif boundary and field == "u":
                _, a, c, s = f
                fd = self.face(c, a, s, "u")
                C = self.penalty(c, a, s, None, "u")
                t = fd["u"]
                dS = fd["dS"]
                gn = np.einsum("qjd,qd->qj", t.G, fd["n"])
                blk = (-(t.V * dS[:, None]).T @ gn
                       - (gn * dS[:, None]).T @ t.V
                       + (t.V * (2.0 * C * dS)[:, None]).T @ t.V)
                acc.add(c, c, blk)
        return acc.csr()

    def sip_u(self, cells=None):
        return self._sip("u", cells)

    def sip_p(self, cells=None):
        """Pressure stiffness K_ij = a_p(psi_j, psi_i)."""
        return self._sip("p", cells)

    def lf_advection(self, w, uD_face=None, cells=None):
        """Linearised advection with local Lax-Friedrichs flux (eq. trilinear).

        One scalar component, without the 1/2 or a33 factor:
        -int u (w.grad v) + sum_I int {{u w}}.[[v]]
        + sum_I int lambda/2 [[u]].[[v]] + sum_B int lambda u v.
        ``uD_face(c, a, s, x) -> (npnt, dim)`` gives the Dirichlet data on a
        boundary face (needed for lambda there).
        """
        acc = self._Acc((self.n_scalar, self.n_scalar), self.nbu, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "a")
            t = cd["u"]
            wq = self._eval_vec(t.V, w, c)
            wgv = np.einsum("qd,qid->qi", wq, t.G)           # w . grad v_i
            acc.add(c, c, -(wgv * cd["JxW"][:, None]).T @ t.V)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a, cm, cp = f
                fm = self.face(cm, a, 1, "a")
                fp = self.face(cp, a, 0, "a")
                dS = fm["dS"]
                nm = fm["n"]
                wm = self._eval_vec(fm["u"].V, w, cm)
                wp = self._eval_vec(fp["u"].V, w, cp)
                lam = np.maximum(np.abs(np.einsum("qd,qd->q", wm, nm)),
                                 np.abs(np.einsum("qd,qd->q", wp, nm)))
                tabs = [(cm, fm["u"], nm, wm), (cp, fp["u"], -nm, wp)]
                for (ct, tt, nt, _) in tabs:
                    for (cs, ts, ns, ws) in tabs:
                        central = 0.5 * np.einsum("qd,qd->q", ws, nt)     # trial side's w . n_test
                        jump = 0.5 * lam * np.einsum("qd,qd->q", ns, nt)
                        blk = (tt.V * ((central + jump) * dS)[:, None]).T @ ts.V
                        acc.add(ct, cs, blk)
            else:
                _, a, c, s = f
                fd = self.face(c, a, s, "a")
                t = fd["u"]
                n = fd["n"]
                wq = self._eval_vec(t.V, w, c)
                if uD_face is None:
                    raise ValueError("boundary faces need Dirichlet data for lambda")
                wext = 2.0 * uD_face(c, a, s, fd["x"]) - wq
                lam = np.maximum(np.abs(np.einsum("qd,qd->q", wq, n)),
                                 np.abs(np.einsum("qd,qd->q", wext, n)))
                acc.add(c, c, (t.V * (lam * fd["dS"])[:, None]).T @ t.V)
        return acc.csr()

    def explicit_diffusion(self, cells=None):
        """L0(u, v) = int grad u.grad v - sum_E int {{grad u}}.[[v]].

        The diffusion part of the functionals F_u (eq. rhs1) is -theta nu L0
        applied to the previous-level velocity: no penalty and no
        symmetrising term, the face sum over the whole skeleton.
        """
        acc = self._Acc((self.n_scalar, self.n_scalar), self.nbu, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            t = cd["u"]
            blk = np.zeros((self.nbu, self.nbu))
            for a in range(self.dim):
                blk += t.G[:, :, a].T @ (cd["JxW"][:, None] * t.G[:, :, a])
            acc.add(c, c, blk)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a, cm, cp = f
                fm = self.face(cm, a, 1, "u")
                fp = self.face(cp, a, 0, "u")
                dS = fm["dS"]
                tabs = [(cm, fm["u"], fm["n"]), (cp, fp["u"], -fm["n"])]
                for (ct, tt, nt) in tabs:
                    for (cs, ts, _) in tabs:
                        g = 0.5 * np.einsum("qjd,qd->qj", ts.G, nt)
                        acc.add(ct, cs, -(tt.V * dS[:, None]).T @ g)
            else:
                _, a, c, s = f
                fd = self.face(c, a, s, "u")
                t = fd["u"]
                g = np.einsum("qjd,qd->qj", t.G, fd["n"])
                acc.add(c, c, -(t.V * fd["dS"][:, None]).T @ g)
        return acc.csr()

    def explicit_advection(self, w, cells=None):
        """A0_w(u, v) = int u (w.grad v) - sum_E int {{u w}}.[[v]].

        The advection part of the functionals F_u (eq. rhs1): no upwinding,
        face sum over the whole skeleton, one scalar component.
        """
        acc = self._Acc((self.n_scalar, self.n_scalar), self.nbu, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "a")
            t = cd["u"]
            wq = self._eval_vec(t.V, w, c)
            wgv = np.einsum("qd,qid->qi", wq, t.G)
            acc.add(c, c, (wgv * cd["JxW"][:, None]).T @ t.V)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a, cm, cp = f
                fm = self.face(cm, a, 1, "a")
                fp = self.face(cp, a, 0, "a")
                dS = fm["dS"]
                nm = fm["n"]
                wm = self._eval_vec(fm["u"].V, w, cm)
                wp = self._eval_vec(fp["u"].V, w, cp)
                tabs = [(cm, fm["u"], nm, wm), (cp, fp["u"], -nm, wp)]
                for (ct, tt, nt, _) in tabs:
                    for (cs, ts, _, ws) in tabs:
                        central = 0.5 * np.einsum("qd,qd->q", ws, nt)
                        acc.add(ct, cs, -(tt.V * (central * dS)[:, None]).T @ ts.V)
            else:
                _, a, c, s = f
                fd = self.face(c, a, s, "a")
                t = fd["u"]
                wq = self._eval_vec(t.V, w, c)
                wn = np.einsum("qd,qd->q", wq, fd["n"])
                acc.add(c, c, -(t.V * (wn * fd["dS"])[:, None]).T @ t.V)
        return acc.csr()

    # ------------------------------------------------------------------
    # mixed velocity-pressure forms
    # ------------------------------------------------------------------
    def weak_gradient(self, cells=None):
        """Gw: pressure -> velocity test space, the pressure part of F_u.

        (Gw p)(v) = sum_K int p div v - sum_E int {{p}} [[v]]  (eq. rhs1),
        rows in the [cell][component][node] layout.
        """
        d = self.dim
        acc = self._Acc((self.N_u, self.N_p), self.nbu, self.nbp, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            for a in range(d):
                blk = (cd["u"].G[:, :, a] * cd["JxW"][:, None]).T @ cd["p"].V
                acc.add(c, c, blk, rsub=a, rstride=d)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a_, cm, cp = f
                fm = self.face(cm, a_, 1, "u")
                fp = self.face(cp, a_, 0, "u")
                dS = fm["dS"]
                tabs = [(cm, fm, fm["n"]), (cp, fp, -fm["n"])]
                for (ct, ft, nt) in tabs:
                    for (cs, fs, _) in tabs:
                        for a in range(d):
                            blk = -(ft["u"].V * (0.5 * nt[:, a] * dS)[:, None]).T @ fs["p"].V
                            acc.add(ct, cs, blk, rsub=a, rstride=d)
            else:
                _, a_, c, s = f
                fd = self.face(c, a_, s, "u")
                for a in range(d):
                    blk = -(fd["u"].V * (fd["n"][:, a] * fd["dS"])[:, None]).T @ fd["p"].V
                    acc.add(c, c, blk, rsub=a, rstride=d)
        return acc.csr()

    def divergence(self, cells=None):
        """D: velocity -> pressure test space, the bracket of F_p.

        (D u)(q) = sum_K int u.grad q - sum_E int {{u}}.[[q]]; F_p is
        (1/(beta dt)) D u**.
        """
        d = self.dim
        acc = self._Acc((self.N_p, self.N_u), self.nbp, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            for a in range(d):
                blk = (cd["p"].G[:, :, a] * cd["JxW"][:, None]).T @ cd["u"].V
                acc.add(c, c, blk, csub=a, cstride=d)
        for f in self.faces(cells):
            if f[0] == "I":
                _, a_, cm, cp = f
                fm = self.face(cm, a_, 1, "u")
                fp = self.face(cp, a_, 0, "u")
                dS = fm["dS"]
                tabs = [(cm, fm, fm["n"]), (cp, fp, -fm["n"])]
                for (ct, ft, nt) in tabs:
                    for (cs, fs, _) in tabs:
                        for a in range(d):
                            blk = -(ft["p"].V * (0.5 * nt[:, a] * dS)[:, None]).T @ fs["u"].V
                            acc.add(ct, cs, blk, csub=a, cstride=d)
            else:
                _, a_, c, s = f
                fd = self.face(c, a_, s, "u")
                for a in range(d):
                    blk = -(fd["p"].V * (fd["n"][:, a] * fd["dS"])[:, None]).T @ fd["u"].V
                    acc.add(c, c, blk, csub=a, cstride=d)
        return acc.csr()

    def projection(self, cells=None):
        """P_ij = sum_K int grad psi_j . phi_i (velocity rows, pressure cols)."""
        d = self.dim
        acc = self._Acc((self.N_u, self.N_p), self.nbu, self.nbp, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            for a in range(d):
                blk = (cd["u"].V * cd["JxW"][:, None]).T @ cd["p"].G[:, :, a]
                acc.add(c, c, blk, rsub=a, rstride=d)
        return acc.csr()

    def mass_u_vector(self, cells=None):
        """Velocity mass for the full [cell][component][node] vector."""
        d = self.dim
        acc = self._Acc((self.N_u, self.N_u), self.nbu, self.nbu, cells)
        for c in self._cells(cells):
            cd = self.cell(c, "u")
            V = cd["u"].V
            blk = V.T @ (cd["JxW"][:, None] * V)
            for a in range(d):
                acc.add(c, c, blk, rsub=a, csub=a, rstride=d, cstride=d)
        return acc.csr()

    # ------------------------------------------------------------------
    # Dirichlet data terms of the momentum functionals
    # ------------------------------------------------------------------
    def dirichlet_rhs(self, theta, w, uD_face):
        """Boundary-data part of F_u (eq. rhs1; stage 2 with theta = a33).

        For each component: -theta nu int u_D (n.grad v) + theta nu int 2C u_D v
        - theta int u_D (w.n) v + theta int lambda u_D v on E^B.
        """
        d = self.dim
        out = np.zeros(self.N_u)
        for f in self.faces():
            if f[0] != "B":
                continue
            _, a, c, s = f
            fd = self.face(c, a, s, "u")
            t = fd["u"]
            n = fd["n"]
            dS = fd["dS"]
            C = self.penalty(c, a, s, None, "u")
            uD = uD_face(c, a, s, fd["x"])
            wq = self._eval_vec(t.V, w, c)
            wn = np.einsum("qd,qd->q", wq, n)
            wext = 2.0 * uD - wq
            lam = np.maximum(np.abs(wn), np.abs(np.einsum("qd,qd->q", wext, n)))
            gn = np.einsum("qid,qd->qi", t.G, n)
            for comp in range(d):
                g = uD[:, comp] * dS
                contrib = (-theta * self.nu * (gn.T @ g)
                           + theta * self.nu * 2.0 * C * (t.V.T @ g)
                           - theta * (t.V.T @ (g * wn))
                           + theta * (t.V.T @ (g * lam)))
                base = (c * d + comp) * self.nbu
                out[base:base + self.nbu] += contrib
        return out

    # ------------------------------------------------------------------
    # nodes
    # ------------------------------------------------------------------
    def node_coords(self, field="u"):
        """Physical coordinates of the nodes, (Nc * nb, dim) in [cell][node]."""
        z = self.zu if field == "u" else self.zp
        xi = tensor_points([z] * self.dim)
        out = []
        for c in range(self.Nc):
            x, _ = _map(self.mesh.cell_vertices(c), xi)
            out.append(x)
        return np.concatenate(out, axis=0)

    def boundary_face_points(self):
        """Physical velocity quadrature points of every boundary face.

        Order: the order of ``faces()`` restricted to boundary faces, points
        lexicographic in the tangential directions (lowest direction fastest).
        """
        pts = []
        for f in self.faces():
            if f[0] == "B":
                _, a, c, s = f
                pts.append(self.face(c, a, s, "u")["x"])
        return np.concatenate(pts, axis=0) if pts else np.zeros((0, self.dim))

    # ------------------------------------------------------------------
    # norms against a closed form (over-integrated quadrature)
    # ------------------------------------------------------------------
    def l2_error(self, vec, exact, field="u", extra=3, remove_mean=False):
        """||u_h - u||_{L2} and ||u||_{L2} with an (n+extra)-point rule.

        ``remove_mean`` subtracts each function's mean first (pressure is
        only defined up to a constant on a periodic box).
        """
        d = self.dim
        nodes = self.zu if field == "u" else self.zp
        q, w = gauss_legendre_01(len(nodes) + extra)
        xi = tensor_points([q] * d)
        W = tensor_weights([w] * d)
        nb = len(nodes) ** d
        ncomp = d if field == "u" else 1
        V = tensor([lagrange_values(nodes, q)] * d)
        vals_h, vals_e, wts = [], [], []
        for c in range(self.Nc):
            x, J = _map(self.mesh.cell_vertices(c), xi)
            wts.append(W * np.linalg.det(J))
            vals_e.append(np.asarray(exact(x)).reshape(len(x), ncomp))
            loc = vec[c * ncomp * nb:(c + 1) * ncomp * nb].reshape(ncomp, nb)
            vals_h.append(V @ loc.T)
        JxW = np.concatenate(wts)
        uh = np.concatenate(vals_h)
        ex = np.concatenate(vals_e)
        if remove_mean:
            vol = JxW.sum()
            uh = uh - (JxW[:, None] * uh).sum(0) / vol
            ex = ex - (JxW[:, None] * ex).sum(0) / vol
        err = np.sqrt(float(np.sum(JxW[:, None] * (uh - ex) ** 2)))
        ref = np.sqrt(float(np.sum(JxW[:, None] * ex ** 2)))
        return err, ref
