"""h/p-multigrid preconditioners for the pressure Helmholtz operator and for
one velocity component of the momentum operator (oracle; TEST
INFRASTRUCTURE ONLY).

The paper solves the pressure systems of Sec. 3 with a multigrid-preconditioned
CG (Sec. 4) and gives no details of the multigrid; this module fixes one
concrete method and computes it in plain FP64 with assembled matrices:

* Levels.  Level 0 is the pressure space Q_{k-1} on the mesh.  If k-1 > 1 the
  next level is Q_1 on the same cells (p-coarsening); then Q_1 on meshes with
  every direction halved (h-coarsening) while every direction has an even
  number of cells and the level has more than ``coarse_cells`` cells.  Every
  level operator is rediscretised: H_l = alpha M^p_l + K_l with the SIP
  penalty of its own degree q and cell size, sigma = (q+1)^2 / h.
* Velocity field (``field="u"``; not in the paper, which preconditions the
  momentum solves with Jacobi).  The stage-s momentum operator on one
  component is m_s M + theta_s (nu A + C(w)) with A the SIP form of eq.
  bilin_diff (Dirichlet walls).  Its symmetric part without advection is
  theta_s nu (alpha M + A) with alpha = m_s / (theta_s nu), and the same
  construction applies to H = alpha M + A: level 0 the velocity space Q_k,
  the velocity penalty (q+1)^2 pen_u / h on every level and the Dirichlet
  boundary terms of A (doubled penalty) instead of the natural condition.
* Transfers.  Prolongation is the embedding of the coarse space in the fine
  one, i.e. the coarse polynomial evaluated at the fine nodes: for p-transfer
  the Q_1 basis at the Q_q nodes of the same cell, for h-transfer the parent
  cell's Q_1 basis at the child cell's nodes.  Restriction is the transpose.
* Smoother.  Chebyshev iteration (the three-term recurrence of Chebyshev
  acceleration for the Jacobi-preconditioned system D^{-1} H x = D^{-1} b) of
  a given degree on the interval [lam/range, safety*lam], where lam is the
  largest Ritz value of ``lanczos_steps`` Lanczos steps on
  D^{-1/2} H D^{-1/2} from a SplitMix64 start vector.
* Coarsest level: dense FP64 Cholesky factorisation.
* V-cycle with zero initial guess, pre- and post-smoothing of the same degree
  (which makes the cycle a symmetric operator), used as the preconditioner of
  a flexible (Polak-Ribiere) CG in FP64.

Every function below computes the plain definition of its step; none shares
code with the GPU library.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import gauss_legendre_01, lagrange_values
from .forms import Discretization
from .mesh import BoxMesh

_MASK = (1 << 64) - 1


def splitmix64(seed, count):
    """The first ``count`` outputs of SplitMix64 (Steele, Lea and Flood,
    OOPSLA 2014; the mixing function of Vigna's public-domain reference code)
    from state ``seed``, as Python integers: the state advances by the golden
    gamma 0x9E3779B97F4A7C15 and each output is the state passed through
    two xor-shift-multiply rounds and a final xor-shift."""
    out = []
    s = int(seed) & _MASK
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def lanczos_start(n, seed=0):
    """Start vector of the Lanczos eigenvalue estimate: entry i is the i-th
    SplitMix64 output from ``seed`` with its top 53 bits scaled to [0, 1),
    minus 1/2."""
    z = splitmix64(seed, n)
    return np.array([(v >> 11) * 2.0 ** -53 for v in z]) - 0.5


def lanczos_largest(H, d, steps, v0):
    """Largest Ritz value of ``steps`` Lanczos steps (no reorthogonalisation)
    on S = D^{-1/2} H D^{-1/2} from v0: the eigenvalue estimate of the
    Jacobi-preconditioned operator D^{-1} H (which is similar to S)."""
    s = 1.0 / np.sqrt(d)
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alphas, betas = [], []
    steps = min(steps, len(v0))
    for j in range(steps):
        w = s * (H @ (s * v))
        a = float(w @ v)
        w = w - a * v - b_prev * v_prev
        alphas.append(a)
        b = float(np.linalg.norm(w))
        if j == steps - 1 or b == 0.0:
            break
        betas.append(b)
        v_prev, v, b_prev = v, w / b, b
    T = np.diag(alphas)
    for i, b in enumerate(betas):
        T[i, i + 1] = T[i + 1, i] = b
    return float(np.linalg.eigvalsh(T).max())


def chebyshev_coefficients(lo, hi, degree):
    """Scalars of the Chebyshev recurrence on [lo, hi]: theta, delta and, for
    steps k = 1 .. degree-1, (c1_k, c2_k) with d_k = c1_k d_{k-1} + c2_k D^{-1} r_k."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    coefs = []
    for _ in range(1, degree):
        rho_new = 1.0 / (2.0 * sigma - rho)
        coefs.append((rho_new * rho, 2.0 * rho_new / delta))
        rho = rho_new
    return theta, delta, coefs


def chebyshev_smooth(H, dinv, b, x, degree, lo, hi):
    """``degree`` steps of Chebyshev acceleration for D^{-1} H x = D^{-1} b on
    [lo, hi] from x (None: zero).  The error is multiplied by
    T_degree((theta - D^{-1}H)/delta) / T_degree(theta/delta)."""
    theta, _, coefs = chebyshev_coefficients(lo, hi, degree)
    if x is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        r = b - H @ x
    d = dinv * r / theta
    for k in range(1, degree + 1):
        x = x + d
        if k == degree:
            break
        r = r - H @ d
        c1, c2 = coefs[k - 1]
        d = c1 * d + c2 * dinv * r
    return x


def _transfer_1d_p(n_fine):
    """E[i, j] = (Q_1 basis j)(fine Gauss node i) on the same cell."""
    zc, _ = gauss_legendre_01(2)
    zf, _ = gauss_legendre_01(n_fine)
    return lagrange_values(zc, zf)


def _transfer_1d_h(b):
    """E_b[i, j] = (parent Q_1 basis j)((b + child node i) / 2), child b in {0, 1}."""
    z, _ = gauss_legendre_01(2)
    return lagrange_values(z, 0.5 * (b + z))


def _kron_cell(tabs):
    """Tensor product of per-direction matrices, x fastest on both axes."""
    out = np.ones((1, 1))
    for t in tabs:             # x first, so kron(t_last, ..., t_x)
        out = np.kron(t, out)
    return out


class Level:
    """One level: mesh, degree q, assembled H_l = alpha M + K and its diagonal
    (field "p": the pressure space's M^p and K; "u": one velocity component's
    mass and SIP form with Dirichlet walls)."""

    def __init__(self, mesh, q, alpha, pen, field="p"):
        self.mesh = mesh
        self.q = int(q)
        if field == "p":
            self.disc = Discretization(mesh, q + 1, nu=1.0, pen_p=pen)
            self.H = (alpha * self.disc.mass_p() + self.disc.sip_p()).tocsr()
        else:
            self.disc = Discretization(mesh, q, nu=1.0, pen_u=pen)
            self.H = (alpha * self.disc.mass_u() + self.disc.sip_u()).tocsr()
        self.d = self.H.diagonal().copy()
        self.N = self.H.shape[0]
        self.nb = (q + 1) ** mesh.dim


def _coarse_mesh(mesh):
    n = tuple(v // 2 for v in mesh.n_cells)
    return BoxMesh(mesh.dim, n, tuple(mesh.lo), tuple(mesh.hi), mesh.periodic)


def _prolongation(fine, coarse):
    """Sparse prolongation from ``coarse`` to ``fine`` (p- or h-transfer)."""
    dim = fine.mesh.dim
    rows, cols, vals = [], [], []
    if fine.mesh.n_cells == coarse.mesh.n_cells:          # p-transfer
        E = _kron_cell([_transfer_1d_p(fine.q + 1)] * dim)
        for c in range(fine.mesh.N):
            I, J = np.nonzero(np.ones_like(E))
            rows.append(c * fine.nb + I)
            cols.append(c * coarse.nb + J)
            vals.append(E[I, J])
    else:                                                  # h-transfer
        Eb = [_transfer_1d_h(0), _transfer_1d_h(1)]
        for c in range(fine.mesh.N):
            ijk = fine.mesh.cell_ijk(c)
            C = coarse.mesh.cell_index([v // 2 for v in ijk])
            E = _kron_cell([Eb[v % 2] for v in ijk])
            I, J = np.nonzero(np.ones_like(E))
            rows.append(c * fine.nb + I)
            cols.append(C * coarse.nb + J)
            vals.append(E[I, J])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.N, coarse.N))


class Multigrid:
    """h/p-multigrid V-cycle for H = alpha M + K on an affine box (periodic
    directions wrap; the others carry the natural Neumann condition for the
    pressure, homogeneous Dirichlet for a velocity component).

    ``disc`` gives the mesh and the velocity degree k (pressure degree k-1);
    ``alpha`` the mass coefficient of the stage; ``field`` "p" or "u"."""

    def __init__(self, disc, alpha, degree=3, lanczos_steps=15, range_=15.0, safety=1.1,
                 coarse_cells=None, seed=0, field="p"):
        mesh = disc.mesh
        if not mesh.affine:
            raise ValueError("the multigrid hierarchy is defined on affine boxes")
        if coarse_cells is None:
            coarse_cells = 64 if mesh.dim == 3 else 16
        self.degree = int(degree)
        self.alpha = float(alpha)
        if field not in ("p", "u"):
            raise ValueError("field must be 'p' or 'u'")
        q0, pen = (disc.k - 1, disc.pen_p) if field == "p" else (disc.k, disc.pen_u)
        levels = [Level(mesh, q0, alpha, pen, field)]
        if q0 > 1:
            levels.append(Level(mesh, 1, alpha, pen, field))
        while True:
            m = levels[-1].mesh
            if m.N <= coarse_cells or any(v % 2 for v in m.n_cells):
                break
            levels.append(Level(_coarse_mesh(m), 1, alpha, pen, field))
        self.levels = levels
        self.P = [_prolongation(levels[i], levels[i + 1]) for i in range(len(levels) - 1)]
        self.lam = []
        self.bounds = []
        for lv in levels[:-1]:
            lam = lanczos_largest(lv.H, lv.d, lanczos_steps, lanczos_start(lv.N, seed))
            self.lam.append(lam)
            self.bounds.append((lam / range_, safety * lam))
        self.coarse = sla.cho_factor(levels[-1].H.toarray(), lower=True)

    def vcycle(self, b, level=0):
        """x = B b: one V-cycle with zero initial guess."""
        if level == len(self.levels) - 1:
            return sla.cho_solve(self.coarse, b)
        lv = self.levels[level]
        lo, hi = self.bounds[level]
        dinv = 1.0 / lv.d
        x = chebyshev_smooth(lv.H, dinv, b, None, self.degree, lo, hi)
        r = b - lv.H @ x
        e = self.vcycle(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ e
        return chebyshev_smooth(lv.H, dinv, b, x, self.degree, lo, hi)


def flexible_pcg(H, b, x, precond, tol, maxiter=500):
    """CG with a (possibly variable) preconditioner and the Polak-Ribiere
    choice beta = z_new.(r_new - r_old) / z_old.r_old; stops on the relative
    true-recurrence residual ||r|| <= tol ||b||.  Returns (x, iterations, history)."""
    bn = np.linalg.norm(b)
    r = b - H @ x
    hist = [np.linalg.norm(r) / bn]
    if hist[-1] <= tol:
        return x, 0, hist
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxiter + 1):
        q = H @ p
        a = rz / (p @ q)
        x = x + a * p
        r_old = r
        r = r - a * q
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            return x, it, hist
        z = precond(r)
        beta = (z @ (r - r_old)) / rz
        rz = r @ z
        p = z + beta * p
    return x, maxiter, hist
