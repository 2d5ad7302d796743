"""Pins of the oracle's adaptive-mesh module (Sec. 4, the adaptive runs).

* forests stay 2:1 balanced and tile the box under random adaptation;
  refining everything and coarsening everything back is the identity;
* with the penalty switched off, the pressure mass matrix and a_p on a mesh
  with hanging nodes equal the conforming forms of the uniformly refined
  mesh (the pinned box-mesh oracle) restricted through the exact embedding
  of the adapted space: the coarse-fine face integrals carry no error;
* the penalty part is symmetric, kills globally continuous fields, and on
  the indicator function of one cell equals the closed-form sum of C |F|
  over that cell's faces;
* the Neumann Helmholtz problem with a manufactured solution converges at
  rate k (pressure degree k - 1) on adapted meshes;
* eta_K of polynomial velocities equals its closed form;
* the marking counts, tie order and size limits;
* transfers: exact for polynomials the spaces hold, coarsening is the L2
  projection, refine-then-coarsen is the identity.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import BoxMesh, Discretization
from oracle.adaptive import AdaptiveDisc, QuadForest, mark, transfer
from oracle.basis import gauss_legendre_01, lagrange_values, tensor


def _random_forest(seed, n_cells=(3, 2), periodic=(False, False), max_level=3, rounds=3,
                   lo=(0.0, 0.0), hi=(1.5, 1.0)):
    rng = np.random.default_rng(seed)
    f = QuadForest(n_cells, lo, hi, periodic, max_level)
    for _ in range(rounds):
        flags = rng.choice([-1, 0, 1], size=f.N, p=[0.35, 0.35, 0.3])
        f = f.adapt(flags)
    return f


def _check_balanced_tiling(f):
    area = 0.0
    for c in range(f.N):
        h = f.size(c)
        area += h[0] * h[1]
        for a in range(2):
            for s in (0, 1):
                nb = f.neighbours(c, a, s)
                if nb[0] in ("C", "c"):
                    assert abs(f.leaves[nb[1]][0] - f.leaves[c][0]) <= 1
                elif nb[0] == "f":
                    for o in nb[1]:
                        assert f.leaves[o][0] == f.leaves[c][0] + 1
    assert abs(area - np.prod(f.hi - f.lo)) < 1e-12
    # no overlap: every finest-level cell is covered exactly once
    L = f.max_level
    cover = np.zeros((f.n_cells[1] << L, f.n_cells[0] << L), dtype=int)
    for (l, i, j) in f.leaves:
        m = 1 << (L - l)
        cover[j * m:(j + 1) * m, i * m:(i + 1) * m] += 1
    assert np.all(cover == 1)
    keys = [f._key(c) for c in f.leaves]
    assert keys == sorted(keys)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("periodic", [(False, False), (True, True), (True, False)])
def test_forest_balanced_tiling(seed, periodic):
    f = _random_forest(seed, periodic=periodic)
    _check_balanced_tiling(f)


def test_refine_all_then_coarsen_all_is_identity():
    f0 = QuadForest((2, 3), (0.0, 0.0), (1.0, 1.5), (False, True), 2)
    f1 = f0.adapt(np.ones(f0.N))
    assert f1.N == 4 * f0.N
    f2 = f1.adapt(-np.ones(f1.N))
    assert f2.leaves == f0.leaves


def test_two_to_one_spreads_refinement():
    """Refining one level-1 cell next to a level-0 cell refines the latter."""
    f = QuadForest((2, 1), (0.0, 0.0), (2.0, 1.0), (False, False), 3)
    flags = np.array([1, 0])
    f = f.adapt(flags)                         # tree 0 refined: 4 + 1 leaves
    c = f.index[(1, 1, 0)]                     # touches tree 1 (level 0)
    flags = np.zeros(f.N, dtype=int)
    flags[c] = 1
    g = f.adapt(flags)
    assert (0, 1, 0) not in g.index and (1, 2, 0) in g.index
    _check_balanced_tiling(g)


def _embedding(f, n, L=None):
    """Prolongation from the adapted space (n nodes per direction) to the
    uniform mesh of level L (default: the finest; BoxMesh order, x fastest)."""
    if L is None:
        L = max(l for (l, _, _) in f.leaves)
    nx, ny = f.n_cells[0] << L, f.n_cells[1] << L
    z, _ = gauss_legendre_01(n)
    nb = n * n
    rows, cols, vals = [], [], []
    for c, (l, i, j) in enumerate(f.leaves):
        m = 1 << (L - l)
        for dj in range(m):
            for di in range(m):
                P = tensor([lagrange_values(z, (di + z) / m), lagrange_values(z, (dj + z) / m)])
                fc = (i * m + di) + nx * (j * m + dj)
                rr, cc = np.meshgrid(np.arange(nb) + fc * nb, np.arange(nb) + c * nb, indexing="ij")
                rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(P.ravel())
    Pi = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(nx * ny * nb, f.N * nb)).tocsr()
    box = BoxMesh(2, (nx, ny), tuple(f.lo), tuple(f.hi), f.periodic)
    return Pi, box


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("periodic", [(False, False), (True, False)])
def test_forms_equal_embedded_conforming_forms_without_penalty(k, periodic):
    f = _random_forest(11 + k, periodic=periodic, max_level=2, rounds=2)
    assert any(f.neighbours(c, a, s)[0] == "f" for c in range(f.N) for a in range(2) for s in (0, 1))
    ad = AdaptiveDisc(f, k, pen_p=0.0)
    Pi, box = _embedding(f, k)
    disc = Discretization(box, k, nu=1.0, pen_p=0.0)
    Mf, Kf = disc.mass_p(), disc.sip_p()
    dM = ad.mass_p() - Pi.T @ Mf @ Pi
    dK = ad.sip_p() - Pi.T @ Kf @ Pi
    assert abs(dM).max() < 1e-13
    assert abs(dK).max() < 1e-11 * abs(Kf).max()


def _penalty_part(f, k):
    return (AdaptiveDisc(f, k, pen_p=1.0).sip_p() - AdaptiveDisc(f, k, pen_p=0.0).sip_p()).tocsr()


@pytest.mark.parametrize("k", [2, 3])
def test_penalty_part_closed_forms(k):
    f = _random_forest(5, max_level=3, rounds=3)
    J = _penalty_part(f, k)
    assert abs(J - J.T).max() < 1e-12 * abs(J).max()
    ad = AdaptiveDisc(f, k)
    xp = ad.node_coords("p")
    # a globally continuous (linear) field has no jumps
    p = 0.3 + xp[:, 0] - 2.0 * xp[:, 1]
    assert np.abs(J @ p).max() < 1e-10 * abs(J).max()
    nbp = k * k
    sig = lambda c, a: k * k / float(f.size(c)[a])
    for c0 in range(0, f.N, max(1, f.N // 7)):
        e = np.zeros(f.N * nbp)
        e[c0 * nbp:(c0 + 1) * nbp] = 1.0
        want = 0.0
        for a in range(2):
            for s in (0, 1):
                nb = f.neighbours(c0, a, s)
                if nb[0] == "C" and nb[1] != c0:
                    want += sig(c0, a) * f.size(c0)[1 - a]
                elif nb[0] == "c":
                    want += 0.5 * (sig(c0, a) + sig(nb[1], a)) * f.size(c0)[1 - a]
                elif nb[0] == "f":
                    for o in nb[1]:
                        want += 0.5 * (sig(c0, a) + sig(o, a)) * f.size(o)[1 - a]
        assert abs(e @ (J @ e) - want) < 1e-12 * want


def test_sip_symmetric_psd_with_constant_kernel():
    f = _random_forest(2, periodic=(True, False))
    K = AdaptiveDisc(f, 3).sip_p()
    assert abs(K - K.T).max() < 1e-12 * abs(K).max()
    assert np.abs(K @ np.ones(K.shape[0])).max() < 1e-11 * abs(K).max()
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev.min() > -1e-10 * ev.max()
    assert np.sum(ev < 1e-9 * ev.max()) == 1


def _mms_error(f, k, alpha=1.0):
    ad = AdaptiveDisc(f, k)
    A = ad.helmholtz_p(alpha)
    ex = lambda x: np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    # right-hand side with an over-integrated rule on every cell
    q, w = gauss_legendre_01(k + 4)
    xr, yr = np.tile(q, len(q)), np.repeat(q, len(q))
    Wq = np.kron(w, w)
    V = tensor([lagrange_values(ad.zp, q)] * 2)
    b = np.zeros(ad.N_p)
    err2 = 0.0
    rhs_f = (2 * np.pi ** 2 + alpha)
    for c in range(f.N):
        o, h = f.origin(c), f.size(c)
        x = np.stack([o[0] + h[0] * xr, o[1] + h[1] * yr], 1)
        b[c * ad.nbp:(c + 1) * ad.nbp] = V.T @ (Wq * h[0] * h[1] * rhs_f * ex(x))
    p = spla.spsolve(A.tocsc(), b)
    for c in range(f.N):
        o, h = f.origin(c), f.size(c)
        x = np.stack([o[0] + h[0] * xr, o[1] + h[1] * yr], 1)
        ph = V @ p[c * ad.nbp:(c + 1) * ad.nbp]
        err2 += float(np.sum(Wq * h[0] * h[1] * (ph - ex(x)) ** 2))
    return np.sqrt(err2)


@pytest.mark.parametrize("k", [2, 3])
def test_neumann_helmholtz_converges_at_rate_k(k):
    f = QuadForest((2, 2), (0.0, 0.0), (1.0, 1.0), (False, False), 5)
    # refine the lower-left quarter twice: hanging faces on two levels
    f = f.adapt(np.array([1, 0, 0, 0]))
    f = f.adapt(np.array([1 if (l, i, j) == (1, 1, 1) or (l, i, j) == (1, 0, 0) else 0
                          for (l, i, j) in f.leaves]))
    errs = []
    for _ in range(3):
        errs.append(_mms_error(f, k))
        f = f.adapt(np.ones(f.N))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(abs(r - k) < 0.35 for r in rates), (errs, rates)


def test_indicator_closed_forms():
    f = _random_forest(3, max_level=2, rounds=2)
    k = 2
    ad = AdaptiveDisc(f, k)
    xu = ad.node_coords("u")
    nb = ad.nbu

    def field(ux, uy):
        u = np.zeros(ad.N_u)
        for c in range(f.N):
            sl = slice(c * nb, (c + 1) * nb)
            u[2 * c * nb:(2 * c + 1) * nb] = ux[sl]
            u[(2 * c + 1) * nb:(2 * c + 2) * nb] = uy[sl]
        return u

    cst = 0.7
    eta = ad.indicator(field(-cst * xu[:, 1], cst * xu[:, 0]))      # omega = 2 c
    for c in range(f.N):
        h = f.size(c)
        assert abs(eta[c] - (h[0] ** 2 + h[1] ** 2) * 4 * cst ** 2 * h[0] * h[1]) < 1e-14
    eta = ad.indicator(field(0.0 * xu[:, 0], xu[:, 0] ** 2))          # omega = 2 x
    for c in range(f.N):
        o, h = f.origin(c), f.size(c)
        x0, x1 = o[0], o[0] + h[0]
        want = (h[0] ** 2 + h[1] ** 2) * 4.0 * (x1 ** 3 - x0 ** 3) / 3.0 * h[1]
        assert abs(eta[c] - want) < 1e-13


def test_marking_fractions_ties_and_limits():
    f = QuadForest((4, 5), (0.0, 0.0), (1.0, 1.25), (False, False), 3)
    f = f.adapt(np.array([1 if c % 3 == 0 else 0 for c in range(f.N)]))
    N = f.N
    rng = np.random.default_rng(0)
    eta = rng.random(N)
    eta[5] = eta[9] = eta.max() + 1.0     # a tie at the top: lower index first
    fl = mark(eta, f, 0.1, 0.3)
    nr, nc = int(0.1 * N), int(0.3 * N)
    order = sorted(range(N), key=lambda c: (-eta[c], c))
    assert set(np.flatnonzero(fl > 0)) == set(order[:nr])
    low = [c for c in sorted(range(N), key=lambda c: (eta[c], c)) if c not in order[:nr]][:nc]
    assert set(np.flatnonzero(fl < 0)) == set(c for c in low if f.leaves[c][0] > 0)
    if nr == 1:
        assert fl[5] == 1 and fl[9] == 0
    # size limits: nothing refined below h_min, nothing coarsened above h_max
    H = f.H.max()
    fl = mark(eta, f, 0.5, 0.5, h_min=H / 2, h_max=H)
    for c in np.flatnonzero(fl > 0):
        assert f.leaves[c][0] == 0
    for c in np.flatnonzero(fl < 0):
        assert f.leaves[c][0] == 1


@pytest.mark.parametrize("n", [2, 3, 4])
def test_transfer_exact_projection_and_roundtrip(n):
    f0 = _random_forest(7, max_level=4, rounds=2)
    rng = np.random.default_rng(1)
    flags = rng.choice([-1, 0, 1], size=f0.N)
    f1 = f0.adapt(flags)
    assert any(c not in f0.index for c in f1.leaves)
    # a polynomial of degree n-1 per direction is held by both spaces
    z, _ = gauss_legendre_01(n)
    def nodes(f):
        out = []
        for c in range(f.N):
            o, h = f.origin(c), f.size(c)
            out.append(np.stack([o[0] + h[0] * np.tile(z, n), o[1] + h[1] * np.repeat(z, n)], 1))
        return np.concatenate(out)
    poly = lambda x: (1 + x[:, 0] ** (n - 1)) * (x[:, 1] ** (n - 1) - 0.5)
    if n >= 2:
        u0 = poly(nodes(f0))
        assert np.abs(transfer(f0, f1, u0, n, 1) - poly(nodes(f1))).max() < 1e-12
    # two components, random field: refine-then-coarsen is the identity
    fr = f0.adapt(np.ones(f0.N))
    v = rng.standard_normal(f0.N * 2 * n * n)
    back = transfer(fr, fr.adapt(-np.ones(fr.N)), transfer(f0, fr, v, n, 2), n, 2)
    assert np.abs(back - v).max() < 1e-12
    # coarsening is the L2 projection: the error is orthogonal to the parent space
    fc = fr.adapt(-np.ones(fr.N))
    w = rng.standard_normal(fr.N * n * n)
    wc = transfer(fr, fc, w, n, 1)
    L = max(l for (l, _, _) in fr.leaves)
    Pi_r, _ = _embedding(fr, n, L)
    Pi_c, _ = _embedding(fc, n, L)
    # mass of the uniform mesh with n Gauss nodes per direction: diagonal weights
    zq, wq = gauss_legendre_01(n)
    hx, hy = fr.H / (1 << L)
    Md = np.tile(np.kron(wq, wq) * hx * hy, Pi_r.shape[0] // (n * n))
    resid = Pi_c.T @ (Md * (Pi_r @ w - Pi_c @ wc))
    assert np.abs(resid).max() < 1e-13


# ---------------------------------------------------------------------------
# velocity forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("periodic", [(False, False), (True, False)])
def test_velocity_forms_equal_embedded_conforming_forms(k, periodic):
    """Without the penalty, the velocity mass and SIP forms (Dirichlet walls
    included) equal the uniform fine mesh's through the exact embedding; with
    a constant advecting field and constant wall data every advection
    integral is exact, so the LF form embeds too."""
    f = _random_forest(21 + k, periodic=periodic, max_level=2, rounds=2)
    ad = AdaptiveDisc(f, k, pen_u=0.0)
    Pi, box = _embedding(f, k + 1)
    disc = Discretization(box, k, nu=1.0, pen_u=0.0)
    assert abs(ad.mass_u() - Pi.T @ disc.mass_u() @ Pi).max() < 1e-13
    Kf = disc.sip_u()
    assert abs(ad.sip_u() - Pi.T @ Kf @ Pi).max() < 1e-11 * abs(Kf).max()
    wc = np.array([0.7, -1.3])
    uDc = np.array([0.4, 2.1])
    wa = np.tile(np.repeat(wc, ad.nbu), f.N)
    wf = np.tile(np.repeat(wc, disc.nbu), box.N)
    uD = np.tile(uDc, (len(ad.boundary_points()), 1))
    Cf = disc.lf_advection(wf, lambda c, a, s, x: np.tile(uDc, (len(x), 1)))
    Ca = ad.lf_advection(wa, uD)
    assert abs(Ca - Pi.T @ Cf @ Pi).max() < 1e-12 * abs(Cf).max()


def test_velocity_penalty_closed_form_and_boundary_points():
    k = 2
    f = _random_forest(8, max_level=3, rounds=3)
    J = (AdaptiveDisc(f, k, pen_u=1.0).sip_u() - AdaptiveDisc(f, k, pen_u=0.0).sip_u()).tocsr()
    nbu = (k + 1) ** 2
    sig = lambda c, a: (k + 1) ** 2 / float(f.size(c)[a])
    for c0 in range(0, f.N, max(1, f.N // 6)):
        e = np.zeros(f.N * nbu)
        e[c0 * nbu:(c0 + 1) * nbu] = 1.0
        want = 0.0
        for a in range(2):
            for s in (0, 1):
                nb = f.neighbours(c0, a, s)
                if nb[0] == "B":
                    want += 2.0 * sig(c0, a) * f.size(c0)[1 - a]
                elif nb[0] == "C":
                    want += sig(c0, a) * f.size(c0)[1 - a]
                elif nb[0] == "c":
                    want += 0.5 * (sig(c0, a) + sig(nb[1], a)) * f.size(c0)[1 - a]
                else:
                    for o in nb[1]:
                        want += 0.5 * (sig(c0, a) + sig(o, a)) * f.size(o)[1 - a]
        assert abs(e @ (J @ e) - want) < 1e-12 * want
    # the boundary points lie on the boundary, n per boundary face
    ad = AdaptiveDisc(f, k)
    x = ad.boundary_points()
    nbf = sum(1 for c in range(f.N) for a in range(2) for s in (0, 1) if f.neighbours(c, a, s)[0] == "B")
    assert x.shape == (nbf * (k + 1), 2)
    on = np.isclose(x[:, 0], f.lo[0]) | np.isclose(x[:, 0], f.hi[0]) | \
        np.isclose(x[:, 1], f.lo[1]) | np.isclose(x[:, 1], f.hi[1])
    assert on.all()


def test_advection_conserves_on_a_periodic_mesh():
    """The constant test function sees no advection on a periodic mesh: its
    gradient vanishes and so do its jumps, so 1^T C(w) u = 0 for every w and
    u; the flux a coarse cell sends through a hanging face is exactly what
    its two fine neighbours receive."""
    k = 3
    f = _random_forest(4, periodic=(True, True), max_level=3, rounds=2)
    assert any(f.neighbours(c, a, s)[0] == "f" for c in range(f.N) for a in range(2) for s in (0, 1))
    ad = AdaptiveDisc(f, k)
    rng = np.random.default_rng(0)
    w = rng.standard_normal(ad.N_u)
    C = ad.lf_advection(w)
    u = rng.standard_normal(C.shape[0])
    assert abs(np.ones(C.shape[0]) @ (C @ u)) < 1e-12 * abs(C).max() * np.abs(u).sum()


@pytest.mark.parametrize("periodic", [(True, True), (False, True)])
def test_advection_cell_self_term_closed_form(periodic):
    """A cellwise constant advecting field W_c and u = v = the indicator of
    one cell: the volume term vanishes and every face (or fine half face) F
    of the cell adds |F| (W_c.n + max(|W_c.n|, |W_nb.n|)) / 2; a wall face
    adds |F| max(|W_c.n|, |(2 u_D - W_c).n|)."""
    k = 2
    f = _random_forest(6, periodic=periodic, max_level=3, rounds=3)
    ad = AdaptiveDisc(f, k)
    rng = np.random.default_rng(3)
    Wc = rng.standard_normal((f.N, 2))
    w = np.stack([np.repeat(Wc[:, 0:1], ad.nbu, 1), np.repeat(Wc[:, 1:2], ad.nbu, 1)], 1).reshape(-1)
    uDc = np.array([0.3, -0.8])
    C = ad.lf_advection(w, np.tile(uDc, (len(ad.boundary_points()), 1)))
    nbu = ad.nbu
    for c0 in range(f.N):
        e = np.zeros(C.shape[0])
        e[c0 * nbu:(c0 + 1) * nbu] = 1.0
        want = 0.0
        for a in range(2):
            for s in (0, 1):
                n = np.zeros(2); n[a] = 1.0 if s else -1.0
                nb = f.neighbours(c0, a, s)
                wn = Wc[c0] @ n
                if nb[0] == "B":
                    want += f.size(c0)[1 - a] * max(abs(wn), abs((2 * uDc - Wc[c0]) @ n))
                elif nb[0] in ("C", "c"):
                    want += f.size(c0)[1 - a] * 0.5 * (wn + max(abs(wn), abs(Wc[nb[1]] @ n)))
                else:
                    for o in nb[1]:
                        want += f.size(o)[1 - a] * 0.5 * (wn + max(abs(wn), abs(Wc[o] @ n)))
        assert abs(e @ (C @ e) - want) < 1e-12 * (1 + abs(want)), c0


# ---------------------------------------------------------------------------
# the explicit and mixed forms, and the TR-BDF2 step on adapted meshes
# ---------------------------------------------------------------------------
def _vector_embedding(Pi, ncell_f, ncell_c, nb):
    """Componentwise embedding of [cell][component][node] vectors."""
    Pi = Pi.tocoo()
    r, c, v = [], [], []
    for comp in range(2):
        fr, fn = np.divmod(Pi.row, nb)
        cr, cn = np.divmod(Pi.col, nb)
        r.append((fr * 2 + comp) * nb + fn)
        c.append((cr * 2 + comp) * nb + cn)
        v.append(Pi.data)
    return sp.coo_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))),
                         shape=(2 * ncell_f * nb, 2 * ncell_c * nb)).tocsr()


@pytest.mark.parametrize("periodic", [(False, False), (True, False)])
def test_explicit_and_mixed_forms_equal_embedded_conforming_forms(periodic):
    k = 3
    f = _random_forest(31, periodic=periodic, max_level=2, rounds=2)
    ad = AdaptiveDisc(f, k, nu=0.1)
    Pu, box = _embedding(f, k + 1)
    Pp, _ = _embedding(f, k)
    disc = Discretization(box, k, nu=0.1)
    Puv = _vector_embedding(Pu, box.N, f.N, ad.nbu)
    L0 = disc.explicit_diffusion()
    assert abs(ad.explicit_diffusion() - Pu.T @ L0 @ Pu).max() < 1e-11 * abs(L0).max()
    for name, A, L, R in (("weak_gradient", ad.weak_gradient(), Puv, Pp),
                          ("divergence", ad.divergence(), Pp, Puv),
                          ("projection", ad.projection(), Puv, Pp),
                          ("mass_u_vector", ad.mass_u_vector(), Puv, Puv)):
        ref = getattr(disc, name)()
        assert abs(A - L.T @ ref @ R).max() < 1e-12 * abs(ref).max(), name
    wc = np.array([-0.4, 0.9])
    wa = np.tile(np.repeat(wc, ad.nbu), f.N)
    wf = np.tile(np.repeat(wc, disc.nbu), box.N)
    A0 = disc.explicit_advection(wf)
    assert abs(ad.explicit_advection(wa) - Pu.T @ A0 @ Pu).max() < 1e-12 * abs(A0).max()


@pytest.mark.parametrize("walls", [False, True])
def test_trbdf2_step_on_a_one_level_forest_equals_the_box_oracle(walls):
    """Every cell at level 1 and no hanging node: the oracle's TR-BDF2 step
    (two fixed-point solves per stage) on the adaptive forms equals the box
    oracle's step on the same cells (Morton vs lexicographic order)."""
    import synthetic
    from oracle import TRBDF2
    k, nu, dt = 3, 0.05, 0.02
    per = (not walls, not walls)
    f = QuadForest((2, 2), (0.0, 0.0), (1.0, 1.0), per, 2)
    f = f.adapt(np.ones(f.N))
    ad = AdaptiveDisc(f, k, nu=nu)
    box = BoxMesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), per)
    disc = Discretization(box, k, nu=nu)
    perm = np.array([i + 4 * j for (_, i, j) in f.leaves])   # adapted cell -> box cell
    def to_box(v, nb, ncomp):
        out = np.empty_like(v)
        V = v.reshape(f.N, ncomp * nb)
        out.reshape(box.N, ncomp * nb)[perm] = V
        return out
    xu = disc.node_coords("u")
    if walls:
        ex = lambda x, t: synthetic.kovasznay(x - 0.5, 40.0)[0]
        u0 = synthetic.nodal_velocity(ex(xu, 0.0), 2, disc.nbu)
        uD = ex
    else:
        u0 = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, 0.0, nu)[0], 2, disc.nbu)
        uD = None
    p0 = np.sin(2 * np.pi * disc.node_coords("p")[:, 0])
    # the same fields on the adapted cells
    ua = u0.reshape(box.N, -1)[perm].reshape(-1)
    pa = p0.reshape(box.N, -1)[perm].reshape(-1)
    sb = TRBDF2(disc, dt, uD=uD, nonlinear_iters=2)
    sa = TRBDF2(ad, dt, uD=uD, nonlinear_iters=2)
    ub, hb, pb, _ = sb.step(u0, u0, p0, 0.0)
    uad, ha, pad, _ = sa.step(ua, ua, pa, 0.0)
    assert np.abs(to_box(uad, disc.nbu, 2) - ub).max() < 1e-11 * np.abs(ub).max()
    assert np.abs(to_box(pad, disc.nbp, 1) - pb).max() < 1e-10 * np.abs(pb).max()


def test_row_restricted_assembly_equals_full_rows():
    """The forms assembled for a few cells give those cells' rows of the
    full matrices (used for sampled comparisons on large meshes)."""
    k = 3
    f = _random_forest(12, max_level=3, rounds=3)
    ad = AdaptiveDisc(f, k)
    rng = np.random.default_rng(5)
    cells = sorted(rng.choice(f.N, size=min(7, f.N), replace=False).tolist())
    rp = np.concatenate([np.arange(c * ad.nbp, (c + 1) * ad.nbp) for c in cells])
    ru = np.concatenate([np.arange(c * ad.nbu, (c + 1) * ad.nbu) for c in cells])
    A, Ar = ad.helmholtz_p(2.0), ad.helmholtz_p(2.0, cells)
    assert abs(A[rp] - Ar[rp]).max() < 1e-14 * abs(A).max()   # summation order only
    w = rng.standard_normal(ad.N_u)
    uD = rng.standard_normal((len(ad.boundary_points()), 2))
    for full, part in ((ad.sip_u(), ad.sip_u(cells)), (ad.mass_u(), ad.mass_u(cells)),
                       (ad.lf_advection(w, uD), ad.lf_advection(w, uD, cells))):
        assert abs(full[ru] - part[ru]).max() < 1e-14 * abs(full).max()
    u = rng.standard_normal(ad.N_u)
    yf = ad.apply_momentum(1.0, 0.1, 0.5, w, u, uD)
    yr = ad.apply_momentum(1.0, 0.1, 0.5, w, u, uD, cells)
    rv = np.concatenate([np.arange(c * 2 * ad.nbu, (c + 1) * 2 * ad.nbu) for c in cells])
    assert np.abs(yf[rv] - yr[rv]).max() < 1e-13 * np.abs(yf).max()
