// Adaptive 2D quadrilateral meshes with hanging nodes (the adaptive runs of
// Sec. 4): the forest of quadtrees on the host, its device view, the
// refinement indicator, fixed-fraction marking, remeshing with field
// transfer, the pressure Helmholtz operator and its Jacobi CG solve, and the
// momentum operator (mass, SIP diffusion, Lax-Friedrichs advection, walls)
// on the adapted mesh; the C ABI of all of it.
//
// The forest lives on the host: remeshing happens every few hundred or
// thousand steps and is integer bookkeeping over the cell list, while every
// per-DoF operation (operators, indicator, transfer, reductions) runs in the
// kernels of amr.hip on the device view built here after each remesh.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "amr.hpp"
#include "internal.hpp"
#include "krylov.hpp"

using trbdg::Error;
namespace A = trbdg::amr;

namespace {

struct Leaf {
    int l, i, j;
};

inline uint64_t pack(int l, int i, int j) {
    return ((uint64_t)l << 58) | ((uint64_t)(uint32_t)i << 29) | (uint64_t)(uint32_t)j;
}

inline uint64_t morton(uint64_t x, uint64_t y, int bits) {
    uint64_t m = 0;
    for (int b = 0; b < bits; ++b) {
        m |= ((x >> b) & 1u) << (2 * b);
        m |= ((y >> b) & 1u) << (2 * b + 1);
    }
    return m;
}

struct Nb {
    int kind;      // A::FACE_*
    int n0, n1;    // neighbour, or the two finer ones (tangential halves 0, 1)
    int half;      // FACE_COARSER: the half of the neighbour's face
};

struct Forest {
    int nc[2] = {0, 0};
    double lo[2] = {0, 0}, H[2] = {0, 0};
    int per[2] = {0, 0};
    int maxl = 0;
    std::vector<Leaf> leaves;
    std::unordered_map<uint64_t, int> index;

    std::pair<int64_t, uint64_t> key(const Leaf& c) const {
        const int tx = c.i >> c.l, ty = c.j >> c.l;
        const uint64_t li = (uint64_t)(c.i - (tx << c.l)) << (maxl - c.l);
        const uint64_t lj = (uint64_t)(c.j - (ty << c.l)) << (maxl - c.l);
        return {(int64_t)ty * nc[0] + tx, morton(li, lj, maxl)};
    }

    void finalize() {
        std::sort(leaves.begin(), leaves.end(),
                  [&](const Leaf& a, const Leaf& b) { return key(a) < key(b); });
        index.clear();
        index.reserve(leaves.size() * 2);
        for (size_t n = 0; n < leaves.size(); ++n)
            index[pack(leaves[n].l, leaves[n].i, leaves[n].j)] = (int)n;
    }

    int find(int l, int i, int j) const {
        auto it = index.find(pack(l, i, j));
        return it == index.end() ? -1 : it->second;
    }

    double size(int c, int a) const { return H[a] / (double)(1 << leaves[c].l); }

    Nb neighbours(int c, int a, int s) const {
        const Leaf& L = leaves[c];
        int ij[2] = {L.i, L.j};
        ij[a] += s ? 1 : -1;
        const int n = nc[a] << L.l;
        if (ij[a] < 0 || ij[a] >= n) {
            if (!per[a]) return {A::FACE_BOUNDARY, -1, -1, 0};
            ij[a] = (ij[a] % n + n) % n;
        }
        int o = find(L.l, ij[0], ij[1]);
        if (o >= 0) return {A::FACE_SAME, o, -1, 0};
        if (L.l > 0) {
            o = find(L.l - 1, ij[0] >> 1, ij[1] >> 1);
            if (o >= 0) return {A::FACE_COARSER, o, -1, ij[1 - a] & 1};
        }
        int kids[2];
        for (int h = 0; h < 2; ++h) {
            int ch[2] = {2 * ij[0], 2 * ij[1]};
            ch[a] += s ? 0 : 1;
            ch[1 - a] += h;
            kids[h] = find(L.l + 1, ch[0], ch[1]);
            if (kids[h] < 0) throw Error(TBDG_EINVAL, "adaptive mesh is not 2:1 balanced");
        }
        return {A::FACE_FINER, kids[0], kids[1], 0};
    }

    void face_leaves(int c, std::vector<int>& out) const {
        out.clear();
        for (int a = 0; a < 2; ++a)
            for (int s = 0; s < 2; ++s) {
                const Nb nb = neighbours(c, a, s);
                if (nb.kind == A::FACE_SAME || nb.kind == A::FACE_COARSER) out.push_back(nb.n0);
                else if (nb.kind == A::FACE_FINER) {
                    out.push_back(nb.n0);
                    out.push_back(nb.n1);
                }
            }
    }

    // The adapted forest: flags > 0 refine, < 0 coarsen; refinement spreads
    // to coarser face neighbours until the refined mesh is balanced; a family
    // of four flagged, unrefined leaves is coarsened unless a face neighbour
    // would end finer than the family's leaves (families dropped until the
    // set is consistent with the final levels).
    Forest adapt(const int8_t* flags) const {
        const int N = (int)leaves.size();
        std::vector<char> ref(N, 0);
        std::vector<int> work, nbs;
        for (int c = 0; c < N; ++c)
            if (flags[c] > 0 && leaves[c].l < maxl) {
                ref[c] = 1;
                work.push_back(c);
            }
        while (!work.empty()) {
            const int c = work.back();
            work.pop_back();
            face_leaves(c, nbs);
            for (int o : nbs)
                if (leaves[o].l < leaves[c].l && !ref[o]) {
                    ref[o] = 1;
                    work.push_back(o);
                }
        }
        std::unordered_map<uint64_t, std::vector<int>> fam;
        for (int c = 0; c < N; ++c) {
            const Leaf& L = leaves[c];
            if (L.l > 0 && flags[c] < 0 && !ref[c])
                fam[pack(L.l - 1, L.i >> 1, L.j >> 1)].push_back(c);
        }
        std::vector<uint64_t> live;
        for (auto& kv : fam)
            if (kv.second.size() == 4) live.push_back(kv.first);
        std::vector<uint64_t> member(N, ~(uint64_t)0);
        for (;;) {
            std::fill(member.begin(), member.end(), ~(uint64_t)0);
            for (uint64_t p : live)
                for (int c : fam[p]) member[c] = p;
            std::vector<uint64_t> keep;
            for (uint64_t p : live) {
                bool ok = true;
                for (int c : fam[p]) {
                    face_leaves(c, nbs);
                    for (int o : nbs) {
                        if (member[o] == p) continue;
                        const int fin = leaves[o].l + (ref[o] ? 1 : 0) - (member[o] != ~(uint64_t)0 ? 1 : 0);
                        if (fin > leaves[c].l) ok = false;
                    }
                }
                if (ok) keep.push_back(p);
            }
            if (keep.size() == live.size()) break;
            live.swap(keep);
        }
        std::fill(member.begin(), member.end(), ~(uint64_t)0);
        for (uint64_t p : live)
            for (int c : fam[p]) member[c] = p;
        Forest F;
        std::memcpy(F.nc, nc, sizeof nc);
        std::memcpy(F.lo, lo, sizeof lo);
        std::memcpy(F.H, H, sizeof H);
        std::memcpy(F.per, per, sizeof per);
        F.maxl = maxl;
        for (int c = 0; c < N; ++c) {
            const Leaf& L = leaves[c];
            if (ref[c]) {
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) F.leaves.push_back({L.l + 1, 2 * L.i + di, 2 * L.j + dj});
            } else if (member[c] != ~(uint64_t)0) {
                // the family's parent, once (from its first child in (di, dj) order)
                if ((L.i & 1) == 0 && (L.j & 1) == 0) F.leaves.push_back({L.l - 1, L.i >> 1, L.j >> 1});
            } else {
                F.leaves.push_back(L);
            }
        }
        F.finalize();
        return F;
    }
};

void tab1(int n, A::Tab1& t) {
    std::memset(&t, 0, sizeof t);
    t.n = n;
    trbdg::gauss_legendre(n, t.z, t.W);
    auto val = [&](int j, double x) { return trbdg::lagrange_value(t.z, n, j, x); };
    auto der = [&](int j, double x) {
        // l_j'(x) by the product rule over the factors of l_j
        double s = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == j) continue;
            double term = 1.0 / (t.z[j] - t.z[m]);
            for (int q = 0; q < n; ++q)
                if (q != j && q != m) term *= (x - t.z[q]) / (t.z[j] - t.z[q]);
            s += term;
        }
        return s;
    };
    for (int m = 0; m < n; ++m)
        for (int j = 0; j < n; ++j) t.D[m * n + j] = der(j, t.z[m]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int m = 0; m < n; ++m) s += t.W[m] * t.D[m * n + i] * t.D[m * n + j];
            t.S[i * n + j] = s;
        }
    for (int j = 0; j < n; ++j) {
        t.L[0][j] = val(j, 0.0);
        t.L[1][j] = val(j, 1.0);
        t.dL[0][j] = der(j, 0.0);
        t.dL[1][j] = der(j, 1.0);
    }
    for (int h = 0; h < 2; ++h)
        for (int q = 0; q < n; ++q)
            for (int m = 0; m < n; ++m) t.T[h][q * n + m] = val(m, 0.5 * (h + t.z[q]));
}

void mixtab(const A::Tab1& tu, const A::Tab1& tp, A::MixTab& x) {
    std::memset(&x, 0, sizeof x);
    x.n = tu.n;
    x.np = tp.n;
    const int n = tu.n, np = tp.n;
    auto dval = [&](int m, double z) {
        double sum = 0.0;
        for (int r = 0; r < np; ++r) {
            if (r == m) continue;
            double term = 1.0 / (tp.z[m] - tp.z[r]);
            for (int q = 0; q < np; ++q)
                if (q != m && q != r) term *= (z - tp.z[q]) / (tp.z[m] - tp.z[q]);
            sum += term;
        }
        return sum;
    };
    for (int q = 0; q < n; ++q)
        for (int m = 0; m < np; ++m) {
            x.I[q * np + m] = trbdg::lagrange_value(tp.z, np, m, tu.z[q]);
            x.DI[q * np + m] = dval(m, tu.z[q]);
            for (int h = 0; h < 2; ++h)
                x.Ih[h][q * np + m] = trbdg::lagrange_value(tp.z, np, m, 0.5 * (h + tu.z[q]));
        }
    for (int m = 0; m < np; ++m) {
        x.Lp[0][m] = trbdg::lagrange_value(tp.z, np, m, 0.0);
        x.Lp[1][m] = trbdg::lagrange_value(tp.z, np, m, 1.0);
    }
}

template <typename T>
T* devalloc(int64_t count) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)(count > 0 ? count : 1));
    if (e != hipSuccess) throw Error(TBDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return static_cast<T*>(p);
}

template <typename T>
void devfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

struct tbdg_amr {
    int device = 0;
    hipStream_t stream = nullptr;
    int k = 2;
    double pen_p = 1.0;
    Forest F, next;
    bool planned = false;
    A::Tab1 tp, tu;
    A::MixTab mx;
    double nu = 0.0, dt = 0.0, c = 1.0e3;   // tbdg_amr_set_flow
    bool flow = false;
    double* sv = nullptr;   // step vectors: velocity x6, pressure x3
    int64_t sv_cap = 0;
    int *level = nullptr, *meta = nullptr, *nbr = nullptr, *bface = nullptr;
    int64_t n_bfaces = 0;
    double pen_u = 1.0;
    int64_t geo_cap = 0;
    int *xkind = nullptr, *xsrc = nullptr;
    int64_t x_cap = 0;
    double *cg = nullptr;   // r, z, p, q, d
    int64_t cg_cap = 0;
    double* gm = nullptr;   // momentum GMRES: basis, z, diagonal
    int64_t gm_cap = 0;
    double* part = nullptr;
    double* ppart = nullptr;     // block partials of the operator kernel
    int64_t ppart_cap = 0;
    double* blk = nullptr;       // cell blocks of the pressure operator (FP64)
    float* blkinv = nullptr;     // their inverses (FP32)
    int64_t blk_cap = 0;
    double* bpart = nullptr;     // block partials of the block-Jacobi apply
    int64_t bpart_cap = 0;
    double* scal = nullptr;      // device scalars: rz[2], pq, rr, bb
    double* gdev = nullptr;      // GMRES: the Gram-Schmidt coefficients, w.w, |w'|^2, 1/|w'|
    double* gpart = nullptr;     // GMRES: block partials of the multi-dots
    double* host = nullptr;      // pinned
    std::string last_error;

    int64_t Nc() const { return (int64_t)F.leaves.size(); }
    int64_t Np() const { return Nc() * k * k; }
    int64_t Nu() const { return Nc() * 2 * (k + 1) * (k + 1); }

    A::Geo geo() const {
        A::Geo g;
        g.level = level;
        g.meta = meta;
        g.nbr = nbr;
        g.bface = bface;
        g.Nc = (int)Nc();
        g.H[0] = F.H[0];
        g.H[1] = F.H[1];
        g.csig = (double)k * k * pen_p;
        g.csig_u = (double)(k + 1) * (k + 1) * pen_u;
        return g;
    }

    // device connectivity of the current forest
    void upload() {
        const int64_t N = Nc();
        std::vector<int> lv(N), mt(4 * N), nb(8 * N, -1), bf(4 * N, -1);
        n_bfaces = 0;
        for (int64_t c = 0; c < N; ++c) {
            lv[c] = F.leaves[c].l;
            for (int a = 0; a < 2; ++a)
                for (int s = 0; s < 2; ++s) {
                    const int f = 2 * a + s;
                    const Nb o = F.neighbours((int)c, a, s);
                    mt[4 * c + f] = o.kind | (o.half << 4);
                    nb[8 * c + 2 * f] = o.n0;
                    nb[8 * c + 2 * f + 1] = o.n1;
                    if (o.kind == A::FACE_BOUNDARY) bf[4 * c + f] = (int)n_bfaces++;
                }
        }
        if (N > geo_cap) {
            devfree(level);
            devfree(meta);
            devfree(nbr);
            devfree(bface);
            const int64_t cap = std::max<int64_t>(N, geo_cap * 3 / 2);
            level = devalloc<int>(cap);
            meta = devalloc<int>(4 * cap);
            nbr = devalloc<int>(8 * cap);
            bface = devalloc<int>(4 * cap);
            geo_cap = cap;
        }
        if (N > 0) {
            TBDG_HIP(hipMemcpyAsync(level, lv.data(), sizeof(int) * N, hipMemcpyHostToDevice, stream));
            TBDG_HIP(hipMemcpyAsync(meta, mt.data(), sizeof(int) * 4 * N, hipMemcpyHostToDevice, stream));
            TBDG_HIP(hipMemcpyAsync(nbr, nb.data(), sizeof(int) * 8 * N, hipMemcpyHostToDevice, stream));
            TBDG_HIP(hipMemcpyAsync(bface, bf.data(), sizeof(int) * 4 * N, hipMemcpyHostToDevice, stream));
        }
        // the host vectors die here: wait for the copies
        TBDG_HIP(hipStreamSynchronize(stream));
    }

    void free_all() {
        devfree(level);
        devfree(meta);
        devfree(nbr);
        devfree(bface);
        devfree(xkind);
        devfree(xsrc);
        devfree(cg);
        devfree(gm);
        devfree(sv);
        devfree(part);
        devfree(ppart);
        devfree(blk);
        devfree(blkinv);
        devfree(bpart);
        devfree(scal);
        devfree(gdev);
        devfree(gpart);
        if (host) (void)hipHostFree(host);
        host = nullptr;
    }
};

namespace {

constexpr int DOT_BLOCKS = 1024;
constexpr int kGmMaxRestart = 60;   // the adaptive GMRES's largest basis
constexpr int kGmBlocks = 256;      // blocks per vector of its multi-dots
constexpr int kGmScalars = 72;      // device / pinned scalars (>= kGmMaxRestart + 4)

template <class F>
tbdg_status aguard(tbdg_amr* m, F&& f) {
    try {
        if (m) TBDG_HIP(hipSetDevice(m->device));
        return f();
    } catch (const Error& e) {
        if (m) m->last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        if (m) m->last_error = "host allocation failed";
        return TBDG_ENOMEM;
    } catch (const std::exception& e) {
        if (m) m->last_error = e.what();
        return TBDG_EINVAL;
    }
}

void need(bool ok, const char* msg) {
    if (!ok) throw Error(TBDG_EINVAL, msg);
}

double dot(tbdg_amr* m, int64_t n, const double* a, const double* b, int slot) {
    A::launch_amr_dot(m->stream, n, a, b, m->part, DOT_BLOCKS, m->scal + slot);
    TBDG_HIP(hipMemcpyAsync(m->host, m->scal + slot, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    TBDG_HIP(hipStreamSynchronize(m->stream));
    return m->host[0];
}

// TR-BDF2 constants (eq. trbdf2, second_stage) and the extrapolation
// weights of the advecting velocity (stage 1 to its midpoint from the
// previous step's stage value, stage 2 to t^{n+1}), as on the box mesh
struct Trbdf2 {
    double g, a31, a32, a33, e1[2], e2[2];
    Trbdf2() {
        g = 2.0 - std::sqrt(2.0);
        a31 = (1.0 - g) / (2.0 * (2.0 - g));
        a32 = a31;
        a33 = 1.0 / (2.0 - g);
        e1[0] = 1.0 + g / (2.0 * (1.0 - g));
        e1[1] = -g / (2.0 * (1.0 - g));
        e2[0] = 1.0 + (1.0 - g) / g;
        e2[1] = -(1.0 - g) / g;
    }
    double beta(int s) const { return s == 1 ? g : 1.0 - g; }
    double theta(int s) const { return s == 1 ? 0.5 : a33; }
};

void rhs_momentum_amr(tbdg_amr* m, int s, const double* u_n, const double* u_g, const double* w,
                      const double* w_ex, const double* p, const double* uD, double* out) {
    const Trbdf2 T;
    const A::Geo g = m->geo();
    const double ms = 1.0 / (T.beta(s) * m->dt);
    A::ExplicitArgs e{};
    e.visc = m->nu;
    e.thd = T.theta(s);
    e.wd = w;
    e.uD = m->n_bfaces ? uD : nullptr;
    e.p = p;
    e.cg = 1.0;
    e.acc = false;
    if (s == 1) {
        e.mcoef = ms;
        e.uprev = u_n;
        e.cl = -T.theta(1) * m->nu;
        e.ca = T.theta(1);
        e.ue = u_n;
        e.we = w_ex ? w_ex : w;
        A::launch_amr_explicit(m->stream, g, m->tu, m->mx, e, out);
    } else {
        e.mcoef = ms;
        e.uprev = u_g;
        e.cl = -m->nu * T.a32;
        e.ca = T.a32;
        e.ue = u_g;
        e.we = u_g;
        A::launch_amr_explicit(m->stream, g, m->tu, m->mx, e, out);
        A::ExplicitArgs e2{};
        e2.cl = -m->nu * T.a31;
        e2.ca = T.a31;
        e2.ue = u_n;
        e2.we = u_n;
        e2.acc = true;
        A::launch_amr_explicit(m->stream, g, m->tu, m->mx, e2, out);
    }
}

void rhs_pressure_amr(tbdg_amr* m, int s, const double* u_ss, const double* p, double* out) {
    const Trbdf2 T;
    const double b = T.beta(s) * m->dt;
    const double alpha = std::isinf(m->c) ? 0.0 : 1.0 / (m->c * m->c * b * b);
    A::launch_amr_rhs_p(m->stream, m->geo(), m->tu, m->mx, alpha, p, 1.0 / b, u_ss, out);
}

}  // namespace

extern "C" {

tbdg_status tbdg_amr_create(const tbdg_amr_desc* d, void* hip_stream, tbdg_amr** out) {
    if (!out) return TBDG_EINVAL;
    *out = nullptr;
    if (!d) return TBDG_EINVAL;
    tbdg_amr* m = nullptr;
    try {
        m = new tbdg_amr();
    } catch (const std::bad_alloc&) {
        return TBDG_ENOMEM;
    }
    const tbdg_status st = aguard(nullptr, [&]() {
        for (int a = 0; a < 2; ++a) {
            need(d->n_cells[a] >= 1, "n_cells must be >= 1");
            need(std::isfinite(d->lo[a]) && std::isfinite(d->hi[a]) && d->lo[a] < d->hi[a],
                 "need finite lo < hi");
            need(!d->periodic[a] || d->n_cells[a] >= 2, "a periodic direction needs >= 2 base cells");
        }
        need(d->k >= 1 && d->k <= 7, "velocity degree k must be 1..7");
        need(d->max_level >= 0 && d->max_level <= 20, "max_level must be 0..20");
        for (int a = 0; a < 2; ++a)
            need(((int64_t)d->n_cells[a] << d->max_level) < ((int64_t)1 << 29),
                 "n_cells << max_level must stay below 2^29");
        need(std::isfinite(d->pen_p) && d->pen_p >= 0.0, "pen_p must be finite and >= 0");
        need(std::isfinite(d->pen_u) && d->pen_u >= 0.0, "pen_u must be finite and >= 0");
        TBDG_HIP(hipGetDevice(&m->device));
        m->stream = static_cast<hipStream_t>(hip_stream);
        m->k = d->k;
        m->pen_p = d->pen_p;
        m->pen_u = d->pen_u;
        Forest& F = m->F;
        for (int a = 0; a < 2; ++a) {
            F.nc[a] = d->n_cells[a];
            F.lo[a] = d->lo[a];
            F.H[a] = (d->hi[a] - d->lo[a]) / d->n_cells[a];
            F.per[a] = d->periodic[a] != 0;
        }
        F.maxl = d->max_level;
        for (int j = 0; j < F.nc[1]; ++j)
            for (int i = 0; i < F.nc[0]; ++i) F.leaves.push_back({0, i, j});
        F.finalize();
        tab1(m->k, m->tp);
        tab1(m->k + 1, m->tu);
        mixtab(m->tu, m->tp, m->mx);
        m->part = devalloc<double>(DOT_BLOCKS);
        m->scal = devalloc<double>(8);
        m->gdev = devalloc<double>(kGmScalars);
        m->gpart = devalloc<double>((int64_t)(kGmMaxRestart + 1) * kGmBlocks);
        TBDG_HIP(hipHostMalloc((void**)&m->host, kGmScalars * sizeof(double), hipHostMallocDefault));
        m->upload();
        return TBDG_OK;
    });
    if (st != TBDG_OK) {
        m->free_all();
        delete m;
        return st;
    }
    *out = m;
    return TBDG_OK;
}

void tbdg_amr_destroy(tbdg_amr* m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    m->free_all();
    delete m;
}

const char* tbdg_amr_last_error(const tbdg_amr* m) { return m ? m->last_error.c_str() : "null handle"; }

tbdg_status tbdg_amr_set_stream(tbdg_amr* m, void* hip_stream) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        m->stream = static_cast<hipStream_t>(hip_stream);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_sizes(const tbdg_amr* m, int64_t* n_cells, int64_t* n_u, int64_t* n_p) {
    if (!m) return TBDG_EINVAL;
    if (n_cells) *n_cells = m->Nc();
    if (n_u) *n_u = m->Nu();
    if (n_p) *n_p = m->Np();
    return TBDG_OK;
}

tbdg_status tbdg_amr_leaves(const tbdg_amr* m, int32_t* lij) {
    if (!m || !lij) return TBDG_EINVAL;
    for (int64_t c = 0; c < m->Nc(); ++c) {
        lij[3 * c] = m->F.leaves[c].l;
        lij[3 * c + 1] = m->F.leaves[c].i;
        lij[3 * c + 2] = m->F.leaves[c].j;
    }
    return TBDG_OK;
}

tbdg_status tbdg_amr_apply_pressure(tbdg_amr* m, double alpha, const double* p, double* y) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(alpha), "alpha must be finite");
        need(m->Nc() == 0 || (p && y), "null vector");
        A::launch_amr_pressure(m->stream, m->geo(), m->tp, alpha, p, y, false);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_face_qpoints(const tbdg_amr* m, int64_t* n_points, double* xy) {
    if (!m || !n_points) return TBDG_EINVAL;
    return aguard(const_cast<tbdg_amr*>(m), [&]() {
        const int n = m->k + 1;
        *n_points = m->n_bfaces * n;
        if (!xy || m->n_bfaces == 0) return TBDG_OK;
        std::vector<double> pts(2 * (size_t)*n_points);
        const Forest& F = m->F;
        int64_t b = 0;
        for (int64_t c = 0; c < m->Nc(); ++c) {
            const Leaf& L = F.leaves[c];
            const double h[2] = {F.size((int)c, 0), F.size((int)c, 1)};
            const double o[2] = {F.lo[0] + L.i * h[0], F.lo[1] + L.j * h[1]};
            for (int a = 0; a < 2; ++a)
                for (int s = 0; s < 2; ++s) {
                    if (F.neighbours((int)c, a, s).kind != A::FACE_BOUNDARY) continue;
                    for (int q = 0; q < n; ++q) {
                        pts[2 * (b * n + q) + a] = o[a] + s * h[a];
                        pts[2 * (b * n + q) + 1 - a] = o[1 - a] + h[1 - a] * m->tu.z[q];
                    }
                    ++b;
                }
        }
        TBDG_HIP(hipMemcpyAsync(xy, pts.data(), sizeof(double) * pts.size(), hipMemcpyHostToDevice,
                                m->stream));
        TBDG_HIP(hipStreamSynchronize(m->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_apply_momentum(tbdg_amr* m, double mc, double tnu, double th, const double* w,
                                    const double* u, const double* uD, double* y) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(mc) && std::isfinite(tnu) && std::isfinite(th), "coefficients must be finite");
        need(m->Nc() == 0 || (w && u && y), "null vector");
        need(m->n_bfaces == 0 || uD, "the mesh has walls: wall data uD needed");
        need(u != y && w != y, "y must not alias u or w");
        A::launch_amr_momentum(m->stream, m->geo(), m->tu, mc, tnu, th, w, u, uD, y);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_solve_momentum(tbdg_amr* m, double mc, double tnu, double th, const double* w,
                                    const double* uD, const double* b, double* x, double tol,
                                    int maxiter, int restart, tbdg_solve_info* info) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(mc) && std::isfinite(tnu) && std::isfinite(th), "coefficients must be finite");
        need(tol > 0.0 && maxiter >= 0 && restart >= 1 && restart <= kGmMaxRestart,
             "need tol > 0, restart 1..60");
        need(w && b && x, "null vector");
        need(m->n_bfaces == 0 || uD, "the mesh has walls: wall data uD needed");
        need(x != w && b != w && x != b, "x, b and w must be distinct");
        const int64_t n = m->Nu();
        const int mr = restart;
        // basis (mr + 1 vectors), z, the diagonal
        const int64_t need_cap = (int64_t)(mr + 3) * n;
        if (need_cap > m->gm_cap) {
            devfree(m->gm);
            m->gm = devalloc<double>(need_cap);
            m->gm_cap = need_cap;
        }
        double* V = m->gm;
        double* z = V + (int64_t)(mr + 1) * n;
        double* dg = z + n;
        const hipStream_t st = m->stream;
        const A::Geo g = m->geo();
        auto op = [&](const double* in, double* out) {
            A::launch_amr_momentum(st, g, m->tu, mc, tnu, th, w, in, uD, out);
        };
        A::launch_amr_momentum_diag(st, g, m->tu, mc, tnu, dg);
        const int Gd = (int)std::min<int64_t>(kGmBlocks, std::max<int64_t>(1, (n + 255) / 256));
        tbdg_solve_info inf{0, 0.0, 0.0, 0, 0};
        const double bnorm = std::sqrt(dot(m, n, b, b, 4));
        if (bnorm == 0.0) {
            TBDG_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
            if (info) *info = inf;
            return TBDG_OK;
        }
        if (!std::isfinite(bnorm)) return TBDG_ENAN;
        std::vector<double> H((size_t)(mr + 1) * mr), cs(mr), sn(mr), gv(mr + 1), y(mr);
        int total = 0;
        tbdg_status status = TBDG_ENOTCONV;
        double res = 0.0;
        for (bool first = true;; first = false) {
            // true residual r = b - A x into V_0
            op(x, z);
            trbdg::vec_axpby(st, n, 1.0, b, -1.0, z, V);
            const double beta = std::sqrt(dot(m, n, V, V, 3));
            res = beta / bnorm;
            if (first) inf.res0 = res;
            if (!std::isfinite(res)) {
                status = TBDG_ENAN;
                break;
            }
            if (res <= tol) {
                status = TBDG_OK;
                break;
            }
            if (total >= maxiter) break;
            trbdg::vec_scale_copy(st, n, 1.0 / beta, V, V);
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            int j = 0;
            bool breakdown = false;
            for (; j < mr && total < maxiter; ++j) {
                ++total;
                double* vj = V + (int64_t)j * n;
                double* vn = V + (int64_t)(j + 1) * n;
                A::launch_amr_div(st, n, vj, dg, z);
                op(z, vn);
                // classical Gram-Schmidt: the dots with V_0..V_j and w.w in one
                // pass, the update and |w'|^2 in another, one host read; a
                // second pass when the norm fell below 1/sqrt(10) of its value
                // (cancellation large enough to cost orthogonality)
                double nn = 0.0;
                for (int i = 0; i <= j; ++i) H[(size_t)i * mr + j] = 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    trbdg::kr_dots(st, n, j + 1, V, n, vn, m->gpart, Gd, m->gdev);
                    trbdg::kr_update_norm(st, n, j + 1, V, n, m->gdev, vn, m->gpart, Gd, m->gdev + j + 2,
                                          m->gdev + kGmScalars - 1);
                    TBDG_HIP(hipMemcpyAsync(m->host, m->gdev, sizeof(double) * (j + 3), hipMemcpyDeviceToHost,
                                            st));
                    TBDG_HIP(hipStreamSynchronize(st));
                    for (int i = 0; i <= j; ++i) H[(size_t)i * mr + j] += m->host[i];
                    const double ww = m->host[j + 1];
                    nn = m->host[j + 2];
                    if (!(nn < 0.1 * ww)) break;
                }
                const double hn = std::sqrt(nn);
                H[(size_t)(j + 1) * mr + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double t1 = cs[i] * H[(size_t)i * mr + j] + sn[i] * H[(size_t)(i + 1) * mr + j];
                    const double t2 = -sn[i] * H[(size_t)i * mr + j] + cs[i] * H[(size_t)(i + 1) * mr + j];
                    H[(size_t)i * mr + j] = t1;
                    H[(size_t)(i + 1) * mr + j] = t2;
                }
                const double a = H[(size_t)j * mr + j], bb = H[(size_t)(j + 1) * mr + j];
                const double r = std::hypot(a, bb);
                if (r == 0.0 || !std::isfinite(r)) {
                    breakdown = true;
                    break;
                }
                cs[j] = a / r;
                sn[j] = bb / r;
                H[(size_t)j * mr + j] = r;
                H[(size_t)(j + 1) * mr + j] = 0.0;
                gv[j + 1] = -sn[j] * gv[j];
                gv[j] = cs[j] * gv[j];
                if (hn == 0.0 || std::fabs(gv[j + 1]) <= tol * bnorm) {
                    ++j;
                    break;
                }
                trbdg::vec_scale_copy(st, n, 1.0 / hn, vn, vn);
            }
            const int k = j;
            for (int i = k - 1; i >= 0; --i) {
                double s2 = gv[i];
                for (int q = i + 1; q < k; ++q) s2 -= H[(size_t)i * mr + q] * y[q];
                y[i] = s2 / H[(size_t)i * mr + i];
            }
            // x += D^{-1} V y
            if (k > 0) {
                trbdg::vec_scale_copy(st, n, y[0], V, z);
                for (int i = 1; i < k; ++i) trbdg::vec_axpby(st, n, 1.0, z, y[i], V + (int64_t)i * n, z);
                A::launch_amr_div(st, n, z, dg, z);
                trbdg::vec_axpby(st, n, 1.0, x, 1.0, z, x);
            }
            if (breakdown && k == 0) {
                status = TBDG_EBREAKDOWN;
                break;
            }
        }
        inf.iters = total;
        inf.res_final = res;
        if (info) *info = inf;
        if (status != TBDG_OK) m->last_error = "adaptive-mesh momentum GMRES did not converge";
        return status;
    });
}

tbdg_status tbdg_amr_set_flow(tbdg_amr* m, double nu, double dt, double c) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(nu) && nu > 0.0 && std::isfinite(dt) && dt > 0.0, "need nu > 0 and dt > 0");
        need(c > 0.0, "need c > 0 (infinite: no artificial compressibility term)");
        m->nu = nu;
        m->dt = dt;
        m->c = c;
        m->flow = true;
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_rhs_momentum(tbdg_amr* m, int stage, const double* u_n, const double* u_g,
                                  const double* w, const double* w_explicit, const double* p_prev,
                                  const double* uD, double* out) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->flow, "tbdg_amr_set_flow first");
        need(stage == 1 || stage == 2, "stage must be 1 or 2");
        need(m->Nc() == 0 || (u_n && w && p_prev && out && (stage == 1 || u_g)), "null vector");
        need(m->n_bfaces == 0 || uD, "the mesh has walls: wall data uD needed");
        need(out != u_n && out != u_g && out != w && out != w_explicit, "out must not alias an input");
        rhs_momentum_amr(m, stage, u_n, u_g, w, w_explicit, p_prev, uD, out);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_rhs_pressure(tbdg_amr* m, int stage, const double* u_ss, const double* p_prev,
                                  double* out) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->flow, "tbdg_amr_set_flow first");
        need(stage == 1 || stage == 2, "stage must be 1 or 2");
        need(m->Nc() == 0 || (u_ss && p_prev && out), "null vector");
        need(out != p_prev, "out must not alias p_prev");
        rhs_pressure_amr(m, stage, u_ss, p_prev, out);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_add_grad_p(tbdg_amr* m, const double* x, double a, const double* p, double* y) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(a), "a must be finite");
        need(m->Nc() == 0 || (x && p && y), "null vector");
        A::launch_amr_grad(m->stream, m->geo(), m->tu, m->mx, x, a, p, y);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_step(tbdg_amr* m, const tbdg_amr_step_opts* o, double* u, double* u_hist,
                          double* p, const double* uD, tbdg_solve_info info[4], double* max_du) {
    if (!m || !o) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->flow, "tbdg_amr_set_flow first");
        need(u && u_hist && p, "null vector");
        need(m->n_bfaces == 0 || uD, "the mesh has walls: wall data uD needed");
        need(o->nonlinear >= 1 && o->mom_tol > 0.0 && o->prs_tol > 0.0, "bad step options");
        const int64_t nu_ = m->Nu(), np_ = m->Np();
        const int64_t cap = 6 * nu_ + 3 * np_;
        if (cap > m->sv_cap) {
            devfree(m->sv);
            m->sv = devalloc<double>(cap);
            m->sv_cap = cap;
        }
        double* w = m->sv;
        double* rhs = w + nu_;
        double* us = rhs + nu_;
        double* uss = us + nu_;
        double* ug = uss + nu_;
        double* un = ug + nu_;
        double* b = un + nu_;
        double* pg = b + np_;
        double* pn = pg + np_;
        const hipStream_t st = m->stream;
        const Trbdf2 T;
        const size_t bu = sizeof(double) * nu_, bp = sizeof(double) * np_;
        tbdg_solve_info loc[4] = {};
        auto stage = [&](int s, const double* u_n, const double* u_h, const double* u_gs,
                         const double* p_prev, double* u_out, double* p_out) -> tbdg_status {
            const double* base = s == 1 ? u_n : u_gs;
            if (s == 1) trbdg::vec_axpby(st, nu_, T.e1[0], u_n, T.e1[1], u_h, w);
            else trbdg::vec_axpby(st, nu_, T.e2[0], u_gs, T.e2[1], u_n, w);
            const double ms = 1.0 / (T.beta(s) * m->dt), th = T.theta(s);
            const double* w_ex = (o->nonlinear > 1 && s == 1) ? u_n : nullptr;
            TBDG_HIP(hipMemcpyAsync(us, base, bu, hipMemcpyDeviceToDevice, st));
            tbdg_solve_info acc{0, 0.0, 0.0, 0, 0}, one{};
            for (int solves = 1;; ++solves) {
                rhs_momentum_amr(m, s, u_n, u_gs, w, w_ex, p_prev, uD, rhs);
                const tbdg_status rc = tbdg_amr_solve_momentum(m, ms, th * m->nu, th, w, uD, rhs, us,
                                                               o->mom_tol, o->mom_maxiter,
                                                               o->restart > 0 ? o->restart : 30, &one);
                if (solves == 1) acc.res0 = one.res0;
                acc.iters += one.iters;
                acc.res_final = one.res_final;
                if (rc != TBDG_OK) {
                    loc[2 * (s - 1)] = acc;
                    return rc;
                }
                if (solves >= o->nonlinear) break;
                TBDG_HIP(hipMemcpyAsync(w, us, bu, hipMemcpyDeviceToDevice, st));
            }
            loc[2 * (s - 1)] = acc;
            const double bdt = T.beta(s) * m->dt;
            A::launch_amr_grad(st, m->geo(), m->tu, m->mx, us, bdt, p_prev, uss);
            rhs_pressure_amr(m, s, uss, p_prev, b);
            // initial guess: stage 1 starts from p^n; stage 2 from the line
            // through p^n and p^{n+gamma}, evaluated at t^{n+1}
            if (s == 1) TBDG_HIP(hipMemcpyAsync(p_out, p_prev, bp, hipMemcpyDeviceToDevice, st));
            else trbdg::vec_axpby(st, np_, 1.0 / T.g, p_prev, -(1.0 - T.g) / T.g, p, p_out);
            const double alpha = std::isinf(m->c) ? 0.0 : 1.0 / (m->c * m->c * bdt * bdt);
            const tbdg_status rc = tbdg_amr_solve_pressure(m, alpha, b, p_out, o->prs_tol, o->prs_maxiter,
                                                           &loc[2 * (s - 1) + 1]);
            if (rc != TBDG_OK) return rc;
            A::launch_amr_grad(st, m->geo(), m->tu, m->mx, uss, -bdt, p_out, u_out);
            return TBDG_OK;
        };
        tbdg_status rc = stage(1, u, u_hist, nullptr, p, ug, pg);
        if (rc == TBDG_OK) rc = stage(2, u, nullptr, ug, pg, un, pn);
        if (info)
            for (int q = 0; q < 4; ++q) info[q] = loc[q];
        if (rc != TBDG_OK) return rc;
        if (max_du) {
            A::launch_amr_maxdiff(st, nu_, un, u, m->part, DOT_BLOCKS, m->scal + 5);
            TBDG_HIP(hipMemcpyAsync(m->host, m->scal + 5, sizeof(double), hipMemcpyDeviceToHost, st));
            TBDG_HIP(hipStreamSynchronize(st));
            *max_du = m->host[0];
        }
        TBDG_HIP(hipMemcpyAsync(u_hist, ug, bu, hipMemcpyDeviceToDevice, st));
        TBDG_HIP(hipMemcpyAsync(u, un, bu, hipMemcpyDeviceToDevice, st));
        TBDG_HIP(hipMemcpyAsync(p, pn, bp, hipMemcpyDeviceToDevice, st));
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_diag_pressure(tbdg_amr* m, double alpha, double* d) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(alpha), "alpha must be finite");
        need(m->Nc() == 0 || d, "null vector");
        A::launch_amr_pressure(m->stream, m->geo(), m->tp, alpha, nullptr, d, true);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_solve_pressure(tbdg_amr* m, double alpha, const double* b, double* x, double tol,
                                    int maxiter, tbdg_solve_info* info) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(std::isfinite(alpha) && alpha > 0.0, "alpha must be finite and > 0");
        need(tol > 0.0 && maxiter >= 0, "need tol > 0 and maxiter >= 0");
        need(b && x, "null vector");
        const int64_t n = m->Np();
        if (n > m->cg_cap) {
            devfree(m->cg);
            m->cg = devalloc<double>(6 * n);
            m->cg_cap = n;
        }
        // two direction buffers: the operator forms the new direction from
        // the old one while other blocks still read the old one
        double *r = m->cg, *z = r + n, *q = z + n, *d = q + n;
        double* P[2] = {d + n, d + 2 * n};
        double* rz[2] = {m->scal, m->scal + 1};
        double* pq = m->scal + 2;
        const hipStream_t st = m->stream;
        const A::Geo g = m->geo();
        tbdg_solve_info inf{0, 0.0, 0.0, 0, 0};
        // cell-block Jacobi (the inverse of every cell's diagonal block) where
        // the blocks are small, else the point Jacobi diagonal
        const int nbp = m->k * m->k;
        const bool blk = A::amr_block_ok(nbp);
        const int64_t nc = m->Nc();
        if (blk) {
            const int64_t nbb = nc * nbp * nbp;
            if (nbb > m->blk_cap) {
                devfree(m->blk);
                devfree(m->blkinv);
                m->blk = devalloc<double>(nbb);
                m->blkinv = devalloc<float>(nbb);
                m->blk_cap = nbb;
            }
            A::launch_amr_block_build(st, g, m->tp, alpha, z, q, m->blk, m->blkinv);
            const int64_t gb = 2 * (int64_t)A::amr_block_grid(nc, nbp);
            if (gb > m->bpart_cap) {
                devfree(m->bpart);
                m->bpart = devalloc<double>(gb);
                m->bpart_cap = gb;
            }
        } else {
            A::launch_amr_pressure(st, g, m->tp, alpha, nullptr, d, true);
        }
        A::launch_amr_pressure(st, g, m->tp, alpha, x, q, false);
        trbdg::vec_axpby(st, n, 1.0, b, -1.0, q, r);
        const double bnorm = std::sqrt(dot(m, n, b, b, 4));
        if (bnorm == 0.0) {
            TBDG_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
            if (info) *info = inf;
            return TBDG_OK;
        }
        if (!std::isfinite(bnorm)) return TBDG_ENAN;
        double res = std::sqrt(dot(m, n, r, r, 3)) / bnorm;
        inf.res0 = res;
        if (blk) {
            const int gb = A::launch_amr_block_apply(st, nc, nbp, m->blkinv, r, z, m->bpart);
            A::launch_amr_finish(st, m->bpart, gb, 1, rz[0], nullptr);
        } else {
            A::launch_amr_div(st, n, r, d, z);
            A::launch_amr_dot(st, n, r, z, m->part, DOT_BLOCKS, rz[0]);
        }
        // per iteration: the operator fused with the new direction, then the
        // update of x and r fused with the preconditioner.  Each writes block
        // partials of its dot products; when they are few, the next kernel
        // sums them itself (the operator stores r.z for the update), else a
        // one-block kernel sums them in between.  All scalars stay on the
        // device and the host reads p.q and r.r every kCheck iterations.
        constexpr int kCheck = 8;
        const int Gp = A::amr_pressure_blocks(g, m->tp);
        if (Gp > m->ppart_cap) {
            devfree(m->ppart);
            m->ppart = devalloc<double>(Gp);
            m->ppart_cap = Gp;
        }
        double* rr = m->scal + 3;
        constexpr int kFusedSums = 1024;
        const int Grz = blk ? A::amr_block_grid(nc, nbp) : DOT_BLOCKS / 2;
        double* rzpart = blk ? m->bpart : m->part;
        const bool fused = Gp <= kFusedSums && Grz <= kFusedSums;
        tbdg_status status = TBDG_ENOTCONV;
        int it = 0, cur = 0, pb = 0;
        for (;;) {
            if (!std::isfinite(res)) {
                status = TBDG_ENAN;
                break;
            }
            if (res <= tol) {
                status = TBDG_OK;
                break;
            }
            if (it >= maxiter) break;
            const int stop = std::min(maxiter, it + kCheck);
            for (; it < stop; ++it) {
                // p_it = z + (rz_it / rz_{it-1}) p_{it-1}, the first one z
                // rz[cur] holds r.z of this iteration (or receives it from the
                // operator kernel), rz[1 - cur] that of the previous one
                const bool first = it == 0;
                A::CgDir dir{first ? z : P[pb], P[1 - pb], rz[cur], nullptr, 0,
                             first ? nullptr : rz[1 - cur], nullptr};
                if (fused && !first) {
                    dir.rz_part = rzpart;
                    dir.rz_G = Grz;
                    dir.rz_store = rz[cur];
                }
                A::launch_amr_pressure_dir(st, g, m->tp, alpha, z, dir, q, m->ppart);
                pb = 1 - pb;
                A::CgUpdate up{rz[cur], pq, nullptr, 0, P[pb], q, x};
                if (fused) {
                    up.pq_part = m->ppart;
                    up.pq_G = Gp;
                } else {
                    A::launch_amr_finish(st, m->ppart, Gp, 1, pq, nullptr);
                }
                if (blk) A::launch_amr_block_xr(st, nc, nbp, m->blkinv, up, r, z, m->bpart);
                else A::launch_amr_cg_step(st, n, up, d, r, z, m->part, DOT_BLOCKS / 2);
                if (!fused) A::launch_amr_finish(st, rzpart, Grz, 2, rz[1 - cur], rr);
                cur = 1 - cur;
            }
            if (fused) {
                A::launch_amr_finish(st, m->ppart, Gp, 1, pq, nullptr);
                A::launch_amr_finish(st, rzpart + Grz, Grz, 1, rr, nullptr);
            }
            TBDG_HIP(hipMemcpyAsync(m->host, pq, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            TBDG_HIP(hipStreamSynchronize(st));
            const double pqv = m->host[0];
            if (!(pqv > 0.0)) {
                status = std::isfinite(pqv) ? TBDG_EBREAKDOWN : TBDG_ENAN;
                break;
            }
            res = std::sqrt(m->host[1]) / bnorm;
        }
        inf.iters = it;
        inf.res_final = res;
        if (info) *info = inf;
        if (status != TBDG_OK) m->last_error = "adaptive-mesh pressure CG did not converge";
        return status;
    });
}

tbdg_status tbdg_amr_indicator(tbdg_amr* m, const double* u, double* eta) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->Nc() == 0 || (u && eta), "null vector");
        A::launch_amr_indicator(m->stream, m->geo(), m->tu, u, eta);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_mark(tbdg_amr* m, const double* eta, double refine_frac, double coarsen_frac,
                          double h_min, double h_max, int8_t* flags) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(refine_frac >= 0.0 && refine_frac <= 1.0 && coarsen_frac >= 0.0 && coarsen_frac <= 1.0,
             "fractions must lie in [0, 1]");
        need(h_min >= 0.0 && h_max > 0.0 && !std::isnan(h_min) && !std::isnan(h_max), "bad size limits");
        const int64_t N = m->Nc();
        need(N == 0 || (eta && flags), "null pointer");
        std::vector<double> e(N);
        if (N > 0) {
            TBDG_HIP(hipMemcpyAsync(e.data(), eta, sizeof(double) * N, hipMemcpyDeviceToHost, m->stream));
            TBDG_HIP(hipStreamSynchronize(m->stream));
        }
        for (double v : e)
            if (std::isnan(v)) throw Error(TBDG_ENAN, "indicator holds NaN");
        const int64_t nr = (int64_t)std::floor(refine_frac * N + 1e-12);
        const int64_t ncs = (int64_t)std::floor(coarsen_frac * N + 1e-12);
        std::vector<int64_t> ord(N);
        for (int64_t c = 0; c < N; ++c) ord[c] = c;
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
            return e[a] > e[b] || (e[a] == e[b] && a < b);
        });
        std::vector<char> top(N, 0);
        std::memset(flags, 0, (size_t)N);
        const Forest& F = m->F;
        for (int64_t r = 0; r < nr; ++r) {
            const int64_t c = ord[r];
            top[c] = 1;
            const double hm = std::max(F.size((int)c, 0), F.size((int)c, 1));
            if (0.5 * hm >= h_min * (1.0 - 1e-12) && F.leaves[c].l < F.maxl) flags[c] = 1;
        }
        std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
            return e[a] < e[b] || (e[a] == e[b] && a < b);
        });
        int64_t taken = 0;
        for (int64_t r = 0; r < N && taken < ncs; ++r) {
            const int64_t c = ord[r];
            if (top[c]) continue;
            ++taken;
            const double hm = std::max(F.size((int)c, 0), F.size((int)c, 1));
            if (F.leaves[c].l > 0 && 2.0 * hm <= h_max * (1.0 + 1e-12)) flags[c] = -1;
        }
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_plan(tbdg_amr* m, const int8_t* flags, int64_t* new_cells) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        const int64_t N = m->Nc();
        need(N == 0 || flags, "null flags");
        m->next = m->F.adapt(flags);
        const Forest& Fn = m->next;
        const int64_t Nn = (int64_t)Fn.leaves.size();
        std::vector<int> kind(Nn), src(4 * Nn, -1);
        for (int64_t c = 0; c < Nn; ++c) {
            const Leaf& L = Fn.leaves[c];
            int o = m->F.find(L.l, L.i, L.j);
            if (o >= 0) {
                kind[c] = 0;
                src[4 * c] = o;
            } else if (L.l > 0 && (o = m->F.find(L.l - 1, L.i >> 1, L.j >> 1)) >= 0) {
                kind[c] = 1 | (((L.i & 1) + 2 * (L.j & 1)) << 4);
                src[4 * c] = o;
            } else {
                kind[c] = 2;
                for (int ch = 0; ch < 4; ++ch) {
                    src[4 * c + ch] = m->F.find(L.l + 1, 2 * L.i + (ch & 1), 2 * L.j + (ch >> 1));
                    if (src[4 * c + ch] < 0) throw Error(TBDG_EINVAL, "inconsistent adaptation");
                }
            }
        }
        if (Nn > m->x_cap) {
            devfree(m->xkind);
            devfree(m->xsrc);
            m->xkind = devalloc<int>(Nn);
            m->xsrc = devalloc<int>(4 * Nn);
            m->x_cap = Nn;
        }
        if (Nn > 0) {
            TBDG_HIP(hipMemcpyAsync(m->xkind, kind.data(), sizeof(int) * Nn, hipMemcpyHostToDevice,
                                    m->stream));
            TBDG_HIP(hipMemcpyAsync(m->xsrc, src.data(), sizeof(int) * 4 * Nn, hipMemcpyHostToDevice,
                                    m->stream));
        }
        TBDG_HIP(hipStreamSynchronize(m->stream));
        m->planned = true;
        if (new_cells) *new_cells = Nn;
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_transfer(tbdg_amr* m, int field, const double* src, double* dst) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->planned, "no adaptation planned (tbdg_amr_plan)");
        need(field == 0 || field == 1, "field must be 0 (velocity) or 1 (pressure)");
        const int64_t Nn = (int64_t)m->next.leaves.size();
        need((m->Nc() == 0 || src) && (Nn == 0 || dst), "null vector");
        need(src != dst, "source and destination must differ");
        A::XferMap xm{m->xkind, m->xsrc, (int)Nn};
        A::launch_amr_transfer(m->stream, xm, field == 0 ? m->tu : m->tp, field == 0 ? 2 : 1, src, dst);
        return TBDG_OK;
    });
}

tbdg_status tbdg_amr_commit(tbdg_amr* m) {
    if (!m) return TBDG_EINVAL;
    return aguard(m, [&]() {
        need(m->planned, "no adaptation planned (tbdg_amr_plan)");
        // kernels still reading the old connectivity must finish first
        TBDG_HIP(hipStreamSynchronize(m->stream));
        m->F = std::move(m->next);
        m->next = Forest();
        m->planned = false;
        m->upload();
        return TBDG_OK;
    });
}

}  // extern "C"
