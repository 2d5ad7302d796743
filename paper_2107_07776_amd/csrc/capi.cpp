// extern "C" entry points of libtrbdg: argument validation, context life
// cycle and translation of C++ errors into status codes.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

namespace trbdg {
void build_tables(tbdg_ctx* c);
void build_line_operators(tbdg_ctx* c);
tbdg_status solve_pressure(tbdg_ctx* c, int s, const double* b, double* x,
                           const tbdg_solver_opts& o, tbdg_solve_info* info);
void extrapolate(tbdg_ctx* c, int s, const double* u_new, const double* u_old, double* w);
void rhs_momentum(tbdg_ctx* c, int s, const double* u_n, const double* u_g, const double* w,
                  const double* p, double* rhs);
void rhs_pressure(tbdg_ctx* c, int s, const double* u_ss, const double* p_prev, double* rhs);
tbdg_status step(tbdg_ctx* c, tbdg_state* S, const tbdg_solver_opts& mo,
                 const tbdg_solver_opts& po, tbdg_solve_info info[4]);
tbdg_status step_single(tbdg_ctx* c, tbdg_state* S, const tbdg_solver_opts& mo,
                        const tbdg_solver_opts& po, tbdg_solve_info info[4]);
}  // namespace trbdg

using trbdg::Error;

namespace {

constexpr int GMRES_MAX = 60;

template <class F>
tbdg_status guarded(tbdg_ctx* c, F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        if (c) c->last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        if (c) c->last_error = "host allocation failed";
        return TBDG_ENOMEM;
    } catch (const std::exception& e) {
        if (c) c->last_error = e.what();
        return TBDG_EINVAL;
    }
}

void require(bool ok, const char* msg) {
    if (!ok) throw Error(TBDG_EINVAL, msg);
}

void check_stage(int s) { require(s == 1 || s == 2, "stage must be 1 or 2"); }

double* dalloc(int64_t n) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (e != hipSuccess) throw Error(TBDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return static_cast<double*>(p);
}

void dfree(double*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_all(tbdg_ctx* c) {
    for (auto& d : c->diag_p) dfree(d);
    dfree(c->diag_u);
    dfree(c->V);
    dfree(c->gsc);
    if (c->mom_blk) (void)hipFree(c->mom_blk);
    c->mom_blk = nullptr;
    if (c->mom_dbox) (void)hipFree(c->mom_dbox);
    c->mom_dbox = nullptr;
    dfree(c->gm_part);
    dfree(c->gv);
    dfree(c->gz);
    dfree(c->cr);
    dfree(c->cp);
    dfree(c->cq);
    dfree(c->cp2);
    dfree(c->red_part);
    dfree(c->red_out);
    dfree(c->invd_u);
    dfree(c->red_op);
    dfree(c->invd_p[1]);
    dfree(c->invd_p[2]);
    if (c->host_out) (void)hipHostFree(c->host_out);
    c->host_out = nullptr;
    dfree(c->s_w);
    dfree(c->s_rhs);
    dfree(c->s_ustar);
    dfree(c->s_ug);
    dfree(c->s_u1);
    dfree(c->s_pb);
    dfree(c->s_pg);
    dfree(c->s_p1);
    dfree(c->s_pv);
    dfree(c->s_wlag);
    trbdg::mg_free(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    trbdg::guess_free(c);
    dfree(c->bnd_uD[0]);
    dfree(c->bnd_uD[1]);
    dfree(c->map_vtx);
    dfree(c->map_gr);
}

void levels_of(const trbdg::MGData& M, int cap, int* n_levels, int64_t* desc, double* lambda) {
    const int nl = (int)M.lv.size();
    *n_levels = nl;
    for (int l = 0; l < nl && l < cap; ++l) {
        const trbdg::MGLevel& L = M.lv[l];
        if (desc) {
            desc[5 * l] = L.np;
            for (int a = 0; a < 3; ++a) desc[5 * l + 1 + a] = L.geom.nc[a];
            desc[5 * l + 4] = L.N;
        }
        if (lambda) {
            lambda[l] = L.lam[1];
            lambda[cap + l] = L.lam[2];
        }
    }
}

tbdg_solver_opts defaults(const tbdg_solver_opts* o) {
    tbdg_solver_opts d{1e-8, 1000, 30, 0, 0};
    if (!o) return d;
    tbdg_solver_opts r = *o;
    require(r.tol > 0.0 && std::isfinite(r.tol), "solver tol must be positive");
    require(r.maxiter > 0, "solver maxiter must be positive");
    require(r.restart >= 0 && r.restart <= GMRES_MAX, "GMRES restart must be in [0, 60]");
    require(r.precond >= TBDG_PRECOND_JACOBI && r.precond <= TBDG_PRECOND_LINE,
            "unknown preconditioner");
    require(r.guess >= TBDG_GUESS_GIVEN && r.guess <= TBDG_GUESS_EXTRAP3, "unknown initial guess");
    return r;
}

}  // namespace

extern "C" {

tbdg_status tbdg_create(const tbdg_mesh_desc* mesh, const tbdg_disc_desc* disc, void* stream,
                        tbdg_ctx** out) {
    if (!out) return TBDG_EINVAL;
    *out = nullptr;
    if (!mesh || !disc) return TBDG_EINVAL;
    tbdg_ctx* c = new (std::nothrow) tbdg_ctx();
    if (!c) return TBDG_ENOMEM;
    const tbdg_status st = guarded(c, [&]() -> tbdg_status {
        require(mesh->dim == 2 || mesh->dim == 3, "dim must be 2 or 3");
        c->dim = mesh->dim;
        c->Nc = 1;
        for (int a = 0; a < 3; ++a) {
            if (a < c->dim) {
                require(mesh->n_cells[a] >= 1, "n_cells must be >= 1");
                require(mesh->hi[a] > mesh->lo[a], "hi must exceed lo");
                c->geom.nc[a] = mesh->n_cells[a];
                c->geom.h[a] = (mesh->hi[a] - mesh->lo[a]) / mesh->n_cells[a];
                c->geom.lo[a] = mesh->lo[a];
                c->periodic_flags[a] = mesh->periodic[a] ? 1 : 0;
                c->Nc *= mesh->n_cells[a];
            } else {
                c->geom.nc[a] = 1;
                c->geom.h[a] = 1.0;
                c->geom.lo[a] = 0.0;
                c->periodic_flags[a] = 1;
            }
        }
        require(mesh->mapping == 0 || mesh->mapping == 1, "mapping must be 0 (affine) or 1 (sine Q1)");
        if (mesh->mapping == 1) {
            if (c->dim != 2) throw Error(TBDG_EUNSUPPORTED, "Q1-mapped cells are built in 2D only");
            require(std::isfinite(mesh->map_amp), "map_amp must be finite");
            c->mapped = 1;
        }
        require(disc->k_u >= 2, "velocity degree k_u must be >= 2");
        const int kmax = c->dim == 2 ? 5 : 3;
        if (disc->k_u > kmax) throw Error(TBDG_EUNSUPPORTED, "velocity degree too high for this dim");
        require(std::isfinite(disc->nu) && disc->nu >= 0.0, "nu must be finite and >= 0");
        require(disc->c > 0.0, "c must be > 0");
        require(std::isfinite(disc->dt) && disc->dt > 0.0, "dt must be > 0");
        require(disc->gamma >= 0.0 && disc->gamma < 1.0, "gamma must be in [0,1)");
        c->k = disc->k_u;
        c->n = c->k + 1;
        c->np = c->k;
        c->nu = disc->nu;
        c->c = disc->c;
        c->dt = disc->dt;
        c->gamma = disc->gamma > 0.0 ? disc->gamma : 2.0 - std::sqrt(2.0);
        c->pen_u = disc->pen_u > 0.0 ? disc->pen_u : 1.0;
        c->pen_p = disc->pen_p > 0.0 ? disc->pen_p : 1.0;
        const double g = c->gamma;
        c->a31 = (1.0 - g) / (2.0 * (2.0 - g));
        c->a32 = c->a31;
        c->a33 = 1.0 / (2.0 - g);
        c->beta[1] = g;
        c->beta[2] = 1.0 - g;
        c->theta[1] = 0.5;
        c->theta[2] = c->a33;
        int64_t nbu = 1, nbp = 1;
        for (int a = 0; a < c->dim; ++a) {
            nbu *= c->n;
            nbp *= c->np;
        }
        c->nbu = nbu;
        c->nbp = nbp;
        c->Ns = c->Nc * nbu;
        c->Nu = c->Ns * c->dim;
        c->Np = c->Nc * nbp;
        c->geom.vol = 1.0;
        for (int a = 0; a < c->dim; ++a) c->geom.vol *= c->geom.h[a];
        // uniform mesh: C = sigma_{Gamma,K} = deg^2 |Gamma| / |K| = deg^2 / h_a
        for (int a = 0; a < 3; ++a) {
            c->sig_u[a] = (c->k + 1.0) * (c->k + 1.0) * c->pen_u / c->geom.h[a];
            c->sig_p[a] = (double)c->k * c->k * c->pen_p / c->geom.h[a];
        }
        c->stream = static_cast<hipStream_t>(stream);
        TBDG_HIP(hipGetDevice(&c->device));
        trbdg::noalloc_init(c->device);   // address of the static scratch on this device
        trbdg::build_tables(c);
        trbdg::build_line_operators(c);
        // workspaces
        c->gm_m = GMRES_MAX;
        c->diag_p[1] = dalloc(c->Np);
        c->diag_p[2] = dalloc(c->Np);
        c->diag_u = dalloc(c->Ns);
        c->V = dalloc((int64_t)(c->gm_m + 1) * c->Nu);
        c->gv = dalloc(c->Nu);
        c->gz = dalloc(c->Nu);
        c->gsc = dalloc(GMRES_MAX + 2);
        c->gm_part_len = (c->Nc + 4) * (trbdg::MOM_FUSE_MAX_DOTS + 1);   // per-wave partials too
        c->gm_part = dalloc(c->gm_part_len);
        c->cr = dalloc(c->Np);
        c->cp = dalloc(c->Np);
        c->cq = dalloc(c->Np);
        c->cp2 = dalloc(c->Np);
        c->red_blocks = 64 * 4096;
        c->red_part = dalloc(c->red_blocks);
        c->red_out = dalloc(128);   // [0..62] GMRES, [63] norms, [64..79] CG scalars
        c->red_op_len = c->Nc + 1;   // at least one slot per block of any operator kernel
        c->red_op = dalloc(c->red_op_len);
        c->invd_u = dalloc(c->Ns);
        c->invd_p[1] = dalloc(c->Np);
        c->invd_p[2] = dalloc(c->Np);
        void* h = nullptr;
        TBDG_HIP(hipHostMalloc(&h, sizeof(double) * 2048, hipHostMallocCoherent | hipHostMallocMapped));
        c->host_out = static_cast<double*>(h);
        void* hd = nullptr;
        TBDG_HIP(hipHostGetDevicePointer(&hd, h, 0));
        c->host_dev = static_cast<double*>(hd);
        c->s_w = dalloc(c->Nu);
        c->s_rhs = dalloc(c->Nu);
        c->s_ustar = dalloc(c->Nu);
        c->s_ug = dalloc(c->Nu);
        c->s_u1 = dalloc(c->Nu);
        c->s_pb = dalloc(c->Np);
        c->s_pg = dalloc(c->Np);
        c->s_p1 = dalloc(c->Np);
        c->s_pv = dalloc(c->Ns);
        // boundary faces of the non-periodic directions: point offsets and
        // zero-initialised Dirichlet data for the two stage times
        {
            int64_t nf = 1;
            for (int a = 0; a < c->dim - 1; ++a) nf *= c->n;
            int64_t off = 0;
            for (int a = 0; a < 3; ++a)
                for (int sd = 0; sd < 2; ++sd) {
                    if (a < c->dim && !c->periodic_flags[a]) {
                        c->bnd_off[a][sd] = off;
                        off += (c->Nc / c->geom.nc[a]) * nf;
                    } else {
                        c->bnd_off[a][sd] = -1;
                    }
                }
            c->bnd_npts = off;
            for (int k = 0; k < 2; ++k) {
                c->bnd_uD[k] = dalloc(off * c->dim);
                TBDG_HIP(hipMemsetAsync(c->bnd_uD[k], 0, sizeof(double) * (off > 0 ? off * c->dim : 1),
                                        c->stream));
            }
        }
        if (c->mapped) {
            std::vector<double> vtx, gr;
            trbdg::build_mapped_geometry(c, mesh->map_amp, vtx, gr);
            // the bilinear Jacobian determinant is linear in each reference
            // coordinate: positive at the corners means positive everywhere
            for (int64_t q = 0; q < c->Nc; ++q) {
                const double* X = &vtx[(size_t)q * 8];
                for (int v = 0; v < 4; ++v) {
                    const double x0 = v & 1, x1 = v >> 1;
                    const double j00 = (1 - x1) * (X[2] - X[0]) + x1 * (X[6] - X[4]);
                    const double j10 = (1 - x1) * (X[3] - X[1]) + x1 * (X[7] - X[5]);
                    const double j01 = (1 - x0) * (X[4] - X[0]) + x0 * (X[6] - X[2]);
                    const double j11 = (1 - x0) * (X[5] - X[1]) + x0 * (X[7] - X[3]);
                    require(j00 * j11 - j01 * j10 > 0.0, "map_amp inverts a cell");
                }
            }
            c->map_vtx = dalloc((int64_t)vtx.size());
            c->map_gr = dalloc((int64_t)gr.size());
            TBDG_HIP(hipMemcpyAsync(c->map_vtx, vtx.data(), sizeof(double) * vtx.size(),
                                    hipMemcpyHostToDevice, c->stream));
            TBDG_HIP(hipMemcpyAsync(c->map_gr, gr.data(), sizeof(double) * gr.size(),
                                    hipMemcpyHostToDevice, c->stream));
            TBDG_HIP(hipStreamSynchronize(c->stream));
        }
        trbdg::launch_diag_pressure(c, c->alpha(1), c->diag_p[1]);
        trbdg::launch_diag_pressure(c, c->alpha(2), c->diag_p[2]);
        trbdg::vec_recip(c->stream, c->Np, c->diag_p[1], c->invd_p[1]);
        trbdg::vec_recip(c->stream, c->Np, c->diag_p[2], c->invd_p[2]);
        TBDG_HIP(hipStreamSynchronize(c->stream));
        return TBDG_OK;
    });
    if (st != TBDG_OK) {
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return TBDG_OK;
}

void tbdg_destroy(tbdg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    trbdg::timer_release(c);
    free_all(c);
    delete c;
}

const char* tbdg_last_error(const tbdg_ctx* c) {
    if (!c) return "null context";
    return c->last_error.c_str();
}

tbdg_status tbdg_set_stream(tbdg_ctx* c, void* stream) {
    if (!c) return TBDG_EINVAL;
    c->stream = static_cast<hipStream_t>(stream);
    return TBDG_OK;
}

tbdg_status tbdg_sizes(const tbdg_ctx* c, int64_t* n_u, int64_t* n_p, int64_t* n_cells) {
    if (!c) return TBDG_EINVAL;
    if (n_u) *n_u = c->Nu;
    if (n_p) *n_p = c->Np;
    if (n_cells) *n_cells = c->Nc;
    return TBDG_OK;
}

tbdg_status tbdg_node_coords(const tbdg_ctx* cc, int field, double* xyz) {
    tbdg_ctx* c = const_cast<tbdg_ctx*>(cc);
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(field == 0 || field == 1, "field must be 0 (velocity) or 1 (pressure)");
        require(xyz != nullptr, "null output");
        trbdg::launch_node_coords(c, field, xyz);
        return TBDG_OK;
    });
}

tbdg_status tbdg_extrapolate(tbdg_ctx* c, int stage, const double* u_new, const double* u_old,
                             double* w) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(u_new && u_old && w, "null pointer");
        trbdg::extrapolate(c, stage, u_new, u_old, w);
        return TBDG_OK;
    });
}

tbdg_status tbdg_face_qpoints(const tbdg_ctx* c, int64_t* n, double* xyz) {
    if (!c) return TBDG_EINVAL;
    return guarded(const_cast<tbdg_ctx*>(c), [&]() {
        require(n != nullptr, "null pointer");
        *n = c->bnd_npts;
        if (!xyz || c->bnd_npts == 0) return TBDG_OK;
        const int d = c->dim, N = c->n;
        int64_t nf = 1;
        for (int a = 0; a < d - 1; ++a) nf *= N;
        std::vector<double> pts((size_t)c->bnd_npts * d);
        std::vector<double> mvtx;
        if (c->mapped) {
            mvtx.resize((size_t)c->Nc * 8);
            TBDG_HIP(hipMemcpy(mvtx.data(), c->map_vtx, sizeof(double) * mvtx.size(), hipMemcpyDeviceToHost));
        }
        for (int a = 0; a < d; ++a) {
            if (c->bnd_off[a][0] < 0) continue;
            int oth[2] = {0, 0}, no = 0;
            for (int b = 0; b < d; ++b)
                if (b != a) oth[no++] = b;
            const int64_t ncf = c->Nc / c->geom.nc[a];
            for (int sd = 0; sd < 2; ++sd)
                for (int64_t tc = 0; tc < ncf; ++tc) {
                    int64_t ci[3] = {0, 0, 0};
                    int64_t r = tc;
                    for (int q = 0; q < no; ++q) {
                        ci[oth[q]] = r % c->geom.nc[oth[q]];
                        r /= c->geom.nc[oth[q]];
                    }
                    for (int64_t tt = 0; tt < nf; ++tt) {
                        const int64_t pt = c->bnd_off[a][sd] + tc * nf + tt;
                        int64_t rr = tt;
                        for (int q = 0; q < no; ++q) {
                            const int b = oth[q];
                            const int ib = (int)(rr % N);
                            rr /= N;
                            pts[pt * d + b] = c->geom.lo[b] + (ci[b] + c->tab.xu[ib]) * c->geom.h[b];
                        }
                        pts[pt * d + a] = c->geom.lo[a] + (sd ? c->geom.nc[a] : 0) * c->geom.h[a];
                        if (c->mapped) {
                            // the bilinear image of the reference face point
                            const int b = 1 - a;
                            const int cell = (int)(a == 0 ? (sd ? c->geom.nc[0] - 1 : 0) + c->geom.nc[0] * tc
                                                          : tc + c->geom.nc[0] * (sd ? c->geom.nc[1] - 1 : 0));
                            double xi[2];
                            xi[a] = sd;
                            xi[b] = c->tab.xu[tt];
                            const double* X = &mvtx[(size_t)cell * 8];
                            const double w0 = (1 - xi[0]) * (1 - xi[1]), w1 = xi[0] * (1 - xi[1]),
                                         w2 = (1 - xi[0]) * xi[1], w3 = xi[0] * xi[1];
                            for (int e = 0; e < 2; ++e)
                                pts[pt * d + e] = w0 * X[e] + w1 * X[2 + e] + w2 * X[4 + e] + w3 * X[6 + e];
                        }
                    }
                }
        }
        TBDG_HIP(hipMemcpyAsync(xyz, pts.data(), sizeof(double) * pts.size(), hipMemcpyHostToDevice,
                                c->stream));
        TBDG_HIP(hipStreamSynchronize(c->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_set_dirichlet(tbdg_ctx* c, int slot, const double* uD) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(slot == 0 || slot == 1, "slot must be 0 (stage-1 time) or 1 (stage-2 time)");
        require(uD != nullptr || c->bnd_npts == 0, "null pointer");
        if (c->bnd_npts == 0) return TBDG_OK;
        TBDG_HIP(hipMemcpyAsync(c->bnd_uD[slot], uD, sizeof(double) * c->bnd_npts * c->dim,
                                hipMemcpyDeviceToDevice, c->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_apply_momentum(tbdg_ctx* c, int stage, const double* w, const double* u, double* y) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(w && u && y, "null pointer");
        require(u != y && w != y, "output must not alias an input");
        trbdg::launch_apply_momentum(c, stage, w, u, y);
        return TBDG_OK;
    });
}

tbdg_status tbdg_apply_pressure(tbdg_ctx* c, int stage, const double* p, double* y) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(p && y, "null pointer");
        require(p != y, "output must not alias the input");
        trbdg::launch_apply_pressure(c, c->alpha(stage), p, y);
        return TBDG_OK;
    });
}

tbdg_status tbdg_diag_momentum(tbdg_ctx* c, int stage, const double* w, double* diag) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(w && diag, "null pointer");
        trbdg::launch_diag_momentum(c, stage, w, diag);
        return TBDG_OK;
    });
}

tbdg_status tbdg_diag_pressure(tbdg_ctx* c, int stage, double* diag) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(diag != nullptr, "null pointer");
        trbdg::launch_diag_pressure(c, c->alpha(stage), diag);
        return TBDG_OK;
    });
}

tbdg_status tbdg_rhs_momentum(tbdg_ctx* c, int stage, const double* u_n, const double* u_g,
                              const double* w, const double* p_prev, double* rhs) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(u_n && w && p_prev && rhs, "null pointer");
        require(stage == 1 || u_g != nullptr, "stage 2 needs u_g");
        trbdg::rhs_momentum(c, stage, u_n, u_g, w, p_prev, rhs);
        return TBDG_OK;
    });
}

tbdg_status tbdg_grad_p(tbdg_ctx* c, const double* p, double* gu) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(p && gu, "null pointer");
        trbdg::launch_add_grad_p(c, nullptr, 1.0, p, gu);
        return TBDG_OK;
    });
}

tbdg_status tbdg_add_grad_p(tbdg_ctx* c, const double* x, double a, const double* p, double* y) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(x && p && y, "null pointer");
        trbdg::launch_add_grad_p(c, x, a, p, y);
        return TBDG_OK;
    });
}

tbdg_status tbdg_rhs_pressure(tbdg_ctx* c, int stage, const double* u_ss, const double* p_prev,
                              double* rhs) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(u_ss && p_prev && rhs, "null pointer");
        trbdg::rhs_pressure(c, stage, u_ss, p_prev, rhs);
        return TBDG_OK;
    });
}

tbdg_status tbdg_solve_momentum(tbdg_ctx* c, int stage, const double* w, const double* rhs,
                                double* u_inout, const tbdg_solver_opts* opts,
                                tbdg_solve_info* info) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(w && rhs && u_inout, "null pointer");
        const tbdg_solver_opts o = defaults(opts);
        if (o.precond == TBDG_PRECOND_MG_BF16)
            throw Error(TBDG_EUNSUPPORTED, "the momentum solve takes the Jacobi, line or FP32 multigrid preconditioner");
        const tbdg_status s = trbdg::solve_momentum(c, stage, w, rhs, u_inout, o, info);
        if (s != TBDG_OK) c->last_error = "momentum GMRES did not converge";
        return s;
    });
}

tbdg_status tbdg_precond_momentum(tbdg_ctx* c, int stage, const double* w, const double* v,
                                  double* z) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(w && v && z, "null pointer");
        require(v != z, "v and z must not alias");
        trbdg::launch_diag_momentum(c, stage, w, c->diag_u);
        const double* d = trbdg::build_mom_lineprec(c, stage, w);
        c->lineprec_stage = 0;   // built for this w, not a stage's advector
        trbdg::launch_mom_lineprec(c, c->mom_blk, d, v, nullptr, z);
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_apply_momentum(tbdg_ctx* c, int stage, const double* v, double* z) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(v && z, "null pointer");
        require(v != z, "v and z must not alias");
        trbdg::mg_apply_velocity(c, stage, v, nullptr, z);
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_fused(tbdg_ctx* c, int field, int* first_level, int64_t* lds_bytes) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(first_level && lds_bytes, "null output");
        require(field == 0 || field == 1, "field must be 0 (pressure) or 1 (momentum)");
        const trbdg::MGData* M = field == 0 ? c->mg : c->mgu;
        if (!M) throw Error(TBDG_EINVAL, "multigrid hierarchy not built");
        *first_level = M->fuse_from;
        *lds_bytes = M->fuse_from > 0 ? (int64_t)M->fuse_lds : 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_set_mg_graphs(tbdg_ctx* c, int enable) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(enable == 0 || enable == 1, "enable must be 0 or 1");
        c->mg_graphs = enable != 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_levels_momentum(tbdg_ctx* c, int cap, int* n_levels, int64_t* desc,
                                    double* lambda) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(n_levels != nullptr && cap >= 0, "null n_levels or negative cap");
        trbdg::mgu_ensure(c);
        levels_of(*c->mgu, cap, n_levels, desc, lambda);
        return TBDG_OK;
    });
}

tbdg_status tbdg_solve_pressure(tbdg_ctx* c, int stage, const double* rhs, double* p_inout,
                                const tbdg_solver_opts* opts, tbdg_solve_info* info) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(rhs && p_inout, "null pointer");
        const tbdg_solver_opts o = defaults(opts);
        if (o.guess != TBDG_GUESS_GIVEN)
            throw Error(TBDG_EINVAL, "initial-guess modes apply to the solves inside tbdg_step");
        if (o.precond == TBDG_PRECOND_LINE)
            throw Error(TBDG_EUNSUPPORTED, "the line preconditioner applies to the momentum solve");
        const tbdg_status s = trbdg::solve_pressure(c, stage, rhs, p_inout, o, info);
        if (s != TBDG_OK) c->last_error = "pressure CG did not converge";
        return s;
    });
}

namespace {

// Points the context's CG and reduction workspaces at the static scratch for
// the lifetime of the guard and restores them afterwards (also when the solve
// throws).
struct ScratchSwap {
    tbdg_ctx* c;
    trbdg::NoallocScratch saved;
    ScratchSwap(tbdg_ctx* ctx, const trbdg::NoallocScratch& s) : c(ctx) {
        saved = {c->cr, c->cp, c->cq, c->cp2, c->red_part, c->red_blocks, c->red_out, c->red_op,
                 c->red_op_len};
        set(s);
    }
    ~ScratchSwap() { set(saved); }
    void set(const trbdg::NoallocScratch& s) {
        c->cr = s.cr;
        c->cp = s.cp;
        c->cq = s.cq;
        c->cp2 = s.cp2;
        c->red_part = s.red_part;
        c->red_blocks = s.red_blocks;
        c->red_out = s.red_out;
        c->red_op = s.red_op;
        c->red_op_len = s.red_op_len;
    }
};

}  // namespace

tbdg_status tbdg_solve_pressure_noalloc(tbdg_ctx* c, int stage, const double* rhs, double* p_inout,
                                        const tbdg_solver_opts* opts, tbdg_solve_info* info) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(rhs && p_inout, "null pointer");
        if (c->Np > TBDG_NOALLOC_MAX_NP)
            throw Error(TBDG_EINVAL, "pressure space larger than the static scratch (N_p > "
                                     "TBDG_NOALLOC_MAX_NP)");
        const tbdg_solver_opts o = defaults(opts);
        if (o.precond != TBDG_PRECOND_JACOBI)
            throw Error(TBDG_EUNSUPPORTED, "the allocation-free solve is Jacobi-preconditioned CG only");
        if (o.guess != TBDG_GUESS_GIVEN)
            throw Error(TBDG_EUNSUPPORTED, "the allocation-free solve takes the given initial guess");
        const trbdg::NoallocScratch scr = trbdg::noalloc_scratch(c->device);
        // a partial slot per operator block and the reduction sizes of the
        // context must fit the slices
        require(c->red_op_len <= scr.red_op_len && c->red_blocks <= scr.red_blocks,
                "workspace layout exceeds the static scratch");
        ScratchSwap swap(c, scr);
        // the scalar slots start from zero on every call
        TBDG_HIP(hipMemsetAsync(scr.red_out, 0, sizeof(double) * 128, c->stream));
        const tbdg_status s = trbdg::solve_pressure(c, stage, rhs, p_inout, o, info);
        if (s != TBDG_OK) c->last_error = "pressure CG did not converge";
        return s;
    });
}

tbdg_status tbdg_step(tbdg_ctx* c, tbdg_state* state, const tbdg_solver_opts* mom,
                      const tbdg_solver_opts* prs, tbdg_solve_info info[4]) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(state && state->u && state->u_hist && state->p, "null state");
        const tbdg_solver_opts mo = defaults(mom);
        const tbdg_solver_opts po = defaults(prs);
        if (mo.precond == TBDG_PRECOND_MG_BF16)
            throw Error(TBDG_EUNSUPPORTED, "the momentum solve takes the Jacobi, line or FP32 multigrid preconditioner");
        if (po.precond == TBDG_PRECOND_LINE)
            throw Error(TBDG_EUNSUPPORTED, "the line preconditioner applies to the momentum solve");
        require(mo.guess != TBDG_GUESS_LEARNED && mo.guess != TBDG_GUESS_EXTRAP2 &&
                    mo.guess != TBDG_GUESS_EXTRAP3,
                "the momentum solve takes the given or the extrapolated guess");
        if (c->scheme != TBDG_SCHEME_TRBDF2 && po.guess == TBDG_GUESS_LEARNED)
            throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for the two TR-BDF2 stages");
        const tbdg_status s = c->scheme == TBDG_SCHEME_TRBDF2 ? trbdg::step(c, state, mo, po, info)
                                                               : trbdg::step_single(c, state, mo, po, info);
        if (s != TBDG_OK && c->last_error.empty()) c->last_error = "a stage solve failed";
        return s;
    });
}

tbdg_status tbdg_set_nonlinear(tbdg_ctx* c, int max_solves, double tol) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(max_solves >= 1, "max_solves must be >= 1");
        require(std::isfinite(tol) && tol >= 0.0, "tol must be finite and >= 0");
        c->nl_max = max_solves;
        c->nl_tol = tol;
        return TBDG_OK;
    });
}

tbdg_status tbdg_nonlinear_solves(tbdg_ctx* c, int* solves) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(solves != nullptr, "null output");
        solves[0] = c->nl_solves[0];
        solves[1] = c->nl_solves[1];
        return TBDG_OK;
    });
}

tbdg_status tbdg_set_scheme(tbdg_ctx* c, int scheme) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(scheme == TBDG_SCHEME_TRBDF2 || scheme == TBDG_SCHEME_BCG || scheme == TBDG_SCHEME_BDF2,
                "unknown time scheme");
        // (beta, theta) of stage slot 1: the TR-BDF2 trapezoidal stage, the
        // Crank-Nicolson step, or the BDF2 step written as
        // (1/(beta dt)) (u* - (4 u^n - u^{n-1})/3) + ... with beta = 2/3
        const double g = c->gamma;
        const double beta1 = scheme == TBDG_SCHEME_TRBDF2 ? g : scheme == TBDG_SCHEME_BCG ? 1.0 : 2.0 / 3.0;
        const double theta1 = scheme == TBDG_SCHEME_BDF2 ? 1.0 : 0.5;
        if (scheme == TBDG_SCHEME_BDF2 && !c->s_wlag) c->s_wlag = dalloc(c->Nu);
        c->scheme = scheme;
        c->beta[1] = beta1;
        c->theta[1] = theta1;
        c->wlag_valid = false;
        trbdg::guess_reset(c);
        trbdg::launch_diag_pressure(c, c->alpha(1), c->diag_p[1]);
        trbdg::vec_recip(c->stream, c->Np, c->diag_p[1], c->invd_p[1]);
        // the level operators and eigenvalue estimates depend on (beta_1, theta_1)
        trbdg::mgu_free(c);
        if (c->mg) trbdg::mg_setup(c, &c->mg_desc);
        TBDG_HIP(hipStreamSynchronize(c->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_setup(tbdg_ctx* c, const tbdg_mg_desc* desc) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        trbdg::mg_setup(c, desc);
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_levels(tbdg_ctx* c, int cap, int* n_levels, int64_t* desc, double* lambda) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(n_levels != nullptr && cap >= 0, "null n_levels or negative cap");
        if (!c->mg) throw Error(TBDG_EINVAL, "multigrid hierarchy not built (tbdg_mg_setup)");
        levels_of(*c->mg, cap, n_levels, desc, lambda);
        return TBDG_OK;
    });
}

tbdg_status tbdg_mg_apply(tbdg_ctx* c, int stage, int precision, const double* r, double* z) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(r && z, "null pointer");
        require(r != z, "r and z may not alias");
        require(precision == 1 || precision == 2, "precision must be 1 (FP32) or 2 (BF16)");
        trbdg::mg_apply(c, stage, precision, r, z);
        return TBDG_OK;
    });
}

tbdg_status tbdg_set_guess_net(tbdg_ctx* c, tbdg_net* net) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        if (net) {
            require(trbdg::net_stream(net) == c->stream, "network and context must share one stream");
            if (c->geom.nc[0] > 93)
                throw Error(TBDG_EUNSUPPORTED, "the network takes at most 93 cells in x");
        }
        if (!c->gs && !net) return TBDG_OK;
        trbdg::guess_reset(c);
        trbdg::guess_ensure(c);
        c->gs->net = net;
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_reset(tbdg_ctx* c) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        trbdg::guess_reset(c);
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_record(tbdg_ctx* c, float* buf, int capacity) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(buf == nullptr || capacity > 0, "capacity must be positive");
        trbdg::guess_ensure(c);
        trbdg::guess_reset(c);
        c->gs->rec = buf;
        c->gs->rec_cap = buf ? capacity : 0;
        c->gs->rec_count = 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_recorded(tbdg_ctx* c, int* count) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(count != nullptr, "null pointer");
        *count = c->gs ? c->gs->rec_count : 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_last(tbdg_ctx* c, double* r_learned, double* r_fallback) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(r_learned && r_fallback, "null pointer");
        *r_learned = c->gs ? c->gs->last_r[0] : 0.0;
        *r_fallback = c->gs ? c->gs->last_r[1] : 0.0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_features(tbdg_ctx* c, int stage, const double* b, const double* p_prev,
                                const double* d0, double beta0, const double* d1, const double* d2,
                                float* x, double* scales) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        check_stage(stage);
        require(b && p_prev && d0 && d1 && d2 && x, "null pointer");
        require(beta0 > 0.0 && std::isfinite(beta0), "stage weight must be positive");
        trbdg::guess_features(c, stage, b, p_prev, d0, beta0, d1, d2);
        TBDG_HIP(hipMemcpyAsync(x, c->gs->feat, sizeof(float) * 6 * c->Nc, hipMemcpyDeviceToDevice,
                                c->stream));
        if (scales) {
            TBDG_HIP(hipMemcpyAsync(c->host_out, c->gs->sc, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream));
            TBDG_HIP(hipStreamSynchronize(c->stream));
            scales[0] = c->host_out[0];
            scales[1] = c->host_out[1];
        }
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_inject(tbdg_ctx* c, const double* p_prev, const double* d1, const double* d2,
                              const double* d3, const float* y, double* out) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(p_prev && d1 && d2 && d3 && y && out, "null pointer");
        trbdg::guess_inject(c, p_prev, d1, d2, d3, y, out);
        TBDG_HIP(hipStreamSynchronize(c->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_guess_target(tbdg_ctx* c, const double* p_new, const double* p_prev, const double* d1,
                              const double* d2, const double* d3, float* out) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(p_new && p_prev && d1 && d2 && d3 && out, "null pointer");
        trbdg::guess_target(c, p_new, p_prev, d1, d2, d3, out);
        TBDG_HIP(hipStreamSynchronize(c->stream));
        return TBDG_OK;
    });
}

tbdg_status tbdg_profile_enable(tbdg_ctx* c, int enable) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        trbdg::timer_collect(c);
        c->timer.on = enable != 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_profile_read(tbdg_ctx* c, int which, double* total_ms, int64_t* launches) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(which == 0 || which == 1, "which must be 0 (pressure) or 1 (momentum)");
        trbdg::timer_collect(c);
        if (total_ms) *total_ms = c->timer.total_ms[which];
        if (launches) *launches = c->timer.count[which];
        c->timer.total_ms[which] = 0.0;
        c->timer.count[which] = 0;
        return TBDG_OK;
    });
}

tbdg_status tbdg_profile_bytes(tbdg_ctx* c, int which, double* bytes) {
    if (!c) return TBDG_EINVAL;
    return guarded(c, [&]() {
        require(which == 0 || which == 1, "which must be 0 (pressure) or 1 (momentum)");
        require(bytes != nullptr, "null output");
        *bytes = c->timer.bytes[which];
        c->timer.bytes[which] = 0.0;
        return TBDG_OK;
    });
}

}  // extern "C"
