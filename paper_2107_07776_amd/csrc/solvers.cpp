// Krylov solvers and the TR-BDF2 step (host orchestration of device kernels).
//
// GMRES (momentum predictor): restarted, right-preconditioned with the exact
// Jacobi diagonal, the line blocks, or FP32 multigrid V-cycles of the
// operator's symmetric part on each component; classical Gram-Schmidt through one multi-vector dot kernel
// and one update kernel that also returns the new norm, repeated once when
// the norm drops below 1/sqrt(10) of its value before orthogonalisation (a
// looser form of the "twice is enough" test, enough for short restarts);
// Givens rotations on the host.
// CG (Helmholtz): Jacobi-preconditioned, three kernels per iteration
// (direction, operator fused with p.q and the step length, update fused with
// r.z, r.r and the next beta); all scalars stay on the device and the host
// reads the residual norm every 16 iterations.
// Both stop on the relative residual and confirm with a freshly computed
// true residual ||b - A x|| before returning.
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace trbdg {

namespace {

// scalar slot of red_out that a finishing kernel also wrote to host_out
double mirrored(tbdg_ctx* c, const double* dev) {
    TBDG_HIP(hipStreamSynchronize(c->stream));
    return c->host_out[dev - c->red_out];
}

double host_scalar(tbdg_ctx* c, const double* dev, int k = 1) {
    TBDG_HIP(hipMemcpyAsync(c->host_out, dev, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    TBDG_HIP(hipStreamSynchronize(c->stream));
    return c->host_out[0];
}

double norm2(tbdg_ctx* c, int64_t n, const double* x) {
    dot2(c, n, x, x, c->red_out + 63);
    return std::sqrt(host_scalar(c, c->red_out + 63));
}

// shift of the Arnoldi operator in the momentum GMRES (the diagonal of the
// Jacobi-scaled operator is one)
constexpr double kArnoldiShift = 1.0;

}  // namespace

// storage of the line-block preconditioner (allocated on first use)
void ensure_mom_blk(tbdg_ctx* c) {
    if (c->mom_blk) return;
    const int64_t nf = c->Nc * c->dim * (c->nbu / c->n) * c->n * c->n;
    void* p = nullptr;
    TBDG_HIP(hipMalloc(&p, sizeof(float) * nf));
    c->mom_blk = static_cast<float*>(p);
}

const double* build_mom_lineprec(tbdg_ctx* c, int s, const double* w) {
    ensure_mom_blk(c);
    const double* d = c->diag_u;
    if (c->mapped) {
        if (!c->mom_dbox) {
            void* p = nullptr;
            TBDG_HIP(hipMalloc(&p, sizeof(double) * c->Ns));
            c->mom_dbox = static_cast<double*>(p);
        }
        launch_diag_momentum_box(c, s, w, c->mom_dbox);
        d = c->mom_dbox;
    }
    launch_mom_lineblk(c, s, w, d, c->mom_blk);
    return d;
}

// ---------------------------------------------------------------------------
tbdg_status solve_momentum(tbdg_ctx* c, int s, const double* w, const double* b, double* x,
                           const tbdg_solver_opts& o, tbdg_solve_info* info, bool reuse_prec) {
    const int64_t n = c->Nu;
    const int m = std::min(o.restart > 0 ? o.restart : 30, c->gm_m);
    const bool line = o.precond == TBDG_PRECOND_LINE;
    const bool mgp = o.precond == TBDG_PRECOND_MG_FP32;
    // line blocks and multigrid are applied by their own kernels into gz;
    // the Jacobi scaling inside the operator kernel (the only user of D^{-1})
    const bool pc = line || mgp;
    const double* dprec = nullptr;
    if (line && reuse_prec && c->lineprec_stage == s) {
        // a later fixed-point solve of the same stage: the blocks built for
        // the previous advector stay a fixed preconditioner of this one
        dprec = c->mapped ? c->mom_dbox : c->diag_u;
    } else if (!mgp) {
        launch_diag_momentum(c, s, w, c->diag_u);
        if (line) {
            dprec = build_mom_lineprec(c, s, w);
            c->lineprec_stage = s;
        } else {
            vec_recip(c->stream, c->Ns, c->diag_u, c->invd_u);
        }
    }
    if (mgp) mgu_ensure(c);
    auto apply_pc = [&](const double* in, const double* sc_dev, double* out, bool acc) {
        if (line) launch_mom_lineprec(c, c->mom_blk, dprec, in, sc_dev, out, acc);
        else mg_apply_velocity(c, s, in, sc_dev, out, acc);
    };
    const double bnorm = norm2(c, n, b);
    tbdg_solve_info inf{0, 0.0, 0.0, 0};
    if (bnorm == 0.0) {
        TBDG_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
        if (info) *info = inf;
        return TBDG_OK;
    }
    if (!std::isfinite(bnorm)) {
        if (info) *info = inf;
        return TBDG_ENAN;
    }
    double* V = c->V;
    const int64_t ld = n;
    double* hdev = c->red_out;        // h (j+1 entries) then w.w
    double* nndev = c->red_out + 62;  // |w'|^2
    std::vector<double> H((m + 1) * m), H0((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1);
    int total = 0;
    tbdg_status st = TBDG_ENOTCONV;
    // initial residual r = b - A x into V_0; the Krylov vectors stay
    // unnormalised, their inverse norms live in c->gsc on the device
    double* gsc = c->gsc;
    launch_residual_momentum(c, s, w, x, b, V);
    gm_norm_inv(c, n, V, c->red_out + 63, gsc);
    double beta = std::sqrt(mirrored(c, c->red_out + 63));
    inf.res0 = beta / bnorm;
    // V_0 = b - A x recomputed (true) or formed from the Krylov basis at a
    // restart; convergence and the final residual always use a true one
    bool true_res = true;
    auto true_residual = [&]() {
        launch_residual_momentum(c, s, w, x, b, V);
        gm_norm_inv(c, n, V, c->red_out + 63, gsc);
        beta = std::sqrt(mirrored(c, c->red_out + 63));
        true_res = true;
    };
    while (true) {
        if (!std::isfinite(beta)) {
            st = TBDG_ENAN;
            break;
        }
        if (beta <= o.tol * bnorm || total >= o.maxiter) {
            if (!true_res) {
                true_residual();
                continue;
            }
            st = beta <= o.tol * bnorm ? TBDG_OK : TBDG_ENOTCONV;
            break;
        }
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        const double g0 = beta;
        int j = 0;
        bool breakdown = false;
        for (; j < m && total < o.maxiter; ++j) {
            ++total;
            double* vj = V + (int64_t)j * ld;
            double* vn = V + (int64_t)(j + 1) * ld;
            // vn = (A P^{-1} - sigma) (gsc_j V_j), P the Jacobi diagonal (applied
            // inside the operator kernel) or the line-block or multigrid
            // preconditioner (applied into gz): the Arnoldi process runs on
            // the shifted operator, whose Krylov spaces are the same; with the
            // preconditioned operator close to the identity the shift removes
            // most of the cancellation, so one Gram-Schmidt pass is normally
            // enough.  The first dots with V_0 .. V_j come out of the
            // operator kernel when they fit.
            const bool fused = j + 1 <= MOM_FUSE_MAX_DOTS;
            MomFuse fz{c->invd_u, gsc + j, kArnoldiShift, V, ld, fused ? j + 1 : 0,
                       c->gm_part, nullptr};
            const double* opnd = vj;
            if (pc) {
                apply_pc(vj, gsc + j, c->gz, false);
                opnd = c->gz;
                fz.invd = nullptr;
                fz.shv = vj;
            }
            const int Gop = launch_apply_momentum_fused(c, s, w, opnd, vn, fz);
            // classical Gram-Schmidt, repeated only when cancellation is large
            std::fill(h.begin(), h.end(), 0.0);
            double nn = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                if (pass == 0 && fused)
                    gm_finish_dots(c, Gop, j + 1, c->gm_part, gsc, hdev);
                else
                    gm_dots(c, n, j + 1, V, ld, vn, gsc, hdev);
                gm_update_norm(c, n, j + 1, V, ld, hdev, gsc, vn, nndev, gsc + j + 1);
                TBDG_HIP(hipStreamSynchronize(c->stream));   // h, w.w and |w'|^2 are in host_out
                for (int i = 0; i <= j; ++i) h[i] += c->host_out[i];
                const double ww = c->host_out[j + 1];
                nn = c->host_out[62];
                // one classical pass leaves an orthogonality error of about
                // eps |w|^2 / |w'|^2; up to a cancellation of |w'|^2 = |w|^2 / 10
                // that is ~10 eps, which a restart of a few vectors cannot feel
                if (!(nn < 0.1 * ww)) break;
            }
            const double hn = std::sqrt(nn);
            for (int i = 0; i <= j; ++i) H[i * m + j] = h[i];
            H[j * m + j] += kArnoldiShift;   // Hessenberg of A D^{-1} itself
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i <= j + 1; ++i) H0[i * m + j] = H[i * m + j];
            for (int i = 0; i < j; ++i) {
                const double t1 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                const double t2 = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t1;
                H[(i + 1) * m + j] = t2;
            }
            const double a = H[j * m + j], bb = H[(j + 1) * m + j];
            const double r = std::hypot(a, bb);
            if (r == 0.0 || !std::isfinite(r)) {
                breakdown = true;
                break;
            }
            cs[j] = a / r;
            sn[j] = bb / r;
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (std::fabs(g[j + 1]) <= o.tol * bnorm || hn == 0.0) {
                ++j;
                break;
            }
        }
        const int k = j;
        for (int i = k - 1; i >= 0; --i) {
            double s2 = g[i];
            for (int q = i + 1; q < k; ++q) s2 -= H[i * m + q] * y[q];
            y[i] = s2 / H[i * m + i];
        }
        if (k > 0 && !breakdown) {
            // residual of the updated x in the basis: r = V_{k+1} (beta e_1 - Hbar y)
            for (int i = 0; i <= k; ++i) {
                double ci = i == 0 ? g0 : 0.0;
                for (int q = (i > 0 ? i - 1 : 0); q < k; ++q) ci -= H0[i * m + q] * y[q];
                c->host_out[k + i] = ci;
            }
            std::memcpy(c->host_out, y.data(), sizeof(double) * k);
            TBDG_HIP(hipMemcpyAsync(c->red_out, c->host_out, sizeof(double) * (2 * k + 1),
                                    hipMemcpyHostToDevice, c->stream));
            gm_restart(c, n, k, V, ld, c->red_out, c->red_out + k, gsc, pc ? nullptr : c->invd_u,
                       x, c->red_out + 63, gsc, pc ? c->gz : nullptr);
            if (pc) {
                apply_pc(c->gz, nullptr, x, true);   // x += P^{-1} (V y)
            }
            beta = std::sqrt(mirrored(c, c->red_out + 63));
            true_res = false;
            continue;
        }
        if (k > 0) {
            std::memcpy(c->host_out, y.data(), sizeof(double) * k);
            TBDG_HIP(hipMemcpyAsync(c->red_out, c->host_out, sizeof(double) * k,
                                    hipMemcpyHostToDevice, c->stream));
            TBDG_HIP(hipMemsetAsync(c->gz, 0, sizeof(double) * n, c->stream));
            vec_add_combo(c->stream, n, k, V, ld, c->red_out, gsc, c->gz);
            if (pc) {
                apply_pc(c->gz, nullptr, x, true);   // x += P^{-1} (V y)
            } else {
                vec_add_div_diag_u(c->stream, n, c->dim, c->nbu, c->gz, c->diag_u, x);
            }
        }
        true_residual();
        if (breakdown && beta > o.tol * bnorm) {
            st = TBDG_EBREAKDOWN;
            break;
        }
    }
    inf.iters = total;
    inf.res_final = beta / bnorm;
    if (info) *info = inf;
    return st;
}

// ---------------------------------------------------------------------------
tbdg_status solve_pressure(tbdg_ctx* c, int s, const double* b, double* x,
                           const tbdg_solver_opts& o, tbdg_solve_info* info) {
    if (o.precond == TBDG_PRECOND_MG_FP32 || o.precond == TBDG_PRECOND_MG_BF16)
        return solve_pressure_mg(c, s, b, x, o, info);
    const int64_t n = c->Np;
    const double alpha = c->alpha(s);
    const double* invd = c->invd_p[s];
    double* r = c->cr;
    double* p = c->cp;
    double* q = c->cq;
    double* sc = c->red_out + 64;   // CG scalars
    tbdg_solve_info inf{0, 0.0, 0.0, 0};
    const double bnorm = norm2(c, n, b);
    if (bnorm == 0.0) {
        TBDG_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
        if (info) *info = inf;
        return TBDG_OK;
    }
    if (!std::isfinite(bnorm)) {
        if (info) *info = inf;
        return TBDG_ENAN;
    }
    TBDG_HIP(hipMemsetAsync(sc, 0, sizeof(double) * 8, c->stream));
    tbdg_status st = TBDG_ENOTCONV;
    int total = 0;
    const int check = 16;
    bool first_cycle = true;
    // partial sums of the update kernel (r.z then r.r), Gu blocks
    const int Gu = 256;
    double* up = c->red_part;
    while (true) {
        // (re)start from the true residual
        launch_apply_pressure(c, alpha, x, q);
        vec_axpby(c->stream, n, 1.0, b, -1.0, q, r);
        cg_start(c, n, invd, r, p, sc, up, Gu);
        TBDG_HIP(hipMemcpyAsync(c->host_out, sc, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
        TBDG_HIP(hipStreamSynchronize(c->stream));
        double rr = c->host_out[2];
        if (first_cycle) inf.res0 = std::sqrt(rr) / bnorm;
        first_cycle = false;
        if (!std::isfinite(rr)) {
            st = TBDG_ENAN;
            break;
        }
        if (std::sqrt(rr) <= o.tol * bnorm) {
            st = TBDG_OK;
            break;
        }
        if (total >= o.maxiter) break;
        bool converged = false, broke = false;
        double* pa = p;
        double* pb = c->cp2;
        int k = 0;
        while (total < o.maxiter) {
            ++k;
            const int slot = 8 + (k & 1), slot_prev = 8 + ((k - 1) & 1);
            const int Ga = launch_cg_apply(c, alpha, r, invd, pa, pb, q, sc, up, Gu, k == 1, slot,
                                           slot_prev);
            cg_upd(c, n, invd, x, r, pb, q, sc, c->red_op, Ga, slot, up, Gu);
            std::swap(pa, pb);
            ++total;
            if (total % check == 0 || total >= o.maxiter) {
                // r.r after this update: add the update kernel's partials here
                TBDG_HIP(hipMemcpyAsync(c->host_out, up + Gu, sizeof(double) * Gu,
                                        hipMemcpyDeviceToHost, c->stream));
                TBDG_HIP(hipMemcpyAsync(c->host_out + Gu, sc + 6, sizeof(double), hipMemcpyDeviceToHost,
                                        c->stream));
                TBDG_HIP(hipStreamSynchronize(c->stream));
                rr = 0.0;
                for (int i = 0; i < Gu; ++i) rr += c->host_out[i];
                if (c->host_out[Gu] != 0.0) {
                    broke = true;
                    break;
                }
                if (!std::isfinite(rr)) break;
                if (std::sqrt(rr) <= o.tol * bnorm) {
                    converged = true;
                    break;
                }
            }
        }
        if (broke) {
            st = TBDG_EBREAKDOWN;
            break;
        }
        if (!converged && !std::isfinite(rr)) {
            st = TBDG_ENAN;
            break;
        }
        if (!converged && total >= o.maxiter) {
            st = TBDG_ENOTCONV;
            break;
        }
    }
    launch_apply_pressure(c, alpha, x, q);
    vec_axpby(c->stream, n, 1.0, b, -1.0, q, r);
    const double rt = norm2(c, n, r);
    inf.iters = total;
    inf.res_final = rt / bnorm;
    if (st == TBDG_ENOTCONV && rt <= o.tol * bnorm) st = TBDG_OK;
    if (info) *info = inf;
    return st;
}

// ---------------------------------------------------------------------------
void extrapolate(tbdg_ctx* c, int s, const double* u_new, const double* u_old, double* w) {
    const double g = c->gamma;
    double e0, e1;
    if (s == 1) {
        e1 = -g / (2.0 * (1.0 - g));
        e0 = 1.0 - e1;
    } else {
        e1 = -(1.0 - g) / g;
        e0 = 1.0 - e1;
    }
    vec_axpby(c->stream, c->Nu, e0, u_new, e1, u_old, w);
}

// stage-s momentum right-hand side without the boundary terms of the
// advector; wx advects the stage-1 explicit advection
void rhs_momentum_base(tbdg_ctx* c, int s, const double* u_n, const double* u_g, const double* wx,
                       const double* p, double* rhs) {
    if (s == 1) {
        const double th = c->theta[1];
        launch_rhs_momentum(c, c->mcoef(1), u_n, u_n, wx, th * c->nu, th, nullptr, nullptr, 0.0,
                            0.0, p, rhs);
    } else {
        launch_rhs_momentum(c, c->mcoef(2), u_g, u_g, u_g, c->a32 * c->nu, c->a32, u_n, u_n,
                            c->a31 * c->nu, c->a31, p, rhs);
    }
}

void rhs_momentum(tbdg_ctx* c, int s, const double* u_n, const double* u_g, const double* w,
                  const double* p, double* rhs) {
    rhs_momentum_base(c, s, u_n, u_g, w, p, rhs);
    if (c->bnd_npts > 0) launch_dirichlet_rhs(c, s, w, rhs);
}

void rhs_pressure(tbdg_ctx* c, int s, const double* u_ss, const double* p_prev, double* rhs) {
    launch_rhs_pressure(c, c->alpha(s), 1.0 / (c->beta[s] * c->dt), u_ss, p_prev, rhs);
}

namespace {

// Momentum predictor of stage s into c->s_ustar, which holds the initial
// guess; c->s_w holds the extrapolated advector.  With c->nl_max > 1 the
// fully nonlinear form of Sec. 2: the stage-1 explicit advection is advected
// by u^n, and every solve after the first is advected by the previous
// solution, until the relative change drops to c->nl_tol or c->nl_max
// solves are done.  info sums the GMRES iterations of all solves.
tbdg_status momentum_stage(tbdg_ctx* c, int s, const double* u_n, const double* u_g,
                           const double* p, const tbdg_solver_opts& mo, tbdg_solve_info* info) {
    c->nl_solves[s - 1] = 1;
    if (c->nl_max <= 1) {
        rhs_momentum(c, s, u_n, u_g, c->s_w, p, c->s_rhs);
        return solve_momentum(c, s, c->s_w, c->s_rhs, c->s_ustar, mo, info);
    }
    const int64_t Nu = c->Nu;
    hipStream_t st = c->stream;
    const bool bnd = c->bnd_npts > 0;
    rhs_momentum_base(c, s, u_n, u_g, u_n, p, c->s_rhs);
    tbdg_solve_info acc{0, 0.0, 0.0, 0}, one{0, 0.0, 0.0, 0};
    tbdg_status rc = TBDG_OK;
    for (int solves = 1;; ++solves) {
        const double* b = c->s_rhs;
        if (bnd) {
            // s_u1 is free until the end of stage 2
            TBDG_HIP(hipMemcpyAsync(c->s_u1, c->s_rhs, sizeof(double) * Nu, hipMemcpyDeviceToDevice,
                                    st));
            launch_dirichlet_rhs(c, s, c->s_w, c->s_u1);
            b = c->s_u1;
        }
        rc = solve_momentum(c, s, c->s_w, b, c->s_ustar, mo, &one, solves > 1 && c->reuse_lineprec);
        if (solves == 1) acc.res0 = one.res0;
        acc.iters += one.iters;
        acc.res_final = one.res_final;
        c->nl_solves[s - 1] = solves;
        if (rc != TBDG_OK) break;
        if (solves >= 2 && c->nl_tol > 0.0) {
            vec_axpby(st, Nu, 1.0, c->s_ustar, -1.0, c->s_w, c->s_u1);
            const double dn = norm2(c, Nu, c->s_u1);
            if (dn <= c->nl_tol * norm2(c, Nu, c->s_ustar)) break;
        }
        if (solves >= c->nl_max) break;
        TBDG_HIP(hipMemcpyAsync(c->s_w, c->s_ustar, sizeof(double) * Nu, hipMemcpyDeviceToDevice, st));
    }
    if (info) *info = acc;
    return rc;
}

}  // namespace

tbdg_status step(tbdg_ctx* c, tbdg_state* S, const tbdg_solver_opts& mo,
                 const tbdg_solver_opts& po, tbdg_solve_info info[4]) {
    const int64_t Nu = c->Nu, Np = c->Np;
    hipStream_t st = c->stream;
    tbdg_solve_info loc[4];
    tbdg_status rc;
    const size_t bu = sizeof(double) * Nu, bp = sizeof(double) * Np;
    // ---- stage 1 ----
    extrapolate(c, 1, S->u, S->u_hist, c->s_w);
    if (mo.guess == TBDG_GUESS_PREVIOUS) {
        // linear extrapolation of (u^{n-1+gamma}, u^n) to t^n + gamma dt
        const double e = c->gamma / (1.0 - c->gamma);
        vec_axpby(st, Nu, 1.0 + e, S->u, -e, S->u_hist, c->s_ustar);
    } else {
        TBDG_HIP(hipMemcpyAsync(c->s_ustar, S->u, bu, hipMemcpyDeviceToDevice, st));
    }
    rc = momentum_stage(c, 1, S->u, nullptr, S->p, mo, &loc[0]);
    if (info) info[0] = loc[0];
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    const double b1 = c->beta[1] * c->dt;
    launch_add_grad_p(c, c->s_ustar, b1, S->p, c->s_ustar);          // u**
    rhs_pressure(c, 1, c->s_ustar, S->p, c->s_pb);
    int used = guess_prepare(c, 1, po.guess, c->s_pb, S->p, c->s_pg);
    rc = solve_pressure(c, 1, c->s_pb, c->s_pg, po, &loc[1]);
    loc[1].guess_used = used;
    if (info) info[1] = loc[1];
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    guess_after_solve(c, 1, c->s_pg, S->p);
    launch_add_grad_p(c, c->s_ustar, -b1, c->s_pg, c->s_ug);          // u^{n+gamma}
    // ---- stage 2 ----
    extrapolate(c, 2, c->s_ug, S->u, c->s_w);
    // stage-2 initial guess: u^{n+gamma}, or its linear extrapolation with u^n
    // to t^{n+1}, which is the stage-2 advector
    TBDG_HIP(hipMemcpyAsync(c->s_ustar, mo.guess == TBDG_GUESS_PREVIOUS ? c->s_w : c->s_ug, bu,
                            hipMemcpyDeviceToDevice, st));
    rc = momentum_stage(c, 2, S->u, c->s_ug, c->s_pg, mo, &loc[2]);
    if (info) info[2] = loc[2];
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    const double b2 = c->beta[2] * c->dt;
    launch_add_grad_p(c, c->s_ustar, b2, c->s_pg, c->s_ustar);
    rhs_pressure(c, 2, c->s_ustar, c->s_pg, c->s_pb);
    used = guess_prepare(c, 2, po.guess, c->s_pb, c->s_pg, c->s_p1);
    rc = solve_pressure(c, 2, c->s_pb, c->s_p1, po, &loc[3]);
    loc[3].guess_used = used;
    if (info) info[3] = loc[3];
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    guess_after_solve(c, 2, c->s_p1, c->s_pg);
    launch_add_grad_p(c, c->s_ustar, -b2, c->s_p1, c->s_u1);
    // ---- commit ----
    TBDG_HIP(hipMemcpyAsync(S->u_hist, c->s_ug, bu, hipMemcpyDeviceToDevice, st));
    TBDG_HIP(hipMemcpyAsync(S->u, c->s_u1, bu, hipMemcpyDeviceToDevice, st));
    TBDG_HIP(hipMemcpyAsync(S->p, c->s_p1, bp, hipMemcpyDeviceToDevice, st));
    S->t += c->dt;
    S->n += 1;
    return TBDG_OK;
}

// One step of the single-stage projection schemes of Sec. 2 (eqs.
// momentum_BCG / helmholtz_BCG and momentum_HI / helmholtz_HI) with their
// (beta, theta) in stage slot 1; S->u_hist holds u^{n-1}.
tbdg_status step_single(tbdg_ctx* c, tbdg_state* S, const tbdg_solver_opts& mo,
                        const tbdg_solver_opts& po, tbdg_solve_info info[4]) {
    const int64_t Nu = c->Nu, Np = c->Np;
    hipStream_t st = c->stream;
    const size_t bu = sizeof(double) * Nu, bp = sizeof(double) * Np;
    const bool bcg = c->scheme == TBDG_SCHEME_BCG;
    const bool bnd = c->bnd_npts > 0;
    tbdg_solve_info loc[4] = {};
    c->nl_solves[0] = c->nl_solves[1] = 0;
    // first advecting field: the extrapolation to t^{n+1/2} (Crank-Nicolson)
    // or the previous step's predictor (BDF2; u^n at the first step); the
    // BDF2 base state (4 u^n - u^{n-1})/3 in s_ug
    if (bcg) {
        vec_axpby(st, Nu, 1.5, S->u, -0.5, S->u_hist, c->s_w);
    } else {
        const bool lag = S->n > 0 && c->wlag_valid;
        TBDG_HIP(hipMemcpyAsync(c->s_w, lag ? c->s_wlag : S->u, bu, hipMemcpyDeviceToDevice, st));
        vec_axpby(st, Nu, 4.0 / 3.0, S->u, -1.0 / 3.0, S->u_hist, c->s_ug);
    }
    if (mo.guess == TBDG_GUESS_PREVIOUS)
        vec_axpby(st, Nu, 2.0, S->u, -1.0, S->u_hist, c->s_ustar);   // extrapolation to t^{n+1}
    else
        TBDG_HIP(hipMemcpyAsync(c->s_ustar, S->u, bu, hipMemcpyDeviceToDevice, st));
    const int max_solves = bcg ? c->nl_max : 1;
    tbdg_solve_info one{};
    tbdg_status rc = TBDG_OK;
    for (int solves = 1;; ++solves) {
        if (bcg)
            rhs_momentum_base(c, 1, S->u, nullptr, c->s_w, S->p, c->s_rhs);
        else
            launch_rhs_momentum(c, c->mcoef(1), c->s_ug, c->s_ug, c->s_w, 0.0, 0.0, nullptr, nullptr,
                                0.0, 0.0, S->p, c->s_rhs);
        if (bnd) launch_dirichlet_rhs(c, 1, c->s_w, c->s_rhs);
        rc = solve_momentum(c, 1, c->s_w, c->s_rhs, c->s_ustar, mo, &one);
        if (solves == 1) loc[0].res0 = one.res0;
        loc[0].iters += one.iters;
        loc[0].res_final = one.res_final;
        c->nl_solves[0] = solves;
        if (rc != TBDG_OK || solves >= max_solves) break;
        // next midpoint velocity (u* + u^n)/2; stop once it has settled
        vec_axpby(st, Nu, 0.5, c->s_ustar, 0.5, S->u, c->s_u1);
        if (c->nl_tol > 0.0) {
            vec_axpby(st, Nu, 1.0, c->s_u1, -1.0, c->s_w, c->s_rhs);
            const double dn = norm2(c, Nu, c->s_rhs);
            if (dn <= c->nl_tol * norm2(c, Nu, c->s_u1)) break;
        }
        TBDG_HIP(hipMemcpyAsync(c->s_w, c->s_u1, bu, hipMemcpyDeviceToDevice, st));
    }
    if (info) info[0] = loc[0];
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    // projection (u** in s_u1, the predictor stays in s_ustar), Helmholtz
    // solve, correction into s_ug
    const double b1 = c->beta[1] * c->dt;
    launch_add_grad_p(c, c->s_ustar, b1, S->p, c->s_u1);
    rhs_pressure(c, 1, c->s_u1, S->p, c->s_pb);
    const int used = guess_prepare(c, 1, po.guess, c->s_pb, S->p, c->s_p1);
    rc = solve_pressure(c, 1, c->s_pb, c->s_p1, po, &loc[1]);
    loc[1].guess_used = used;
    if (info) {
        info[1] = loc[1];
        info[2] = info[3] = tbdg_solve_info{};
    }
    if (rc != TBDG_OK) {
        guess_reset(c);
        return rc;
    }
    guess_after_solve(c, 1, c->s_p1, S->p);
    launch_add_grad_p(c, c->s_u1, -b1, c->s_p1, c->s_ug);
    // ---- commit ----
    if (!bcg) {
        TBDG_HIP(hipMemcpyAsync(c->s_wlag, c->s_ustar, bu, hipMemcpyDeviceToDevice, st));
        c->wlag_valid = true;
    }
    TBDG_HIP(hipMemcpyAsync(S->u_hist, S->u, bu, hipMemcpyDeviceToDevice, st));
    TBDG_HIP(hipMemcpyAsync(S->u, c->s_ug, bu, hipMemcpyDeviceToDevice, st));
    TBDG_HIP(hipMemcpyAsync(S->p, c->s_p1, bp, hipMemcpyDeviceToDevice, st));
    S->t += c->dt;
    S->n += 1;
    return TBDG_OK;
}

}  // namespace trbdg
