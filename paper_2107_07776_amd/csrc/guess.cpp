// Initial guesses of the Helmholtz solves inside tbdg_step: the previous
// pressure, the previous pressure plus the same stage's increment of the
// previous step (the fallback), that increment extrapolated linearly from its
// last two or quadratically from its last three values, or the learned
// correction of the quadratic extrapolation with the fallback as the
// alternative (the guess with the smaller FP64 residual is used).
// Also records (input, target) samples of the network from the solver's own
// solves.
#include <cmath>
#include <utility>

#include "internal.hpp"

namespace trbdg {

namespace {

void fill_state(tbdg_ctx* c, GuessState* g);

void ensure_state(tbdg_ctx* c) {
    if (c->gs) return;
    GuessState* g = new GuessState();
    try {
        fill_state(c, g);
    } catch (...) {
        for (void* p : g->allocs) (void)hipFree(p);
        delete g;
        throw;
    }
    c->gs = g;   // published only when complete
}

void fill_state(tbdg_ctx* c, GuessState* g) {
    auto dal = [&](int64_t n) {
        void* p = nullptr;
        TBDG_HIP(hipMalloc(&p, sizeof(double) * (size_t)(n > 0 ? n : 1)));
        g->allocs.push_back(p);
        return static_cast<double*>(p);
    };
    auto fal = [&](int64_t n) {
        void* p = nullptr;
        TBDG_HIP(hipMalloc(&p, sizeof(float) * (size_t)(n > 0 ? n : 1)));
        g->allocs.push_back(p);
        return static_cast<float*>(p);
    };
    for (int i = 0; i < GuessState::kHist; ++i) g->inc[i] = dal(c->Np);
    g->cells = dal(7 * c->Nc);
    g->partial = dal(2 * c->Nc + 2);   // two partials per block of at least one cell
    g->sc = dal(8);
    g->trial = dal(c->Np);
    g->feat = fal(6 * c->Nc);
    g->y = fal(2 * c->Nc);
}

// ||b - H x||^2 into the device slot
void residual_sq(tbdg_ctx* c, int s, const double* b, const double* x, double* slot) {
    launch_apply_pressure(c, c->alpha(s), x, c->cq);
    vec_axpby(c->stream, c->Np, 1.0, b, -1.0, c->cq, c->cr);
    dot2(c, c->Np, c->cr, c->cr, slot);
}

}  // namespace

void guess_ensure(tbdg_ctx* c) { ensure_state(c); }

void guess_free(tbdg_ctx* c) {
    if (!c->gs) return;
    for (void* p : c->gs->allocs) (void)hipFree(p);
    delete c->gs;
    c->gs = nullptr;
}

void guess_reset(tbdg_ctx* c) {
    if (c->gs) c->gs->n = 0;
}

void guess_features(tbdg_ctx* c, int s, const double* b, const double* p, const double* d0,
                    double beta0, const double* d1, const double* d2) {
    ensure_state(c);
    GuessState& g = *c->gs;
    const double bdt = c->beta[s] * c->dt;
    const int G = launch_guess_cells(c, d1, d2, d0, b, p, 1.0 / bdt, 1.0 / (beta0 * c->dt), -bdt,
                                     c->alpha(s), g.cells, g.partial);
    launch_guess_feat(c, g.cells, g.partial, G, g.feat, g.sc);
}

void guess_inject(tbdg_ctx* c, const double* p, const double* d1, const double* d2, const double* d3,
                  const float* y, double* out) {
    launch_guess_inject(c, p, d1, d2, d3, y, out);
}

void guess_target(tbdg_ctx* c, const double* pn, const double* p, const double* d1, const double* d2,
                  const double* d3, float* out) {
    ensure_state(c);
    launch_guess_target(c, pn, p, d1, d2, d3, c->gs->cells, c->gs->partial, out);
}

int guess_prepare(tbdg_ctx* c, int s, int mode, const double* b, const double* p_prev, double* x) {
    const int64_t bp = (int64_t)sizeof(double) * c->Np;
    const bool two_stage = c->scheme == TBDG_SCHEME_TRBDF2;
    const bool recording = two_stage && c->gs && c->gs->rec && c->gs->rec_count < c->gs->rec_cap;
    // the same stage's increments one and two steps back: every other entry
    // of the history with two stages per step, consecutive entries with one
    const int lag1 = two_stage ? 1 : 0, lag2 = two_stage ? 3 : 1, lag3 = two_stage ? 5 : 2;
    if (mode == 0 && !recording) {
        TBDG_HIP(hipMemcpyAsync(x, p_prev, bp, hipMemcpyDeviceToDevice, c->stream));
        return 0;
    }
    ensure_state(c);
    GuessState& g = *c->gs;
    g.feat_valid = false;
    // the network needs the same stage's increments of the last three steps
    const bool history = two_stage && g.n > lag3;
    const bool learned = mode == TBDG_GUESS_LEARNED && g.net != nullptr && history;
    if (history && (learned || recording)) {
        guess_features(c, s, b, p_prev, g.inc[0], g.beta[0], g.inc[lag1], g.inc[lag2]);
        g.feat_valid = true;
    }
    if (mode == 0 || g.n <= lag1) {
        TBDG_HIP(hipMemcpyAsync(x, p_prev, bp, hipMemcpyDeviceToDevice, c->stream));
        return 0;
    }
    if (mode == TBDG_GUESS_EXTRAP3 && g.n > lag3) {
        // quadratic extrapolation of the same stage's increment from its last
        // three values: p + 3 inc[lag1] - 3 inc[lag2] + inc[lag3]
        vec_axpby(c->stream, c->Np, 3.0, g.inc[lag1], -3.0, g.inc[lag2], x);
        vec_axpby(c->stream, c->Np, 1.0, g.inc[lag3], 1.0, x, x);
        vec_axpby(c->stream, c->Np, 1.0, p_prev, 1.0, x, x);
        return TBDG_GUESS_EXTRAP3;
    }
    if ((mode == TBDG_GUESS_EXTRAP2 || mode == TBDG_GUESS_EXTRAP3) && g.n > lag2) {
        // the same stage's increment extrapolated linearly from its last two
        // values: p + 2 inc[lag1] - inc[lag2]
        vec_axpby(c->stream, c->Np, 2.0, g.inc[lag1], -1.0, g.inc[lag2], x);
        vec_axpby(c->stream, c->Np, 1.0, p_prev, 1.0, x, x);
        return TBDG_GUESS_EXTRAP2;
    }
    // fallback: the increment of the same stage one step earlier (the two
    // TR-BDF2 stages' pressures carry different offsets, so the other
    // stage's increment is a poor predictor)
    vec_axpby(c->stream, c->Np, 1.0, p_prev, 1.0, g.inc[lag1], x);
    if (!learned) return 1;
    net_infer(g.net, g.feat, g.y, c->geom.nc[0], c->geom.nc[1], c->geom.nc[2]);
    guess_inject(c, p_prev, g.inc[lag1], g.inc[lag2], g.inc[lag3], g.y, g.trial);
    residual_sq(c, s, b, g.trial, c->red_out + 60);
    residual_sq(c, s, b, x, c->red_out + 61);
    TBDG_HIP(hipMemcpyAsync(c->host_out, c->red_out + 60, 2 * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    TBDG_HIP(hipStreamSynchronize(c->stream));
    const double rl = c->host_out[0], rf = c->host_out[1];
    g.last_r[0] = std::sqrt(rl);
    g.last_r[1] = std::sqrt(rf);
    if (std::isfinite(rl) && rl < rf) {
        TBDG_HIP(hipMemcpyAsync(x, g.trial, bp, hipMemcpyDeviceToDevice, c->stream));
        return 2;
    }
    return 1;
}

void guess_after_solve(tbdg_ctx* c, int s, const double* p_new, const double* p_prev) {
    if (!c->gs) return;
    GuessState& g = *c->gs;
    if (g.feat_valid && g.rec && g.rec_count < g.rec_cap) {
        // sample = network input [6][Nc], then the Gram target [6][Nc]; the
        // same stage's increments are inc[1], inc[3] and inc[5] until the
        // shift below
        float* dst = g.rec + (int64_t)g.rec_count * 12 * c->Nc;
        TBDG_HIP(hipMemcpyAsync(dst, g.feat, sizeof(float) * 6 * c->Nc, hipMemcpyDeviceToDevice, c->stream));
        guess_target(c, p_new, p_prev, g.inc[1], g.inc[3], g.inc[5], dst + 6 * c->Nc);
        ++g.rec_count;
    }
    g.feat_valid = false;
    constexpr int H = GuessState::kHist;
    double* oldest = g.inc[H - 1];
    for (int i = H - 1; i > 0; --i) {
        g.inc[i] = g.inc[i - 1];
        g.beta[i] = g.beta[i - 1];
    }
    g.inc[0] = oldest;
    vec_axpby(c->stream, c->Np, 1.0, p_new, -1.0, p_prev, g.inc[0]);
    g.beta[0] = c->beta[s];
    g.n = g.n < H ? g.n + 1 : H;
}

}  // namespace trbdg
