/*
 * trbdg — matrix-free DG operators, stage solvers and the TR-BDF2 projection
 * step of Orlando, Della Rocca, Barbante, Bonaventura, Parolini,
 * "An efficient and accurate implicit DG solver for the incompressible
 * Navier-Stokes equations" (arXiv 2107.07776), for AMD Instinct MI355X
 * (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer to contiguous float64 data,
 *    owned by the caller, unless stated otherwise.  The library never frees
 *    caller memory.  Input and output arrays of one call must not overlap
 *    unless the call says so.
 *  - Work is enqueued on the context's HIP stream and is asynchronous with
 *    respect to the host unless stated otherwise (the solvers and the step
 *    synchronise the stream to read their convergence scalars).
 *  - Layouts: a velocity field is [cell][component][node] (N_u = dim *
 *    N_cells * (k+1)^dim values); a scalar velocity-space field such as the
 *    momentum diagonal is [cell][node]; a pressure field is [cell][node]
 *    (N_p = N_cells * k^dim values).  Cells are numbered lexicographically
 *    with x fastest; nodes are the tensor-product Gauss-Legendre points of
 *    the reference cell, lexicographic with x fastest.
 *  - Velocity space: Q_k per component, Lagrange basis at the k+1
 *    Gauss-Legendre points, k+1 point Gauss quadrature (collocated, so the
 *    velocity mass matrix is diagonal).  Pressure: Q_{k-1}, Lagrange at the
 *    k Gauss points, k point quadrature in the pressure-only forms; forms
 *    coupling velocity and pressure use the velocity quadrature (Sec. 3).
 *  - Stage index s: 1 = TR stage (beta = gamma, theta = 1/2), 2 = BDF2-like
 *    stage (beta = 1 - gamma, theta = a33 = 1/(2 - gamma)), eq. trbdf2.
 *  - No exception or abort crosses this interface.  Every call returns a
 *    tbdg_status; on failure a message is available from tbdg_last_error.
 */
#ifndef TRBDG_H
#define TRBDG_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define TBDG_API __attribute__((visibility("default")))
#else
#define TBDG_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TBDG_OK = 0,
    TBDG_EINVAL = -1,        /* invalid argument, descriptor or null pointer   */
    TBDG_EDEVICE = -2,       /* a HIP runtime call failed                       */
    TBDG_ENOMEM = -3,        /* device allocation failed                        */
    TBDG_ENOTCONV = -4,      /* Krylov solver reached maxiter above tolerance   */
    TBDG_EBREAKDOWN = -5,    /* Krylov breakdown (zero or negative curvature)   */
    TBDG_ENAN = -6,          /* a non-finite residual was detected              */
    TBDG_EUNSUPPORTED = -7   /* valid request outside what the library supports  */
} tbdg_status;

typedef struct tbdg_ctx tbdg_ctx;

/* Structured box mesh T_h (Sec. 3).  dim 2 or 3; n_cells[a] >= 1;
 * lo < hi per direction; periodic[a] != 0 wraps direction a, otherwise its
 * two end faces are boundary faces with Dirichlet velocity data
 * (tbdg_set_dirichlet).  mapping 0 is the affine box.  mapping 1 (dim 2
 * only; TBDG_EUNSUPPORTED in 3D) moves every vertex of the box grid by
 * map_amp sin(2 pi x) sin(2 pi y) in both coordinates and keeps each cell
 * the bilinear (Q1) image of the reference square through its four moved
 * vertices.  map_amp must be finite (TBDG_EINVAL otherwise); the caller
 * keeps every cell's Jacobian positive (the displacement gradient is at
 * most 2 pi sqrt(2) |map_amp|, so |map_amp| < 0.11 suffices), which is not
 * checked.  Other mapping values: TBDG_EINVAL.                             */
typedef struct {
    int dim;
    int n_cells[3];
    double lo[3], hi[3];
    int periodic[3];
    int mapping;
    double map_amp;
} tbdg_mesh_desc;

/* Discretisation parameters.  k_u: velocity degree k >= 2 (pressure k-1);
 * supported: dim 2 with k <= 5, dim 3 with k <= 3.  nu = 1/Re.  c: the
 * artificial sound speed of eq. ns_artcomp (> 0).  dt > 0.  gamma: 0 selects
 * 2 - sqrt(2).  pen_u, pen_p: multipliers of the SIP penalties
 * sigma^u = (k+1)^2 |Gamma|/|K| and sigma^p = k^2 |Gamma|/|K| (eq. penconst1
 * and its pressure analogue, with diam(Gamma)/diam(K) read as the ratio of
 * face to cell measure); 0 selects 1.                                      */
typedef struct {
    int k_u;
    double nu, c, dt, gamma;
    double pen_u, pen_p;
} tbdg_disc_desc;

/* Create a context: validates the descriptors, builds the 1D Gauss tables,
 * the neighbour structure and the operator diagonals that do not depend on
 * the advecting field, and allocates all solver workspaces.  hip_stream is
 * a hipStream_t (NULL: the default stream).  On success *out owns the
 * device memory until tbdg_destroy.  On failure *out is NULL.                */
TBDG_API tbdg_status tbdg_create(const tbdg_mesh_desc* mesh, const tbdg_disc_desc* disc,
                        void* hip_stream, tbdg_ctx** out);
TBDG_API void tbdg_destroy(tbdg_ctx* ctx);
TBDG_API const char* tbdg_last_error(const tbdg_ctx* ctx);
TBDG_API tbdg_status tbdg_set_stream(tbdg_ctx* ctx, void* hip_stream);

/* Host outputs: total velocity DoFs (all components), pressure DoFs, cells. */
TBDG_API tbdg_status tbdg_sizes(const tbdg_ctx* ctx, int64_t* n_u, int64_t* n_p, int64_t* n_cells);

/* Physical node coordinates, field 0 = velocity nodes, 1 = pressure nodes,
 * written as [cell][node][dim] into a device array of (N_cells * nodes) * dim. */
TBDG_API tbdg_status tbdg_node_coords(const tbdg_ctx* ctx, int field, double* xyz);

/* Advecting velocity of stage s (Sec. 2 after eq. first_stage and
 * eq. second_stage): w = e0 u_new + e1 u_old with (e0, e1) =
 * (1 + gamma/(2(1-gamma)), -gamma/(2(1-gamma))) for s = 1 (u_new = u^n,
 * u_old = u^{n-1+gamma}) and (1 + (1-gamma)/gamma, -(1-gamma)/gamma) for
 * s = 2 (u_new = u^{n+gamma}, u_old = u^n).  All arrays N_u.                */
/* Dirichlet velocity data (Sec. 3: the boundary E^B of the non-periodic
 * directions; the pressure is natural, homogeneous Neumann, there).  The data
 * enter the momentum operator only through the Lax-Friedrichs speed at the
 * boundary, max(|w.n|, |(2 u_D - w).n|), and the momentum right-hand side
 * through the boundary terms of eq. rhs1 (penalty 2C on boundary faces).
 * Boundary points are the tangential velocity Gauss nodes of every boundary
 * face: for each non-periodic direction a, side 0 (low) then 1 (high), the
 * boundary cells in lexicographic order of their other coordinates, the
 * points lexicographic (lower direction fastest).  tbdg_face_qpoints returns
 * the count and, if xyz != NULL, the coordinates ([n][dim], device).        */
TBDG_API tbdg_status tbdg_face_qpoints(const tbdg_ctx* ctx, int64_t* n, double* xyz);
/* Dirichlet data at the boundary points ([n][dim], device, copied): slot 0
 * for the stage-1 time t^n + gamma dt, slot 1 for t^{n+1}; both start zero.
 * Stage s of tbdg_apply_momentum, tbdg_diag_momentum, tbdg_rhs_momentum,
 * tbdg_solve_momentum and tbdg_step uses slot s - 1.                        */
TBDG_API tbdg_status tbdg_set_dirichlet(tbdg_ctx* ctx, int slot, const double* uD);

TBDG_API tbdg_status tbdg_extrapolate(tbdg_ctx* ctx, int stage, const double* u_new,
                             const double* u_old, double* w);

/* Momentum operator of stage s applied to u (algebraic systems at the end of
 * Sec. 3): y = m_s M u + theta_s (nu A u + C(w) u), with A the SIP form of
 * eq. bilin_diff and C(w) the local Lax-Friedrichs form of eq. trilinear,
 * applied to each component.  w, u, y: N_u.                                 */
TBDG_API tbdg_status tbdg_apply_momentum(tbdg_ctx* ctx, int stage, const double* w,
                                const double* u, double* y);

/* Pressure Helmholtz operator of stage s: y = alpha_s M^p p + K p with
 * alpha_s = 1/(c^2 beta_s^2 dt^2) and K the SIP form a_p.  p, y: N_p.       */
TBDG_API tbdg_status tbdg_apply_pressure(tbdg_ctx* ctx, int stage, const double* p, double* y);

/* Exact diagonals (Jacobi preconditioners).  Momentum: diag is N_u/dim in
 * the [cell][node] layout, identical for every component.  Pressure: N_p.   */
TBDG_API tbdg_status tbdg_diag_momentum(tbdg_ctx* ctx, int stage, const double* w, double* diag);
TBDG_API tbdg_status tbdg_diag_pressure(tbdg_ctx* ctx, int stage, double* diag);

/* Right-hand side of the momentum predictor: rhs = m_s M u_prev + F_u^(s)
 * (eq. rhs1 for s = 1 with u_prev = u_n and advecting field w; the stage-2
 * functional for s = 2 with u_prev = u_g = u^{n+gamma}, which uses
 * u_g (x) u_g and u_n (x) u_n in the explicit advection).  p_prev is p^n
 * (s = 1) or p^{n+gamma} (s = 2).  u_g may be NULL for s = 1.               */
TBDG_API tbdg_status tbdg_rhs_momentum(tbdg_ctx* ctx, int stage, const double* u_n,
                              const double* u_g, const double* w,
                              const double* p_prev, double* rhs);

/* gu = M^{-1} P p: the broken pressure gradient projected into V_h (end of
 * Sec. 3); with collocated quadrature it is grad p at the velocity nodes.
 * p: N_p, gu: N_u.                                                         */
TBDG_API tbdg_status tbdg_grad_p(tbdg_ctx* ctx, const double* p, double* gu);

/* y = x + a * M^{-1} P p (velocity update of the projection, Sec. 3); y may
 * alias x.                                                                 */
TBDG_API tbdg_status tbdg_add_grad_p(tbdg_ctx* ctx, const double* x, double a,
                            const double* p, double* y);

/* Helmholtz right-hand side: rhs = alpha_s M^p p_prev + F_p^(s)(u_ss) with
 * F_p(q) = (1/(beta_s dt)) [ sum_K int u_ss . grad q - sum_E int {{u_ss}}.[[q]] ].
 * u_ss: N_u, p_prev, rhs: N_p.                                             */
TBDG_API tbdg_status tbdg_rhs_pressure(tbdg_ctx* ctx, int stage, const double* u_ss,
                              const double* p_prev, double* rhs);

/* Krylov options.  tol: relative true residual ||b - A x||_2 <= tol ||b||_2.
 * maxiter: total iterations (GMRES: over all restarts).  restart: GMRES
 * basis size m (<= 60).  precond: TBDG_PRECOND_*; TBDG_PRECOND_LINE applies
 * to the momentum solves only, TBDG_PRECOND_MG_BF16 to the pressure solves
 * only, TBDG_PRECOND_MG_FP32 to both (momentum: see
 * tbdg_mg_apply_momentum).  guess: 0 = use the content of x_inout.        */
enum {
    TBDG_GUESS_GIVEN = 0,       /* the content of x_inout (in tbdg_step: the previous pressure) */
    TBDG_GUESS_PREVIOUS = 1,    /* tbdg_step only: previous pressure + same stage's last increment */
    TBDG_GUESS_LEARNED = 2,     /* tbdg_step only: the guess network, TBDG_GUESS_PREVIOUS as fallback */
    TBDG_GUESS_EXTRAP2 = 3,     /* tbdg_step only: previous pressure + 2 inc_2 - inc_4 (pressure only) */
    TBDG_GUESS_EXTRAP3 = 4      /* tbdg_step only: previous pressure + 3 inc_2 - 3 inc_4 + inc_6
                                   (pressure only)                                               */
};
enum {
    TBDG_PRECOND_JACOBI = 0,
    TBDG_PRECOND_MG_FP32 = 1,   /* h/p-multigrid V-cycle in FP32 under FP64 flexible CG;
                                   momentum: one velocity-component V-cycle per component
                                   under FP64 GMRES (right preconditioning)             */
    TBDG_PRECOND_MG_BF16 = 2,   /* the same with BF16 storage on the finest level; if
                                   that cycle breaks flexible CG down (z.r <= 0) or the
                                   residual norm fails to halve over 10 steps, the
                                   solve restarts from its true residual with the FP32
                                   cycle (tbdg_solve_info.precond_fallbacks)            */
    TBDG_PRECOND_LINE = 3       /* momentum solves only: line-block preconditioner, see
                                   tbdg_precond_momentum                                 */
};
typedef struct {
    double tol;
    int maxiter;
    int restart;
    int precond;
    int guess;          /* TBDG_GUESS_*                                       */
} tbdg_solver_opts;

typedef struct {
    int iters;
    double res0;        /* ||b - A x0||_2 / ||b||_2                          */
    double res_final;   /* ||b - A x||_2 / ||b||_2, recomputed at the end    */
    int guess_used;     /* TBDG_GUESS_* actually used (tbdg_step)              */
    int precond_fallbacks; /* TBDG_PRECOND_MG_BF16: restarts with the FP32 cycle
                              after a breakdown or stall of the BF16 one (0/1)  */
} tbdg_solve_info;

/* Momentum predictor solve (right-preconditioned restarted GMRES with CGS2
 * orthogonalisation, Jacobi preconditioner, all components in one Krylov
 * space): V_s(w) u = rhs.  u_inout: initial guess in, solution out (the
 * best iterate is written even when the solve fails).                      */
TBDG_API tbdg_status tbdg_solve_momentum(tbdg_ctx* ctx, int stage, const double* w,
                                const double* rhs, double* u_inout,
                                const tbdg_solver_opts* opts, tbdg_solve_info* info);

/* Helmholtz solve: (alpha_s M^p + K) p = rhs by CG with the Jacobi
 * preconditioner, or by flexible CG (Polak-Ribiere beta) preconditioned with
 * one multigrid V-cycle (tbdg_mg_setup; built with default parameters on
 * first use).  Residuals, dot products, the recurrences and the coarsest
 * solve are FP64 in every case.                                             */
TBDG_API tbdg_status tbdg_solve_pressure(tbdg_ctx* ctx, int stage, const double* rhs,
                                double* p_inout, const tbdg_solver_opts* opts,
                                tbdg_solve_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Jacobi-preconditioned CG of tbdg_solve_pressure, same arguments and
 * results, with its residual, direction and operator vectors and its
 * reduction partials and scalars kept in a static device array of the
 * library (about 44 MB per GPU, held from the first context on that GPU
 * until the process ends) instead of the context's workspace.  It calls no
 * hipMalloc, hipFree or allocating routine.  Limits: N_p <= TBDG_NOALLOC_MAX_NP
 * (else TBDG_EINVAL, nothing launched); opts->precond must be
 * TBDG_PRECOND_JACOBI and opts->guess TBDG_GUESS_GIVEN (else
 * TBDG_EUNSUPPORTED).  Every call on one GPU shares that array, whatever
 * the context: calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  The call clears the scalars
 * it reads before it uses them; nothing else of the array has to start
 * at zero.                                                                  */
#define TBDG_NOALLOC_MAX_NP (1 << 20)
TBDG_API tbdg_status tbdg_solve_pressure_noalloc(tbdg_ctx* ctx, int stage, const double* rhs,
                                double* p_inout, const tbdg_solver_opts* opts,
                                tbdg_solve_info* info);

/* Multigrid preconditioner of the pressure Helmholtz operator.  The paper
 * preconditions the pressure CG with a multigrid (Sec. 4) without details;
 * this one is an h/p hierarchy on the affine box: level 0 is
 * Q_{k-1} on the mesh, then Q_1 on the same cells (when k-1 > 1), then Q_1
 * on meshes with every direction halved while all directions have an even
 * cell count and the level has more than coarse_cells cells.  Each level
 * operator is rediscretised (alpha_s M^p + K with the level's SIP penalty
 * (q+1)^2/h); prolongation evaluates the coarse polynomial at the fine
 * nodes, restriction is its transpose; smoothing is `degree` steps of
 * Chebyshev acceleration of the Jacobi-preconditioned level operator on
 * [lam/range, safety*lam], lam the largest Ritz value of lanczos_steps
 * Lanczos steps (FP64, start vector: SplitMix64 outputs from state 0, top
 * 53 bits scaled to [0,1), minus 1/2) on D^{-1/2} H D^{-1/2}; the coarsest
 * level is solved with the inverse formed from its FP64 Cholesky factor.
 * V-cycle: zero initial guess, pre- and post-smoothing.  Smoother vectors
 * are FP32 (BF16 storage on level 0 for TBDG_PRECOND_MG_BF16).             */
typedef struct {
    int degree;          /* Chebyshev steps per smoothing pass, 2..16 (0 => 4)   */
    int lanczos_steps;   /* 0 => 15                                             */
    double range;        /* 0 => 15                                             */
    double safety;       /* 0 => 1.1                                            */
    int coarse_cells;    /* 0 => 64 (3D) / 16 (2D)                              */
    int max_coarse_dofs; /* largest coarsest level solved densely (0 => 2048)    */
    int no_fuse;         /* 0: in 2D the longest run of Q1 levels below level 0
                            (down to the coarsest) whose FP32 vectors fit one
                            workgroup's LDS runs as one single-workgroup launch
                            per V-cycle (same smoother, transfers and coarse
                            solve), in 3D every level is launched on its own
                            (there the single workgroup is slower: 101 against
                            ~65 us per cycle on the 64^3 vortex's 8^3 and 4^3
                            levels); 1: every level on its own; 2: the single
                            workgroup in 2D and 3D                              */
} tbdg_mg_desc;

/* (Re)builds the hierarchy for both stages (desc NULL: defaults).  Fails
 * with TBDG_EUNSUPPORTED when fewer than two levels result or the coarsest
 * level exceeds max_coarse_dofs; allocates device memory held until
 * tbdg_destroy or the next tbdg_mg_setup.                                  */
TBDG_API tbdg_status tbdg_mg_setup(tbdg_ctx* ctx, const tbdg_mg_desc* desc);

/* Hierarchy description (after tbdg_mg_setup): *n_levels; for level l < cap,
 * desc[5l..5l+4] = nodes per direction, cells in x, y, z (1 if unused), DoFs;
 * lambda[l] and lambda[cap + l] = eigenvalue estimates of stages 1 and 2
 * (0 on the coarsest level).  Host arrays; desc or lambda may be NULL.     */
TBDG_API tbdg_status tbdg_mg_levels(tbdg_ctx* ctx, int cap, int* n_levels, int64_t* desc,
                                    double* lambda);

/* z = B_s r: one V-cycle of the stage-s hierarchy (precision 1: FP32,
 * 2: BF16 storage on level 0).  r, z: device, N_p, FP64; may not alias.     */
TBDG_API tbdg_status tbdg_mg_apply(tbdg_ctx* ctx, int stage, int precision, const double* r,
                                   double* z);

/* Multigrid preconditioner of the momentum solves (not in the paper, which
 * uses Jacobi; for TBDG_PRECOND_MG_FP32 in the momentum options).  The
 * stage-s momentum operator of Sec. 3 on one velocity component is
 * m_s M + theta_s (nu A + C(w)), with A the SIP form of eq. bilin_diff
 * (Dirichlet walls: boundary terms with the doubled penalty).  Its
 * symmetric part without advection is theta_s nu H with H = alpha_s M + A,
 * alpha_s = m_s / (theta_s nu): a Helmholtz operator of the same kind as the
 * pressure's, built into a second hierarchy by the rules of tbdg_mg_setup
 * (same parameters; level 0 the velocity space Q_k with the velocity
 * penalty, Dirichlet instead of natural conditions at walls; on Q1-mapped
 * cells the levels of the undistorted box).  z = P^{-1} v applies one FP32
 * V-cycle of H to each component of v / (theta_s nu).  The hierarchy is
 * built on first use (TBDG_EINVAL if nu = 0) and dropped by tbdg_mg_setup
 * and tbdg_set_scheme.  v, z: device, N_u, velocity layout, FP64; may not
 * alias.                                                                    */
TBDG_API tbdg_status tbdg_mg_apply_momentum(tbdg_ctx* ctx, int stage, const double* v, double* z);

/* The momentum hierarchy's description, as tbdg_mg_levels (builds it if
 * needed).                                                                  */
TBDG_API tbdg_status tbdg_mg_levels_momentum(tbdg_ctx* ctx, int cap, int* n_levels, int64_t* desc,
                                             double* lambda);

/* The single-workgroup coarse cycle of a built hierarchy (field 0: pressure,
 * 1: momentum): *first_level = the first level it runs (-1: none, every
 * level launched on its own), *lds_bytes = its LDS.  Host outputs.         */
TBDG_API tbdg_status tbdg_mg_fused(tbdg_ctx* ctx, int field, int* first_level, int64_t* lds_bytes);

/* enable = 1 (the default): every V-cycle of the pressure flexible CG, of
 * the momentum GMRES and of tbdg_mg_apply_momentum runs as one replay of a
 * HIP graph captured from its kernel launches on first use (per hierarchy,
 * stage, precision and output buffer); 0: the same kernels launched one by
 * one.  The results are the same bit for bit.  Captures are dropped with
 * their hierarchy; tbdg_mg_apply always launches kernel by kernel.         */
TBDG_API tbdg_status tbdg_set_mg_graphs(tbdg_ctx* ctx, int enable);

/* Learned initial guess of the pressure solves: a small 3D convolutional
 * network on the cell grid (not part of the paper).  Layers 6 -> 32 -> 32 ->
 * 32 -> 2, 3x3x3 kernels, circular padding, ReLU between layers; bf16
 * weights and activations with FP32 accumulation (matrix cores), FP32
 * master parameters and Adam.  Parameters are one flat FP32 vector
 * [W0, b0, W1, b1, W2, b2, W3, b3], each W laid out [out][in][dz][dy][dx];
 * the convolution is the cross-correlation
 *   y[o](z,y,x) = b[o] + sum_{i,dz,dy,dx} W[o][i][dz+1][dy+1][dx+1]
 *                        * x[i]((z+dz) mod nz, (y+dy) mod ny, (x+dx) mod nx).
 * All arrays are device pointers; work is enqueued on the network's stream. */
typedef struct tbdg_net tbdg_net;

/* channels must be 32.  Weights of the three hidden layers He-uniform
 * U(-a, a), a = sqrt(6 / (27 in)), drawn from SplitMix64 outputs from state
 * `seed` (top 53 bits scaled to [0, 1)), layer after layer; the output
 * layer's weights, every bias and the Adam moments zero.                   */
TBDG_API tbdg_status tbdg_net_create(int channels, uint64_t seed, void* hip_stream, tbdg_net** out);
TBDG_API void tbdg_net_destroy(tbdg_net* net);
TBDG_API const char* tbdg_net_last_error(const tbdg_net* net);
TBDG_API tbdg_status tbdg_net_num_params(const tbdg_net* net, int64_t* n);
/* Copy the FP32 master parameters in (resets Adam) / out; gradients out.      */
TBDG_API tbdg_status tbdg_net_set_params(tbdg_net* net, const float* theta);
TBDG_API tbdg_status tbdg_net_get_params(tbdg_net* net, float* theta);
TBDG_API tbdg_status tbdg_net_get_grads(tbdg_net* net, float* grads);
TBDG_API tbdg_status tbdg_net_zero_grad(tbdg_net* net);
/* y = net(x): x FP32 [B][6][nz][ny][nx] (rounded to bf16), y FP32
 * [B][2][nz][ny][nx].  nx <= 93.  Keeps the activations for tbdg_net_backward. */
TBDG_API tbdg_status tbdg_net_forward(tbdg_net* net, const float* x, float* y, int B, int nx, int ny,
                                      int nz);
/* Adds d(sum dy * y)/d(theta) of the last forward to the gradients; dy has
 * the shape of y (rounded to bf16 on entry).                                 */
TBDG_API tbdg_status tbdg_net_backward(tbdg_net* net, const float* dy);
/* dy = 2 (yhat - target) / n; *loss (host, may be NULL) = mean squared error. */
TBDG_API tbdg_status tbdg_net_mse(tbdg_net* net, const float* yhat, const float* target, int64_t n,
                                  float* dy, double* loss);
/* The guess's training loss: yhat FP32 [B][2][n] (the blend (y0, y1) of each
 * of n cells), gram FP32 [B][6][n] (g11, g12, g22, r1, r2, ee per cell, as
 * recorded by tbdg_guess_record); per cell
 *   l = ee - 2 (y0 r1 + y1 r2) + y0^2 g11 + 2 y0 y1 g12 + y1^2 g22,
 * *loss (host, may be NULL) = mean of l over the B n cells, dy [B][2][n] its
 * gradient with respect to yhat.                                            */
TBDG_API tbdg_status tbdg_net_quad_loss(tbdg_net* net, const float* yhat, const float* gram, int64_t n,
                                        int B, float* dy, double* loss);
/* One Adam step (Kingma and Ba, with bias correction) on the master
 * parameters from the accumulated gradients.                                */
TBDG_API tbdg_status tbdg_net_adam_step(tbdg_net* net, float lr, float beta1, float beta2, float eps);

/* Initial guesses of the Helmholtz solves in tbdg_step (not part of the
 * paper).  The context keeps the six newest pressure increments
 * p_new - p_prev of its solves; for the stage-s solve with right-hand side b
 * and previous pressure p, d1, d2 and d3 are the same stage's increments of
 * the last three steps and d0 the newest increment (the other stage's,
 * weight beta0).  With <a, c>_K = sum_{i in K} W_i a_i c_i (W_i the product of the
 * Gauss weights of node i on the unit cell):
 *   TBDG_GUESS_PREVIOUS: p + d1 (the fallback);
 *   TBDG_GUESS_EXTRAP2:  p + 2 d1 - d2;
 *   TBDG_GUESS_EXTRAP3:  p + 3 d1 - 3 d2 + d3;
 *   TBDG_GUESS_LEARNED:  per cell K the network input is (m1 / s_inc,
 *     m2 / s_inc, m0 / s_inc, div / s_div, cos_K, lr_K) with
 *     m1 = <d1, 1>_K / (beta_s dt), m2 = <d2, 1>_K / (beta_s dt),
 *     m0 = <d0, 1>_K / (beta0 dt), div = -(beta_s dt / |K|) sum_{i in K}
 *     (b_i - alpha_s (M^p p)_i) (cell average of div u** in flux form),
 *     s_inc and s_div the RMS over cells of m1 and div (1 where zero),
 *     cos_K = <d1, d2>_K / sqrt(<d1, d1>_K <d2, d2>_K) and
 *     lr_K = log(<d1, d1>_K / <d2, d2>_K) / 2 clamped to [-4, 4] (both 0
 *     where a norm vanishes); the network output (y0_K, y1_K) gives the
 *     guess p + (3 + y0_K) d1 - (3 - y1_K) d2 + d3 at the nodes of K (a
 *     correction of TBDG_GUESS_EXTRAP3); the candidate with the smaller FP64
 *     residual ||b - H x|| (learned or TBDG_GUESS_PREVIOUS) is used.
 * Without the history a mode needs, TBDG_GUESS_PREVIOUS (or, without any,
 * the previous pressure) is used.  A failed step clears the history.       */

/* Attach (net != NULL) or detach the guess network; it must use the
 * context's stream.  The network is borrowed, not owned.  Clears the history. */
TBDG_API tbdg_status tbdg_set_guess_net(tbdg_ctx* ctx, tbdg_net* net);
/* Forget the stored increments (start of a new trajectory).                 */
TBDG_API tbdg_status tbdg_guess_reset(tbdg_ctx* ctx);
/* Record training samples: after each TR-BDF2 Helmholtz solve of tbdg_step
 * whose stage has three earlier increments, sample k of buf (device, FP32,
 * [capacity][12][N_c]) receives the network input [6][N_c] and the Gram
 * target [6][N_c] of tbdg_guess_target for the solve's p_new, p, d1, d2, d3.
 * buf NULL stops recording; the history is cleared.                        */
TBDG_API tbdg_status tbdg_guess_record(tbdg_ctx* ctx, float* buf, int capacity);
TBDG_API tbdg_status tbdg_guess_recorded(tbdg_ctx* ctx, int* count);
/* ||b - H x|| of the learned and the fallback candidate of the last
 * TBDG_GUESS_LEARNED decision (host outputs; 0 before the first).          */
TBDG_API tbdg_status tbdg_guess_last(tbdg_ctx* ctx, double* r_learned, double* r_fallback);
/* The network input for given vectors (device, N_p each): x FP32 [6][N_c];
 * scales (host, may be NULL) = (s_inc, s_div).                              */
TBDG_API tbdg_status tbdg_guess_features(tbdg_ctx* ctx, int stage, const double* b,
                                         const double* p_prev, const double* d0, double beta0,
                                         const double* d1, const double* d2, float* x, double* scales);
/* out = p_prev + (3 + y0_K) d1 - (3 - y1_K) d2 + d3 (y: FP32 [2][N_c], the
 * rest N_p).                                                                 */
TBDG_API tbdg_status tbdg_guess_inject(tbdg_ctx* ctx, const double* p_prev, const double* d1,
                                       const double* d2, const double* d3, const float* y,
                                       double* out);
/* Gram target of a solve (device, N_p each; out FP32 [6][N_c]): per cell
 * (<d1,d1>, <d1,d2>, <d2,d2>, <e,d1>, <e,d2>, <e,e>)_K / S with
 * e = p_new - (p_prev + 3 d1 - 3 d2 + d3) and S the mean over cells of
 * <d1,d1>_K (1 where zero), so that the squared error <x - p_new, x - p_new>_K
 * of the injected guess x is S times the per-cell loss of
 * tbdg_net_quad_loss.                                                        */
TBDG_API tbdg_status tbdg_guess_target(tbdg_ctx* ctx, const double* p_new, const double* p_prev,
                                       const double* d1, const double* d2, const double* d3,
                                       float* out);

/* TR-BDF2 state: u = u^n, u_hist = u^{n-1+gamma} (history level of the
 * stage-1 extrapolation), p = p^n; t and n are host values.                 */
typedef struct {
    double* u;
    double* u_hist;
    double* p;
    double t;
    int64_t n;
} tbdg_state;

/* Momentum initial guesses in tbdg_step (mom->guess): TBDG_GUESS_GIVEN
 * starts stage 1 from u^n and stage 2 from u^{n+gamma}; TBDG_GUESS_PREVIOUS
 * from their linear extrapolations to the stage times,
 * (1 + e) u^n - e u^{n-1+gamma} with e = gamma / (1 - gamma), and the
 * stage-2 advector.                                                          */
/* One TR-BDF2 projection step (Sec. 2 and the algebraic form of Sec. 3):
 * per stage, extrapolate, momentum right-hand side, GMRES, projection,
 * Helmholtz right-hand side, CG, velocity correction.  info[0..3] receive
 * the momentum and pressure solves of stages 1 and 2.  The state is updated
 * only when all four solves succeed; otherwise it is left untouched and the
 * first failing status is returned.                                        */
TBDG_API tbdg_status tbdg_step(tbdg_ctx* ctx, tbdg_state* state, const tbdg_solver_opts* mom,
                      const tbdg_solver_opts* prs, tbdg_solve_info info[4]);

/* The line-block preconditioner of the momentum solves (not in the paper,
 * which uses Jacobi; for TBDG_PRECOND_LINE): z = P^{-1} v with
 * P^{-1} = B_z^{-1} D B_y^{-1} D B_x^{-1} (2D: B_y^{-1} D B_x^{-1}) applied to
 * each velocity component, D the Jacobi diagonal of the stage operator
 * V_s(w) and B_a its exact restriction to each grid line of direction a
 * inside a cell (D on the diagonal, the couplings of direction a off it:
 * stiffness, advection volume term and the own-trace parts of the SIP and
 * Lax-Friedrichs face terms of eqs. bilin_diff and trilinear).  Builds the
 * inverse blocks for w (computed in FP64, stored in FP32), then applies
 * them in FP64.  On Q1-mapped cells D and B_a are those of the undistorted
 * box (the same operator with the cells' vertex displacement removed), a
 * fixed approximation of the distorted operator.  w, v, z: N_u (device); v
 * and z must not alias.  The GMRES of TBDG_PRECOND_LINE uses the same
 * operator (right preconditioning).                                         */
TBDG_API tbdg_status tbdg_precond_momentum(tbdg_ctx* ctx, int stage, const double* w,
                                           const double* v, double* z);

/* Fully nonlinear momentum predictors (Sec. 2: the advecting velocity of
 * each stage may be the stage unknown itself, found by fixed-point
 * iteration).  max_solves = 1 (the default) is the linearised scheme with
 * the extrapolated advecting velocity.  With max_solves > 1 every tbdg_step
 * stage does up to max_solves momentum solves: the first advected by the
 * extrapolated velocity, each later one by the previous solution (which is
 * also its initial guess); the stage-1 explicit advection is advected by
 * u^n.  A stage stops early once ||u*_j - u*_{j-1}||_2 <= tol ||u*_j||_2
 * (tol = 0: always max_solves).  The momentum info of tbdg_step then sums
 * the GMRES iterations of all solves of the stage.  Errors: TBDG_EINVAL
 * for max_solves < 1 or tol < 0 or not finite.                             */
TBDG_API tbdg_status tbdg_set_nonlinear(tbdg_ctx* ctx, int max_solves, double tol);
/* solves[0..1] (host): momentum solves of stages 1 and 2 in the last
 * tbdg_step (also of a failed one, up to the failing solve).               */
TBDG_API tbdg_status tbdg_nonlinear_solves(tbdg_ctx* ctx, int* solves);

/* Time scheme of tbdg_step.  Besides TR-BDF2 the paper compares two
 * single-stage projection methods on the same DG forms (Sec. 2, eqs.
 * momentum_BCG, helmholtz_BCG, momentum_HI, helmholtz_HI):
 *   TBDG_SCHEME_BCG (Bell-Colella-Glaz, Crank-Nicolson): momentum
 *     [M/dt + (nu A + C(w))/2] u* = M u^n/dt + (explicit diffusion and
 *     advection of u^n advected by w)/2 + (weak gradient of p^n) + boundary
 *     data, w the midpoint velocity: the first solve is advected by
 *     (3 u^n - u^{n-1})/2, each later one (tbdg_set_nonlinear: up to
 *     max_solves, early stop on ||w_j - w_{j-1}||_2 <= tol ||w_j||_2) by
 *     (u*_{j-1} + u^n)/2; projection and Helmholtz solve with beta = 1;
 *   TBDG_SCHEME_BDF2 (Guermond-Quartapelle): [3M/(2dt) + nu A + C(w)] u* =
 *     M (4 u^n - u^{n-1})/(2 dt) + (weak gradient of p^n) + boundary data,
 *     one solve, w the momentum predictor of the context's previous step
 *     (u^n when state->n = 0); projection and Helmholtz solve with
 *     beta = 2/3 (alpha = 1/(c^2 beta^2 dt^2), divergence term 1/(beta dt),
 *     correction u^{n+1} = u** - beta dt M^{-1} P p^{n+1}).
 * With a single-stage scheme, tbdg_state.u_hist holds u^{n-1} (the exact
 * solution at t = -dt, or u^0, at the first step), the momentum and
 * pressure solves of tbdg_step go to info[0] and info[1] (info[2..3] are
 * zero), the stage-1 entry points (apply, diagonals, right-hand sides,
 * solves with stage = 1) use the scheme's (beta, theta), the Dirichlet data
 * of slot 1 (t^{n+1}) are used, mom->guess TBDG_GUESS_PREVIOUS starts from
 * 2 u^n - u^{n-1}, prs->guess TBDG_GUESS_PREVIOUS / TBDG_GUESS_EXTRAP2
 * extrapolate the pressure increments of the last one / two steps, and
 * TBDG_GUESS_LEARNED is TBDG_EUNSUPPORTED.  Setting a scheme recomputes the
 * stage-1 pressure diagonal, rebuilds an existing multigrid hierarchy with
 * its parameters, and clears the initial-guess history and the lagged
 * predictor.  Errors: TBDG_EINVAL for an unknown scheme.                   */
enum {
    TBDG_SCHEME_TRBDF2 = 0,
    TBDG_SCHEME_BCG = 1,
    TBDG_SCHEME_BDF2 = 2
};
TBDG_API tbdg_status tbdg_set_scheme(tbdg_ctx* ctx, int scheme);

/* Measurement hook.  While enabled, every third launch of the pressure
 * operator kernel (which = 0: tbdg_apply_pressure and the CG iterations) and
 * of the momentum operator kernel (which = 1: tbdg_apply_momentum and the
 * GMRES iterations), counted per calling thread, is bracketed by a pair of
 * HIP events on the context's stream (a timed dispatch has a cost of its
 * own; the stride keeps the mix of plain and fused launches).
 * tbdg_profile_read synchronises on the recorded events, returns the summed
 * kernel time in milliseconds and the number of timed launches for `which`
 * since the previous read, and resets those counters.                      */
TBDG_API tbdg_status tbdg_profile_enable(tbdg_ctx* ctx, int enable);
TBDG_API tbdg_status tbdg_profile_read(tbdg_ctx* ctx, int which, double* total_ms,
                                       int64_t* launches);
/* Algorithmic bytes (the compulsory FP64 reads and writes: pressure apply
 * 16 B, fused CG step 40 B, flexible CG step 32 B per pressure DoF; momentum
 * apply 24 B per velocity DoF, in GMRES plus 8 B per scalar node for the
 * inverse diagonal and 8 B per velocity DoF per fused dot) of the launches
 * timed for `which` since the previous call (host output), then reset.     */
TBDG_API tbdg_status tbdg_profile_bytes(tbdg_ctx* ctx, int which, double* bytes);

/* ------------------------------------------------------------------------
 * Adaptive 2D meshes with hanging nodes (Sec. 4, the adaptive runs: the
 * indicator eta_K = diam(K)^2 ||omega||^2_K, refinement of the 10 % of
 * cells with the largest indicator and coarsening of the 30 % with the
 * smallest, bounded element sizes).
 *
 * A quadtree over every cell of an n_cells[0] x n_cells[1] box; the leaves
 * (level l, integer position i, j: the cell [i, i+1] x [j, j+1] in units of
 * the base cell size / 2^l) stay 2:1 balanced across faces, so a face meets
 * at most two cells of half its size.  Cells are ordered by base cell (x
 * fastest), then by the Morton index (x bit below y bit) of their lower-left
 * corner at level max_level.  Fields use the layouts of the box mesh:
 * velocity [cell][component][node], pressure [cell][node], nodes the
 * (k+1)^2 resp. k^2 Gauss-Legendre points of the cell, x fastest.  Vectors
 * are device pointers on the handle's device, used on its stream; the mesh
 * itself (the forest) is host data of the handle.
 * ------------------------------------------------------------------------ */
typedef struct tbdg_amr tbdg_amr;
typedef struct {
    int n_cells[2];     /* base grid, >= 1; >= 2 in a periodic direction     */
    double lo[2], hi[2];
    int periodic[2];    /* non-periodic ends: pressure faces without terms
                           (homogeneous Neumann)                               */
    int k;              /* velocity degree 1..7 (pressure k - 1)             */
    int max_level;      /* deepest level, 0..20, n_cells[a] << max_level < 2^29 */
    double pen_p;       /* multiplier of the pressure SIP penalty (1 = paper) */
    double pen_u;       /* multiplier of the velocity SIP penalty (1 = paper) */
} tbdg_amr_desc;

/* The base grid (every cell at level 0) on the current device; hip_stream
 * may be NULL (default stream).  Errors: TBDG_EINVAL for a bad descriptor. */
TBDG_API tbdg_status tbdg_amr_create(const tbdg_amr_desc* desc, void* hip_stream, tbdg_amr** out);
TBDG_API void tbdg_amr_destroy(tbdg_amr* amr);
TBDG_API const char* tbdg_amr_last_error(const tbdg_amr* amr);
TBDG_API tbdg_status tbdg_amr_set_stream(tbdg_amr* amr, void* hip_stream);
/* Cell count and the velocity / pressure vector lengths of the current mesh. */
TBDG_API tbdg_status tbdg_amr_sizes(const tbdg_amr* amr, int64_t* n_cells, int64_t* n_u,
                                    int64_t* n_p);
/* (level, i, j) of every cell, host array of 3 n_cells int32.              */
TBDG_API tbdg_status tbdg_amr_leaves(const tbdg_amr* amr, int32_t* lij);

/* y = (alpha M^p + K) p with a_p of Sec. 3 on the adapted mesh: on a face
 * shared by a coarse and two fine cells every integral is the sum over the
 * two fine faces with their Gauss rule, the coarse traces evaluated there;
 * penalty C = average of the two cells' k^2 pen_p / h_a.  p, y distinct.  */
TBDG_API tbdg_status tbdg_amr_apply_pressure(tbdg_amr* amr, double alpha, const double* p, double* y);
/* Velocity Gauss points of the boundary faces of a non-periodic direction:
 * cells in order, faces (direction a, side s) in the order 2a + s, the k+1
 * points along each face; *n_points always, xy (device, [point][2]) when
 * not NULL.  Wall data for tbdg_amr_apply_momentum use this order.          */
TBDG_API tbdg_status tbdg_amr_face_qpoints(const tbdg_amr* amr, int64_t* n_points, double* xy);
/* y_c = mc M u_c + tnu A u_c + th C(w) u_c for both velocity components:
 * A the SIP bracket of eq. bilin_diff (penalty (k+1)^2 pen_u / h_a averaged
 * over the two cells; on walls -grad u.n v - u n.grad v + 2 C u v), C(w)
 * the Lax-Friedrichs form of eq. trilinear (lambda = max |w.n| of the two
 * traces at each face point; on walls lambda u v with the exterior state
 * 2 u_D - w).  Faces between a coarse and two fine cells are integrated on
 * the fine faces' Gauss points.  uD: wall data at tbdg_amr_face_qpoints
 * ([point][2], device), may be NULL on a fully periodic mesh.  y must not
 * alias u or w.                                                            */
TBDG_API tbdg_status tbdg_amr_apply_momentum(tbdg_amr* amr, double mc, double tnu, double th,
                                             const double* w, const double* u, const double* uD,
                                             double* y);
/* Restarted GMRES(restart), restart 1..60, for (mc M + tnu A + th C(w)) x = b
 * (both components in one Krylov space), right-preconditioned by the
 * diagonal of mc M + tnu A, classical Gram-Schmidt repeated once where
 * cancellation is large, FP64 throughout, from the given x to a true
 * residual ||b - A x|| <= tol ||b|| (checked at every restart).
 * Errors: TBDG_ENOTCONV, TBDG_EBREAKDOWN, TBDG_ENAN; x holds the last
 * iterate.                                                                  */
TBDG_API tbdg_status tbdg_amr_solve_momentum(tbdg_amr* amr, double mc, double tnu, double th,
                                             const double* w, const double* uD, const double* b,
                                             double* x, double tol, int maxiter, int restart,
                                             tbdg_solve_info* info);
/* The flow of the stage forms below: viscosity nu = 1/Re, time step dt and
 * artificial sound speed c (alpha_s = 1/(c beta_s dt)^2; INFINITY: none).  */
TBDG_API tbdg_status tbdg_amr_set_flow(tbdg_amr* amr, double nu, double dt, double c);
/* m_s M u_prev + F_u^(s) on the adapted mesh (eq. rhs1 and its stage-2
 * analogue, the TR-BDF2 coefficients of tbdg_rhs_momentum): stage 1 u_prev
 * = u_n and the explicit advection advected by w_explicit (NULL: w);
 * stage 2 u_prev = u_g with a32 (u_g, u_g) + a31 (u_n, u_n); the weak
 * gradient of p_prev; the wall-data terms with the implicit advector w and
 * uD (at tbdg_amr_face_qpoints; NULL on a fully periodic mesh).  out must
 * not alias an input.                                                      */
TBDG_API tbdg_status tbdg_amr_rhs_momentum(tbdg_amr* amr, int stage, const double* u_n,
                                           const double* u_g, const double* w,
                                           const double* w_explicit, const double* p_prev,
                                           const double* uD, double* out);
/* alpha_s M^p p_prev + (1/(beta_s dt)) D u_ss, D the bracket of F_p.      */
TBDG_API tbdg_status tbdg_amr_rhs_pressure(tbdg_amr* amr, int stage, const double* u_ss,
                                           const double* p_prev, double* out);
/* y = x + a M^{-1} P p (x, y may alias).                                    */
TBDG_API tbdg_status tbdg_amr_add_grad_p(tbdg_amr* amr, const double* x, double a, const double* p,
                                         double* y);
typedef struct {
    int nonlinear;      /* momentum solves per stage (>= 1): fixed point      */
    double mom_tol, prs_tol;
    int mom_maxiter, prs_maxiter, restart;   /* restart <= 0: 30; max 60    */
} tbdg_amr_step_opts;
/* One TR-BDF2 step on the adapted mesh (the stages of tbdg_step: the
 * advecting velocity extrapolated from u and u_hist = u^{n-1+gamma}, the
 * momentum GMRES of tbdg_amr_solve_momentum from the stage's previous
 * value, the pressure CG of tbdg_amr_solve_pressure from the previous
 * pressure, time-independent wall data uD).  On success u, u_hist, p hold
 * u^{n+1}, u^{n+gamma}, p^{n+1}; on failure they are unchanged.  info: the
 * four solves (stage-1 momentum, pressure, stage-2 momentum, pressure);
 * max_du (host, may be NULL): max over all velocity DoFs of
 * |u^{n+1} - u^n|, the quantity of the early remeshing check of Sec. 4.    */
TBDG_API tbdg_status tbdg_amr_step(tbdg_amr* amr, const tbdg_amr_step_opts* opts, double* u,
                                   double* u_hist, double* p, const double* uD,
                                   tbdg_solve_info info[4], double* max_du);
/* d = diag(alpha M^p + K).                                                 */
TBDG_API tbdg_status tbdg_amr_diag_pressure(tbdg_amr* amr, double alpha, double* d);
/* Preconditioned CG for (alpha M^p + K) x = b from the given x (alpha > 0),
 * FP64 vectors and recurrences, to ||b - A x|| <= tol ||b|| (the recurrence
 * residual, read every 8 iterations).  Preconditioner: the inverses of the
 * cells' diagonal blocks (stored FP32) for k <= 4, else the Jacobi
 * diagonal.  Errors: TBDG_ENOTCONV, TBDG_EBREAKDOWN, TBDG_ENAN; x holds
 * the last iterate.                                                          */
TBDG_API tbdg_status tbdg_amr_solve_pressure(tbdg_amr* amr, double alpha, const double* b, double* x,
                                             double tol, int maxiter, tbdg_solve_info* info);
/* eta[c] = (h_x^2 + h_y^2) int_K (d_x u_y - d_y u_x)^2 (the diagonal as
 * diam(K); the velocity Gauss rule, exact for the squared vorticity).      */
TBDG_API tbdg_status tbdg_amr_indicator(tbdg_amr* amr, const double* u, double* eta);
/* Fixed-fraction marking from eta (device): the floor(refine_frac N) cells
 * of largest eta (ties: lower index first) get +1 unless their children's
 * larger edge would fall below h_min or the level is max_level; of the
 * others, the floor(coarsen_frac N) of smallest eta get -1 unless the
 * parent's larger edge would exceed h_max or the level is 0; the rest 0.
 * flags: host array of N int8.  Errors: TBDG_ENAN for a NaN indicator.     */
TBDG_API tbdg_status tbdg_amr_mark(tbdg_amr* amr, const double* eta, double refine_frac,
                                   double coarsen_frac, double h_min, double h_max, int8_t* flags);
/* Remeshing in three calls, so that the caller owns every vector:
 * tbdg_amr_plan builds the adapted forest from host flags (> 0 refine, < 0
 * coarsen; refinement spreads to coarser face neighbours until balanced; a
 * family of four flagged, unrefined leaves is coarsened unless a face
 * neighbour would end finer than the family's leaves) and returns its cell
 * count; tbdg_amr_transfer moves a field (0: velocity, 1: pressure) from
 * the current mesh to the planned one (kept cells copy, children
 * interpolate their parent's polynomial, a parent is the L2 projection of
 * its four children); tbdg_amr_commit makes the planned mesh current.      */
TBDG_API tbdg_status tbdg_amr_plan(tbdg_amr* amr, const int8_t* flags, int64_t* new_cells);
TBDG_API tbdg_status tbdg_amr_transfer(tbdg_amr* amr, int field, const double* src, double* dst);
TBDG_API tbdg_status tbdg_amr_commit(tbdg_amr* amr);

#ifdef __cplusplus
}
#endif

#endif /* TRBDG_H */
