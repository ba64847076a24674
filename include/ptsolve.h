/*
 * ptsolve.h -- C ABI of the MI355X (gfx950) solver for the implicit-Euler
 * time-periodic nonlinear eddy-current problem.
 *
 * Problem 1 of the paper (eqs. (disc1)-(disc2)): find U = (u^1, ..., u^N) with
 *     M (u^n - u^{n-1}) / tau + K(u^n) = f^n,  n = 1..N,   u^0 = u^N,
 * where, for the 2-D model of Sec. 4 ("Test problem"),
 *     K(u)  = -div(nu(|grad u|) grad u)  (P1 finite elements, u = 0 on the boundary),
 *     M     = sigma-weighted consistent P1 mass (sigma may vanish: degenerate, (A2)),
 *     f^n   = J0 w(2 pi t_n / T) b,  t_n = n tau, tau = T / N.
 * The solver is the fixed-point iteration of Sec. 3, eqs. (iter1)-(iter2), with
 * the linear operator Khat = nu_max * (P1 stiffness) (or a P1 stiffness with a
 * coefficient per region, pt_region.nu_hat), run in correction form
 *     U^{k+1} = U^k + P^{-1}(F - A(U^k)),  P = I (x) (M/tau + Khat) - C_N (x) M/tau,
 * whose fixed point is A(U) = F however P^{-1} is approximated. Each P^{-1} is
 * applied by a DFT along time (remark rem:parallel: the periodic time-invariant
 * system is block diagonal in frequency) and one batched solve of the N/2 + 1
 * complex-shifted systems (Khat + z_k M) X_k = R_k, z_k = (1 - exp(-2 pi i k/N))/tau,
 * preconditioned by a geometric-multigrid V-cycle.
 *
 * Mesh: uniform n x n cells on the unit square, each cell split along its SW-NE
 * diagonal; node (i, j) at (i/n, j/n) has index j (n+1) + i. Triangle ids are
 * 2 (j n + i) + 0 for {(i,j),(i+1,j),(i+1,j+1)} and + 1 for {(i,j),(i+1,j+1),(i,j+1)}.
 * A triangle belongs to a rectangle iff its centroid lies in the closed rectangle.
 *
 * Memory and ownership. Every device buffer (solution, workspace, optional
 * tables) is allocated and owned by the caller and must stay valid until the
 * stream-ordered work of the call has completed. The library allocates no device
 * memory at run time (the one device array it holds, the 64 MiB scratch of
 * pt_solve_noalloc, is part of its code object); a plan owns only small host state. All entry points are stream-ordered
 * on the given HIP stream (hipStream_t passed as void*, NULL = default stream);
 * pt_solve and pt_residual additionally synchronise that stream before returning
 * because they read scalars back to the host.
 *
 * Errors. Every function returns a pt_status; no C++ exception crosses the ABI.
 * Arguments are validated before anything is launched. pt_last_error() returns a
 * thread-local description of the most recent failure on the calling thread.
 *
 * Layouts.
 *   time field    double [N][n+1][n+1]: slice j holds u^{j+1} (so slice N-1 is
 *                 u^N = u^0); boundary entries are read as 0 and written as 0.
 *   frequency     complex [ (n+1)^2 ][N/2] interleaved (re, im), node-major, in
 *   field         the plan's solver precision (double for PT_FP64, float for
 *                 PT_FP32_REFINE). Slot s >= 1 holds X_s = sum_j x^{j+1} e^{-2 pi i j s/N};
 *                 slot 0 holds (Re X_0) + i (Re X_{N/2}) (both real for real input).
 */
#ifndef PTSOLVE_H
#define PTSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PT_OK = 0,
    PT_ERR_INVALID = -1,        /* an argument or option is out of range */
    PT_ERR_HIP = -3,            /* a HIP runtime call failed (message in pt_last_error) */
    PT_ERR_NOT_CONVERGED = -4,  /* max_outer reached; the solution holds the last iterate */
    PT_ERR_BREAKDOWN = -5,      /* COCG bilinear form p^T A p vanished (to breakdown_tol) for an
                                   active frequency */
    PT_ERR_NONFINITE = -6,      /* residual norm is NaN or Inf */
    PT_ERR_DIVERGED = -7,       /* residual grew by diverge_factor over its minimum */
    PT_ERR_WORKSPACE = -8       /* workspace NULL, too small or not 256-byte aligned */
} pt_status;

typedef enum { PT_FP64 = 0, PT_FP32_REFINE = 1 } pt_precision;

/* Inner approximation of P^{-1} per frequency k (all frequencies in one launch):
 *  PT_INNER_GALERKIN1: one V-cycle p = B_k r, then x = alpha p with
 *                      alpha = (p^H r) / (p^H A_k p) (Galerkin condition in the
 *                      Hermitian inner product; p^H A_k p has positive real part).
 *  PT_INNER_COCG:      COCG (unconjugated bilinear form x^T y, preconditioned by
 *                      the same V-cycle) from zero, per frequency until
 *                      ||r_k|| <= inner_rtol ||R_k|| (that frequency is then
 *                      masked: its iterate no longer changes) or inner_iters
 *                      steps. A frequency whose right-hand side is zero is
 *                      masked from the start.                                   */
typedef enum { PT_INNER_GALERKIN1 = 0, PT_INNER_COCG = 1 } pt_inner;

/* Shape of the multigrid cycle B_k (P1 interpolation P, restriction P^T, damped Jacobi with
 * D = diag(Khat) + z_k diag(M), i.e. 4 nu_max + z_k diag(M) for Khat = nu_max S, exact solve on
 * the 2 x 2-cell grid), the same on every level:
 *  PT_VC_V11: V(1,1): x1 = omega D^{-1} r, coarse cycle on P^T (r - A x1), x2 = x1 + P x_c,
 *             x3 = x2 + omega D^{-1} (r - A x2). Symmetric in the bilinear form x^T y, as
 *             COCG requires.
 *  PT_VC_V01: V(0,1): coarse cycle on P^T r, x2 = P x_c, x3 = x2 + omega D^{-1} (r - A x2).
 *             Not symmetric; PT_INNER_GALERKIN1 only. Per cycle it skips the pre-smoothing
 *             sweep and its operator evaluation on every level.
 *  PT_VC_DEFAULT: V(0,1) with PT_INNER_GALERKIN1, V(1,1) with PT_INNER_COCG.            */
typedef enum { PT_VC_DEFAULT = 0, PT_VC_V11 = 1, PT_VC_V01 = 2 } pt_vcycle;

typedef enum { PT_WAVE_SIN = 0, PT_WAVE_COS = 1 } pt_waveform;

/* Reluctivity law of every region of a problem:
 *  PT_NU_RATIONAL: nu(s) = a + b s^2/(1 + s^2) (the synthetic iron law; rectangle problems use it
 *                  with a = nu_a, b = nu_b in nu_rect and a = nu_out, b = 0 elsewhere)
 *  PT_NU_EXPCAP:   nu(s) = a min(exp(b s^2), c) + d, the law of Sec. 4 ("Test problem"); region
 *                  mode only. Evaluated in FP64 in both precision modes.                          */
typedef enum { PT_NU_RATIONAL = 0, PT_NU_EXPCAP = 1 } pt_nu_law;

/* Material of one region (region mode; Sec. 4, table tab:coef): conductivity, law parameters
 * (b, c, d unused by PT_NU_RATIONAL: nu = a + b s^2/(1+s^2) there), the amplitude j of the
 * current density j w(2 pi t / T), and the region's coefficient nu_hat of the linear operator
 * Khat of the fixed-point iteration (eq. (iter1); Thm. thm:iter admits any Khat = S_nuhat with a
 * piecewise-constant coefficient bounding the law's range suitably): Khat is the P1 stiffness
 * with coefficient nu_hat on the region's triangles. nu_hat = 0 takes the problem's nu_max; when
 * every region has nu_hat = 0, Khat = nu_max S (a constant stencil). Every inner method and
 * cycle shape takes the per-region Khat (on coarse levels its Galerkin products). */
typedef struct {
    double sigma;          /* >= 0 */
    double a, b, c, d;     /* PT_NU_RATIONAL: a > 0, a + b > 0; PT_NU_EXPCAP: a, b >= 0, c >= 1, d > 0 */
    double j;
    double nu_hat;         /* >= 0 (0: nu_max) */
} pt_region;

typedef struct { double x0, y0, x1, y1; } pt_rect;   /* closed rectangle */

typedef struct {
    int32_t n;            /* cells per side, power of two, 4 <= n <= 4096 */
    int32_t N;            /* time steps per period, power of two, 4 <= N <= 1024 */
    double T;             /* period > 0 */
    double sigma_in;      /* conductivity inside sigma_rect (0 outside), >= 0 */
    pt_rect sigma_rect;
    double nu_a, nu_b;    /* nu(s) = theta (nu_a + nu_b s^2/(1+s^2)) inside nu_rect */
    double nu_out;        /* nu = theta nu_out outside nu_rect */
    pt_rect nu_rect;
    double J0;            /* source amplitude on coil_rect */
    pt_rect coil_rect;
    int32_t waveform;     /* pt_waveform: w = sin or cos */
    double nu_max;        /* Khat = nu_max * stiffness (region mode: per region, see nu_hat); > 0 */
    const double* d_theta; /* optional device [2 n^2] per-triangle nu scale (> 0), NULL = 1 */
    const double* d_sigma; /* optional device [2 n^2] per-triangle conductivity (>= 0),
                              NULL = sigma_in on sigma_rect */
    const double* d_load;  /* optional device time field [N][n+1][n+1]: f^n given
                              explicitly (replaces J0 w b); NULL = built-in source */
    int32_t law;           /* pt_nu_law; PT_NU_EXPCAP requires region mode */
    int32_t nregions;      /* 0: rectangle mode (sigma_in/sigma_rect, nu_a/nu_b/nu_out/nu_rect,
                              J0/coil_rect above); 1..16: region mode, where every triangle takes
                              the conductivity, law and current of its region and those fields are
                              not used (single-problem plans; d_sigma must be NULL) */
    const uint8_t* d_region;     /* region mode: device [2 n^2], the region (< nregions) of every
                                    triangle, ids as for d_theta */
    const pt_region* regions;    /* region mode: host [nregions], copied by pt_plan_create */
} pt_problem;

typedef struct {
    double tol;            /* stop when ||F - A(U)||_2 <= tol ||F||_2 (absolute if F = 0) */
    int32_t max_outer;     /* >= 1 */
    int32_t check_every;   /* read the residual back every this many steps, >= 1 */
    int32_t precision;     /* pt_precision */
    int32_t inner;         /* pt_inner */
    int32_t inner_iters;   /* COCG steps per outer step (PT_INNER_COCG), 1..64 */
    int32_t vc_sweeps;     /* damped-Jacobi sweeps per smoothing step of the cycle (vc_cycle);
                              must be 1 (the fused sweeps) */
    double vc_omega;       /* Jacobi damping, 0 < omega < 1 */
    int32_t use_initial_guess; /* 0: U^0 = 0; 1: start from the contents of d_u */
    double diverge_factor; /* PT_ERR_DIVERGED if rel > diverge_factor * min(rel) (0 = off) */
    int32_t xcd_remap;     /* 1: map workgroups to contiguous node ranges per XCD */
    int32_t timing;        /* 1: bracket every kernel launch of pt_solve with HIP events on
                              the solve stream and report per-kernel device time in pt_stats */
    int32_t grid_slot;     /* workgroups the slot-vector sweeps (V-cycle, operator) and the
                              residual sweep aim for per slot chunk; 0 = 8192. Performance
                              only (>= 8). */
    int32_t grid_team;     /* workgroups the per-node time-axis sweeps (DFT, inverse DFT)
                              aim for; 0 = 262144. Performance only (>= 8). */
    int32_t adjoint;       /* 1: reserve the workspace of pt_adjoint_solve / pt_loss_gradients
                              (two more time fields and a per-triangle table); single-problem
                              plans only */
    int32_t init_static;   /* 1: start from the static solution (Sec. 4, "Initialization"): the
                              decoupled problems K(u^n) = f^n of sigma = 0, solved by the same
                              iteration to init_tol; cannot be combined with use_initial_guess */
    double init_tol;       /* relative residual of the static start (default 1e-8) */
    int32_t stop_relative_initial; /* 1: stop when ||F - A(U^k)|| <= tol ||F - A(U^0)|| (the paper's
                              rule); 0: tol ||F|| (the same for U^0 = 0) */
    int32_t krylov_dim;    /* > 0: reserve the workspace of pt_newton_solve with flexible GMRES of
                              this restart length (1..64); single-problem plans only */
    double forcing;        /* Newton: relative tolerance of each linear solve (default 1e-2) */
    int32_t max_krylov;    /* Newton: Krylov steps per Newton step at most (default 100) */
    int32_t graph;         /* 1: capture the kernels of check_every outer steps into a HIP
                              graph on the first call (per plan and workspace address) and
                              replay it; same iterates as 0. Cannot be combined with timing. */
    double inner_rtol;     /* PT_INNER_COCG: relative residual at which a frequency stops, in
                              [0, 1); 0 = run inner_iters steps on every frequency with a nonzero
                              residual. Eager launches end the inner loop once every frequency has
                              stopped (one host read-back per step); graph replay runs inner_iters
                              steps with the stopped frequencies masked (the same iterates). */
    double breakdown_tol;  /* PT_INNER_COCG: PT_ERR_BREAKDOWN when an active frequency has
                              |p^T A p| <= breakdown_tol Re(p^H A p) (the bilinear form vanishes to
                              rounding); 0 = 64 units in the last place of the solver precision */
    int32_t vc_cycle;      /* pt_vcycle; PT_VC_V01 requires PT_INNER_GALERKIN1 */
    int32_t timing_mask;   /* with timing = 1: bit k set = time the launches of kernel class k
                              (pt_kernel_class_name(k)) only; 0 = every class. Each timed launch
                              adds two event records to the stream, so timing fewer classes
                              perturbs the timed solve less. Bits >= PT_KERNEL_CLASSES: invalid. */
    int32_t grid_restrict; /* workgroups the restriction sweeps aim for (every level); 0 = grid_slot */
    int32_t grid_up;       /* workgroups the prolongation + smoothing sweeps aim for; 0 = grid_slot */
    int32_t grid_matvec;   /* workgroups the operator sweep (p^H A p, COCG's A p) aims for; 0 =
                              grid_slot. All three: performance only (>= 8). */
} pt_options;

typedef struct {
    int32_t outer_iters;        /* fixed-point updates applied */
    double rel_residual;        /* ||F - A(U)|| / ||F|| of the returned U */
    double f_norm;              /* ||F||_2 */
    double time_ms;             /* device time of the whole call (HIP events) */
    double* residual_history;   /* caller-owned host array or NULL; rel at each check */
    int32_t history_cap;
    int32_t history_len;
    double* kernel_ms;          /* caller-owned host array [PT_KERNEL_CLASSES] or NULL: total
                                   device time per kernel class (options.timing = 1) */
    int64_t* kernel_launches;   /* caller-owned host array [PT_KERNEL_CLASSES] or NULL */
    int32_t converged_at;       /* outer step at whose check rel <= tol first held, -1 if never */
    int32_t init_iters;         /* steps of the static start (options.init_static) */
    double rel_initial;         /* ||F - A(U^0)|| / ||F|| of the iteration's starting iterate */
    int32_t krylov_iters;       /* pt_newton_solve: Krylov steps over all Newton steps */
    int32_t inner_iters_max;    /* most inner steps (COCG steps; 1 for the Galerkin step) taken by
                                   one periodic solve of the call */
    int64_t inner_iters_sum;    /* inner steps over all periodic solves of the call */
} pt_stats;

/* Kernel classes reported by the per-kernel timer; pt_kernel_class_name() names them. */
#define PT_KERNEL_CLASSES 15

typedef struct pt_plan pt_plan;

/* Fill *o with the defaults (tol 1e-8, max_outer 1000, check_every 1, FP64,
 * PT_INNER_GALERKIN1, inner_iters 1, vc_sweeps 1, vc_omega 0.8, PT_VC_DEFAULT, no initial guess,
 * diverge_factor 1e3, xcd_remap 1, timing 0, default grid targets, adjoint 0, no static start
 * (init_tol 1e-8), stop relative to ||F||, graph 0). */
void pt_options_default(pt_options* o);

/* Validate the problem and options (host only, no device work) and create a plan. */
pt_status pt_plan_create(const pt_problem* prob, const pt_options* opts, pt_plan** out);
void pt_plan_destroy(pt_plan* plan);

/* Host-only check of a plan before any launch: walks every workgroup of every sweeping kernel
 * with the kernels' own range helpers and checks that each index range, partial-sum slot and
 * LDS request it can address lies within its buffer, and that the workspace buffers are
 * aligned, inside the workspace and disjoint. PT_OK, or PT_ERR_INVALID with the first violation
 * in msg (caller-owned, cap bytes, may be NULL) and pt_last_error. No device work. */
pt_status pt_plan_check_bounds(const pt_plan* plan, char* msg, size_t cap);

/* Bytes of device workspace every entry point below needs (256-byte aligned base). */
pt_status pt_plan_workspace_bytes(const pt_plan* plan, size_t* bytes);

/* Solve Problem 1 by the fixed-point iteration (eqs. (iter1)-(iter2)).
 * d_u: device time field [N][n+1][n+1], in (initial guess if use_initial_guess) and
 * out (the periodic solution, zero boundary). stats may be NULL. Returns PT_OK on
 * convergence; on PT_ERR_NOT_CONVERGED / _DIVERGED / _NONFINITE d_u holds the last
 * iterate and stats are filled. Blocks until the stream has finished. */
pt_status pt_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream,
                   pt_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pt_solve_batch (and so pt_solve for a single-problem
 * plan) with the workspace in a static device array of 64 MiB that the library holds on every
 * GPU it runs on until the process ends, instead of a caller-owned workspace. d_u, stats,
 * statuses and blocking as pt_solve_batch; time_ms is host wall time. Calls no allocating
 * routine and creates no HIP object: plans with options.timing or options.graph are rejected
 * (PT_ERR_INVALID), and plans whose pt_plan_workspace_bytes exceeds 64 MiB get
 * PT_ERR_WORKSPACE before anything is launched. Every call on one GPU uses the same array,
 * which keeps the previous call's contents (the solve initialises everything it reads):
 * calls that overlap on one GPU, from any thread or stream, race and must be serialised by
 * the caller. */
pt_status pt_solve_noalloc(pt_plan* plan, double* d_u, void* stream, pt_stats* stats);

/* Batching: count independent instances of Problem 1 that share the grid (n), the
 * period (N, T), the conductivity (sigma_in, sigma_rect) and nu_max -- hence M, Khat and
 * the multigrid hierarchy -- but may differ in the reluctivity law and region (nu_a,
 * nu_b, nu_out, nu_rect), the source (J0, coil_rect, waveform). The instances are
 * stacked along the frequency axis, so each kernel of the outer step treats all of
 * them in one launch (the DFT diagonalisation of Remark rem:parallel applied per
 * instance). count is a power of two, 1 <= count <= 1024, count N / 2 <= 65536;
 * d_theta, d_sigma and d_load must be NULL when count > 1. probs is copied. */
pt_status pt_plan_create_batch(const pt_problem* probs, int32_t count, const pt_options* opts,
                               pt_plan** out);

/* Number of instances of a plan (1 for pt_plan_create). */
pt_status pt_plan_batch_size(const pt_plan* plan, int32_t* count);

/* pt_solve for a batch plan: d_u is [count][N][n+1][n+1] (instance-major), stats NULL
 * or a caller-owned array of count entries (each with its own history buffer). The
 * iteration runs until every instance meets tol; an instance's converged_at gives the
 * step at which it first did. The status is the first failure over the instances
 * (non-finite, breakdown, divergence of any instance; max_outer). Every other entry
 * point below requires a single-problem plan. Blocks until the stream has finished. */
pt_status pt_solve_batch(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream,
                         pt_stats* stats);

/* Work-list solve of several plans (single or batch) at once, for many problems of
 * uneven size: nstreams host threads each own streams[w] (NULL: all on the null
 * stream) and repeatedly take the next unclaimed plan, in the order given, and run
 * pt_solve_batch on it, so that the kernels of different plans overlap on the device.
 * Plan i uses d_ws[i] (ws_bytes[i]) and d_u[i]; stats[i] is NULL or its stats array;
 * status[i] receives its status. A plan may appear only once. Returns PT_OK if every
 * plan returned PT_OK, else the status of the first failing item (pt_last_error names
 * it). Blocks until all are done. 1 <= nstreams <= 64. */
pt_status pt_solve_many(int32_t count, pt_plan* const* plans, void* const* d_ws,
                        const size_t* ws_bytes, double* const* d_u, pt_stats* const* stats,
                        pt_status* status, void* const* streams, int32_t nstreams);

/* R = F - A(U) (eq. (disc1) moved to one side, u^0 = u^N) on every slice; d_r has
 * the time-field layout, boundary entries 0. rel_out / fnorm_out (host, may be NULL)
 * receive ||R||_2 / ||F||_2 and ||F||_2. Blocks until the stream has finished. */
pt_status pt_residual(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                      double* d_r, void* stream, double* rel_out, double* fnorm_out);

/* The first two steps of one outer iteration (eq. (iter1) with the DFT of remark
 * rem:parallel): the residual R = F - A(U) of pt_residual and its packed real DFT along
 * time, written to d_rhat (frequency-field layout, plan precision: what pt_time_rfft(R)
 * gives, to rounding in the transform). For 4 <= N/2 <= 256 this is the fused sweep the
 * solver runs in every step (the time-domain R never reaches memory); other N take the
 * two-kernel path. rel_out / fnorm_out as in pt_residual (the fused sweep adds the norm
 * terms in another order, so rel_out may differ from pt_residual's in the last bits). Blocks
 * until done. */
pt_status pt_residual_spectrum(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                               void* d_rhat, void* stream, double* rel_out, double* fnorm_out);

/* d_ku[j] = K(d_u[j]) for j < nslices (time-field layout, 1 <= nslices <= N); the
 * nonlinear P1 operator of Sec. 4 with the plan's material law. */
pt_status pt_apply_K(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                     double* d_ku, int32_t nslices, void* stream);

/* Device check of the two FP64 reciprocals the kernels use in place of a divide (no plan): for
 * 0 <= i < n, d_y[2i] = the residual sweep's 1/x (hardware estimate refined by one Newton step;
 * the law's 1 / (1 + s^2), so x >= 1) and d_y[2i+1] = the V-cycle's 1/x (two Newton steps; the
 * Jacobi inverse, x > 0). d_x: n doubles, d_y: 2n doubles, both device memory owned by the
 * caller. PT_ERR_INVALID for n < 0 or NULL buffers with n > 0; n = 0 does nothing. Enqueued on
 * stream, does not block. */
pt_status pt_device_reciprocals(const double* d_x, double* d_y, int64_t n, void* stream);

/* Packed real DFT along time: time field (double) -> frequency field (plan precision). */
pt_status pt_time_rfft(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_x,
                       void* d_xhat, void* stream);

/* Inverse of pt_time_rfft including the 1/N factor: frequency field -> time field. */
pt_status pt_time_irfft(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_xhat,
                        double* d_x, void* stream);

/* y_s = (Khat + z_s M) x_s for every slot (slot 0: the k = 0 and k = N/2 systems act
 * on the real and imaginary parts). Frequency-field layout, plan precision. */
pt_status pt_shifted_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_x,
                           void* d_y, void* stream);

/* x_s = B_s r_s: one cycle of the multigrid preconditioner (the plan's vc_cycle) for every slot. */
pt_status pt_precond_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_r,
                           void* d_x, void* stream);

/* Approximate X = P^{-1} R for time fields R (input) and X (output) with the plan's
 * inner method: DFT in time, the batched preconditioned solve, inverse DFT.
 * inner_iters overrides the plan's COCG step count when > 0. */
pt_status pt_periodic_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_r,
                            double* d_x, int32_t inner_iters, void* stream);

/* Adjoint of the cycle-averaged eddy-current loss
 *     l(U) = tau sum_n (d u^n)^T M (d u^n),   d u^n = (u^n - u^{n-1}) / tau,  u^0 = u^N,
 * (the time integral over one period of int sigma |du/dt|^2 with the implicit-Euler
 * difference quotient and the consistent mass; Sec. 4 model, Problem 1). For the state U
 * with A(U) = F the adjoint state lambda solves J^T lambda = dl/dU, J = dA/dU (eqs.
 * (disc1)-(disc2) linearised):
 *     (M/tau)(lambda^n - lambda^{n+1}) + K'(u^n) lambda^n = (dl/dU)^n,  lambda^{N+1} = lambda^1,
 * a periodic system running backward in time. It is solved by the same fixed-point
 * correction as the forward problem (eqs. (iter1)-(iter2) with Khat = nu_max S), whose
 * periodic linear part is now I (x) (M/tau + Khat) - C_N^T (x) (M/tau): in the time-DFT
 * basis the systems (Khat + conj(z_k) M), solved as the conjugates of the forward ones.
 * The plan must have been created with options.adjoint = 1 (single problem).
 *
 * pt_adjoint_solve: d_u is the state (time field [N][n+1][n+1], e.g. from pt_solve);
 * d_lambda receives lambda in the same layout (and holds the initial guess when
 * use_initial_guess = 1). Stops when ||dl/dU - J^T lambda|| <= tol ||dl/dU|| (absolute if
 * dl/dU = 0); statuses and stats as pt_solve. Blocks until the stream has finished. */
pt_status pt_adjoint_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                           double* d_lambda, void* stream, pt_stats* stats);

/* Loss and gradients at the state d_u with the adjoint state d_lambda (may be NULL: then
 * only the loss and the direct part tau sum du^T M_T du of dl/dsigma_T are formed):
 *     dl/dtheta_T = - sum_n |T| nuhat_T(|grad u^n|^2) grad u^n . grad lambda^n
 *     dl/dsigma_T = tau sum_n du^T M_T du - sum_n (lambda^n)^T M_T du
 * with theta_T the nu scale (nu = theta nuhat) and M_T the unit-conductivity element mass
 * of triangle T. d_gtheta / d_gsigma: device arrays (may be NULL) of 2 n^2 entries (per
 * triangle, id 2 (j n + i) + {0, 1}) or, with per_cell = 1, of n^2 entries (sum over the
 * two triangles of cell (i, j)). loss_out (host, may be NULL) receives l. Blocks. */
pt_status pt_loss_gradients(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                            const double* d_lambda, double* d_gtheta, double* d_gsigma,
                            int32_t per_cell, double* loss_out, void* stream);

/* Newton's method on A(U) = F (the outer loop of method (M2), Sec. 4): each step solves
 * J(U^k) D = F - A(U^k), J the linearised operator of eqs. (disc1)-(disc2), by flexible
 * GMRES(krylov_dim) right-preconditioned with the periodic solve of the fixed-point
 * iteration (I (x) (M/tau + Khat) - C_N (x) (M/tau), applied by the time DFT and the
 * inner method), to relative accuracy options.forcing, then backtracks U^k + lambda D
 * (lambda = 1, 1/2, ...) until ||F - A|| <= (1 - 1e-4 lambda) ||F - A(U^k)|| (Armijo).
 * The plan needs options.krylov_dim > 0. Stops as pt_solve (options.tol, max_outer Newton
 * steps); stats.outer_iters counts Newton steps, stats.krylov_iters the Krylov steps.
 * d_u, statuses and blocking as pt_solve; a failed line search gives PT_ERR_NOT_CONVERGED. */
pt_status pt_newton_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream,
                          pt_stats* stats);

/* d_out = J(U) d_v (transpose = 0) or J(U)^T d_v (transpose = 1) at the state d_u, all time
 * fields [N][n+1][n+1] (boundary entries of d_out are 0). The plan needs options.adjoint or
 * options.krylov_dim. Blocks until the stream has finished. */
pt_status pt_jacobian_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u,
                            const double* d_v, double* d_out, int32_t transpose, void* stream);

/* Name of kernel class id (0 <= id < PT_KERNEL_CLASSES), or NULL. */
const char* pt_kernel_class_name(int32_t id);

const char* pt_status_string(pt_status s);
const char* pt_last_error(void);
int32_t pt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PTSOLVE_H */
