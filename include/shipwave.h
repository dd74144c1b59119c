/*
 * shipwave.h -- C ABI of the MI355X (gfx950) library for steady nonlinear
 * free-surface flow past a submerged source, solved by a preconditioned
 * Jacobian-free Newton-Krylov method.
 *
 * Paper: Pethiyagoda, McCue, Moroney & Back, "Jacobian-free Newton-Krylov
 * methods with GPU acceleration for computing nonlinear ship wave patterns".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh (numerical discretisation section): N points in x (x_1 .. x_N, spacing
 * dx = (x_N - x_1)/(N-1)), M points in y (y_1 = 0 .. y_M, dy = y_M/(M-1)); the
 * half domain y >= 0 with image terms.  Collocation points are the half-mesh
 * points (x_{k+1/2}, y_l), k = 1..N-1, l = 1..M.
 *
 * Unknowns (reduced form of eq. unknowns): the first and third radiation
 * equations (E3, E5 of Appendix A) are solved for phi_{1,l} and zeta_{1,l},
 * which leaves 2NM unknowns, x fastest within each row l:
 *     u = [ (phi_x)_{1..N,1}, ..., (phi_x)_{1..N,M}, (zeta_x)_{1..N,1}, ..., (zeta_x)_{1..N,M} ].
 * Residual, same length and row layout (Appendix A order with E3/E5 removed):
 *     E = [ E4_l, E1_{1..N-1,l} ]_{l=1..M}, [ E6_l, E2_{1..N-1,l} ]_{l=1..M}.
 * E1 is the Bernoulli condition (eq. freeSurfCond), E2 the boundary-integral
 * equation (eq. IntegroEqn) with the singular part of the second integral
 * subtracted (eq. I2DashDash, S2) and added back in closed form (eq. IS2),
 * E4/E6 the upstream radiation rows (eq. numUpRadiation, forward difference).
 *
 * Memory: every vector argument is device memory owned by the caller (for
 * example torch tensors), FP64, contiguous.  The library never keeps a caller
 * pointer after the call's stream work has completed.  Library-owned objects
 * (sw_precond, sw_server) are released only by their destroy call.
 * shipwave_precond_destroy keeps the preconditioner's device block (at most one
 * block of up to 2 GiB per device) for the next set-up of a similar size; it is
 * freed when a later device allocation fails, or at process exit.
 *
 * Streams: every call enqueues its work on `stream` and returns without
 * waiting, except shipwave_solve and the server calls, which wait on their own
 * stream for scalar control, and shipwave_precond_build_banded, which waits for
 * its set-up to check the diagonal blocks.  Preconditioner set-up also runs
 * work on library-owned helper streams (a per-device pool, default priority),
 * ordered with `stream` by events; it is complete when the build call returns.  Internal scratch memory is kept per (device,
 * stream); it grows on demand (hipMalloc, after a stream synchronisation).
 * Calls on one stream are ordered by the stream; calls on different streams
 * use different scratch and may run concurrently.
 *
 * Errors: return 0 (SW_OK) or a negative SW_E* code; no exception crosses the
 * ABI and nothing exits the process.  shipwave_last_error() returns a message
 * for the calling thread's most recent failure.
 */
#ifndef SHIPWAVE_H
#define SHIPWAVE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHIPWAVE_ABI_VERSION 3

enum {
    SW_OK = 0,
    SW_EINVAL = -1,      /* invalid argument (sizes, domain, parameters, null pointer) */
    SW_ENOMEM = -2,      /* device allocation failed, or a request cannot be admitted */
    SW_EHIP = -3,        /* HIP runtime error */
    SW_ENOCONV = -4,     /* Newton did not converge (iteration limit or line-search failure) */
    SW_ENONFINITE = -5,  /* a residual norm was NaN or Inf */
    SW_EBUSY = -6        /* server: result not ready yet */
};

enum { SW_WEIGHTS_TRAPEZOID = 0, SW_WEIGHTS_SIMPSON = 1 };
/* Spline end conditions for zeta_y, phi_y (the paper does not state them):
 * 0 = zero slope at y = 0 (zeta, phi even in y) and not-a-knot at y_M;
 * 1 = not-a-knot at both ends. */
enum { SW_SPLINE_CLAMPED0 = 0, SW_SPLINE_NOTAKNOT = 1 };
/* Arithmetic of the all-pairs sum: 0 = FP64; 1 = FP32 with Kahan-compensated
 * row sums (grid fields, the closed-form I and the assembly stay FP64). */
enum { SW_PREC_FP64 = 0, SW_PREC_FP32 = 1 };

typedef struct { int32_t N, M; } sw_mesh;
/* Truncated domain x_1 <= x <= x_N, 0 <= y <= y_M (section on discretisation). */
typedef struct { double x1, xN, yM; } sw_domain;
/* F: depth-based Froude number (eq. Froude); eps: source strength (eq. epsilon);
 * nu: upstream decay constant of the radiation condition (0.05 in the paper). */
typedef struct {
    double F, eps, nu;
    int32_t weights;     /* SW_WEIGHTS_*; Simpson needs odd N and M */
    int32_t spline_bc;   /* SW_SPLINE_* */
    int32_t precision;   /* SW_PREC_* */
    int32_t reserved;
} sw_params;
typedef struct { sw_mesh mesh; sw_domain domain; sw_params params; } sw_problem;

/* Validation shared by all calls: N, M >= 4; N <= 65536 and N M <= 2^28; F > 0;
 * eps >= 0; nu > 0; x_1 < 0 < x_N is not required, but x_1 < x_N, y_M > 0; Simpson
 * needs odd N and M.  Calls that build or use a preconditioner (precond_build_banded,
 * solve, server requests) also need N <= 1024.  Violations return SW_EINVAL. */

int32_t shipwave_abi_version(void);
const char* shipwave_last_error(void);

/* E(u): the nonlinear residual of section 3 (steps: unpack + eliminate E3/E5,
 * trapezoid integration in x (eq. zetaapprox), cubic spline in y, two-point
 * interpolation to the half mesh, Bernoulli E1, closed-form I, the all-pairs
 * boundary-integral sum, E2 assembly, radiation rows E4/E6).
 * u, E: device, 2NM doubles each; must not overlap.  prob->params.precision
 * selects the arithmetic of the all-pairs sum. */
int32_t shipwave_residual(const sw_problem* prob, const double* u, double* E, hipStream_t stream);

/* E(u) for nb independent problems (each with its own mesh, F, eps, precision).
 * The all-pairs sums of all problems of one precision run in one shared launch
 * over a combined work list (up to 24 problems per launch); the O(NM) prelude
 * and assembly kernels run per problem.  probs: host array of nb problems;
 * u, E: host arrays of nb device pointers.  Each result is bitwise identical
 * to shipwave_residual on that problem alone. */
int32_t shipwave_residual_batched(int32_t nb, const sw_problem* probs, const double* const* u,
                                  double* const* E, hipStream_t stream);

/* E(u) as shipwave_residual, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * intermediate arrays live in a fixed device array of 64 MiB inside the library, one per
 * GPU, held from the first call on that GPU until the process ends; the call allocates
 * nothing and creates no runtime object.  The spline slopes come from a tridiagonal sweep
 * per column instead of the cached dense operator, so results equal shipwave_residual's
 * to rounding (not bitwise).  Meshes whose arrays exceed 64 MiB return SW_ENOMEM (721 x
 * 241 needs 43 MiB in FP64, 48 MiB in FP32).  Every call on one GPU uses the same array:
 * calls that overlap on one GPU (other streams, other threads) race and must be ordered
 * by the caller; calls on one stream are ordered by it.  u, E: as shipwave_residual. */
int32_t shipwave_residual_noalloc(const sw_problem* prob, const double* u, double* E,
                                  hipStream_t stream);

/* Jacobian-vector product by a first-order difference quotient (eq. JvApprox):
 * Jz = (E(u + h z) - Eu) / h.  Eu must be E(u) computed with the same
 * precision setting.  h <= 0 selects h = sqrt(macheps) (sqrt(n) + ||u||_2) / ||z||_2,
 * n = 2NM, which moves each entry of u by about sqrt(macheps) (1 + rms(u))
 * (macheps of the pair-sum precision).  u, Eu, z, Jz: device, 2NM doubles;
 * Jz may not alias u or z.  A zero z gives Jz = 0. */
int32_t shipwave_jvp(const sw_problem* prob, const double* u, const double* Eu, const double* z,
                     double h, double* Jz, hipStream_t stream);

/* Preconditioner from the linear Jacobian (preconditioning section; Appendix B
 * entries PreA-PreD; Appendix C storage): P = [[A, B], [C, D_q]] with A, B, C
 * block diagonal (identical N x N blocks) and D_q the linear D with the blocks
 * |l - m| <= q_blocks kept (block bandwidth b = 2 q_blocks + 1; q_blocks >=
 * M - 1 keeps all of D).  Set-up forms the Schur complement
 * S = D_q - C A^{-1} B and factorises it by block LU (FP64; partial pivoting
 * inside each N x N diagonal block), eliminating the block rows from both ends
 * of the band towards q_blocks middle rows, which go last.  P depends on the mesh, domain, F, nu and
 * weights, not on eps or u.  *out receives a library-owned handle. */
typedef struct sw_precond sw_precond;
int32_t shipwave_precond_build_banded(const sw_problem* prob, int32_t q_blocks, sw_precond** out,
                                      hipStream_t stream);
/* x = P^{-1} b by the three-step block solve of Appendix C.  b, x: device,
 * 2NM doubles; may alias.  The handle owns the apply's temporaries, so applies
 * of one handle must not run concurrently on different streams. */
int32_t shipwave_precond_apply(const sw_precond* P, const double* b, double* x, hipStream_t stream);
/* x_i = P_i^{-1} b_i for n requests, each the three-step block solve of Appendix C as
 * in shipwave_precond_apply, with the steps of several requests sharing launches:
 * requests whose handles use super-row substitution (block widths N up to a few
 * hundred) run in rounds of distinct handles, one launch per step for the whole round
 * (the first step, step k of every request's substitution, the last step); any other
 * request, and a round of one, runs as shipwave_precond_apply.  Requests that share a
 * handle go in different rounds, since the handle owns the temporaries.  P: host array
 * of n handles; b, x: host arrays of n device pointers (2NM doubles each; b_i may
 * alias x_i; the vectors of different requests must not overlap).  Each x_i is bitwise
 * the result of shipwave_precond_apply on that request alone.  Null pointers or n < 0
 * return SW_EINVAL. */
int32_t shipwave_precond_apply_batched(int32_t n, const sw_precond* const* P,
                                       const double* const* b, double* const* x,
                                       hipStream_t stream);
void shipwave_precond_destroy(sw_precond* P);

typedef struct {
    double tol;            /* stop when ||E||_inf <= tol (default 1e-10) */
    int32_t max_newton;    /* default 50 */
    int32_t gmres_restart; /* Krylov dimension m before restart (default 30) */
    int32_t max_gmres;     /* GMRES iterations per Newton step (default 200) */
    int32_t q_blocks;      /* preconditioner block half-bandwidth (default 5; <0 -> 1) */
    int32_t precision;     /* SW_PREC_FP64, or SW_PREC_FP32: FP32-Kahan inner JVPs, FP64 outer */
    int32_t weights;       /* SW_WEIGHTS_* */
    int32_t spline_bc;     /* SW_SPLINE_* */
    int32_t init;          /* initial guess (Jacobian-free Newton-Krylov overview): 0 the flat
                              surface; 1 the caller's u_inout (eps continuation); 2 the linear
                              solution u_flat - eps P^{-1} s, s the source term of E2 at the
                              flat surface, P this solve's preconditioner: the root of the
                              discretised linear problem when P is the full linear Jacobian
                              (q_blocks >= M - 1, built for this F), its banded approximation
                              otherwise.  With init = 2 and no prebuilt preconditioner, P is
                              built before the first evaluation instead of beside it. */
    double nu;             /* 0 -> 0.05 */
    double eta_max;        /* Eisenstat-Walker forcing cap (default 0.9; <=0 -> default) */
    const sw_precond* precond; /* optional prebuilt preconditioner for this mesh and domain
                                  (any F: it only affects convergence speed); NULL -> build */
} sw_solve_opts;

typedef struct {
    int32_t status;        /* SW_OK, SW_ENOCONV, SW_ENONFINITE, ... */
    int32_t newton_iters;
    int32_t gmres_iters;
    int32_t residual_evals;/* all E evaluations (Newton, JVP and line-search points) */
    double final_norm;     /* ||E||_inf in FP64 at the returned u */
    double time_total_s;
    double time_precond_s; /* preconditioner set-up time (0 if supplied) */
    double fp32_error;     /* max|E32(u) - E64(u)| / max(1, ||E64(u)||_inf) at the returned u,
                              E32 the FP32-Kahan all-pairs residual and E64 the FP64 one: the
                              error the FP32 arithmetic carries at the result.  Costs one FP32
                              evaluation after the solve (not in residual_evals); computed in
                              both precision modes; -1 if the solve ended on a non-finite
                              residual. */
    int32_t linesearch_backtracks; /* halvings of the Newton step length lambda */
    int32_t reserved;
} sw_solve_info;

/* Fill opts with the defaults above. */
void shipwave_solve_opts_default(sw_solve_opts* opts);

/* Solve E(u) = 0 for (F, eps) on the given mesh and domain by damped Newton
 * (eq. newtonstep0) with a line search, the Newton step from right-
 * preconditioned GMRES (Jacobian-free, eq. JvApprox) with Eisenstat-Walker
 * forcing.  u_inout: device, 2NM doubles; initial guess if opts->init == 1,
 * overwritten with the result (the best iterate on failure).  zeta_out:
 * device N*M doubles (row-major [l][k]) or NULL: the surface heights.
 * info_out: host, may be NULL.  Synchronises `stream`.  opts may be NULL
 * (defaults). */
int32_t shipwave_solve(double F, double eps, const sw_mesh* mesh, const sw_domain* domain,
                       const sw_solve_opts* opts, double* u_inout, double* zeta_out,
                       sw_solve_info* info_out, hipStream_t stream);

/* Surface heights zeta_{k,l} ([l][k], N*M doubles, device) of a state u. */
int32_t shipwave_zeta(const sw_problem* prob, const double* u, double* zeta, hipStream_t stream);

/* ---- diagnostics ----------------------------------------------------------
 * Times every all-pairs kernel launch (the dominant kernel of E(u)) with a
 * pair of HIP events recorded on the launch stream around it.
 * shipwave_profile_enable(1) clears the record and starts recording,
 * enable(0) stops.  shipwave_profile_read waits for the recorded events and
 * returns the number of launches, their summed duration in milliseconds and
 * the summed number of (collocation, grid) pairs they evaluated. */
int32_t shipwave_profile_enable(int32_t on);
int32_t shipwave_profile_read(int64_t* launches, double* total_ms, double* pairs);

/* Host-forced non-finite residuals, for tests of the failure paths (line-search
 * backtracking, SW_ENONFINITE, the server's FP64 fallback).  Every solve started after
 * this call (shipwave_solve and server solves, any thread) writes a NaN into the first
 * entry of the output of its nth evaluation (1-based, counted per solve and kind) of each
 * kind in `kinds`, by a one-thread kernel after the residual kernels:
 *   1  E(u) at the initial state          (-> SW_ENONFINITE)
 *   2  E at a line-search trial point     (-> lambda halves, the step is retried)
 *   4  the shifted point of an FP64 JVP   (-> SW_ENONFINITE)
 *   8  the shifted point of an FP32 JVP   (-> SW_ENONFINITE in mixed precision; a server
 *                                             with fallback_fp64 then re-solves in FP64)
 * kinds = 0 or nth = 0 switches it off.  Every kernel runs to completion as usual.
 * SW_EINVAL for kinds outside [0, 15] or nth < 0. */
int32_t shipwave_debug_inject_nonfinite(int32_t kinds, int32_t nth);

/* ---- serving: continuous batching of many solves on one GPU ------------
 * Preconditioners are built for F rounded to 0.025 and cached per (mesh, domain,
 * rounded F, q) while memory allows; the rounding changes only the GMRES count. */
typedef struct sw_server sw_server;
typedef struct {
    double hbm_budget_bytes;  /* device memory the server may hold for admitted solves */
    int32_t max_slots;        /* solves advanced together */
    int32_t fallback_fp64;    /* 1: a mixed-precision solve that fails is retried in FP64 */
    double tol;               /* Newton tolerance (default 1e-10) */
    int32_t q_blocks;         /* preconditioner half-bandwidth; < 0: by mesh, 5 for N <= 200,
                                 8 beyond */
    int32_t precision;        /* SW_PREC_* of the inner JVPs */
} sw_server_opts;
typedef struct {
    sw_mesh mesh;
    sw_domain domain;
    double F, eps;
} sw_request;
typedef struct {
    int32_t status;
    int32_t newton_iters, gmres_iters, residual_evals;
    int32_t used_fallback;
    double final_norm;
    double t_submit_s, t_admit_s, t_done_s; /* seconds on the server clock */
    double fp32_error;    /* as sw_solve_info.fp32_error, at the returned u */
} sw_result;

int32_t shipwave_server_create(const sw_server_opts* opts, sw_server** out);
/* Device bytes a server with these options charges against hbm_budget_bytes when it
 * admits this request with no cached preconditioner: the solve state plus the
 * preconditioner (band factors and substitution operators).  Host-only; SW_EINVAL for
 * an invalid request. */
int32_t shipwave_server_request_bytes(const sw_server_opts* opts, const sw_request* req,
                                      uint64_t* bytes);
/* Queue one request; returns a ticket.  The server copies the request. */
int32_t shipwave_server_submit(sw_server* s, const sw_request* req, uint64_t* ticket);
/* SW_OK with *res filled (and zeta copied to zeta_host if non-NULL, N*M
 * doubles) once done, SW_EBUSY while pending, SW_EINVAL for an unknown ticket. */
int32_t shipwave_server_poll(sw_server* s, uint64_t ticket, sw_result* res, double* zeta_host);
/* Block until every submitted request is done. */
int32_t shipwave_server_drain(sw_server* s);
void shipwave_server_destroy(sw_server* s);

#ifdef __cplusplus
}
#endif
#endif /* SHIPWAVE_H */
