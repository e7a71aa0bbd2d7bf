/*
 * ipmsk.h - C ABI of the sketch-preconditioned interior point hot path for MI355X (gfx950).
 *
 * The library computes, on one GPU, the pieces of one iteration of the infeasible long-step
 * interior point method of Chowdhury, Dexter, London, Avron and Drineas ("Faster Randomized
 * Interior Point Methods for Tall/Wide Linear Programs"):
 *
 *   LP      min c^T x  s.t.  A x = b, x >= 0;   dual  max b^T y  s.t.  A^T y + s = c, s >= 0
 *           (Section 1, eqs. primal and dual), A is m x n with m << n and rank m.
 *   Normal  A D^2 A^T dy = p,  D = X^{1/2} S^{-1/2}  (Section 1, eq. normal).
 *   Solve   Algorithm 1 (Section 3): sketch B = A D W, preconditioner Q = B B^T
 *           (eqn. pdprecond), conjugate gradients on the preconditioned system
 *           (eq. precond_alt). Q is factored by Cholesky (Q = L L^T) instead of the SVD; the
 *           CG iterates and the residual norm ||Q^{-1/2} r|| = ||L^{-1} r|| are the same.
 *   Step    Algorithm 3 (Section 5) with the perturbation v of eq. compv.
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] are device pointers on the context's device, owned by the
 *     caller; the library never frees them and never keeps them after the call returns.
 *   - All work is ordered on the context's stream. Entry points that return scalar results
 *     (info structs, bad_pivot) synchronize that stream before returning; the others may return
 *     before the device work finishes.
 *   - Return value: IPM_OK (0), a warning (> 0) or an error (< 0). Arguments are validated
 *     before any device work is queued; on an error a message is available from
 *     ipm_last_error(). No C++ exception crosses this interface.
 *   - Dense matrices are row-major: element (i, j) of an m x n matrix with row stride ld is at
 *     offset i*ld + j. For the dense A of ipm_matrix, ld must be a multiple of 16/elem_size and
 *     the base pointer 16-byte aligned (the HBM passes use 16-byte vector loads); columns
 *     n..ld-1 are never read.
 *   - One context per host thread. Calls on one context must not overlap.
 */
#ifndef IPMSK_H
#define IPMSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define IPM_OK              0
#define IPM_CONVERGED       1   /* ipm_step: the stop test already holds; no step was taken   */
#define IPM_PCG_MAXIT       2   /* warning: CG reached maxit_pcg before the tolerance         */
#define IPM_PCG_STAGNATED   3   /* warning: CG residual fell by < stag_ratio over stag_window */
#define IPM_ERR_ARG        -1   /* invalid argument (null pointer, bad size, s not dividing w) */
#define IPM_ERR_HIP        -2   /* HIP runtime failure                                       */
#define IPM_ERR_NOT_SPD    -3   /* Cholesky of Q met a non-positive pivot                     */
#define IPM_ERR_BREAKDOWN  -4   /* CG met d^T A D^2 A^T d <= 0                                */
#define IPM_ERR_STALL      -5   /* step length below min_step                                 */
#define IPM_ERR_NOMEM      -6   /* workspace allocation failed                                */

/* ---- element types and layouts ------------------------------------------------------------ */
#define IPM_F64   0
#define IPM_F32   1
#define IPM_BF16  2
#define IPM_DENSE_ROWMAJOR 0
#define IPM_CSR            1

typedef struct ipm_ctx ipm_ctx;

/* Constraint matrix A (m x n).
 * IPM_DENSE_ROWMAJOR: val [device] m*ld elements of `dtype`; the sparse fields are ignored.
 * IPM_CSR (A by its nonzeros; the method's cost is stated in nnz(A), Section 3 and the running
 *   time discussion of Section 4): the nnz nonzeros twice, all [device]:
 *   row order    val (nnz of `dtype`), row_ptr (m+1, int64), col_idx (nnz, int32, < n);
 *   column order csc_val (nnz of `dtype`), col_ptr (n+1, int64), row_idx (nnz, int32, < m);
 *   both orders hold the same values. ld is ignored and n must be below 2^31. The index arrays
 *   are trusted: row_ptr / col_ptr must be non-decreasing from 0 to nnz and every index in
 *   range (an index out of range is an out-of-bounds device access, not a returned error).
 *   Duplicate entries are summed; the order within a row or column is free.
 * Sizes: 1 <= m <= n and m <= 10236 for every layout (the CG kernels keep two FP64 m-vectors
 *   in one block's 160 KB of LDS). A dense A keeps a column strip of all m rows on chip in its
 *   passes, so m <= 2048 with IPM_F64 or IPM_F32 values and m <= 6400 with IPM_BF16 values, and
 *   a thread addresses the rows of its row group (up to 64 rows) with a 32-bit element offset, so
 *   63*ld + 128/elem_size must stay below 2^32 (ld below about 6.8e7 elements); for
 *   1025 <= m <= 2048 the CG matvec reads a 64-row group through one buffer descriptor, so
 *   64*ld*elem_size must stay below 2^32 (ld below 8.3e6 FP64, 1.6e7 FP32, 3.3e7 BF16 elements). A CSR A needs n < 2^31. Larger sizes are IPM_ERR_ARG, reported before any device
 *   work. */
typedef struct {
    int64_t m, n, ld;
    int32_t layout;          /* IPM_DENSE_ROWMAJOR | IPM_CSR */
    int32_t dtype;           /* IPM_F64 | IPM_F32 | IPM_BF16 */
    const void* val;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    const void* csc_val;
    const int64_t* col_ptr;
    const int32_t* row_idx;
} ipm_matrix;

/* LP data: b [device] m doubles, c [device] n doubles. */
typedef struct {
    ipm_matrix A;
    const double* b;
    const double* c;
} ipm_problem;

/* Iterate (x, y, s) [device, n / m / n doubles, updated in place], iteration counter k, and
 * the neighbourhood's reference values mu0 = x0^T s0 / n and ||r0|| = ||(r_p0, r_d0)||
 * (Section 5). If r0norm < 0 the first ipm_step sets mu0 and r0norm from the current point. */
typedef struct {
    double* x;
    double* y;
    double* s;
    int64_t k;
    double mu0;
    double r0norm;
} ipm_state;

/* Method parameters. ipm_params_default() fills the values used throughout:
 * sigma 0.5 (Section 7), gamma 0.9, theta 0.9999, tol_pcg 1e-10, gap_tol 1e-8,
 * min_step 1e-14, maxit_pcg 500, stag_window 10, stag_ratio 0.99, max_redraws 3, vcorr 1,
 * precision IPM_PLAIN, warm_start IPM_WARM_NONE, inner_tol 1e-4, max_refine 12, max_shifts 3. */
typedef struct {
    double sigma;        /* centering parameter, in (0, 4/5) (Algorithm 3 input)            */
    double gamma;        /* neighbourhood parameter, in (0, 1)                              */
    double theta;        /* backoff applied to alpha_max when alpha_max < 1                 */
    double tol_pcg;      /* CG stops when ||L^-1 r|| <= tol_pcg ||L^-1 p|| (eq. pdcond2)   */
    double gap_tol;      /* stop test: relative gap and both relative residuals <= gap_tol  */
    double min_step;     /* alpha_bar below this is IPM_ERR_STALL                            */
    double stag_ratio;   /* CG stagnation: residual > stag_ratio * residual stag_window ago */
    int32_t w;           /* sketch width (columns of W); s must divide w; w >= m           */
    int32_t s;           /* nonzeros per row of W, 1..8                                     */
    int32_t maxit_pcg;
    int32_t stag_window;
    int32_t max_redraws; /* extra draws of W (doubled w, s >= 2) after a failed solve      */
    int32_t vcorr;       /* 1: perturbation v of eq. compv; 0: v = 0                         */
    int32_t precision;   /* A is read in its storage type (F64, F32 or BF16) by every form.
                            IPM_PLAIN: FP64 accumulation everywhere, B stored FP64.
                            IPM_MIXED: the sketch accumulates in FP64 (LDS buckets) and B is
                            stored rounded to FP32 (the Gram widens it to an FP64 Q); the CG
                            matvecs accumulate in FP64, which costs nothing on these
                            bandwidth-bound passes and keeps the plain form's CG iteration
                            counts.
                            IPM_MIXED_F32ACC: as IPM_MIXED, and the CG runs as iterative
                            refinement: inner CG with FP32-accumulated matvecs to inner_tol,
                            outer residual p - A D^2 A^T dy recomputed with FP64 accumulation,
                            stop on ||L^-1 r|| <= tol_pcg ||L^-1 p|| for that true residual.
                            The Cholesky, the residuals and the step stay FP64 in all forms.  */
    int32_t warm_start;  /* IPM_WARM_NONE | IPM_WARM_PREV (previous iteration's dy) |
                            IPM_WARM_GIVEN (ipm_step_warm's candidates). The initial iterate
                            is the combination of the candidate vectors closest to the
                            solution in the M-norm (M = A D^2 A^T; for one candidate v it is
                            (v^T p / v^T M v) v), kept only if its preconditioned residual
                            beats that of dy = 0                                              */
    double inner_tol;    /* relative tolerance of each inner CG solve (IPM_MIXED_F32ACC)     */
    int32_t max_refine;  /* refinement rounds (IPM_MIXED_F32ACC)                             */
    int32_t max_shifts;  /* when Q = B B^T fails to factor: retries with Q + delta_j I,
                            delta_j = 2^-53 trace(Q) 100^j, j < max_shifts, before the next
                            draw of W (the FP64 Gram squares the condition of B)              */
    int32_t feasible;    /* 0: Algorithm 3 (infeasible IPM). 1: Algorithm 2 (feasible IPM,
                            Section 4), for a strictly feasible (x, y, s): p = A x -
                            sigma mu A S^-1 1 (eqn. pdef), ds = -A^T dy (eq. dels), dx as in
                            eq. delxhat, and N(gamma) without its residual term (eq. neigh).
                            The residuals are still measured for the stop test.            */
    int32_t solver;      /* IPM_SOLVER_CG | IPM_SOLVER_CHEBYSHEV (plain and IPM_MIXED forms;
                            the refinement form's inner solves stay CG)                      */
    int32_t sketch;      /* IPM_SKETCH_SPARSE: the hashed sparse embedding (s nonzeros per
                            row, Section 2). IPM_SKETCH_GAUSSIAN: W with N(0, 1/w) entries
                            (the experiments' choice, Section 7), generated on the fly for Q
                            and v; s is ignored; dense A only.                               */
    int32_t reserved;    /* must be 0                                                       */
    uint64_t seed;       /* sketch seed                                                     */
} ipm_params;

#define IPM_PLAIN 0
#define IPM_MIXED 1
#define IPM_MIXED_F32ACC 2
#define IPM_SOLVER_CG      0   /* preconditioned conjugate gradients (Algorithm 1, step 3)   */
#define IPM_SOLVER_CHEBYSHEV 1 /* Chebyshev iteration (Section 3.2) after a 10-step CG probe:
                                  the probe's Lanczos Ritz values theta_min, theta_max give the
                                  interval [0.5 theta_min, 1.1 theta_max]; same stop test     */
#define IPM_SKETCH_SPARSE   0  /* hashed sparse embedding, s signed nonzeros per row       */
#define IPM_SKETCH_GAUSSIAN 1  /* i.i.d. N(0, 1/w) entries                                  */
#define IPM_WARM_NONE 0
#define IPM_WARM_PREV 1
#define IPM_WARM_GIVEN 2

typedef struct {
    int32_t iters;       /* CG iterations performed                                         */
    int32_t status;      /* IPM_OK, IPM_PCG_MAXIT, IPM_PCG_STAGNATED or IPM_ERR_BREAKDOWN    */
    int32_t warm_used;   /* 1 if the initial dy was kept (its residual beat dy = 0)          */
    int32_t rounds;      /* refinement rounds (mixed form); 1 for the plain form             */
    double relres;       /* ||L^-1 r|| / ||L^-1 p|| at exit: the recursive residual of the
                            plain form, the FP64-recomputed true residual of the mixed form   */
    double rho_star;     /* ||L^-1 p||^2                                                     */
} ipm_pcg_info;

typedef struct {
    int32_t status;      /* IPM_OK, IPM_CONVERGED, warnings, or an error                    */
    int32_t pcg_status;
    int32_t pcg_iters;   /* CG iterations of the accepted draw                              */
    int32_t attempts;    /* draws of W used (1 + redraws)                                   */
    int64_t k;           /* iteration index of the point this info describes                */
    int32_t w_used, s_used;
    double mu, gap, relgap, rp_rel, rd_rel, obj;   /* at the point before the step          */
    double alpha_max, alpha;                       /* Algorithm 3, steps 6-7                 */
    double pcg_relres, vnorm;
    int32_t refine_rounds;     /* mixed form: outer refinement rounds                      */
    int32_t warm_used;         /* 1 if the warm start was kept                              */
    double dy_norm;            /* ||dy|| of the accepted direction                          */
    double shift;              /* delta added to Q's diagonal for the accepted draw (0: none) */
} ipm_step_info;

/* ---- context ------------------------------------------------------------------------------ */

/* Create a context on HIP device `device` that orders its work on `hip_stream` (a hipStream_t;
 * NULL = the default stream). The context owns its workspace (grown on demand, freed by
 * ipm_ctx_destroy). Returns IPM_ERR_HIP if the device cannot be used. */
int  ipm_ctx_create(ipm_ctx** out, int device, void* hip_stream);
void ipm_ctx_destroy(ipm_ctx* ctx);
int  ipm_ctx_set_stream(ipm_ctx* ctx, void* hip_stream);
const char* ipm_last_error(const ipm_ctx* ctx);
void ipm_params_default(ipm_params* p);

/* ---- the hot path ----------------------------------------------------------------------- */

/* Sketch B = A diag(d) W (Algorithm 1, step 1; Section 2's sparse embedding).
 * W is the n x w matrix with exactly s nonzeros per row: row j, copy r (0 <= r < s) sits in
 * bucket r*(w/s) + floor(hi32(h) * (w/s) / 2^32) with value +1/sqrt(s) if bit 0 of h is 0,
 * else -1/sqrt(s), where h = mix64(K + (j+1)*phi), K = mix64((seed ^ mix64(k)) + (r+1)*phi),
 * phi = 0x9E3779B97F4A7C15 and mix64 is the SplitMix64 output function (Steele, Lea, Flood
 * 2014). k is the IPM iteration (W is redrawn every iteration, Algorithm 3 step 2).
 *   A    dense m x n, any dtype;  d [device] n doubles (the diagonal of D)
 *   B    [device] m x w row-major, out_dtype IPM_F64 or IPM_F32; overwritten.
 * The buckets accumulate in FP64 whatever out_dtype. A dense A whose w FP64 buckets exceed 64 KB
 * (one or two rows per block) first tabulates d_j / sqrt(s) and, for s <= 2, each column's
 * buckets and signs in the context workspace (8 n + 4 n bytes, grown on demand).
 * Errors: IPM_ERR_ARG if w < 1, s < 1, s > 8, s does not divide w, or pointers are null. */
int ipm_sketch(ipm_ctx* ctx, const ipm_matrix* A, const double* d, uint64_t seed, int64_t k,
               int32_t w, int32_t s, int32_t out_dtype, void* B);

/* Gaussian sketch B = A diag(d) W (the experiments' sketching matrix, Section 7), W with i.i.d.
 * N(0, 1/w) entries that are generated, never stored: entry (j, c), e = j*w + c, takes outputs
 * 2e and 2e+1 (h1, h2) of the SplitMix64 stream started at K = mix64((seed ^ mix64(k)) +
 * 0xD1B54A32D192ED03), u1 = ((h1 >> 11) + 1) * 2^-53, u2 = (h2 >> 11) * 2^-53, and equals
 * sqrt(-2 ln u1) cos(2 pi u2) / sqrt(w) (Box and Muller, 1958).
 *   A    dense row-major m x n (CSR is rejected), any dtype;  d [device] n doubles
 *   B    [device] m x w row-major FP64; overwritten. Accumulation is FP64 (MFMA).
 * Errors: IPM_ERR_ARG for a CSR A, w < 1 or null pointers. */
int ipm_sketch_gaussian(ipm_ctx* ctx, const ipm_matrix* A, const double* d, uint64_t seed, int64_t k,
                        int32_t w, double* B);

/* Preconditioner factor: Q = B B^T (eqn. pdprecond), Q = L L^T, and Linv = L^{-1}.
 *   B    [device] m x w row-major, b_dtype IPM_F64 or IPM_F32
 *   L    [device] m x m, or NULL; on return its lower triangle holds L (upper part unspecified)
 *   Linv [device] m x m; on return the lower triangle holds L^{-1}, the upper part is zero
 *   bad_pivot  [host] may be NULL; set to the first failing pivot index or -1.
 * Errors: IPM_ERR_ARG unless 1 <= m <= 10236 (the row limit of every entry point), w >= 1 and
 *   B, Linv are set; IPM_ERR_NOT_SPD if a pivot is not positive (B lacks full row rank).
 *   Synchronizes. */
int ipm_precond_factor(ipm_ctx* ctx, int64_t m, int32_t w, int32_t b_dtype, const void* B,
                       double* L, double* Linv, int64_t* bad_pivot);

/* Preconditioned CG for A D^2 A^T dy = p with preconditioner Q = L L^T (Algorithm 1, step 3).
 * params->precision IPM_MIXED_F32ACC runs iterative refinement around FP32-accumulated inner
 * solves (see ipm_params.precision); the other forms run one CG with FP64-accumulated
 * matvecs. A's storage type is used as given.
 *   d2   [device] n doubles, the diagonal of D^2
 *   Linv [device] m x m lower triangle of L^{-1} (as written by ipm_precond_factor)
 *   p    [device] m doubles
 *   dy   [device] m doubles; input: initial iterate dy0 if warm != 0 (scaled to beta dy0,
 *        beta = dy0^T p / dy0^T M dy0, and kept only if its preconditioned residual is below
 *        that of 0), output: the solution.
 *   Stops when ||L^-1 (p - A D^2 A^T dy)|| <= tol_pcg * ||L^-1 p|| (eq. pdcond2), at maxit_pcg,
 *   or when the residual stagnates (params stag_window / stag_ratio). Synchronizes. */
int ipm_pcg_solve(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* Linv,
                  const double* p, double* dy, int32_t warm, const ipm_params* params,
                  ipm_pcg_info* info);

/* One iteration of Algorithm 3 (Section 5) from the state's point:
 *   residuals r_p = A x - b, r_d = A^T y + s - c; stop test (relative gap, ||r_p||/(1+||b||),
 *   ||r_d||/(1+||c||) all <= gap_tol -> IPM_CONVERGED, no step); W drawn for iteration k;
 *   p = b - A (sigma mu / s + d^2 r_d); sketch, factor and CG as above; v of eq. compv with
 *   (ADW)^+ = B^T Q^{-1} and the true residual A D^2 A^T dy - p; ds = -r_d - A^T dy;
 *   dx = -x + sigma mu / s - d^2 ds - v / s; alpha_max = end of the segment inside N(gamma)
 *   (x_i s_i >= (1-gamma) mu and ||r||/||r0|| <= mu/mu0 with r(alpha) = (1-alpha) r), times
 *   theta if below 1; alpha = argmin of mu(alpha) on [0, alpha_max]; x, y, s updated in place
 *   and k incremented only when the step succeeds. If CG fails (stagnation, maxit) or Q is not
 *   SPD, W is redrawn up to max_redraws times with w doubled and s at least 2; a redrawn W
 *   whose Q still factors only with a shift (max_shifts) is kept whatever CG did, since the
 *   shift then means that kappa(A D) itself, not the draw, puts kappa(Q) beyond 1/u.
 * Synchronizes. */
int ipm_step(ipm_ctx* ctx, const ipm_problem* prob, ipm_state* state, const ipm_params* params,
             ipm_step_info* info);

/* ipm_step whose CG solve starts from the M-norm-optimal combination of ncand (1 or 2)
 * candidate vectors dy0 [device, ncand x m doubles, one vector after the other], used when
 * params->warm_start is IPM_WARM_GIVEN (the learned warm start passes the previous dy and the
 * network's output). Two candidates nearly parallel in the M-norm (squared sine of their angle
 * below 1e-8) are reduced to the first. The candidates' products M dy0_k come from one pass
 * over A for both (FP64 accumulation), computed once per step and shared by every draw of W.
 * dy0 is read only. */
int ipm_step_warm(ipm_ctx* ctx, const ipm_problem* prob, ipm_state* state, const ipm_params* params,
                  const double* dy0, int32_t ncand, ipm_step_info* info);

/* The accepted dy of the last successful ipm_step on this context [device, m doubles] is copied
 * to out. Returns IPM_ERR_ARG if no step was taken yet or m differs. */
int ipm_last_dy(ipm_ctx* ctx, int64_t m, double* out);

/* ---- measurement ------------------------------------------------------------------------ */

/* ---- learned warm start (a further form of the method; not in the paper) ----------------
 *
 * A three-layer ReLU network (FP32) maps features of IPM iteration k >= 1 to a second
 * warm-start candidate beside the previous direction dy_prev; ipm_step_warm (warm_start =
 * IPM_WARM_GIVEN, ncand = 2) starts the CG solve from their M-norm-optimal combination.
 * Features (m + 18): u = dy_prev / ||dy_prev|| (m), 0.1 log ||dy_prev||, 0.1 [mean, std, min,
 * max] of l = log(x / s) (= log d^2), 0.1 x 12 quantiles of l at levels i/13 (i = 1..12) read
 * from a 64-bin histogram on [min l, max l] with linear interpolation in the bin, and k / kmax.
 * Network: h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3; candidate
 * ||dy_prev|| y. Training target t = (dy - (u^T dy) u) / ||dy_prev|| (the part of the new
 * direction dy the previous one misses). Loss of a batch: mean over samples of log(e + 1e-10)
 * with e = 1 - cos^2(y, t), the squared sine of the angle to the target (only the direction of
 * a candidate matters; the CG iterations a start saves grow like log(1 / e)). Optimiser: Adam. */
typedef struct {
    int32_t n_in;        /* inputs; m + 18 for ipm_mlp_features / ipm_mlp_predict            */
    int32_t n_hidden;    /* width H                                                          */
    int32_t n_out;       /* outputs (m)                                                      */
    int32_t reserved;
    float* params;       /* [device] ipm_mlp_param_count() floats, flat: W1 [H x n_in]
                            row-major, b1 [H], W2 [H x H], b2 [H], W3 [n_out x H], b3 [n_out]   */
} ipm_mlp;

int64_t ipm_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out);

/* Features of iteration k (see above) into feat [device, m + 18 floats]. dy_prev [device, m],
 * x, s [device, n] with x, s > 0. Stream-ordered, no synchronization. */
int ipm_mlp_features(ipm_ctx* ctx, int64_t m, int64_t n, const double* dy_prev, const double* x,
                     const double* s, int64_t k, int64_t kmax, float* feat);

/* Training target of one sample: t = (dy - (u^T dy) u) / ||dy_prev||, u = dy_prev / ||dy_prev||
 * [device, m floats]; dy, dy_prev [device, m doubles] are the accepted directions of
 * iterations k and k-1. */
int ipm_mlp_target(ipm_ctx* ctx, int64_t m, const double* dy_prev, const double* dy, float* t);

/* Y [device, batch x n_out] = network(X [device, batch x n_in]), row-major. */
int ipm_mlp_forward(ipm_ctx* ctx, const ipm_mlp* net, int32_t batch, const float* X, float* Y);

/* Gradient of the batch loss for inputs X and targets T [device, batch x n_out] into grad
 * [device, ipm_mlp_param_count floats, same layout as params]. If loss is not NULL the call
 * synchronizes and writes the loss there (host). A sample whose target or output is zero
 * contributes log(1 + 1e-10) and no gradient. */
int ipm_mlp_backward(ipm_ctx* ctx, const ipm_mlp* net, int32_t batch, const float* X, const float* T,
                     float* grad, double* loss);

/* One Adam step t >= 1 (Kingma and Ba, 2015) on count parameters with moment buffers m1, m2
 * [device, zero before the first step]: m1 = b1 m1 + (1-b1) g, m2 = b2 m2 + (1-b2) g^2,
 * p -= lr (m1 / (1-b1^t)) / (sqrt(m2 / (1-b2^t)) + eps). */
int ipm_mlp_adam(ipm_ctx* ctx, int64_t count, float* params, const float* grad, float* m1, float* m2,
                 int64_t t, double lr, double beta1, double beta2, double eps);

/* Warm-start candidate of iteration k: features, forward pass, dy0 = ||dy_prev|| y
 * [device, n_out doubles]. net->n_in must equal net->n_out + 18. */
int ipm_mlp_predict(ipm_ctx* ctx, const ipm_mlp* net, int64_t n, const double* dy_prev, const double* x,
                    const double* s, int64_t k, int64_t kmax, double* dy0);

/* q = A diag(d2) A^T v in one pass over A (the CG matvec). v, q [device] m doubles;
 * d2 [device] n doubles. */
int ipm_normal_matvec(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v,
                      double* q);

/* ipm_normal_matvec for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result bit for bit, with the pass's per-block partial sums in a static 16 MB device array
 * instead of a context workspace. The call allocates and frees nothing.
 *   A, d2, v, q  as for ipm_normal_matvec (caller-owned, [device]).
 *   Scratch need: dense A  8 * (G m + G + ceil(m/4)) bytes, G <= 2 * CUs the pass's blocks
 *                 (at most about 4.2 MB for FP64/FP32 up to 2048 rows);
 *                 CSR A    8 * (n + ceil(n/256 capped at 2048) + ceil(m/4)) bytes.
 *   A need above 16 MB (BF16 A with more than about 4000 rows, CSR A with about 2 million or
 *   more columns) is IPM_ERR_ARG, before device work.
 * Every call on one GPU shares that GPU's array and leaves its partial sums there; calls that
 * overlap on one GPU (two streams, two contexts or two host threads at once) race and give
 * wrong results. Calls ordered on one stream are safe. */
int ipm_normal_matvec_noalloc(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v,
                              double* q);

/* Attainable-bandwidth probes: the measured denominators, beside the vendor's 8 TB/s, for the
 * streaming passes over A (the matvec, the sketch, the residual and direction passes). Not
 * steps of the method; both run on the context's stream and use its access pattern (contiguous
 * per-block ranges of non-temporal 16-byte loads).
 *
 * ipm_stream_read: out[0] = the sum of the `count` FP64 words at x, accumulated in FP64 (per
 * block, then over the blocks in a fixed order, so the result is reproducible). x [device],
 * 16-byte aligned (may be null when count = 0); out [device] one double. count = 0 gives 0.
 * Errors: IPM_ERR_ARG for a null out, a null x with count > 0, count < 0 or a misaligned x. */
int ipm_stream_read(ipm_ctx* ctx, const double* x, int64_t count, double* out);
/* ipm_stream_copy: dst[0, bytes) = src[0, bytes), bit for bit (16-byte non-temporal loads and
 * stores; the last bytes % 16 bytes one by one). src, dst [device], 16-byte aligned, not
 * overlapping; bytes = 0 does nothing (null pointers allowed). Errors: IPM_ERR_ARG for null
 * pointers with bytes > 0, bytes < 0, misalignment or overlap. */
int ipm_stream_copy(ipm_ctx* ctx, const void* src, void* dst, int64_t bytes);

#define IPM_KERNEL_MATVEC  0   /* the CG matvec pass over A (FP64 accumulation)           */
#define IPM_KERNEL_SKETCH  1   /* the sketch pass over A                                  */
#define IPM_KERNEL_GRAM    2   /* the Gram product B B^T                                  */
#define IPM_KERNEL_MATVEC32 3  /* the mixed form's inner CG matvec (FP32 accumulation)   */
#define IPM_KERNEL_RESID64 4   /* the mixed form's FP64-accumulated residual pass          */
#define IPM_KERNEL_STREAM_READ 5  /* the read pass of ipm_stream_read                       */
#define IPM_KERNEL_STREAM_COPY 6  /* the copy pass of ipm_stream_copy                       */
#define IPM_KERNEL_WARM    7   /* the warm start's candidate products (one pass for both)  */
#define IPM_KERNEL_COUNT   8

/* Per-kernel timing with HIP events recorded at the start and end of launches of the kernels
 * above on the context's stream: on = 0 disables it; on = N >= 1 times every N-th launch of each
 * kernel (1: every launch; recording events costs a few microseconds of queue time per timed
 * launch, so a period of 8 or more keeps the measured run close to an untimed one). Enabling
 * resets the totals. Errors: IPM_ERR_ARG if on < 0. */
int ipm_ctx_set_timing(ipm_ctx* ctx, int32_t on);
/* Total milliseconds and number of launches of `kernel` since timing was enabled.
 * Synchronizes. */
int ipm_kernel_time(ipm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* IPMSK_H */
