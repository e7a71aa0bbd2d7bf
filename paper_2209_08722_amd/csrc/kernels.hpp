// Launchers of the ipmsk device kernels (internal interface between the C ABI and the kernels).
#pragma once

#include "common.hpp"

namespace ipmsk {

// Slots of the per-step device scalar block (doubles).
enum Scalar {
    SC_XS = 0, SC_CTX, SC_C2, SC_MU, SC_SMU, SC_BTY, SC_B2, SC_RP2, SC_RD2,
    SC_GAP, SC_RELGAP, SC_RPREL, SC_RDREL, SC_OBJ, SC_RNORM, SC_MU0, SC_R0NORM,
    SC_A1, SC_A2, SC_V2, SC_AMAX, SC_ABAR, SC_STALL, SC_ROOT, SC_DY2, SC_COUNT = 32
};

// Post-processing of the row reduction of strip-pass partials.
enum RowPost {
    POST_PLAIN = 0, POST_MATVEC = 1, POST_RESID = 2, POST_RHAT = 3, POST_RESP = 4, POST_SUBR = 5,
    POST_PAIR = 6   // both accumulations stored: out0, out1
};

// Kinds of single-pass strip kernels over row-major A.
enum StripKind { STRIP_MATVEC = 0, STRIP_RESID = 1, STRIP_DIR = 2, STRIP_MATVEC2 = 3 };

// Row accumulations (outputs) of a pass of this kind.
inline int strip_nacc(int kind) { return (kind == STRIP_RESID || kind == STRIP_MATVEC2) ? 2 : 1; }

struct StripPlan {
    int nt;        // threads per block
    int rpt;       // rows per thread (template instance)
    int grid;      // blocks (persistent)
    int nstrips;   // column strips of width sw
    int sw;        // strip width in columns
    size_t lds;    // dynamic LDS bytes
    int lpr;       // lanes per row segment
    int rr;        // 1: re-read form (k_strip_rr)
    int kk;        // rows per thread of the re-read form (a multiple of its chunk)
};

// Arguments of every strip pass. Unused pointers may be null. launch_strip queues the pass and
// the row reduction of its per-block partials (which applies the RowPost step).
struct StripCall {
    int kind;
    int dtype;               // IPM_F64 / IPM_F32 / IPM_BF16
    int acc64;               // 1: FP64 accumulation, 0: FP32 (mixed-precision matvec)
    int post;                // RowPost
    const void* A;
    int m;
    int64_t n, ld;
    const double* vec0;      // m-vector dotted with every column
    const double* vec1;      // m (matvec2: the second vector)
    const double* d2;        // n: diagonal of D^2
    const double* x;         // n (resid)
    const double* s;         // n (resid)
    const double* c;         // n (resid)
    const double* rd;        // n (dir: input r_d)
    double* rd_out;          // n (resid: output r_d)
    double* ds_out;          // n (dir: output ds)
    const double* scal;      // device scalar block (resid reads SC_SMU)
    const double* b;         // m (resid post)
    const double* pvec;      // m (rhat post)
    const double* dvec;      // m (matvec post: d^T q)
    double* out0;            // m outputs of the post step
    double* out1;
    double* outsc;           // resid post: [1] = ||r_d||^2
    double* part;            // [nacc][m][grid] per-block partial row sums
    double* colpart;         // [grid] per-block column reductions (resid: sum of r_d^2)
    double* gpart;           // resid post: per-reduction-block sums of r_p^2 [rowsum_blocks(m)]
    const int* done;         // early-exit flag (may be null)
    // sparse A (CSR with a CSC mirror of the same nonzeros); A above is the CSR values
    const int64_t* row_ptr;  // m + 1
    const int32_t* col_idx;  // nnz
    const void* csc_val;     // nnz, column order
    const int64_t* col_ptr;  // n + 1
    const int32_t* row_idx;  // nnz
    double* coefs;           // [nacc][n] column coefficients between the two sparse passes
    int feasible;            // resid / dir passes of Algorithm 2: r_d taken as 0, p = A x - A sigma mu / s
};

StripPlan strip_plan(int dtype, int m, int64_t n, int num_cu, int kind);
hipError_t launch_strip(const StripCall& c, const StripPlan& p, hipStream_t st);   // pass + rowsum
hipError_t launch_strip_pass(const StripCall& c, const StripPlan& p, hipStream_t st);
hipError_t launch_strip_rowsum(const StripCall& c, const StripPlan& p, hipStream_t st);
int rowsum_blocks(int m);
constexpr int kStripMaxGrid = 4096;

// ---- sparse A (sparse.hip) ----
// The same passes for CSR A: a column pass over the CSC mirror (column dots, per-column step,
// coefficients into c.coefs, column reductions into c.colpart[sparse_col_blocks(n)]) and a row
// pass over CSR (row sums with the coefficients and the RowPost step, one wave per row, with the
// reduction-block layout of launch_strip_rowsum).
int sparse_col_blocks(int64_t n);
hipError_t launch_sparse_pass(const StripCall& c, hipStream_t st);
// B = A D W for CSR A: one block per (row, bucket range of one copy), LDS buckets in FP64.
hipError_t launch_sketch_csr(int dtype, const void* val, const int64_t* row_ptr, const int32_t* col_idx, int m,
                             const double* dvals, int dvals_are_d2, const HashKeys& hk, int w, int out_f64, void* B,
                             hipStream_t st);

// ---- sketch and perturbation -----------------------------------------------------------------
// table: the bucket kernel reads d_j / sqrt(s) from an n-vector (dsc) that launch_sketch_prep
// fills first, and, where sketch_table_fits(hk) (s <= 2, w / s <= 32768), each column's buckets
// and signs from an n-vector of packed 32-bit entries (tab) filled by the same launch.
struct SketchPlan { int rows_per_block; int chunks; int64_t cols_per_chunk; size_t lds; bool atomic; bool global_only; int range_width; bool table; };
SketchPlan sketch_plan(int m, int64_t n, int w, int out_f64, int num_cu);
bool sketch_table_fits(const HashKeys& hk);
hipError_t launch_sketch_prep(int64_t n, const double* dvals, int dvals_are_d2, double scale, double* dsc,
                              const HashKeys& hk, uint32_t* tab, hipStream_t st);
hipError_t launch_sketch(int dtype, const void* A, int m, int64_t n, int64_t ld, const double* dvals,
                         int dvals_are_d2, const HashKeys& hk, int w, int out_f64, void* B,
                         const SketchPlan& sp, const double* dsc, const uint32_t* tab, hipStream_t st);
// u = B^T g (B m x w, FP64 or FP32); u is overwritten.
hipError_t launch_btg(const void* B, int b_f64, int m, int w, const double* g, double* u, hipStream_t st);
// dx and the sums a1 = x^T ds + s^T dx, a2 = dx^T ds, ||v||^2 as per-block partials [grid][3].
int pointwise_blocks(int64_t n);
// wu: (W u) precomputed (Gaussian W), or null to apply the hashed sparse W to u
hipError_t launch_dx(int64_t n, const double* x, const double* s, const double* d2, const double* ds,
                     const double* u, int vcorr, const HashKeys& hk, const double* wu, const double* scal, double* dx,
                     double* part3, hipStream_t st);

// ---- dense FP64 linear algebra ----------------------------------------------------------------
// C = alpha * A * op(B) + beta * C, row-major; op(B) = B^T (B stored N x K) if trans_b.
// lower_only skips tiles strictly above the diagonal. ksplit > 1 accumulates atomically (C must
// hold beta*C already; beta is ignored).
hipError_t launch_dgemm(bool trans_b, bool lower_only, int M, int N, int K, double alpha,
                        const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                        double* C, int64_t ldc, int ksplit, hipStream_t st);
hipError_t launch_sgram_f32(int m, int w, const float* B, double* C, int ksplit, hipStream_t st);
// The same products with 128 x 128 tiles and a pipelined K loop (for large M and N).
int gemm_big_tiles(int M, int N, bool lower_only);
hipError_t launch_dgemm_big(bool trans_b, bool lower_only, int M, int N, int K, double alpha, const double* A,
                            int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int ksplit,
                            hipStream_t st);
hipError_t launch_sgram_f32_big(int m, int w, const float* B, double* C, int ksplit, hipStream_t st);
hipError_t launch_fill_2d(double* C, int M, int N, int64_t ldc, hipStream_t st);   // M x N block of C <- 0

// ---- Gaussian sketch (gauss.hip) ----
uint64_t gauss_key(uint64_t seed, int64_t k);   // mix64((seed ^ mix64(k)) + kGaussDomain)
int gauss_tiles(int m, int w);
// B (m x w, FP64, cleared by the caller when ksplit > 1) = A diag(d) W, W generated from key
hipError_t launch_sketch_gauss(int dtype, int m, int64_t n, int w, const void* A, int64_t lda, const double* dvals,
                               int dvals_are_d2, uint64_t key, double* B, int ksplit, hipStream_t st);
// t (n) = W u
hipError_t launch_gauss_apply(int64_t n, int w, uint64_t key, const double* u, double* t, hipStream_t st);
hipError_t launch_potrf_diag(double* Lw, int64_t ld, int k0, int kb, double* X, int64_t ldx, int* status,
                             hipStream_t st);
hipError_t launch_transpose(const double* X, double* XT, int m, hipStream_t st);
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t st);
hipError_t launch_diag_sum(const double* A, int m, int lda, double* out, hipStream_t st);
hipError_t launch_diag_add(double* A, int m, int lda, double delta, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st);

// Bandwidth probes (probe.hip). stream_read_parts: the number of partials launch_stream_read writes.
int stream_read_parts(int64_t count, int num_cu);
hipError_t launch_stream_read(const double* x, int64_t count, double* part, double* out, int num_cu,
                              hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, int num_cu, hipStream_t st);

// ---- PCG -----------------------------------------------------------------------------------------
enum PcgInt { PI_DONE = 0, PI_STATUS, PI_ITERS, PI_WARM, PI_COUNT = 8 };
enum PcgDbl { PD_RHO0 = 0, PD_RHO1, PD_RHOSTAR, PD_HIST = 8 };

struct PcgBufs {
    int m;
    const double* X;      // L^{-1}, lower, ld m
    const double* XT;     // (L^{-1})^T, upper, ld m
    const double* p;
    double* dy[2];
    double* r[2];
    double* dv;           // search direction
    double* q;            // A D^2 A^T dv
    double* wv;           // L^{-1} r
    double* wv2;          // second right-hand side (warm start)
    double* rho_part;
    int n_rho;
    double* cd;           // PcgDbl block (hist at PD_HIST)
    int* ci;              // PcgInt block
    double tol;
    double stag_ratio;
    int stag_window;
    int maxit;
    double* ahist;        // CG step lengths alpha_j (Lanczos estimate for Chebyshev), or null
};
int gemv_blocks(int m);
hipError_t launch_pcg_init1(const PcgBufs& b, int warm, hipStream_t st);
// Chebyshev iteration (Section 3.2), continuing CG's iterate: g = X r with per-block ||g||^2
// (cheb1), then the stop test at total iteration jt, z = X^T g, dx = c1 z + c2 dx, dy += dx
// (cheb2); the matvec pass then subtracts M dx from r (POST_SUBR).
hipError_t launch_cheb1(const PcgBufs& b, const double* r, double* g, hipStream_t st);
hipError_t launch_cheb2(const PcgBufs& b, const double* g, double* dx, double* dy, double c1, double c2, int jt,
                        int t, hipStream_t st);
hipError_t launch_pcg_init2(const PcgBufs& b, int warm, const double* dy_in, hipStream_t st);
hipError_t launch_pcg_gemv1(const PcgBufs& b, int j, hipStream_t st);
hipError_t launch_pcg_gemv2(const PcgBufs& b, int j, hipStream_t st);
hipError_t launch_pcg_finish(const PcgBufs& b, double* dy_out, double* info_out, hipStream_t st);
hipError_t launch_warm_galerkin(int m, int nc, const double* v1, const double* v2, const double* p, const double* q1,
                                const double* q2, double* dy_out, double* q_out, double* r_out, hipStream_t st);
// y = L^{-1} x (lower) or (L^{-1})^T x (upper, given XT) - plain triangular GEMV.
hipError_t launch_trigemv(const double* M, int m, int lower, const double* xin, double* yout, hipStream_t st);

// ---- IPM step pointwise kernels -------------------------------------------------------------
hipError_t launch_stats(int64_t n, const double* x, const double* s, const double* c, double* d2,
                        double* part3, hipStream_t st);
hipError_t launch_fin_stats(int64_t n, int m, const double* part3, int G, const double* b, const double* y,
                            double sigma, double* scal, hipStream_t st);
hipError_t launch_metrics(int64_t n, int m, const double* rp2part, int Grp, const double* rd2, int set_ref,
                          double mu0_in, double r0_in, int feasible, double* scal, hipStream_t st);
hipError_t launch_fin_dx(const double* part3, int G, double* scal, hipStream_t st);
hipError_t launch_roots(int64_t n, const double* x, const double* s, const double* dx, const double* ds,
                        double gamma, const double* scal, double* partmin, hipStream_t st);
hipError_t launch_alpha(int64_t n, const double* partmin, int G, double gamma, double theta,
                        double min_step, double* scal, hipStream_t st);
hipError_t launch_update(int64_t n, int m, double* x, double* y, double* s, const double* dx,
                         const double* dy, const double* ds, const double* scal, hipStream_t st);
// y += alpha * x (m-vectors); out[0] = x^T y (one block).
hipError_t launch_axpy(int m, double alpha, const double* x, double* y, hipStream_t st);
hipError_t launch_dot(int m, const double* x, const double* y, double* out, hipStream_t st);

// ---- learned warm start (mlp.hip) ----
int64_t mlp_param_count(int I, int H, int O);
int feat_blocks(int64_t n);   // work needs 4 * feat_blocks(n) + 4 doubles
hipError_t launch_mlp_features(int m, int64_t n, const double* dy_prev, const double* x, const double* s,
                               double kfrac, double* work, int* hist, float* feat, double* nrm_out, hipStream_t st);
hipError_t launch_mlp_forward(int I, int H, int O, const float* theta, int B, const float* X, float* act1,
                              float* act2, float* Y, hipStream_t st);
hipError_t launch_mlp_backward(int I, int H, int O, const float* theta, int B, const float* X, const float* T,
                               const float* act1, const float* act2, const float* Y, float* dY, float* dZ2,
                               float* dZ1, double* ratio, float* grad, double* loss, hipStream_t st);
hipError_t launch_mlp_adam(int64_t count, float* p, const float* g, float* m1, float* m2, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st);
hipError_t launch_mlp_scale_out(int m, const float* y, const double* nrm, double* dy0, hipStream_t st);
hipError_t launch_mlp_target(int m, const double* dy_prev, const double* dy, float* t, hipStream_t st);

}  // namespace ipmsk
