// C ABI of the sketch-preconditioned IPM hot path: context, workspace and orchestration of the
// HIP kernels. Declarations and the contract of every entry point are in include/ipmsk.h.
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ipmsk.h"
#include "kernels.hpp"

using namespace ipmsk;

namespace ipmsk {
thread_local LaunchTiming g_launch_timing;
}

namespace {

enum WsId {
    W_PART = 0, W_COLPART, W_RED, W_D2, W_RD, W_DS, W_DX, W_RP, W_P, W_DY, W_RHAT, W_G1, W_G2, W_U, W_B,
    W_L, W_X, W_XT, W_T, W_SCAL, W_PCG_VEC, W_PCG_RHO, W_PCG_CD, W_PCG_CI, W_STATUS, W_PART3, W_PARTMIN,
    W_INFO, W_GPART, W_SQ, W_REF, W_WARM, W_PREV, W_BF, W_MLPF, W_MLPD, W_MLPI, W_WQ, W_COEF, W_GU, W_STREAM, W_SKTAB,
    W_COUNT
};

struct TimedPair {
    hipEvent_t a, b;
    int tag;   // CG iteration index (or -1)
};

}  // namespace

struct ipm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string err;
    void* ws[W_COUNT] = {};
    size_t ws_bytes[W_COUNT] = {};
    void* pinned = nullptr;   // host staging for scalar readbacks
    bool timing = false;
    int timing_period = 1;                      // time every timing_period-th launch per kernel
    int64_t timing_seq[IPM_KERNEL_COUNT] = {};  // launches seen per kernel since timing was set
    std::vector<TimedPair> pending[IPM_KERNEL_COUNT];
    double total_ms[IPM_KERNEL_COUNT] = {};
    int64_t launches[IPM_KERNEL_COUNT] = {};
    std::vector<hipEvent_t> pool;
    int last_pcg_iters = 8;    // size of the first batch of queued CG iterations
    int last_inner_iters = 8;  // the same for the inner solves of the mixed form
    int last_cheb_steps = 0;   // Chebyshev steps of the previous solve (first batch after the probe)
    int64_t prev_m = 0;        // length of the accepted dy kept in W_PREV (0: none)
    double* scratch = nullptr; // this device's copy of the static scratch array (device address)
};

namespace {

constexpr size_t kPinnedBytes = 4096;
// Largest m of any entry point: the CG kernels hold two FP64 m-vectors in one block's LDS
// (160 KB, less the per-wave reduction slots).
constexpr int64_t kMaxRows = (160 * 1024 - 64) / 16;

// Static scratch of the allocation-free matvec (ipm_normal_matvec_noalloc): the pass's per-block
// partial sums live here instead of in a context workspace. Every GPU the library runs on holds
// its own copy (16 MB) until the process ends. In host code the name is only a symbol: the
// device address of each GPU's copy is taken once with hipGetSymbolAddress and used from then on.
constexpr size_t kScratchDoubles = (size_t)2 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (device must be current); taken once per device.
int scratch_address(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return IPM_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return IPM_ERR_HIP;
        }
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return IPM_OK;
}

int fail(ipm_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(ctx, IPM_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                      \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ < 0) return rc_;       \
    } while (0)

int ensure(ipm_ctx* ctx, int id, size_t bytes, void** out) {
    if (bytes == 0) bytes = 8;
    if (ctx->ws_bytes[id] < bytes) {
        if (ctx->ws[id]) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            HIPCHK(hipFree(ctx->ws[id]));
            ctx->ws[id] = nullptr;
            ctx->ws_bytes[id] = 0;
        }
        const size_t grow = bytes + bytes / 4;
        void* p = nullptr;
        if (hipMalloc(&p, grow) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, IPM_ERR_NOMEM, "workspace allocation of %zu bytes failed", grow);
        }
        ctx->ws[id] = p;
        ctx->ws_bytes[id] = grow;
    }
    *out = ctx->ws[id];
    return IPM_OK;
}

template <typename T>
int ws(ipm_ctx* ctx, int id, size_t count, T** out) {
    void* p = nullptr;
    int rc = ensure(ctx, id, count * sizeof(T), &p);
    *out = reinterpret_cast<T*>(p);
    return rc;
}

hipEvent_t pool_event(ipm_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Timing of the next launch of a measured kernel: the events are handed to the launch
// (hipExtLaunchKernelGGL records them at the kernel's own start and end).
struct Timer {
    ipm_ctx* ctx;
    int kernel;
    int tag;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(ipm_ctx* c, int k, int t = -1) : ctx(c), kernel(k), tag(t) {
        if (ctx->timing && ctx->timing_seq[k]++ % ctx->timing_period == 0) {
            a = pool_event(ctx);
            b = pool_event(ctx);
            if (a && b) g_launch_timing = LaunchTiming{a, b};
        }
    }
    void stop() {
        g_launch_timing = LaunchTiming{};
        if (ctx->timing && a && b) {
            ctx->pending[kernel].push_back(TimedPair{a, b, tag});
            a = b = nullptr;
        }
    }
};

// Resolve pending timings; pairs tagged with a CG iteration >= keep_below are dropped (those
// launches returned immediately because CG had already stopped).
void resolve_timing(ipm_ctx* ctx, int kernel, int keep_below) {
    for (auto& tp : ctx->pending[kernel]) {
        if (tp.tag < 0 || tp.tag < keep_below) {
            float ms = 0.f;
            if (hipEventSynchronize(tp.b) == hipSuccess && hipEventElapsedTime(&ms, tp.a, tp.b) == hipSuccess) {
                ctx->total_ms[kernel] += ms;
                ctx->launches[kernel] += 1;
            }
        }
        ctx->pool.push_back(tp.a);
        ctx->pool.push_back(tp.b);
    }
    ctx->pending[kernel].clear();
}

bool is_finite(double v) { return std::isfinite(v); }

int elem_size(int dtype) { return dtype == IPM_F64 ? 8 : (dtype == IPM_F32 ? 4 : (dtype == IPM_BF16 ? 2 : 0)); }

int check_matrix(ipm_ctx* ctx, const ipm_matrix* A) {
    if (!A) return fail(ctx, IPM_ERR_ARG, "A is null");
    if (A->layout != IPM_DENSE_ROWMAJOR && A->layout != IPM_CSR)
        return fail(ctx, IPM_ERR_ARG, "unsupported layout %d", A->layout);
    const int es = elem_size(A->dtype);
    if (!es) return fail(ctx, IPM_ERR_ARG, "unsupported dtype %d", A->dtype);
    if (A->m < 1 || A->n < 1 || A->m > A->n) return fail(ctx, IPM_ERR_ARG, "need 1 <= m <= n (m=%lld n=%lld)",
                                                          (long long)A->m, (long long)A->n);
    if (A->m > kMaxRows)
        return fail(ctx, IPM_ERR_ARG, "m=%lld exceeds the limit of %lld rows (the CG kernels keep two m-vectors in LDS)",
                    (long long)A->m, (long long)kMaxRows);
    if (!A->val) return fail(ctx, IPM_ERR_ARG, "A->val is null");
    if (A->layout == IPM_CSR) {
        if (A->n >= ((int64_t)1 << 31)) return fail(ctx, IPM_ERR_ARG, "n too large for 32-bit column indices");
        if (A->nnz < 0) return fail(ctx, IPM_ERR_ARG, "nnz < 0");
        if (!A->row_ptr || !A->col_idx || !A->csc_val || !A->col_ptr || !A->row_idx)
            return fail(ctx, IPM_ERR_ARG, "CSR A needs row_ptr, col_idx and the CSC mirror (csc_val, col_ptr, row_idx)");
        return IPM_OK;
    }
    if (A->ld < A->n) return fail(ctx, IPM_ERR_ARG, "ld < n");
    if ((A->ld * es) % 16 != 0) return fail(ctx, IPM_ERR_ARG, "ld*elem_size must be a multiple of 16 bytes");
    if (reinterpret_cast<uintptr_t>(A->val) % 16 != 0) return fail(ctx, IPM_ERR_ARG, "A->val must be 16-byte aligned");
    const StripPlan pl = strip_plan(A->dtype, (int)A->m, A->n, ctx->num_cu, STRIP_MATVEC);
    if (pl.nt <= 0)
        return fail(ctx, IPM_ERR_ARG, "m=%lld exceeds the dense passes' limit (%d rows with %s values)",
                    (long long)A->m, A->dtype == IPM_BF16 ? 6400 : 2048, A->dtype == IPM_BF16 ? "BF16" : "FP64/FP32");
    // the strip passes address a thread's rows inside a row group with a 32-bit element offset;
    // with more than 16 rows per thread the CG matvec reads a row group through a buffer
    // descriptor, so the group's bytes must fit 32 bits
    const int64_t rg = pl.nt / pl.lpr;
    const int64_t lim = (!pl.rr && pl.rpt > 16) ? ((int64_t)UINT32_MAX / es) / rg
                                                 : ((int64_t)UINT32_MAX - pl.sw) / (rg > 1 ? rg - 1 : 1);
    if (A->ld > lim)
        return fail(ctx, IPM_ERR_ARG, "ld=%lld too large for the dense passes (at most %lld elements per row at m=%lld)",
                    (long long)A->ld, (long long)lim, (long long)A->m);
    return IPM_OK;
}

HashKeys make_keys(uint64_t seed, int64_t k, int w, int s) {
    HashKeys hk{};
    const uint64_t base = seed ^ mix64((uint64_t)k);
    for (int r = 0; r < s; ++r) hk.key[r] = mix64(base + (uint64_t)(r + 1) * kPhi);
    hk.s = s;
    hk.blk = w / s;
    hk.scale = 1.0 / std::sqrt((double)s);
    return hk;
}

int do_sketch(ipm_ctx* ctx, const ipm_matrix* A, const double* dvals, int is_d2, const HashKeys& hk, int w,
              int out_f64, void* B) {
    const int m = (int)A->m;
    if (A->layout == IPM_CSR) {
        Timer t(ctx, IPM_KERNEL_SKETCH);
        HIPCHK(launch_sketch_csr(A->dtype, A->val, A->row_ptr, A->col_idx, m, dvals, is_d2, hk, w, out_f64, B,
                                 ctx->stream));
        t.stop();
        return IPM_OK;
    }
    const SketchPlan sp = sketch_plan(m, A->n, w, out_f64, ctx->num_cu);
    if (sp.atomic) {
        if (out_f64) {
            HIPCHK(launch_fill(reinterpret_cast<double*>(B), (int64_t)m * w, 0.0, ctx->stream));
        } else {
            // FP32 zero is all-zero bits: cleared by the integer fill kernel (a kernel, not a
            // memset, so the call can be captured in a HIP graph)
            HIPCHK(launch_fill_i32(reinterpret_cast<int*>(B), (int64_t)m * w, 0, ctx->stream));
        }
    }
    double* dsc = nullptr;
    uint32_t* tab = nullptr;
    if (sp.table) {
        // d_j / sqrt(s) once per call and, where they pack into 32 bits, the columns' buckets and
        // signs (n doubles, padded to an even count so that the n 32-bit entries after them start
        // 16-byte aligned)
        const bool packed = sketch_table_fits(hk);
        const size_t npad = ((size_t)A->n + 1) & ~(size_t)1;
        CHK(ws(ctx, W_SKTAB, npad + (packed ? ((size_t)A->n + 1) / 2 : 0), &dsc));
        if (packed) tab = reinterpret_cast<uint32_t*>(dsc + npad);
        HIPCHK(launch_sketch_prep(A->n, dvals, is_d2, hk.scale, dsc, hk, tab, ctx->stream));
    }
    Timer t(ctx, IPM_KERNEL_SKETCH);   // times the bucket kernel (the first timed launch below)
    HIPCHK(launch_sketch(A->dtype, A->val, m, A->n, A->ld, dvals, is_d2, hk, w, out_f64, B, sp, dsc, tab,
                         ctx->stream));
    t.stop();
    return IPM_OK;
}

// Gaussian sketch into an FP64 B (m x w): the MFMA kernel with split-K over n when the output
// tiles alone cannot occupy every CU (one 8-wave block per CU); B is cleared first in that case.
int do_sketch_gauss(ipm_ctx* ctx, const ipm_matrix* A, const double* dvals, int is_d2, uint64_t key, int w,
                    double* B) {
    if (A->layout != IPM_DENSE_ROWMAJOR) return fail(ctx, IPM_ERR_ARG, "the Gaussian sketch needs a dense A");
    const int m = (int)A->m;
    const int tiles = gauss_tiles(m, w);
    int ks = 1;
    double best = 0.0;
    for (int c = 1; c <= 64 && (c == 1 || A->n / c >= 512); ++c) {
        const int blocks = tiles * c, slots = ctx->num_cu;
        const int rounds = (blocks + slots - 1) / slots;
        const double eff = (double)blocks / ((double)rounds * slots);
        if (eff > best + 0.02) {
            best = eff;
            ks = c;
        }
    }
    if (ks > 1) HIPCHK(launch_fill(B, (int64_t)m * w, 0.0, ctx->stream));
    Timer t(ctx, IPM_KERNEL_SKETCH);
    HIPCHK(launch_sketch_gauss(A->dtype, m, A->n, w, A->val, A->ld, dvals, is_d2, key, B, ks, ctx->stream));
    t.stop();
    return IPM_OK;
}

// Q = B B^T (lower) plus delta I, Q = L L^T in place in Lw, X = L^{-1}. *bad receives the
// first bad pivot or -1 and *trace the trace of B B^T.
// C = alpha A B (no transposes; C overwritten): the 128-tile kernel when it has work for half the
// CUs, else the 64-tile kernel, with split-K (C cleared first) when the tiles alone cannot fill
// the chip and `split` allows it.
int gemm_nn(ipm_ctx* ctx, int M, int N, int K, double alpha, const double* A, int64_t lda, const double* B,
            int64_t ldb, double* C, int64_t ldc, bool split);

// Rows [64 lo, 64 hi) of the triangular inverse X = L^{-1} (row-major m x m, diagonal 64-blocks
// already inverted, zero above the diagonal): the 2 x 2 block identity
// X21 = -X22 (L21 X11), halves inverted first. T: scratch of at least (m/2 + 64)^2 doubles.
int tri_inverse(ipm_ctx* ctx, int m, const double* L, double* X, double* T, int lo, int hi) {
    if (hi - lo <= 1) return IPM_OK;
    const int mid = (lo + hi) / 2;
    CHK(tri_inverse(ctx, m, L, X, T, lo, mid));
    CHK(tri_inverse(ctx, m, L, X, T, mid, hi));
    const int r1 = lo * 64, r2 = mid * 64, r3 = hi * 64 < m ? hi * 64 : m;
    const int n1 = r2 - r1, n2 = r3 - r2;
    CHK(gemm_nn(ctx, n2, n1, n1, 1.0, L + (int64_t)r2 * m + r1, m, X + (int64_t)r1 * m + r1, m, T, n1, true));
    CHK(gemm_nn(ctx, n2, n1, n2, -1.0, X + (int64_t)r2 * m + r2, m, T, n1, X + (int64_t)r2 * m + r1, m, true));
    return IPM_OK;
}

// Split-K factor for the 128-tile product: the smallest split (at most 8, chunks of at least 512)
// that fills the last round of one-block-per-CU waves best.
int big_ksplit(int tiles, int K, int num_cu) {
    int best = 1;
    double best_eff = 0.0;
    for (int ks = 1; ks <= 8 && (ks == 1 || K / ks >= 512); ++ks) {
        const int blocks = tiles * ks;
        const int rounds = (blocks + num_cu - 1) / num_cu;
        const double eff = (double)blocks / ((double)rounds * num_cu);
        if (eff > best_eff + 0.02) {
            best_eff = eff;
            best = ks;
        }
    }
    return best;
}

int gemm_nn(ipm_ctx* ctx, int M, int N, int K, double alpha, const double* A, int64_t lda, const double* B,
            int64_t ldb, double* C, int64_t ldc, bool split) {
    hipStream_t st = ctx->stream;
    const int big_tiles = gemm_big_tiles(M, N, false);
    if (big_tiles >= ctx->num_cu / 2) {
        const int ks = split ? big_ksplit(big_tiles, K, ctx->num_cu) : 1;
        if (ks > 1) HIPCHK(launch_fill_2d(C, M, N, ldc, st));
        HIPCHK(launch_dgemm_big(false, false, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, ks, st));
        return IPM_OK;
    }
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int ks = split ? (2 * ctx->num_cu + tiles - 1) / tiles : 1;
    const int kmax = (K + 63) / 64;
    if (ks > kmax) ks = kmax;
    if (ks < 1) ks = 1;
    if (ks > 1) HIPCHK(launch_fill_2d(C, M, N, ldc, st));
    HIPCHK(launch_dgemm(false, false, M, N, K, alpha, A, lda, B, ldb, 0.0, C, ldc, ks, st));
    return IPM_OK;
}

int factor_once(ipm_ctx* ctx, int m, int w, int b_f64, const void* B, double* Lw, double* X, double delta,
                int64_t* bad, double* trace) {
    hipStream_t st = ctx->stream;
    // Gram Q = B B^T (lower tiles): the 128-tile pipelined kernel once it has work for every CU,
    // else the 64-tile kernel with split-K
    const int big_tiles = gemm_big_tiles(m, m, true);
    const bool big = big_tiles >= ctx->num_cu / 2;
    int ksplit;
    if (big) {
        ksplit = big_ksplit(big_tiles, w, ctx->num_cu);
    } else {
        const int T = (m + 63) / 64;
        const int tiles = T * (T + 1) / 2;
        ksplit = (2 * ctx->num_cu + tiles - 1) / tiles;
        const int kmax = (w + 63) / 64;
        if (ksplit > kmax) ksplit = kmax;
        if (ksplit < 1) ksplit = 1;
    }
    if (ksplit > 1) HIPCHK(launch_fill(Lw, (int64_t)m * m, 0.0, st));
    {
        Timer t(ctx, IPM_KERNEL_GRAM);
        if (b_f64) {
            const double* Bd = reinterpret_cast<const double*>(B);
            if (big) HIPCHK(launch_dgemm_big(true, true, m, m, w, 1.0, Bd, w, Bd, w, 0.0, Lw, m, ksplit, st));
            else HIPCHK(launch_dgemm(true, true, m, m, w, 1.0, Bd, w, Bd, w, 0.0, Lw, m, ksplit, st));
        } else {
            const float* Bf = reinterpret_cast<const float*>(B);
            if (big) HIPCHK(launch_sgram_f32_big(m, w, Bf, Lw, ksplit, st));
            else HIPCHK(launch_sgram_f32(m, w, Bf, Lw, ksplit, st));
        }
        t.stop();
    }
    int* status = nullptr;
    CHK(ws(ctx, W_STATUS, 8, &status));
    double* tr = reinterpret_cast<double*>(status + 2);
    HIPCHK(launch_diag_sum(Lw, m, m, tr, st));
    if (delta > 0.0) HIPCHK(launch_diag_add(Lw, m, m, delta, st));
    HIPCHK(launch_fill_i32(status, 1, INT_MAX, st));
    HIPCHK(launch_fill(X, (int64_t)m * m, 0.0, st));
    for (int k0 = 0; k0 < m; k0 += 64) {
        const int kb = (m - k0) < 64 ? (m - k0) : 64;
        HIPCHK(launch_potrf_diag(Lw, m, k0, kb, X, m, status, st));
        const int rem = m - k0 - kb;
        if (rem > 0) {
            double* panel = Lw + (int64_t)(k0 + kb) * m + k0;
            HIPCHK(launch_dgemm(true, false, rem, kb, kb, 1.0, panel, m, X + (int64_t)k0 * m + k0, m, 0.0, panel, m, 1,
                                st));
            double* trail = Lw + (int64_t)(k0 + kb) * m + (k0 + kb);
            if (gemm_big_tiles(rem, rem, true) >= 2 * ctx->num_cu)
                HIPCHK(launch_dgemm_big(true, true, rem, rem, kb, -1.0, panel, m, panel, m, 1.0, trail, m, 1, st));
            else
                HIPCHK(launch_dgemm(true, true, rem, rem, kb, -1.0, panel, m, panel, m, 1.0, trail, m, 1, st));
        }
    }
    // X = L^{-1} off the diagonal blocks, recursively: X21 = -X22 (L21 X11)
    double* Tm = nullptr;
    const int64_t half = (int64_t)(m / 2 + 64);
    CHK(ws(ctx, W_T, (size_t)(half * half), &Tm));
    CHK(tri_inverse(ctx, m, Lw, X, Tm, 0, (m + 63) / 64));
    int* hs = reinterpret_cast<int*>(ctx->pinned);
    HIPCHK(hipMemcpyAsync(hs, status, 2 * sizeof(int) + sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    resolve_timing(ctx, IPM_KERNEL_GRAM, INT_MAX);
    *bad = (hs[0] == INT_MAX) ? -1 : hs[0];
    *trace = *reinterpret_cast<double*>(hs + 2);
    return IPM_OK;
}

// Factor Q = B B^T; on breakdown retry with Q + delta_j I, delta_j = u trace(Q) 100^j
// (u = 2^-53, j < max_shifts; trace(Q) >= ||Q||_2): forming B B^T in FP64 squares the
// condition number of B, and a shift of the order of the Gram's own rounding error restores a
// factorization where B is still numerically of full rank. *shift receives the delta used.
int do_factor(ipm_ctx* ctx, int m, int w, int b_f64, const void* B, double* Lw, double* X, int max_shifts,
              int64_t* bad, double* shift) {
    double trace = 0.0;
    *shift = 0.0;
    CHK(factor_once(ctx, m, w, b_f64, B, Lw, X, 0.0, bad, &trace));
    double delta = 0x1p-53 * trace;
    for (int j = 0; *bad >= 0 && j < max_shifts; ++j, delta *= 100.0) {
        double t2 = 0.0;
        CHK(factor_once(ctx, m, w, b_f64, B, Lw, X, delta, bad, &t2));
        if (*bad < 0) *shift = delta;
    }
    return IPM_OK;
}

// One pass over A for the StripCall c (kind, post step and vectors set by the caller): the dense
// strip pass and its row reduction, or the two sparse passes. Returns IPM_ERR_ARG if m is too
// large for the dense pass.
int run_pass(ipm_ctx* ctx, const ipm_matrix* A, StripCall& c, int kernel_id, int tag) {
    c.dtype = A->dtype;
    c.A = A->val;
    c.m = (int)A->m;
    c.n = A->n;
    c.ld = A->ld;
    const int nacc = strip_nacc(c.kind);
    CHK(ws(ctx, W_GPART, (size_t)rowsum_blocks(c.m), &c.gpart));
    if (A->layout == IPM_CSR) {
        c.row_ptr = A->row_ptr;
        c.col_idx = A->col_idx;
        c.csc_val = A->csc_val;
        c.col_ptr = A->col_ptr;
        c.row_idx = A->row_idx;
        CHK(ws(ctx, W_COEF, (size_t)nacc * (size_t)A->n, &c.coefs));
        CHK(ws(ctx, W_COLPART, (size_t)sparse_col_blocks(A->n), &c.colpart));
        HIPCHK(launch_sparse_pass(c, ctx->stream));
        return IPM_OK;
    }
    const StripPlan pl = strip_plan(A->dtype, c.m, A->n, ctx->num_cu, c.kind);
    if (pl.nt <= 0) return fail(ctx, IPM_ERR_ARG, "m=%d too large for the dense pass", c.m);
    CHK(ws(ctx, W_PART, (size_t)nacc * pl.grid * c.m, &c.part));
    CHK(ws(ctx, W_COLPART, (size_t)pl.grid, &c.colpart));
    if (kernel_id >= 0) {
        Timer t(ctx, kernel_id, tag);
        HIPCHK(launch_strip_pass(c, pl, ctx->stream));
        t.stop();
    } else {
        HIPCHK(launch_strip_pass(c, pl, ctx->stream));
    }
    HIPCHK(launch_strip_rowsum(c, pl, ctx->stream));
    return IPM_OK;
}

// One matvec pass over A: out <- A diag(d2) A^T v, accumulated in FP64 (acc64) or FP32.
int matvec_pass(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v, double* out, const int* done,
                int tag, int acc64 = 1) {
    StripCall c{};
    c.kind = STRIP_MATVEC;
    c.acc64 = acc64;
    c.post = POST_PLAIN;
    c.vec0 = v;
    c.d2 = d2;
    c.out0 = out;
    c.done = done;
    return run_pass(ctx, A, c, acc64 || A->dtype == IPM_F64 ? IPM_KERNEL_MATVEC : IPM_KERNEL_MATVEC32, tag);
}

// The warm start's candidate products q_k <- A diag(d2) A^T v_k (k < ncand <= 2), FP64
// accumulation: two candidates share one pass over A (each vector's dots and row sums in the
// order the single-vector pass uses). Where the shared memory of the dense pass cannot hold both
// vectors (BF16 re-read form beyond about 4800 rows) it runs one pass per vector.
int warm_products(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v0, const double* v1, int ncand,
                  double* q0, double* q1) {
    const bool pair = ncand > 1 &&
                      (A->layout == IPM_CSR || strip_plan(A->dtype, (int)A->m, A->n, ctx->num_cu, STRIP_MATVEC2).nt > 0);
    for (int k = 0; k < (ncand > 1 && !pair ? 2 : 1); ++k) {
        StripCall c{};
        c.kind = pair ? STRIP_MATVEC2 : STRIP_MATVEC;
        c.acc64 = 1;
        c.post = pair ? POST_PAIR : POST_PLAIN;
        c.vec0 = k == 0 ? v0 : v1;
        c.vec1 = pair ? v1 : nullptr;
        c.d2 = d2;
        c.out0 = k == 0 ? q0 : q1;
        c.out1 = pair ? q1 : nullptr;
        CHK(run_pass(ctx, A, c, IPM_KERNEL_WARM, -1));
    }
    resolve_timing(ctx, IPM_KERNEL_WARM, INT_MAX);
    return IPM_OK;
}

// r <- p - A diag(d2) A^T dy with FP64 accumulation whatever the storage type of A (the true
// residual of the refinement rounds).
int resid_pass(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* dy, const double* p, double* r) {
    StripCall c{};
    c.kind = STRIP_MATVEC;
    c.acc64 = 1;
    c.post = POST_RESP;
    c.vec0 = dy;
    c.d2 = d2;
    c.pvec = p;
    c.out0 = r;
    return run_pass(ctx, A, c, IPM_KERNEL_RESID64, -1);
}

struct PcgOut {
    int iters, status, warm_used, rounds;
    double relres, rho_star;
    double cheb_lo = 0.0, cheb_hi = 0.0;   // Chebyshev interval used (0: CG only)
};

struct PcgCfg {
    double tol;
    int maxit;
    int acc64;          // matvec accumulation: 1 FP64, 0 FP32 (low-precision storage only)
    bool xt_ready;      // W_XT already holds X^T
    int* last_iters;    // first batch size hint, updated with the count of this solve
    int cheb_probe = 0; // > 0: Chebyshev iteration after this many CG steps
};

// Chebyshev interval from the CG probe (Section 3.2 needs bounds on the spectrum of the
// preconditioned matrix; at practical sketch sizes they are estimated): the extreme Ritz values
// of the Lanczos tridiagonal the probe's CG steps build, widened by these factors.
constexpr int kChebProbe = 10;
constexpr double kChebLo = 0.5, kChebHi = 1.1;

// Smallest and largest eigenvalue of the symmetric tridiagonal (diag d[0..k-1], off-diagonal
// e[0..k-2]) by bisection on the Sturm sequence count, from the Gershgorin interval.
void tridiag_extremes(const double* d, const double* e, int k, double* lo, double* hi) {
    double gl = d[0], gu = d[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
        gl = std::fmin(gl, d[i] - r);
        gu = std::fmax(gu, d[i] + r);
    }
    auto below = [&](double x) {   // number of eigenvalues < x
        int c = 0;
        double q = d[0] - x;
        if (q < 0) ++c;
        for (int i = 1; i < k; ++i) {
            if (q == 0.0) q = 1e-300;
            q = d[i] - x - e[i - 1] * e[i - 1] / q;
            if (q < 0) ++c;
        }
        return c;
    };
    auto kth = [&](int target) {   // smallest x with below(x) >= target
        double a = gl, b = gu;
        for (int it = 0; it < 200 && b - a > 1e-15 * std::fmax(std::fabs(a), std::fabs(b)); ++it) {
            const double mid = 0.5 * (a + b);
            if (below(mid) >= target) b = mid;
            else a = mid;
        }
        return 0.5 * (a + b);
    };
    *lo = kth(1);
    *hi = kth(k);
}

// Initial iterate from ncand (1 or 2) candidate vectors cand[0:m], cand[m:2m]: their
// M-norm-optimal combination into dy_out, M dy_out into q_out and, if r_out is given,
// p - M dy_out into r_out. The products accumulate in FP64, one pass over A for both candidates.
int warm_combination(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* p, const double* cand,
                     int ncand, double* dy_out, double* q_out, double* r_out) {
    const int m = (int)A->m;
    double* q2 = nullptr;
    if (ncand > 1) CHK(ws(ctx, W_WQ, (size_t)m, &q2));
    CHK(warm_products(ctx, A, d2, cand, ncand > 1 ? cand + m : nullptr, ncand, q_out, q2));
    HIPCHK(launch_warm_galerkin(m, ncand, cand, ncand > 1 ? cand + m : nullptr, p, q_out, q2, dy_out, q_out, r_out,
                                ctx->stream));
    return IPM_OK;
}

// A warm start of the CG solve: the candidates' combination dy and q = M dy. It depends on A, D
// and p only, so one IPM step computes it once for all of its draws of W.
struct WarmStart {
    const double* dy;
    const double* q;
};

// Chebyshev iteration (Section 3.2) continuing the CG probe held in b (iterate dy[k & 1],
// residual r[k & 1] after k = out->iters steps): the interval comes from the probe's Lanczos
// tridiagonal; the three-term recurrence in correction form (theta, delta the interval's centre
// and half-width, s = delta / theta; omega_1 = 1, omega_2 = 1 / (1 - s^2 / 2),
// omega_{t+1} = 1 / (1 - s^2 omega_t / 4); dx_t = (omega_{t+1} / theta) Q^{-1} r_t +
// (omega_{t+1} - 1) dx_{t-1}) has host-computed coefficients, so no inner products enter it and
// whole batches are queued; the stop test is the CG's, on ||X r|| (device flag).
int chebyshev_stage(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, PcgBufs b, const PcgCfg& cfg,
                    double* dy_out, PcgOut* out) {
    hipStream_t st = ctx->stream;
    const int m = b.m, k = out->iters;
    double* hd = reinterpret_cast<double*>(ctx->pinned);
    static_assert(kChebProbe + 1 <= 32, "probe history must fit the pinned staging");
    HIPCHK(hipMemcpyAsync(hd, b.cd + PD_HIST, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hd + 32, b.ahist, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double dg[kChebProbe], of[kChebProbe];
    for (int i = 0; i < k; ++i) {
        const double beta_prev = i > 0 ? (hd[i] / hd[i - 1]) * (hd[i] / hd[i - 1]) : 0.0;
        dg[i] = 1.0 / hd[32 + i] + (i > 0 ? beta_prev / hd[32 + i - 1] : 0.0);
        if (i + 1 < k) of[i] = (hd[i + 1] / hd[i]) / hd[32 + i];   // sqrt(beta_i) / alpha_i
    }
    double rlo = 0.0, rhi = 0.0;
    tridiag_extremes(dg, of, k, &rlo, &rhi);
    const double lo = kChebLo * rlo, hi = kChebHi * rhi;
    if (!(lo > 0.0) || !(hi > lo) || !is_finite(hi)) return IPM_OK;   // keep the CG result
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), s2 = (delta / theta) * (delta / theta);
    const int par = k & 1;
    double* dy = b.dy[par];
    double* r = b.r[par];
    double* dx = b.dv;
    double* g = b.wv;
    b.maxit = cfg.maxit;
    HIPCHK(launch_fill(dx, m, 0.0, st));
    HIPCHK(launch_fill_i32(b.ci, 2, 0, st));   // PI_DONE, PI_STATUS
    // first batch: the previous solve's step count, capped by the count the residual bound
    // 2 rho^t (rho = (sqrt(kappa)-1)/(sqrt(kappa)+1)) predicts for the remaining reduction (the
    // bound on the estimated interval overshoots by about half, and every queued step after the
    // stop still launches its kernels), then short batches
    const double kap = hi / lo, rc = (std::sqrt(kap) - 1.0) / (std::sqrt(kap) + 1.0);
    const double need = std::log(2.0 * hd[k] / (cfg.tol * std::sqrt(out->rho_star) + 1e-300)) / std::log(1.0 / rc);
    int batch = need < 1e6 ? (int)std::ceil(need) + 1 : 1000000;
    if (ctx->last_cheb_steps > 0 && ctx->last_cheb_steps < batch) batch = ctx->last_cheb_steps;
    if (batch < 4) batch = 4;
    const int* done = b.ci + PI_DONE;
    int t = 0;
    double omega = 1.0;
    int* hi_ = reinterpret_cast<int*>(ctx->pinned);
    for (;;) {
        for (int u = 0; u < batch && k + t <= cfg.maxit; ++u, ++t) {
            omega = t == 0 ? 1.0 : (t == 1 ? 1.0 / (1.0 - 0.5 * s2) : 1.0 / (1.0 - 0.25 * s2 * omega));
            HIPCHK(launch_cheb1(b, r, g, st));
            HIPCHK(launch_cheb2(b, g, dx, dy, omega / theta, omega - 1.0, k + t, t, st));
            StripCall c{};
            c.kind = STRIP_MATVEC;
            c.acc64 = cfg.acc64;
            c.post = POST_SUBR;
            c.vec0 = dx;
            c.d2 = d2;
            c.out0 = r;
            c.done = done;
            CHK(run_pass(ctx, A, c, cfg.acc64 || A->dtype == IPM_F64 ? IPM_KERNEL_MATVEC : IPM_KERNEL_MATVEC32, k + t));
        }
        HIPCHK(hipMemcpyAsync(hi_, b.ci, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hi_[PI_DONE] || k + t > cfg.maxit) break;
        batch = 8;
    }
    const int iters = hi_[PI_DONE] ? hi_[PI_ITERS] : cfg.maxit;
    const int status = hi_[PI_DONE] ? hi_[PI_STATUS] : IPM_PCG_MAXIT;
    HIPCHK(hipMemcpyAsync(hd, b.cd + PD_HIST + iters, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(dy_out, dy, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    out->iters = iters;
    out->status = status;
    out->relres = out->rho_star > 0.0 ? hd[0] / std::sqrt(out->rho_star) : 0.0;
    out->cheb_lo = lo;
    out->cheb_hi = hi;
    ctx->last_cheb_steps = iters - k;
    return IPM_OK;
}

// CG with preconditioner X^T X (X = L^{-1}); dy_out receives the solution. With a warm start the
// solve starts from its combination (kept only if its preconditioned residual is below that of
// the zero start).
int do_pcg(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* X, const double* p, double* dy_out,
           const WarmStart* w0, const ipm_params* prm, const PcgCfg& cfg, PcgOut* out) {
    const int warm = w0 != nullptr ? 1 : 0;
    hipStream_t st = ctx->stream;
    const int m = (int)A->m;
    double* XT = nullptr;
    CHK(ws(ctx, W_XT, (size_t)m * m, &XT));
    if (!cfg.xt_ready) HIPCHK(launch_transpose(X, XT, m, st));
    double *vec = nullptr, *rho = nullptr, *cd = nullptr, *info = nullptr;
    int* ci = nullptr;
    CHK(ws(ctx, W_PCG_VEC, (size_t)8 * m, &vec));
    const int gb = gemv_blocks(m);
    CHK(ws(ctx, W_PCG_RHO, (size_t)2 * gb, &rho));
    CHK(ws(ctx, W_PCG_CD, (size_t)PD_HIST + 2 * (cfg.maxit + 2), &cd));
    const bool cheb = cfg.cheb_probe > 0 && cfg.cheb_probe < cfg.maxit;
    const int cg_maxit = cheb ? cfg.cheb_probe : cfg.maxit;
    CHK(ws(ctx, W_PCG_CI, PI_COUNT, &ci));
    CHK(ws(ctx, W_INFO, 8, &info));
    PcgBufs b{};
    b.m = m;
    b.X = X;
    b.XT = XT;
    b.p = p;
    b.dy[0] = vec;
    b.dy[1] = vec + m;
    b.r[0] = vec + 2 * m;
    b.r[1] = vec + 3 * m;
    b.dv = vec + 4 * m;
    b.q = vec + 5 * m;
    b.wv = vec + 6 * m;
    b.wv2 = vec + 7 * m;
    b.rho_part = rho;
    b.n_rho = gb;
    b.cd = cd;
    b.ci = ci;
    b.tol = cfg.tol;
    b.stag_ratio = prm->stag_ratio;
    b.stag_window = prm->stag_window;
    b.maxit = cg_maxit;
    b.ahist = cheb ? cd + PD_HIST + cfg.maxit + 2 : nullptr;
    HIPCHK(launch_fill_i32(ci, PI_COUNT, 0, st));
    {
        PcgBufs bi = b;   // the start's M dy0 in place of the matvec output
        if (warm) bi.q = const_cast<double*>(w0->q);   // read only by the start kernels
        HIPCHK(launch_pcg_init1(bi, warm, st));
        HIPCHK(launch_pcg_init2(bi, warm, warm ? w0->dy : nullptr, st));
    }
    double* hd = reinterpret_cast<double*>(ctx->pinned);
    int j = 0;
    // first batch: the previous solve's iteration count (CG counts change slowly between IPM
    // iterations); later batches are short so that few no-op launches follow the stop. Every
    // batch ends with the finish kernel (it only reads the CG state), so the batch whose
    // readback shows the stop already carries the result: one synchronization per batch.
    int batch = cheb ? cg_maxit : (*cfg.last_iters > 4 ? *cfg.last_iters : 4);
    const int* done = ci + PI_DONE;
    for (;;) {
        for (int t = 0; t < batch && j < cg_maxit; ++t, ++j) {
            CHK(matvec_pass(ctx, A, d2, b.dv, b.q, done, j, cfg.acc64));
            HIPCHK(launch_pcg_gemv1(b, j, st));
            HIPCHK(launch_pcg_gemv2(b, j, st));
        }
        HIPCHK(launch_pcg_finish(b, dy_out, info, st));
        HIPCHK(hipMemcpyAsync(hd, info, sizeof(double) * 6, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hd[5] != 0.0 || j >= cg_maxit) break;
        batch = 4;
    }
    out->iters = (int)hd[0];
    out->status = (int)hd[1];
    out->warm_used = (int)hd[2];
    out->relres = hd[3];
    out->rho_star = hd[4];
    out->rounds = 1;
    if (cheb && out->status == IPM_PCG_MAXIT && out->iters == cg_maxit)
        CHK(chebyshev_stage(ctx, A, d2, b, cfg, dy_out, out));
    *cfg.last_iters = out->iters;
    resolve_timing(ctx, IPM_KERNEL_MATVEC, out->iters);
    resolve_timing(ctx, IPM_KERNEL_MATVEC32, out->iters);
    resolve_timing(ctx, IPM_KERNEL_SKETCH, INT_MAX);
    return IPM_OK;
}

// ||X v||^2 into *out (device): two launches, no host synchronization.
int precond_norm2(ipm_ctx* ctx, const double* X, int m, const double* v, double* g, double* out) {
    HIPCHK(launch_trigemv(X, m, 1, v, g, ctx->stream));
    HIPCHK(launch_dot(m, g, g, out, ctx->stream));
    return IPM_OK;
}

// Mixed form of the CG solve: iterative refinement. Each round solves M delta = r with inner CG
// whose matvecs read the low-precision A and accumulate in FP32, to the relative tolerance
// inner_tol; then dy += delta and r = p - M dy is recomputed with FP64 accumulation. The stop test
// is the plain method's, ||L^{-1} r|| <= tol_pcg ||L^{-1} p||, on that recomputed residual. A round
// that does not shrink the residual by half (FP32 accumulation error comparable to the
// preconditioned system's scale, late in the IPM) switches the inner solves to FP64 accumulation.
int do_pcg_mixed(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* X, const double* p,
                 double* dy, const WarmStart* w0, const ipm_params* prm, PcgOut* out) {
    hipStream_t st = ctx->stream;
    const int m = (int)A->m;
    double *ref = nullptr, *XT = nullptr;
    CHK(ws(ctx, W_REF, (size_t)4 * m + 8, &ref));
    CHK(ws(ctx, W_XT, (size_t)m * m, &XT));
    double* r = ref;             // true residual p - M dy
    double* delta = ref + m;     // inner solution
    double* g = ref + 2 * m;     // X v
    double* sc = ref + 4 * m;    // [0] ||X p||^2, [1] ||X r||^2, [2] ||X r0||^2 (warm start)
    double* hd = reinterpret_cast<double*>(ctx->pinned) + 64;
    HIPCHK(launch_transpose(X, XT, m, st));
    CHK(precond_norm2(ctx, X, m, p, g, sc));
    out->warm_used = 0;
    if (w0) {
        // residual of the candidates' combination (its product accumulated in FP64)
        HIPCHK(hipMemcpyAsync(r, p, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
        HIPCHK(launch_axpy(m, -1.0, w0->q, r, st));
        CHK(precond_norm2(ctx, X, m, r, g, sc + 2));
        HIPCHK(hipMemcpyAsync(hd, sc, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        out->warm_used = hd[2] < hd[0] ? 1 : 0;
    }
    if (out->warm_used) {
        HIPCHK(hipMemcpyAsync(dy, w0->dy, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    } else {
        HIPCHK(launch_fill(dy, m, 0.0, st));
        HIPCHK(hipMemcpyAsync(r, p, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    }
    bool fp64_inner = A->dtype == IPM_F64;
    int total = 0, rounds = 0, status = IPM_PCG_MAXIT;
    double rn_prev = -1.0, pn = 0.0, rn = 0.0;
    for (;;) {
        CHK(precond_norm2(ctx, X, m, r, g, sc + 1));
        HIPCHK(hipMemcpyAsync(hd, sc, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        pn = std::sqrt(hd[0]);
        rn = std::sqrt(hd[1]);
        if (!is_finite(rn)) {
            status = IPM_ERR_BREAKDOWN;
            break;
        }
        if (rn <= prm->tol_pcg * pn) {
            status = IPM_OK;
            break;
        }
        if (rounds >= prm->max_refine || total >= prm->maxit_pcg) break;
        if (rn_prev > 0.0 && rn > 0.5 * rn_prev) {
            if (fp64_inner) {   // no progress even with FP64 accumulation
                status = IPM_PCG_STAGNATED;
                break;
            }
            fp64_inner = true;
        }
        rn_prev = rn;
        // FP64 rounds aim at the final tolerance directly; FP32 rounds at inner_tol
        const double need = 0.5 * prm->tol_pcg * pn / rn;
        PcgCfg cfg{};
        cfg.tol = fp64_inner ? need : (need > prm->inner_tol ? need : prm->inner_tol);
        cfg.maxit = prm->maxit_pcg - total;
        cfg.acc64 = fp64_inner ? 1 : 0;
        cfg.xt_ready = true;
        cfg.last_iters = fp64_inner ? &ctx->last_pcg_iters : &ctx->last_inner_iters;
        PcgOut io{};
        CHK(do_pcg(ctx, A, d2, X, r, delta, nullptr, prm, cfg, &io));
        total += io.iters;
        ++rounds;
        if (io.status == IPM_ERR_BREAKDOWN) {
            if (fp64_inner) {
                status = IPM_ERR_BREAKDOWN;
                break;
            }
            fp64_inner = true;
            continue;
        }
        HIPCHK(launch_axpy(m, 1.0, delta, dy, st));
        CHK(resid_pass(ctx, A, d2, dy, p, r));
    }
    out->iters = total;
    out->rounds = rounds;
    out->status = status;
    out->relres = pn > 0.0 ? rn / pn : 0.0;
    out->rho_star = pn * pn;
    resolve_timing(ctx, IPM_KERNEL_RESID64, INT_MAX);
    return IPM_OK;
}

// The parameters of the CG solve alone (ipm_pcg_solve).
int check_solver_params(ipm_ctx* ctx, const ipm_params* p) {
    if (p->maxit_pcg < 1 || p->maxit_pcg > 100000) return fail(ctx, IPM_ERR_ARG, "maxit_pcg out of range");
    if (p->stag_window < 1) return fail(ctx, IPM_ERR_ARG, "stag_window must be >= 1");
    if (!(p->tol_pcg >= 0 && is_finite(p->tol_pcg))) return fail(ctx, IPM_ERR_ARG, "bad tol_pcg");
    if (!(p->stag_ratio > 0 && is_finite(p->stag_ratio))) return fail(ctx, IPM_ERR_ARG, "bad stag_ratio");
    if (p->precision != IPM_PLAIN && p->precision != IPM_MIXED && p->precision != IPM_MIXED_F32ACC)
        return fail(ctx, IPM_ERR_ARG, "bad precision");
    if (p->warm_start < IPM_WARM_NONE || p->warm_start > IPM_WARM_GIVEN) return fail(ctx, IPM_ERR_ARG, "bad warm_start");
    if (!(p->inner_tol > 0 && p->inner_tol < 1)) return fail(ctx, IPM_ERR_ARG, "inner_tol must be in (0, 1)");
    if (p->max_refine < 1 || p->max_refine > 1000) return fail(ctx, IPM_ERR_ARG, "max_refine out of range");
    if (p->max_shifts < 0 || p->max_shifts > 8) return fail(ctx, IPM_ERR_ARG, "max_shifts out of range");
    if (p->feasible != 0 && p->feasible != 1) return fail(ctx, IPM_ERR_ARG, "feasible must be 0 or 1");
    if (p->solver != IPM_SOLVER_CG && p->solver != IPM_SOLVER_CHEBYSHEV)
        return fail(ctx, IPM_ERR_ARG, "unknown solver %d", p->solver);
    return IPM_OK;
}

int check_params(ipm_ctx* ctx, const ipm_params* p, int64_t m) {
    if (!p) return fail(ctx, IPM_ERR_ARG, "params is null");
    if (!(p->sigma > 0 && p->sigma < 1)) return fail(ctx, IPM_ERR_ARG, "sigma must be in (0, 1)");
    if (!(p->gamma > 0 && p->gamma < 1)) return fail(ctx, IPM_ERR_ARG, "gamma must be in (0, 1)");
    if (!(p->theta > 0 && p->theta <= 1)) return fail(ctx, IPM_ERR_ARG, "theta must be in (0, 1]");
    if (!(p->tol_pcg >= 0 && is_finite(p->tol_pcg))) return fail(ctx, IPM_ERR_ARG, "bad tol_pcg");
    if (!(p->gap_tol >= 0 && is_finite(p->gap_tol))) return fail(ctx, IPM_ERR_ARG, "bad gap_tol");
    if (!(p->stag_ratio > 0 && is_finite(p->stag_ratio))) return fail(ctx, IPM_ERR_ARG, "bad stag_ratio");
    if (!(is_finite(p->min_step))) return fail(ctx, IPM_ERR_ARG, "bad min_step");
    if (p->maxit_pcg < 1 || p->maxit_pcg > 100000) return fail(ctx, IPM_ERR_ARG, "maxit_pcg out of range");
    if (p->stag_window < 1) return fail(ctx, IPM_ERR_ARG, "stag_window must be >= 1");
    if (p->max_redraws < 0 || p->max_redraws > 6) return fail(ctx, IPM_ERR_ARG, "max_redraws out of range");
    if (p->sketch != IPM_SKETCH_SPARSE && p->sketch != IPM_SKETCH_GAUSSIAN)
        return fail(ctx, IPM_ERR_ARG, "unknown sketch %d", p->sketch);
    if (p->reserved != 0) return fail(ctx, IPM_ERR_ARG, "reserved must be 0");
    if (p->s < 1 || p->s > 8) return fail(ctx, IPM_ERR_ARG, "s must be in 1..8");
    if (p->w < 1 || (p->sketch == IPM_SKETCH_SPARSE && p->w % p->s != 0)) return fail(ctx, IPM_ERR_ARG, "s must divide w");
    if (p->w < m) return fail(ctx, IPM_ERR_ARG, "w (%d) must be >= m (%lld)", p->w, (long long)m);
    return check_solver_params(ctx, p);
}

}  // namespace

extern "C" {

void ipm_params_default(ipm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->sigma = 0.5;
    p->gamma = 0.9;
    p->theta = 0.9999;
    p->tol_pcg = 1e-10;
    p->gap_tol = 1e-8;
    p->min_step = 1e-14;
    p->stag_ratio = 0.99;
    p->w = 0;
    p->s = 2;
    p->maxit_pcg = 500;
    p->stag_window = 10;
    p->max_redraws = 3;
    p->vcorr = 1;
    p->precision = IPM_PLAIN;
    p->warm_start = IPM_WARM_NONE;
    p->inner_tol = 1e-4;
    p->max_refine = 12;
    p->max_shifts = 3;
    p->seed = 0;
}

int ipm_ctx_create(ipm_ctx** out, int device, void* hip_stream) {
    if (!out) return IPM_ERR_ARG;
    *out = nullptr;
    ipm_ctx* ctx = new (std::nothrow) ipm_ctx();
    if (!ctx) return IPM_ERR_NOMEM;
    ctx->device = device;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return IPM_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    if (hipHostMalloc(&ctx->pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return IPM_ERR_HIP;
    }
    if (scratch_address(device, &ctx->scratch) != IPM_OK) {
        (void)hipHostFree(ctx->pinned);
        delete ctx;
        return IPM_ERR_HIP;
    }

    *out = ctx;
    return IPM_OK;
}

void ipm_ctx_destroy(ipm_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int k = 0; k < IPM_KERNEL_COUNT; ++k) resolve_timing(ctx, k, INT_MAX);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    for (int i = 0; i < W_COUNT; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

int ipm_ctx_set_stream(ipm_ctx* ctx, void* hip_stream) {
    if (!ctx) return IPM_ERR_ARG;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return IPM_OK;
}

const char* ipm_last_error(const ipm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ipm_ctx_set_timing(ipm_ctx* ctx, int32_t on) {
    if (!ctx) return IPM_ERR_ARG;
    if (on < 0) return fail(ctx, IPM_ERR_ARG, "timing period must be >= 0");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    for (int k = 0; k < IPM_KERNEL_COUNT; ++k) {
        resolve_timing(ctx, k, INT_MAX);
        ctx->total_ms[k] = 0.0;
        ctx->launches[k] = 0;
    }
    ctx->timing = on != 0;
    ctx->timing_period = on > 0 ? on : 1;
    for (int k = 0; k < IPM_KERNEL_COUNT; ++k) ctx->timing_seq[k] = 0;
    return IPM_OK;
}

int ipm_kernel_time(ipm_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches) {
    if (!ctx || kernel < 0 || kernel >= IPM_KERNEL_COUNT) return IPM_ERR_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "sync failed");
    resolve_timing(ctx, kernel, INT_MAX);
    if (total_ms) *total_ms = ctx->total_ms[kernel];
    if (launches) *launches = ctx->launches[kernel];
    return IPM_OK;
}

int ipm_sketch(ipm_ctx* ctx, const ipm_matrix* A, const double* d, uint64_t seed, int64_t k, int32_t w, int32_t s,
               int32_t out_dtype, void* B) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_matrix(ctx, A));
    if (!d || !B) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (s < 1 || s > 8 || w < 1 || w % s != 0) return fail(ctx, IPM_ERR_ARG, "need 1 <= s <= 8 and s | w");
    if (out_dtype != IPM_F64 && out_dtype != IPM_F32) return fail(ctx, IPM_ERR_ARG, "B must be F64 or F32");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    const HashKeys hk = make_keys(seed, k, w, s);
    CHK(do_sketch(ctx, A, d, 0, hk, w, out_dtype == IPM_F64, B));
    return IPM_OK;
}

int ipm_sketch_gaussian(ipm_ctx* ctx, const ipm_matrix* A, const double* d, uint64_t seed, int64_t k, int32_t w,
                        double* B) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_matrix(ctx, A));
    if (!d || !B) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (w < 1) return fail(ctx, IPM_ERR_ARG, "need w >= 1");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    CHK(do_sketch_gauss(ctx, A, d, 0, gauss_key(seed, k), w, B));
    return IPM_OK;
}

int ipm_precond_factor(ipm_ctx* ctx, int64_t m, int32_t w, int32_t b_dtype, const void* B, double* L, double* Linv,
                       int64_t* bad_pivot) {
    if (!ctx) return IPM_ERR_ARG;
    if (bad_pivot) *bad_pivot = -1;
    if (m < 1 || m > kMaxRows || w < 1 || !B || !Linv)
        return fail(ctx, IPM_ERR_ARG, "bad arguments (need 1 <= m <= %lld, w >= 1, B and Linv set)", (long long)kMaxRows);
    if (b_dtype != IPM_F64 && b_dtype != IPM_F32) return fail(ctx, IPM_ERR_ARG, "B must be F64 or F32");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    double* Lw = L;
    if (!Lw) CHK(ws(ctx, W_L, (size_t)m * m, &Lw));
    int64_t bad = -1;
    double shift = 0.0;
    CHK(do_factor(ctx, (int)m, w, b_dtype == IPM_F64, B, Lw, Linv, 0, &bad, &shift));
    if (bad_pivot) *bad_pivot = bad;
    if (bad >= 0) return fail(ctx, IPM_ERR_NOT_SPD, "Q is not positive definite (pivot %lld)", (long long)bad);
    return IPM_OK;
}

int ipm_pcg_solve(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* Linv, const double* p, double* dy,
                  int32_t warm, const ipm_params* params, ipm_pcg_info* info) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_matrix(ctx, A));
    if (!d2 || !Linv || !p || !dy || !params) return fail(ctx, IPM_ERR_ARG, "null pointer");
    CHK(check_solver_params(ctx, params));
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    PcgOut o{};
    // the caller's dy scaled to its M-norm-optimal multiple (FP64 accumulation)
    WarmStart w0s{};
    if (warm) {
        double* wb = nullptr;
        CHK(ws(ctx, W_WARM, (size_t)2 * A->m, &wb));
        CHK(warm_combination(ctx, A, d2, p, dy, 1, wb, wb + A->m, nullptr));
        w0s = WarmStart{wb, wb + A->m};
    }
    const WarmStart* w0 = warm ? &w0s : nullptr;
    if (params->precision == IPM_MIXED_F32ACC) {
        CHK(do_pcg_mixed(ctx, A, d2, Linv, p, dy, w0, params, &o));
    } else {
        PcgCfg cfg{params->tol_pcg, params->maxit_pcg, 1, false, &ctx->last_pcg_iters};
        cfg.cheb_probe = params->solver == IPM_SOLVER_CHEBYSHEV ? kChebProbe : 0;
        CHK(do_pcg(ctx, A, d2, Linv, p, dy, w0, params, cfg, &o));
    }
    if (info) {
        info->iters = o.iters;
        info->status = o.status;
        info->warm_used = o.warm_used;
        info->rounds = o.rounds;
        info->relres = o.relres;
        info->rho_star = o.rho_star;
    }
    if (o.status == IPM_ERR_BREAKDOWN) return fail(ctx, IPM_ERR_BREAKDOWN, "CG breakdown (d^T M d <= 0)");
    return o.status;
}

int ipm_normal_matvec(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v, double* q) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_matrix(ctx, A));
    if (!d2 || !v || !q) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    CHK(matvec_pass(ctx, A, d2, v, q, nullptr, -1));
    return IPM_OK;
}

int ipm_normal_matvec_noalloc(ipm_ctx* ctx, const ipm_matrix* A, const double* d2, const double* v, double* q) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_matrix(ctx, A));
    if (!d2 || !v || !q) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (!ctx->scratch) return fail(ctx, IPM_ERR_HIP, "no scratch address for device %d", ctx->device);
    StripCall c{};
    c.kind = STRIP_MATVEC;
    c.acc64 = 1;
    c.post = POST_PLAIN;
    c.vec0 = v;
    c.d2 = d2;
    c.out0 = q;
    c.dtype = A->dtype;
    c.A = A->val;
    c.m = (int)A->m;
    c.n = A->n;
    c.ld = A->ld;
    // carve the pass's buffers out of the scratch array; every entry the kernels read is written
    // by the same launch sequence first, so nothing needs clearing
    const size_t nrow = (size_t)rowsum_blocks(c.m);
    size_t need = 0;
    StripPlan pl{};
    if (A->layout == IPM_CSR) {
        need = nrow + (size_t)sparse_col_blocks(A->n) + (size_t)A->n;
    } else {
        pl = strip_plan(A->dtype, c.m, A->n, ctx->num_cu, STRIP_MATVEC);
        need = nrow + (size_t)pl.grid + (size_t)pl.grid * (size_t)c.m;
    }
    if (need > kScratchDoubles)
        return fail(ctx, IPM_ERR_ARG, "this matvec needs %zu bytes of scratch, the static scratch holds %zu",
                    need * sizeof(double), kScratchDoubles * sizeof(double));
    double* p = ctx->scratch;
    c.gpart = p;
    p += nrow;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    if (A->layout == IPM_CSR) {
        c.row_ptr = A->row_ptr;
        c.col_idx = A->col_idx;
        c.csc_val = A->csc_val;
        c.col_ptr = A->col_ptr;
        c.row_idx = A->row_idx;
        c.colpart = p;
        p += sparse_col_blocks(A->n);
        c.coefs = p;
        HIPCHK(launch_sparse_pass(c, ctx->stream));
        return IPM_OK;
    }
    c.colpart = p;
    p += pl.grid;
    c.part = p;
    HIPCHK(launch_strip_pass(c, pl, ctx->stream));
    HIPCHK(launch_strip_rowsum(c, pl, ctx->stream));
    return IPM_OK;
}

int ipm_stream_read(ipm_ctx* ctx, const double* x, int64_t count, double* out) {
    if (!ctx) return IPM_ERR_ARG;
    if (count < 0) return fail(ctx, IPM_ERR_ARG, "count < 0");
    if ((!x && count > 0) || !out) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (reinterpret_cast<uintptr_t>(x) % 16 != 0) return fail(ctx, IPM_ERR_ARG, "x is not 16-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    double* part;
    CHK(ws(ctx, W_STREAM, (size_t)stream_read_parts(count, ctx->num_cu), &part));
    Timer t(ctx, IPM_KERNEL_STREAM_READ);
    HIPCHK(launch_stream_read(x, count, part, out, ctx->num_cu, ctx->stream));
    t.stop();
    return IPM_OK;
}

int ipm_stream_copy(ipm_ctx* ctx, const void* src, void* dst, int64_t bytes) {
    if (!ctx) return IPM_ERR_ARG;
    if (bytes < 0) return fail(ctx, IPM_ERR_ARG, "bytes < 0");
    if (bytes == 0) return IPM_OK;
    if (!src || !dst) return fail(ctx, IPM_ERR_ARG, "null pointer");
    const uintptr_t s = reinterpret_cast<uintptr_t>(src), d = reinterpret_cast<uintptr_t>(dst);
    if (s % 16 != 0 || d % 16 != 0) return fail(ctx, IPM_ERR_ARG, "src or dst is not 16-byte aligned");
    if (bytes > 0 && s < d + (uintptr_t)bytes && d < s + (uintptr_t)bytes)
        return fail(ctx, IPM_ERR_ARG, "src and dst overlap");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    Timer t(ctx, IPM_KERNEL_STREAM_COPY);
    HIPCHK(launch_stream_copy(src, dst, bytes, ctx->num_cu, ctx->stream));
    t.stop();
    return IPM_OK;
}

}  // extern "C"

namespace {

int step_impl(ipm_ctx* ctx, const ipm_problem* prob, ipm_state* state, const ipm_params* prm, const double* dy_given,
              int n_given, ipm_step_info* info) {
    if (!ctx) return IPM_ERR_ARG;
    if (!prob || !state || !info) return fail(ctx, IPM_ERR_ARG, "null pointer");
    std::memset(info, 0, sizeof(*info));
    const ipm_matrix* A = &prob->A;
    CHK(check_matrix(ctx, A));
    CHK(check_params(ctx, prm, A->m));
    if (!prob->b || !prob->c || !state->x || !state->y || !state->s) return fail(ctx, IPM_ERR_ARG, "null vector");
    if (prm->warm_start == IPM_WARM_GIVEN && !dy_given)
        return fail(ctx, IPM_ERR_ARG, "warm_start IPM_WARM_GIVEN needs ipm_step_warm's dy0");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = ctx->stream;
    const int m = (int)A->m;
    const bool mixed = prm->precision != IPM_PLAIN;            // FP32 sketch, B and Gram input
    const bool refine = prm->precision == IPM_MIXED_F32ACC;    // FP32-accumulated inner CG
    const int64_t n = A->n;
    const int Gn = pointwise_blocks(n);

    double *d2, *rd, *ds, *dx, *rp, *p, *dyv, *rhat, *g1, *g2, *scal, *part3, *partmin, *sq;
    CHK(ws(ctx, W_D2, n, &d2));
    CHK(ws(ctx, W_RD, n, &rd));
    CHK(ws(ctx, W_DS, n, &ds));
    CHK(ws(ctx, W_DX, n, &dx));
    CHK(ws(ctx, W_RP, m, &rp));
    CHK(ws(ctx, W_P, m, &p));
    CHK(ws(ctx, W_DY, m, &dyv));
    CHK(ws(ctx, W_RHAT, m, &rhat));
    CHK(ws(ctx, W_G1, m, &g1));
    CHK(ws(ctx, W_G2, m, &g2));
    CHK(ws(ctx, W_SCAL, SC_COUNT, &scal));
    CHK(ws(ctx, W_PART3, (size_t)3 * Gn, &part3));
    CHK(ws(ctx, W_PARTMIN, Gn, &partmin));
    CHK(ws(ctx, W_SQ, 4, &sq));

    // residuals, mu, p and the stop test at the current point (Algorithm 3, step 3)
    HIPCHK(launch_stats(n, state->x, state->s, prob->c, d2, part3, st));
    HIPCHK(launch_fin_stats(n, m, part3, Gn, prob->b, state->y, prm->sigma, scal, st));
    {
        StripCall c{};
        c.kind = STRIP_RESID;
        c.acc64 = 1;
        c.vec0 = state->y;
        c.d2 = d2;
        c.x = state->x;
        c.s = state->s;
        c.c = prob->c;
        c.rd_out = rd;
        c.scal = scal;
        c.post = POST_RESID;
        c.b = prob->b;
        c.out0 = rp;
        c.out1 = p;
        c.outsc = sq;
        c.feasible = prm->feasible;
        CHK(run_pass(ctx, A, c, -1, -1));
    }
    const int set_ref = state->r0norm < 0.0 ? 1 : 0;
    HIPCHK(launch_metrics(n, m, ctx->ws[W_GPART] ? reinterpret_cast<double*>(ctx->ws[W_GPART]) : nullptr,
                          rowsum_blocks(m), sq + 1, set_ref, state->mu0, state->r0norm, prm->feasible, scal, st));
    double* hs = reinterpret_cast<double*>(ctx->pinned);
    HIPCHK(hipMemcpyAsync(hs, scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    info->k = state->k;
    info->mu = hs[SC_MU];
    info->gap = hs[SC_GAP];
    info->relgap = hs[SC_RELGAP];
    info->rp_rel = hs[SC_RPREL];
    info->rd_rel = hs[SC_RDREL];
    info->obj = hs[SC_OBJ];
    if (set_ref) {
        state->mu0 = hs[SC_MU0];
        state->r0norm = hs[SC_R0NORM];
    }
    if (!is_finite(info->mu) || !is_finite(info->relgap)) return fail(ctx, IPM_ERR_ARG, "non-finite iterate or data");
    const double worst = std::fmax(info->relgap, std::fmax(info->rp_rel, info->rd_rel));
    if (worst <= prm->gap_tol) {
        info->status = IPM_CONVERGED;
        return IPM_CONVERGED;
    }

    // initial CG iterate: the previous accepted dy or the caller's, the same for every draw
    const double* dy0 = nullptr;
    int ncand = 0;
    if (prm->warm_start == IPM_WARM_GIVEN) {
        dy0 = dy_given;
        ncand = n_given;
    } else if (prm->warm_start == IPM_WARM_PREV && ctx->prev_m == m) {
        dy0 = reinterpret_cast<const double*>(ctx->ws[W_PREV]);
        ncand = 1;
    }
    // their M-norm-optimal combination and its product (one pass over A for both candidates,
    // FP64 accumulation), shared by every draw
    WarmStart w0s{};
    if (ncand > 0) {
        double* wb = nullptr;
        CHK(ws(ctx, W_WARM, (size_t)2 * m, &wb));
        CHK(warm_combination(ctx, A, d2, p, dy0, ncand, wb, wb + m, nullptr));
        w0s = WarmStart{wb, wb + m};
    }
    const WarmStart* w0 = ncand > 0 ? &w0s : nullptr;

    // Algorithm 1 with redraws of W: sketch, factor, CG. The mixed form keeps a sparse sketch's B
    // in FP32; the Gaussian sketch (an MFMA product) produces B in FP64 in every form.
    const bool gauss = prm->sketch == IPM_SKETCH_GAUSSIAN;
    const int b_f64 = (mixed && !gauss) ? 0 : 1;
    // B is sized for the draw being made: a redraw (w doubled) grows it only when it happens
    void* B = nullptr;
    auto size_b = [&](int wd) -> int {
        if (!b_f64) {
            float* Bf = nullptr;
            CHK(ws(ctx, W_BF, (size_t)m * (size_t)wd, &Bf));
            B = Bf;
        } else {
            double* Bd = nullptr;
            CHK(ws(ctx, W_B, (size_t)m * (size_t)wd, &Bd));
            B = Bd;
        }
        return IPM_OK;
    };
    double *Lw = nullptr, *X = nullptr;
    CHK(ws(ctx, W_L, (size_t)m * m, &Lw));
    CHK(ws(ctx, W_X, (size_t)m * m, &X));
    HashKeys hk{};
    uint64_t gkey = 0;
    int w_used = prm->w, s_used = prm->s;
    PcgOut po{};
    int attempts = 0;
    double shift = 0.0;
    for (int a = 0; a <= prm->max_redraws; ++a) {
        attempts = a + 1;
        w_used = prm->w << a;
        s_used = a == 0 ? prm->s : (prm->s > 2 ? prm->s : 2);
        const uint64_t seed_a = a == 0 ? prm->seed : prm->seed + (uint64_t)a * 0x632BE59BD9B4E019ull;
        hk = make_keys(seed_a, state->k, w_used, s_used);
        gkey = gauss_key(seed_a, state->k);
        CHK(size_b(w_used));
        if (gauss) CHK(do_sketch_gauss(ctx, A, d2, 1, gkey, w_used, reinterpret_cast<double*>(B)));
        else CHK(do_sketch(ctx, A, d2, 1, hk, w_used, b_f64, B));
        int64_t bad = -1;
        CHK(do_factor(ctx, m, w_used, b_f64, B, Lw, X, prm->max_shifts, &bad, &shift));
        if (bad >= 0) {
            if (a == prm->max_redraws) {
                info->attempts = attempts;
                info->status = IPM_ERR_NOT_SPD;
                return fail(ctx, IPM_ERR_NOT_SPD, "Q is not positive definite after %d draws", attempts);
            }
            continue;
        }
        if (refine) {
            CHK(do_pcg_mixed(ctx, A, d2, X, p, dyv, w0, prm, &po));
        } else {
            PcgCfg cfg{prm->tol_pcg, prm->maxit_pcg, 1, false, &ctx->last_pcg_iters};
            cfg.cheb_probe = prm->solver == IPM_SOLVER_CHEBYSHEV ? kChebProbe : 0;
            CHK(do_pcg(ctx, A, d2, X, p, dyv, w0, prm, cfg, &po));
        }
        if (po.status == IPM_ERR_BREAKDOWN) {
            info->status = IPM_ERR_BREAKDOWN;
            return fail(ctx, IPM_ERR_BREAKDOWN, "CG breakdown");
        }
        // a redrawn W whose Q still factors only with a shift is kept: kappa(Q) beyond 1/u then
        // comes from kappa(AD), which further draws do not change (a first draw that needs a
        // shift is redrawn, since a narrow or s = 1 draw can itself leave B nearly rank deficient)
        if (po.status == IPM_OK || (shift > 0.0 && a > 0)) break;
    }
    info->attempts = attempts;
    info->w_used = w_used;
    info->s_used = s_used;
    info->pcg_iters = po.iters;
    info->pcg_status = po.status;
    info->pcg_relres = po.relres;
    info->refine_rounds = po.rounds;
    info->warm_used = po.warm_used;
    info->shift = shift;

    // directions (eq. ipm_inf): ds, true residual, v, dx
    {
        StripCall c{};
        c.kind = STRIP_DIR;
        c.acc64 = 1;
        c.vec0 = dyv;
        c.d2 = d2;
        c.rd = rd;
        c.ds_out = ds;
        c.post = POST_RHAT;
        c.pvec = p;
        c.out0 = rhat;
        c.feasible = prm->feasible;
        CHK(run_pass(ctx, A, c, -1, -1));
    }
    double* u = nullptr;
    CHK(ws(ctx, W_U, (size_t)w_used, &u));
    if (prm->vcorr) {
        double* XT = nullptr;
        CHK(ws(ctx, W_XT, (size_t)m * m, &XT));   // written by do_pcg for this draw
        HIPCHK(launch_trigemv(X, m, 1, rhat, g1, st));
        HIPCHK(launch_trigemv(XT, m, 0, g1, g2, st));
        HIPCHK(launch_btg(B, b_f64, m, w_used, g2, u, st));
    }
    double* wu = nullptr;   // W u for the Gaussian W (the sparse W is applied inside k_dx)
    if (prm->vcorr && gauss) {
        CHK(ws(ctx, W_GU, (size_t)n, &wu));
        HIPCHK(launch_gauss_apply(n, w_used, gkey, u, wu, st));
    }
    HIPCHK(launch_dx(n, state->x, state->s, d2, ds, u, prm->vcorr, hk, wu, scal, dx, part3, st));
    HIPCHK(launch_fin_dx(part3, Gn, scal, st));
    HIPCHK(launch_roots(n, state->x, state->s, dx, ds, prm->gamma, scal, partmin, st));
    HIPCHK(launch_alpha(n, partmin, Gn, prm->gamma, prm->theta, prm->min_step, scal, st));
    HIPCHK(launch_update(n, m, state->x, state->y, state->s, dx, dyv, ds, scal, st));
    HIPCHK(launch_dot(m, dyv, dyv, scal + SC_DY2, st));
    HIPCHK(hipMemcpyAsync(hs, scal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    info->dy_norm = std::sqrt(hs[SC_DY2]);
    info->alpha_max = hs[SC_AMAX];
    info->alpha = hs[SC_ABAR];
    info->vnorm = std::sqrt(hs[SC_V2]);
    if (hs[SC_STALL] != 0.0) {
        info->status = IPM_ERR_STALL;
        return fail(ctx, IPM_ERR_STALL, "step length %.3e below min_step", info->alpha);
    }
    state->k += 1;
    double* prev = nullptr;
    CHK(ws(ctx, W_PREV, (size_t)m, &prev));
    HIPCHK(hipMemcpyAsync(prev, dyv, sizeof(double) * m, hipMemcpyDeviceToDevice, st));
    ctx->prev_m = m;
    info->status = po.status;
    return po.status;
}

}  // namespace

extern "C" {

int ipm_step(ipm_ctx* ctx, const ipm_problem* prob, ipm_state* state, const ipm_params* prm, ipm_step_info* info) {
    return step_impl(ctx, prob, state, prm, nullptr, 0, info);
}

int ipm_step_warm(ipm_ctx* ctx, const ipm_problem* prob, ipm_state* state, const ipm_params* prm, const double* dy0,
                  int32_t ncand, ipm_step_info* info) {
    if (!ctx) return IPM_ERR_ARG;
    if (!dy0) return fail(ctx, IPM_ERR_ARG, "dy0 is null");
    if (ncand < 1 || ncand > 2) return fail(ctx, IPM_ERR_ARG, "ncand must be 1 or 2");
    return step_impl(ctx, prob, state, prm, dy0, ncand, info);
}

}  // extern "C"

// ---- learned warm start ----

namespace {

int check_net(ipm_ctx* ctx, const ipm_mlp* net) {
    if (!net || !net->params) return fail(ctx, IPM_ERR_ARG, "network or its parameters are null");
    if (net->n_out < 1 || net->n_hidden < 1 || net->n_in < 1 || net->n_in > (1 << 20) ||
        net->n_hidden > 8192 || net->n_out > (1 << 20))
        return fail(ctx, IPM_ERR_ARG, "bad network shape (%d, %d, %d)", net->n_in, net->n_hidden, net->n_out);
    return IPM_OK;
}

struct MlpWs {
    float *act1, *act2, *Y, *dY, *dZ2, *dZ1, *feat;
    double *ratio, *loss, *nrm, *work;
    int* hist;
};

int mlp_ws(ipm_ctx* ctx, const ipm_mlp* net, int B, int64_t n, MlpWs* w) {
    const int64_t H = net->n_hidden, O = net->n_out, I = net->n_in;
    float* f = nullptr;
    CHK(ws(ctx, W_MLPF, (size_t)B * (4 * H + 2 * O) + (size_t)I + 64, &f));
    w->act1 = f;
    w->act2 = w->act1 + B * H;
    w->dZ2 = w->act2 + B * H;
    w->dZ1 = w->dZ2 + B * H;
    w->Y = w->dZ1 + B * H;
    w->dY = w->Y + B * O;
    w->feat = w->dY + B * O;
    double* d = nullptr;
    const int fb = n > 0 ? feat_blocks(n) : 1;
    CHK(ws(ctx, W_MLPD, (size_t)B + 8 + 4 * (size_t)fb + 4, &d));
    w->ratio = d;
    w->loss = d + B;
    w->nrm = d + B + 1;
    w->work = d + B + 8;
    CHK(ws(ctx, W_MLPI, 64, &w->hist));
    return IPM_OK;
}

}  // namespace

extern "C" {

int64_t ipm_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out) {
    if (n_in < 1 || n_hidden < 1 || n_out < 1) return -1;
    return mlp_param_count(n_in, n_hidden, n_out);
}

int ipm_mlp_features(ipm_ctx* ctx, int64_t m, int64_t n, const double* dy_prev, const double* x, const double* s,
                     int64_t k, int64_t kmax, float* feat) {
    if (!ctx) return IPM_ERR_ARG;
    if (!dy_prev || !x || !s || !feat) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (m < 1 || m > (1 << 20) || n < 1 || kmax < 1 || k < 0) return fail(ctx, IPM_ERR_ARG, "bad sizes");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    ipm_mlp shape{(int32_t)m + 18, 1, (int32_t)m, 0, nullptr};
    MlpWs w{};
    CHK(mlp_ws(ctx, &shape, 1, n, &w));
    HIPCHK(launch_mlp_features((int)m, n, dy_prev, x, s, (double)k / (double)kmax, w.work, w.hist, feat, nullptr,
                               ctx->stream));
    return IPM_OK;
}

int ipm_mlp_target(ipm_ctx* ctx, int64_t m, const double* dy_prev, const double* dy, float* t) {
    if (!ctx) return IPM_ERR_ARG;
    if (!dy_prev || !dy || !t || m < 1 || m > (1 << 20)) return fail(ctx, IPM_ERR_ARG, "bad arguments");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    HIPCHK(launch_mlp_target((int)m, dy_prev, dy, t, ctx->stream));
    return IPM_OK;
}

int ipm_mlp_forward(ipm_ctx* ctx, const ipm_mlp* net, int32_t batch, const float* X, float* Y) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_net(ctx, net));
    if (batch < 1 || batch > 65536 || !X || !Y) return fail(ctx, IPM_ERR_ARG, "bad batch or null pointer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    MlpWs w{};
    CHK(mlp_ws(ctx, net, batch, 0, &w));
    HIPCHK(launch_mlp_forward(net->n_in, net->n_hidden, net->n_out, net->params, batch, X, w.act1, w.act2, Y,
                              ctx->stream));
    return IPM_OK;
}

int ipm_mlp_backward(ipm_ctx* ctx, const ipm_mlp* net, int32_t batch, const float* X, const float* T, float* grad,
                     double* loss) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_net(ctx, net));
    if (batch < 1 || batch > 65536 || !X || !T || !grad) return fail(ctx, IPM_ERR_ARG, "bad batch or null pointer");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    MlpWs w{};
    CHK(mlp_ws(ctx, net, batch, 0, &w));
    const int I = net->n_in, H = net->n_hidden, O = net->n_out;
    hipStream_t st = ctx->stream;
    HIPCHK(launch_mlp_forward(I, H, O, net->params, batch, X, w.act1, w.act2, w.Y, st));
    HIPCHK(launch_mlp_backward(I, H, O, net->params, batch, X, T, w.act1, w.act2, w.Y, w.dY, w.dZ2, w.dZ1, w.ratio,
                               grad, w.loss, st));
    if (loss) {
        double* hd = reinterpret_cast<double*>(ctx->pinned) + 128;
        HIPCHK(hipMemcpyAsync(hd, w.loss, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *loss = hd[0];
    }
    return IPM_OK;
}

int ipm_mlp_adam(ipm_ctx* ctx, int64_t count, float* params, const float* grad, float* m1, float* m2, int64_t t,
                 double lr, double beta1, double beta2, double eps) {
    if (!ctx) return IPM_ERR_ARG;
    if (count < 1 || !params || !grad || !m1 || !m2 || t < 1) return fail(ctx, IPM_ERR_ARG, "bad Adam arguments");
    if (!(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0 && lr >= 0))
        return fail(ctx, IPM_ERR_ARG, "bad Adam hyperparameters");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow(beta2, (double)t));
    HIPCHK(launch_mlp_adam(count, params, grad, m1, m2, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                           (float)c2, ctx->stream));
    return IPM_OK;
}

int ipm_mlp_predict(ipm_ctx* ctx, const ipm_mlp* net, int64_t n, const double* dy_prev, const double* x,
                    const double* s, int64_t k, int64_t kmax, double* dy0) {
    if (!ctx) return IPM_ERR_ARG;
    CHK(check_net(ctx, net));
    if (net->n_in != net->n_out + 18) return fail(ctx, IPM_ERR_ARG, "n_in must be n_out + 18");
    if (!dy_prev || !x || !s || !dy0) return fail(ctx, IPM_ERR_ARG, "null pointer");
    if (n < 1 || kmax < 1 || k < 0) return fail(ctx, IPM_ERR_ARG, "bad sizes");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    MlpWs w{};
    CHK(mlp_ws(ctx, net, 1, n, &w));
    const int m = net->n_out;
    hipStream_t st = ctx->stream;
    HIPCHK(launch_mlp_features(m, n, dy_prev, x, s, (double)k / (double)kmax, w.work, w.hist, w.feat, w.nrm, st));
    HIPCHK(launch_mlp_forward(net->n_in, net->n_hidden, m, net->params, 1, w.feat, w.act1, w.act2, w.Y, st));
    HIPCHK(launch_mlp_scale_out(m, w.Y, w.nrm, dy0, st));
    return IPM_OK;
}

int ipm_last_dy(ipm_ctx* ctx, int64_t m, double* out) {
    if (!ctx) return IPM_ERR_ARG;
    if (!out) return fail(ctx, IPM_ERR_ARG, "out is null");
    if (ctx->prev_m == 0 || ctx->prev_m != m) return fail(ctx, IPM_ERR_ARG, "no accepted dy of length %lld", (long long)m);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, IPM_ERR_HIP, "hipSetDevice failed");
    HIPCHK(hipMemcpyAsync(out, ctx->ws[W_PREV], sizeof(double) * m, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return IPM_OK;
}

}  // extern "C"
