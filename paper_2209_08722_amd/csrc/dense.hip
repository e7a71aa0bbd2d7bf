// Dense FP64 linear algebra on the m x m preconditioner (m <= a few thousand):
//   - the Gram product Q = B B^T of the sketch (eqn. pdprecond),
//   - the Cholesky factor Q = L L^T (right-looking, 64-wide panels) and L^{-1},
// all built from one MFMA GEMM kernel (v_mfma_f64_16x16x4f64) and a one-wave kernel that
// factors and inverts a 64 x 64 diagonal block in LDS.
#include <climits>

#include "kernels.hpp"

namespace ipmsk {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int GT = 64;    // output tile edge
constexpr int GK = 16;    // K step staged in LDS

// C[M x N] = alpha * A[M x K] * op(B) (+ beta * C). A row-major (lda); op(B) = B^T with B stored
// N x K (TRANS_B) or B stored K x N. 256 threads = 4 waves in a 2 x 2 grid of 32 x 32 sub-tiles,
// each made of 2 x 2 MFMA 16 x 16 blocks.
// MFMA f64 16x16x4 operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16]; element r
// of lane l's 4-vector result is D[l/16 + 4*r][l%16] (checked on gfx950).
template <bool TRANS_B, bool LOWER, typename TIN>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha, const TIN* A,
                                              int64_t lda, const TIN* __restrict__ B, int64_t ldb, double beta,
                                              double* C, int64_t ldc, int kchunk, int atomic) {
    const int tm = blockIdx.y * GT, tn = blockIdx.x * GT;
    if (LOWER && tn >= tm + GT) return;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    __shared__ double As[GT][GK + 1];
    __shared__ double Bs[GT][GK + 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    d4_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4_t{0.0, 0.0, 0.0, 0.0};

    for (int k0 = kbeg; k0 < kend; k0 += GK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid * 4 + q;
            const int r = e >> 4, kk = e & 15;
            const int gr = tm + r, gk = k0 + kk;
            As[r][kk] = (gr < M && gk < kend) ? (double)A[(int64_t)gr * lda + gk] : 0.0;
        }
        if (TRANS_B) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tid * 4 + q;
                const int r = e >> 4, kk = e & 15;
                const int gn = tn + r, gk = k0 + kk;
                Bs[r][kk] = (gn < N && gk < kend) ? (double)B[(int64_t)gn * ldb + gk] : 0.0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tid * 4 + q;
                const int kk = e >> 6, nn = e & 63;
                const int gn = tn + nn, gk = k0 + kk;
                Bs[nn][kk] = (gn < N && gk < kend) ? (double)B[(int64_t)gk * ldb + gn] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK / 4; ++ks) {
            const int kq = ks * 4 + (lane >> 4);
            const double a0 = As[wr * 32 + (lane & 15)][kq];
            const double a1 = As[wr * 32 + 16 + (lane & 15)][kq];
            const double b0 = Bs[wc * 32 + (lane & 15)][kq];
            const double b1 = Bs[wc * 32 + 16 + (lane & 15)][kq];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = tm + wr * 32 + bi * 16 + (lane >> 4) + 4 * r;
                const int col = tn + wc * 32 + bj * 16 + (lane & 15);
                if (row < M && col < N) {
                    const double v = alpha * acc[bi][bj][r];
                    double* cp = C + (int64_t)row * ldc + col;
                    if (atomic) unsafeAtomicAdd(cp, v);
                    else *cp = (beta == 0.0) ? v : v + beta * (*cp);
                }
            }
}

// Large-tile form for big products (the Gram of a wide sketch, trailing updates of big
// factorizations). C[M x N] = alpha * A[M x K] * op(B) (+ beta * C), op(B) = B^T with B stored
// N x K (TRANS_B) or B stored K x N. 128 x 128 output tile, 256 threads = 4 waves in a 2 x 2 grid
// of 64 x 64 wave tiles, each 4 x 4 MFMA f64 16x16x4 blocks (16 accumulators). K advances in slabs
// of 16: both operand slabs sit in LDS k-major ([k][row], row stride 144 doubles so that the
// 16-row groups read by one MFMA operand fall in disjoint banks), and the next slab is loaded into
// registers while the current one is multiplied, so global latency overlaps the MFMA work. FP32
// inputs are widened when staged. Split-K over gridDim.z with atomic accumulation as in k_gemm.
// Two waves per SIMD (at most 256 registers per lane, accumulators included): measured 1.4x
// faster than the one-wave register allocation on the 5000 x 40000 Gram.
constexpr int BT = 128;   // output tile edge
constexpr int BK = 16;    // K slab
constexpr int BLD = 144;  // LDS row stride (doubles) of the k-major slabs

template <typename TIN>
__device__ __forceinline__ void load8(const TIN* __restrict__ p, bool full, int cnt, double* v) {
    // 8 consecutive elements p[0..7]; all in range if full, else the first cnt (cnt may be <= 0)
    if (full) {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (double)p[q];
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (q < cnt) ? (double)p[q] : 0.0;
    }
}

template <bool TRANS_B, bool LOWER, typename TIN>
__global__ __launch_bounds__(256, 2) void k_gemm_big(int M, int N, int K, double alpha, const TIN* __restrict__ A,
                                                  int64_t lda, const TIN* __restrict__ B, int64_t ldb, double beta,
                                                  double* C, int64_t ldc, int kchunk, int atomic) {
    const int tm = blockIdx.y * BT, tn = blockIdx.x * BT;
    if (LOWER && tn >= tm + BT) return;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    __shared__ double As[BK][BLD];
    __shared__ double Bs[BK][BLD];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    // staging assignment: A slab (128 rows x 16 k): thread -> row tid/2, k half (tid&1)*8.
    // B slab, TRANS_B: same as A over B's rows; otherwise (16 k x 128 n): k row tid/16, 8
    // consecutive n at (tid%16)*8.
    const int sr = tid >> 1, sh = (tid & 1) * 8;
    const int bk_r = tid >> 4, bn_c = (tid & 15) * 8;
    double pa[8], pb[8];
    auto stage = [&](int k0) {
        {
            const int gr = tm + sr, gk = k0 + sh;
            const bool rowok = gr < M;
            const int cnt = rowok ? kend - gk : 0;
            load8<TIN>(A + (int64_t)(rowok ? gr : 0) * lda + (cnt > 0 ? gk : 0), cnt >= 8, cnt, pa);
        }
        if (TRANS_B) {
            const int gn = tn + sr, gk = k0 + sh;
            const bool rowok = gn < N;
            const int cnt = rowok ? kend - gk : 0;
            load8<TIN>(B + (int64_t)(rowok ? gn : 0) * ldb + (cnt > 0 ? gk : 0), cnt >= 8, cnt, pb);
        } else {
            const int gk = k0 + bk_r, gn = tn + bn_c;
            const bool kok = gk < kend;
            const int cnt = kok ? N - gn : 0;
            load8<TIN>(B + (int64_t)(kok ? gk : 0) * ldb + (cnt > 0 ? gn : 0), cnt >= 8, cnt, pb);
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[sh + q][sr] = pa[q];
        if (TRANS_B) {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[sh + q][sr] = pb[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[bk_r][bn_c + q] = pb[q];
        }
    };

    d4_t acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = d4_t{0.0, 0.0, 0.0, 0.0};

    if (kbeg < kend) stage(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();            // previous slab fully consumed
        commit();
        __syncthreads();
        if (k0 + BK < kend) stage(k0 + BK);   // next slab in flight during the MFMAs below
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kq = ks * 4 + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = As[kq][wr * 64 + bi * 16 + (lane & 15)];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) b[bj] = Bs[kq][wc * 64 + bj * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = tm + wr * 64 + bi * 16 + (lane >> 4) + 4 * r;
                const int col = tn + wc * 64 + bj * 16 + (lane & 15);
                if (row < M && col < N) {
                    const double v = alpha * acc[bi][bj][r];
                    double* cp = C + (int64_t)row * ldc + col;
                    if (atomic) unsafeAtomicAdd(cp, v);
                    else *cp = (beta == 0.0) ? v : v + beta * (*cp);
                }
            }
}

// Broadcast lane `lane` of a double held in a VGPR (lane is a compile-time constant here).
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Factor the kb x kb diagonal block at (k0, k0) of the partially updated matrix in place
// (lower triangle) and write its inverse into X's diagonal block (zero above the diagonal).
// Two waves. The block is loaded with coalesced row reads into LDS and padded to 64 x 64 with the
// identity (the factor and inverse of diag(A, I) are diag(L, I) and diag(L^-1, I)), so no step
// below tests bounds. Wave 0, lane t, keeps row t of the matrix in registers: step c of the
// right-looking factorization takes the pivot from lane c, scales column c, publishes it in LDS
// (entry c is l_cc) and updates the row with uniform-address (broadcast) reads of that column; for
// j > t the update only touches the unused upper part. Wave 1, lane t, keeps column t of the
// inverse and does step c of the column-oriented forward substitution L x = e_t with the same
// published column and 1/l_cc (x_c = y_c / l_cc, then y_i -= l_ic x_c for i > c), storing X's row c
// (coalesced). L goes back through LDS for a coalesced write. A pivot that is not positive is
// recorded in *status (smallest index wins) and replaced by 1 so the remaining work stays finite.
__global__ __launch_bounds__(128) void k_potrf_diag(double* __restrict__ Lw, int64_t ld, int k0, int kb,
                                                    double* __restrict__ X, int64_t ldx, int* __restrict__ status) {
    __shared__ double col[2][64];
    __shared__ double rinv[64];          // 1 / l_cc
    __shared__ double Ls[64][65];
    const int lane = threadIdx.x & 63;
    const bool fac = threadIdx.x < 64;   // wave 0 factors, wave 1 inverts
    for (int i = threadIdx.x >> 6; i < 64; i += 2) {
        double v = (i == lane) ? 1.0 : 0.0;
        if (i < kb && lane < kb && lane <= i) v = Lw[(int64_t)(k0 + i) * ld + k0 + lane];
        Ls[i][lane] = v;
    }
    __syncthreads();
    double z[64];   // wave 0: row `lane` of the matrix; wave 1: column `lane` of the inverse
#pragma unroll
    for (int j = 0; j < 64; ++j) z[j] = fac ? Ls[lane][j] : ((j == lane) ? 1.0 : 0.0);
    double* xcol = X + (int64_t)k0 * ldx + k0 + lane;
    const bool xw = !fac && lane < kb;
    int bad = INT_MAX;
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        double* cc = col[c & 1];
        if (fac) {
            double piv = readlane_d(z[c], c);
            if (!(piv > 0.0)) {
                bad = min(bad, k0 + c);
                piv = 1.0;
            }
            // 1/sqrt and sqrt from one reciprocal square root (shorter dependency chain than a
            // square root followed by a division; the factor only has to be accurate to rounding)
            const double inv = rsqrt(piv);
            const double lcc = piv * inv;
            z[c] = (lane == c) ? lcc : z[c] * inv;
            cc[lane] = z[c];
            if (lane == 0) rinv[c] = inv;
            Ls[lane][c] = z[c];            // L[lane][c], final
        }
        __syncthreads();
        if (fac) {
            const double ltc = z[c];
#pragma unroll
            for (int j = c + 1; j < 64; ++j) z[j] = fma(-ltc, cc[j], z[j]);
        } else {
            z[c] = z[c] * rinv[c];         // X[c][lane], final
            if (xw && c < kb) xcol[(int64_t)c * ldx] = z[c];
            const double xc = z[c];
#pragma unroll
            for (int j = c + 1; j < 64; ++j) z[j] = fma(-cc[j], xc, z[j]);
        }
    }
    if (fac && lane == 0 && bad != INT_MAX) atomicMin(status, bad);
    __syncthreads();
    for (int i = threadIdx.x >> 6; i < kb; i += 2)
        if (lane <= i) Lw[(int64_t)(k0 + i) * ld + k0 + lane] = Ls[i][lane];
}

__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ X, double* __restrict__ XT, int m) {
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        tile[r][tx] = (i < m && j < m) ? X[(int64_t)i * m + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bx + r, j = by + tx;   // XT[i][j] = X[j][i]
        if (i < m && j < m) XT[(int64_t)i * m + j] = tile[tx][r];
    }
}

__global__ void k_fill(double* p, int64_t count, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// out = sum_i A[i][i] (one block, fixed summation order).
__global__ __launch_bounds__(256) void k_diag_sum(const double* __restrict__ A, int m, int lda, double* out) {
    __shared__ double sh[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) a += A[(int64_t)i * lda + i];
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) *out = t;
}

__global__ void k_diag_add(double* A, int m, int lda, double delta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) A[(int64_t)i * lda + i] += delta;
}

__global__ void k_fill_2d(double* C, int M, int N, int64_t ldc) {
    const int64_t total = (int64_t)M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        C[(e / N) * ldc + e % N] = 0.0;
}

__global__ void k_fill_i32(int* p, int64_t count, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <bool TB, bool LO, typename TIN>
hipError_t gemm_go(int M, int N, int K, double alpha, const TIN* A, int64_t lda, const TIN* B, int64_t ldb,
                   double beta, double* C, int64_t ldc, int ksplit, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (ksplit < 1) ksplit = 1;
    int kchunk = (K + ksplit - 1) / ksplit;
    kchunk = ((kchunk + GK - 1) / GK) * GK;
    if (kchunk < GK) kchunk = GK;
    ksplit = K > 0 ? (K + kchunk - 1) / kchunk : 1;
    const dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, ksplit);
    IPM_LAUNCH((k_gemm<TB, LO, TIN>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
               ksplit > 1 ? 1 : 0);
    return hipGetLastError();
}

template <bool TB, bool LO, typename TIN>
hipError_t gemm_big_go(int M, int N, int K, double alpha, const TIN* A, int64_t lda, const TIN* B, int64_t ldb,
                       double beta, double* C, int64_t ldc, int ksplit, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (ksplit < 1) ksplit = 1;
    int kchunk = (K + ksplit - 1) / ksplit;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    if (kchunk < BK) kchunk = BK;
    ksplit = K > 0 ? (K + kchunk - 1) / kchunk : 1;
    const dim3 grid((N + BT - 1) / BT, (M + BT - 1) / BT, ksplit);
    IPM_LAUNCH((k_gemm_big<TB, LO, TIN>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
               kchunk, ksplit > 1 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

int gemm_big_tiles(int M, int N, bool lower_only) {
    const int tm = (M + BT - 1) / BT, tn = (N + BT - 1) / BT;
    if (!lower_only) return tm * tn;
    int t = 0;
    for (int i = 0; i < tm; ++i) t += (i + 1 < tn ? i + 1 : tn);
    return t;
}

hipError_t launch_dgemm_big(bool trans_b, bool lower_only, int M, int N, int K, double alpha, const double* A,
                            int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int ksplit,
                            hipStream_t st) {
    if (trans_b) {
        return lower_only ? gemm_big_go<true, true, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st)
                          : gemm_big_go<true, false, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st);
    }
    return lower_only ? gemm_big_go<false, true, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st)
                      : gemm_big_go<false, false, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st);
}

hipError_t launch_sgram_f32_big(int m, int w, const float* B, double* C, int ksplit, hipStream_t st) {
    return gemm_big_go<true, true, float>(m, m, w, 1.0, B, w, B, w, 0.0, C, m, ksplit, st);
}

hipError_t launch_dgemm(bool trans_b, bool lower_only, int M, int N, int K, double alpha, const double* A,
                        int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int ksplit,
                        hipStream_t st) {
    if (trans_b) {
        return lower_only ? gemm_go<true, true, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st)
                          : gemm_go<true, false, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st);
    }
    return lower_only ? gemm_go<false, true, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st)
                      : gemm_go<false, false, double>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ksplit, st);
}

hipError_t launch_sgram_f32(int m, int w, const float* B, double* C, int ksplit, hipStream_t st) {
    return gemm_go<true, true, float>(m, m, w, 1.0, B, w, B, w, 0.0, C, m, ksplit, st);
}

hipError_t launch_potrf_diag(double* Lw, int64_t ld, int k0, int kb, double* X, int64_t ldx, int* status,
                             hipStream_t st) {
    if (kb < 1 || kb > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(128), 0, st, Lw, ld, k0, kb, X, ldx, status);
    return hipGetLastError();
}

hipError_t launch_transpose(const double* X, double* XT, int m, hipStream_t st) {
    const dim3 grid((m + 31) / 32, (m + 31) / 32);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, X, XT, m);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

hipError_t launch_diag_sum(const double* A, int m, int lda, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_sum, dim3(1), dim3(256), 0, st, A, m, lda, out);
    return hipGetLastError();
}

hipError_t launch_diag_add(double* A, int m, int lda, double delta, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_add, dim3((m + 255) / 256), dim3(256), 0, st, A, m, lda, delta);
    return hipGetLastError();
}

hipError_t launch_fill_2d(double* C, int M, int N, int64_t ldc, hipStream_t st) {
    const int64_t total = (int64_t)M * N;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_2d, dim3((unsigned)blocks), dim3(256), 0, st, C, M, N, ldc);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

}  // namespace ipmsk
