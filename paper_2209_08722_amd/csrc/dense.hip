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
// published column (x_c = y_c / l_cc, then y_i -= l_ic x_c for i > c), storing X's row c
// (coalesced). L goes back through LDS for a coalesced write. A pivot that is not positive is
// recorded in *status (smallest index wins) and replaced by 1 so the remaining work stays finite.
__global__ __launch_bounds__(128) void k_potrf_diag(double* __restrict__ Lw, int64_t ld, int k0, int kb,
                                                    double* __restrict__ X, int64_t ldx, int* __restrict__ status) {
    __shared__ double col[2][64];
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
            const double lcc = sqrt(piv);
            z[c] = (lane == c) ? lcc : z[c] * (1.0 / lcc);
            cc[lane] = z[c];
            Ls[lane][c] = z[c];            // L[lane][c], final
        }
        __syncthreads();
        if (fac) {
            const double ltc = z[c];
#pragma unroll
            for (int j = c + 1; j < 64; ++j) z[j] = fma(-ltc, cc[j], z[j]);
        } else {
            z[c] = z[c] / cc[c];           // X[c][lane], final
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

}  // namespace

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

hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, v);
    return hipGetLastError();
}

}  // namespace ipmsk
