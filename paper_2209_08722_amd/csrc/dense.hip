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
    // Tile of this block. The grid is one-dimensional over the tiles (lower tiles only when
    // LOWER), blockIdx.z the split-K slice. Consecutive workgroups go to the chip's 8 XCDs in
    // turn, so workgroup L is given tile (L mod 8) * (T / 8) + L / 8 (remainder spread over the
    // first XCDs): each XCD works through a contiguous band of the row-major tile order, and
    // tiles that read the same row panels of A and B share that XCD's L2.
    const int ntx = (N + BT - 1) / BT;
    const unsigned T = gridDim.x, L = blockIdx.x;
    const unsigned xcd = L % 8u, per = T / 8u, rem = T % 8u;
    const unsigned l = xcd * per + (xcd < rem ? xcd : rem) + L / 8u;
    int ty, tx;
    if (LOWER) {
        ty = (int)((sqrt(8.0 * (double)l + 1.0) - 1.0) * 0.5);
        while ((unsigned)((ty + 1) * (ty + 2) / 2) <= l) ++ty;
        while ((unsigned)(ty * (ty + 1) / 2) > l) --ty;
        tx = (int)l - ty * (ty + 1) / 2;
    } else {
        ty = (int)l / ntx;
        tx = (int)l - ty * ntx;
    }
    const int tm = ty * BT, tn = tx * BT;
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

// Value of lane K of each group of four lanes (DPP quad permutation; K is a constant after the
// step loop is unrolled).
template <int K>
__device__ __forceinline__ double quad_bcast_k(double v) {
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double quad_bcast(double v, int k) {
    switch (k) {
        case 0: return quad_bcast_k<0>(v);
        case 1: return quad_bcast_k<1>(v);
        case 2: return quad_bcast_k<2>(v);
        default: return quad_bcast_k<3>(v);
    }
}

// Factor the kb x kb diagonal block at (k0, k0) of the partially updated matrix in place
// (lower triangle) and write its inverse into X's diagonal block (zero above the diagonal).
// The block is padded to 64 x 64 with the identity (the factor and inverse of diag(A, I) are
// diag(L, I) and diag(L^-1, I)), so no step tests bounds. Eight waves, four threads per row:
// thread (i, q) of waves 0-3 keeps entries 16q..16q+15 of row i of the matrix in registers, thread
// (t, q) of waves 4-7 entries 16q..16q+15 of column t of the inverse. Step p of the right-looking
// factorization eliminates the two columns c = 2p and c + 1 at once. Before its barrier the owners
// (quarter c/16) published column c as updated by the columns before it (colA: the pivot a_cc,
// the a_jc below it, zeros above) and column c + 1 as updated by the columns before c (colB: zeros
// at rows <= c). Every thread forms the two pivots from them: g_a = 1/sqrt(a_cc),
// l1 = l_{c+1,c} = a_{c+1,c} g_a, a' = a_{c+1,c+1} - l1^2, g_b = 1/sqrt(a'). The two rank-1 updates
// a_ij -= l_ic l_jc + l_{i,c+1} l_{j,c+1}, with l_jc = colA[j] g_a and
// l_{j,c+1} = (colB[j] - l_jc l1) g_b, are one pair of FMAs per entry:
// a_ij -= colA[j] s1 + colB[j] s2, s1 = g_a (l_ic - l_{i,c+1} l1 g_b), s2 = l_{i,c+1} g_b, where
// the row thread takes its own a_ic and a_{i,c+1} from the owner lane of its quad (DPP). Entries
// j < c are unchanged (both columns are zero there); entries c and c + 1, where the pair of FMAs
// is not the update, are then overwritten by l_ic and l_{i,c+1}. The inverse threads do the
// matching two steps of the forward substitution L x = e_t: x_c = y_c g_a,
// x_{c+1} = (y_{c+1} - x_c l1) g_b, then y_r -= colA[r] s1 + colB[r] s2 with x in place of l.
// One barrier per two columns; each thread's reads of the two columns are independent, so they
// are all in flight together. A pivot that is not positive is recorded in *status (smallest
// index wins) and replaced by 1 so the remaining work stays finite.
__global__ __launch_bounds__(512) void k_potrf_diag(double* __restrict__ Lw, int64_t ld, int k0, int kb,
                                                    double* __restrict__ X, int64_t ldx, int* __restrict__ status) {
    __shared__ __align__(16) double colb[2][2][64];   // [buffer][colA, colB][row]
    const int tid = threadIdx.x;
    const bool fac = tid < 256;
    const int u = tid & 255;
    const int row = u >> 2;   // row i of the block (factor) or column t of the inverse
    const int q = u & 3;      // quarter: entries 16q .. 16q+15
    double z[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = 16 * q + k;
        double v = (j == row) ? 1.0 : 0.0;
        if (fac && row < kb && j < kb && j <= row) v = Lw[(int64_t)(k0 + row) * ld + k0 + j];
        z[k] = v;
    }
    if (fac && q == 0) {
        colb[0][0][row] = z[0];
        colb[0][1][row] = row > 0 ? z[1] : 0.0;
    }
    __syncthreads();
    int bad = INT_MAX;
#pragma unroll
    for (int c = 0; c < 64; c += 2) {
        const double* ca = colb[(c >> 1) & 1][0];
        const double* cbv = colb[(c >> 1) & 1][1];
        double pa = ca[c];
        if (!(pa > 0.0)) {
            bad = min(bad, k0 + c);
            pa = 1.0;
        }
        const double ga = rsqrt(pa);
        const double l1 = ca[c + 1] * ga;
        double pb = fma(-l1, l1, cbv[c + 1]);
        if (!(pb > 0.0)) {
            bad = min(bad, k0 + c + 1);
            pb = 1.0;
        }
        const double gb = rsqrt(pb);
        double va[16], vb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            va[k] = ca[16 * q + k];
            vb[k] = cbv[16 * q + k];
        }
        const int oq = c >> 4, ok = c & 15;
        const double own0 = quad_bcast(z[ok], oq);
        const double own1 = quad_bcast(z[ok + 1], oq);
        double l0, lb;
        if (fac) {
            l0 = (row == c) ? pa * ga : own0 * ga;                         // l_ic (l_cc on the diagonal)
            lb = (row == c + 1) ? pb * gb : fma(-l0, l1, own1) * gb;     // l_{i,c+1}
        } else {
            l0 = own0 * ga;                                                // x_c
            lb = fma(-l0, l1, own1) * gb;                                  // x_{c+1}
        }
        const double s2 = lb * gb;
        const double s1 = ga * fma(-lb * l1, gb, l0);
#pragma unroll
        for (int k = 0; k < 16; ++k) z[k] = fma(-s1, va[k], fma(-s2, vb[k], z[k]));
        if (q == oq) {
            z[ok] = l0;
            z[ok + 1] = lb;
        }
        if (fac && c + 2 < 64 && q == ((c + 2) >> 4)) {
            const int nk = (c + 2) & 15;
            double* na = colb[((c >> 1) + 1) & 1][0];
            double* nb = colb[((c >> 1) + 1) & 1][1];
            na[row] = row > c + 1 ? z[nk] : 0.0;
            nb[row] = row > c + 2 ? z[nk + 1] : 0.0;
        }
        __syncthreads();
    }
    if (tid == 0 && bad != INT_MAX) atomicMin(status, bad);
    if (row >= kb) return;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int j = 16 * q + k;
        if (j >= kb) continue;
        if (fac) {
            if (j <= row) Lw[(int64_t)(k0 + row) * ld + k0 + j] = z[k];
        } else {
            X[(int64_t)(k0 + j) * ldx + k0 + row] = z[k];   // X[j][t], zero above the diagonal
        }
    }
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
    // LOWER products are square (Gram, trailing updates): the grid covers the lower tiles only
    if (LO && M != N) return hipErrorInvalidValue;
    const int nt = (M + BT - 1) / BT, ntx = (N + BT - 1) / BT;
    const unsigned tiles = LO ? (unsigned)(nt * (nt + 1) / 2) : (unsigned)(nt * ntx);
    const dim3 grid(tiles, 1, ksplit);
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
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(512), 0, st, Lw, ld, k0, kb, X, ldx, status);
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
