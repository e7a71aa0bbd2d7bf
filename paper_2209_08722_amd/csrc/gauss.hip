// Gaussian sketch (the paper's experimental choice, Section 7): B = A D W with W (n x w) of
// i.i.d. N(0, 1/w) entries that are never stored, and W u for the perturbation v (eq. compv).
//
// Entry (j, c) of W, e = j w + c: outputs 2e and 2e+1 of the SplitMix64 stream started at the
// iteration's key give u1 = ((h1 >> 11) + 1) 2^-53 in (0, 1] and u2 = (h2 >> 11) 2^-53 in
// [0, 1); the entry is sqrt(-2 ln u1) cos(2 pi u2) / sqrt(w) (Box-Muller).
//
// The sketch is a dense contraction over n, so it runs on the FP64 MFMA units: 256 x 128 output
// tiles (8 waves of 64 x 64), K slabs of 16 columns of A and the matching 16 rows of W
// generated into LDS by the block itself and scaled by d (B = A (D W)), split-K over gridDim.z with
// atomic accumulation into an FP64 B that the caller cleared. Generating W (two SplitMix64
// outputs, a log, a square root and a cosine in FP64 per entry) costs about as much as the MFMA
// work it feeds, so the tile is tall: each generated entry is used by 256 rows of A (128-row
// tiles ran at 21 TFLOP/s on 500 x 100000 x 2000, generation-bound). The slabs are double-
// buffered in LDS (one barrier per slab). At 256 rows neither unit is saturated (MFMA about 38 %
// busy, vector ALUs about 11 % active) and halving the barriers gained only 3 %: the kernel is
// latency-bound, most likely on the A loads issued one slab ahead.
#include "kernels.hpp"

namespace ipmsk {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int GBM = 256;  // output tile rows
constexpr int GBN = 128;  // output tile columns
constexpr int GKS = 16;   // K slab
constexpr int GNT = 512;  // threads (8 waves in a 4 x 2 grid of 64 x 64)
constexpr int GLDA = 272; // LDS row strides (doubles) of the k-major slabs: = 16 mod 32, so one
constexpr int GLDW = 144; // MFMA operand's 16-row groups fall in disjoint banks

__device__ __forceinline__ double gauss_entry(uint64_t key, uint64_t e, double inv_sqrt_w) {
    const uint64_t h1 = mix64(key + (2ull * e + 1ull) * kPhi);
    const uint64_t h2 = mix64(key + (2ull * e + 2ull) * kPhi);
    const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1p-53;
    const double u2 = (double)(h2 >> 11) * 0x1p-53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2) * inv_sqrt_w;
}

template <typename T>
__global__ __launch_bounds__(GNT, 1) void k_sketch_gauss(int m, int64_t n, int w, const T* __restrict__ A,
                                                         int64_t lda, const double* __restrict__ dv, int d_is_d2,
                                                         uint64_t key, double inv_sqrt_w, double* B, int64_t kchunk,
                                                         int atomic) {
    const int tm = blockIdx.y * GBM, tn = blockIdx.x * GBN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = min(n, kbeg + kchunk);
    __shared__ double As[2][GKS][GLDA];   // double-buffered slabs: one barrier per slab
    __shared__ double Ws[2][GKS][GLDW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int sr = tid >> 1, sh = (tid & 1) * 8;          // A slab: row (of 256), first of 8 columns
    const int wk = tid >> 5, wn = (tid & 31) * 4;         // W slab: row (of 16), first of 4 columns
    double pa[8], pw[4];
    // D scales the rows of W (B = A (D W)): one d_j per W row of the slab, where scaling A would
    // take a load and a square root for every element of every row tile
    auto stage = [&](int64_t k0) {
        const int gr = tm + sr;
        const bool rowok = gr < m;
        const T* arow = A + (int64_t)(rowok ? gr : 0) * lda;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t j = k0 + sh + q;
            pa[q] = (rowok && j < kend) ? (double)Elem<T>::load1(arow + j) : 0.0;
        }
        const int64_t j = k0 + wk;
        double dj = 0.0;
        if (j < kend) {
            const double dd = dv[j];
            dj = d_is_d2 ? sqrt(dd) : dd;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tn + wn + q;
            pw[q] = (j < kend && c < w) ? gauss_entry(key, (uint64_t)j * (uint64_t)w + (uint64_t)c, inv_sqrt_w) * dj
                                        : 0.0;
        }
    };
    auto commit = [&](int bb) {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[bb][sh + q][sr] = pa[q];
#pragma unroll
        for (int q = 0; q < 4; ++q) Ws[bb][wk][wn + q] = pw[q];
    };

    d4_t acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = d4_t{0.0, 0.0, 0.0, 0.0};

    if (kbeg < kend) {
        stage(kbeg);
        commit(0);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += GKS) {
        const bool more = k0 + GKS < kend;
        if (more) stage(k0 + GKS);   // next slab (loads and generation) during the MFMAs
#pragma unroll
        for (int ks = 0; ks < GKS / 4; ++ks) {
            const int kq = ks * 4 + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = As[cur][kq][wr * 64 + bi * 16 + (lane & 15)];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) b[bj] = Ws[cur][kq][wc * 64 + bj * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
        // the other buffer was last read in the previous slab, before the barrier that ended it
        if (more) commit(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = tm + wr * 64 + bi * 16 + (lane >> 4) + 4 * r;
                const int col = tn + wc * 64 + bj * 16 + (lane & 15);
                if (row < m && col < w) {
                    double* cp = B + (int64_t)row * w + col;
                    if (atomic) unsafeAtomicAdd(cp, acc[bi][bj][r]);
                    else *cp = acc[bi][bj][r];
                }
            }
}

// t_j = sum_c W[j][c] u[c]: one wave per row j of W, u staged in LDS in chunks.
constexpr int AU_NT = 256;
constexpr int AU_CHUNK = 8192;
__global__ __launch_bounds__(AU_NT) void k_gauss_apply(int64_t n, int w, uint64_t key, double inv_sqrt_w,
                                                       const double* __restrict__ u, double* __restrict__ t) {
    __shared__ double us[AU_CHUNK];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t j0 = (int64_t)blockIdx.x * (AU_NT / 64); j0 < n; j0 += (int64_t)gridDim.x * (AU_NT / 64)) {
        const int64_t j = j0 + wid;
        double acc = 0.0;
        for (int c0 = 0; c0 < w; c0 += AU_CHUNK) {
            const int cn = min(AU_CHUNK, w - c0);
            __syncthreads();
            for (int c = threadIdx.x; c < cn; c += AU_NT) us[c] = u[c0 + c];
            __syncthreads();
            if (j < n)
                for (int c = lane; c < cn; c += 64)
                    acc += gauss_entry(key, (uint64_t)j * (uint64_t)w + (uint64_t)(c0 + c), inv_sqrt_w) * us[c];
        }
        acc = wave_sum(acc);
        if (j < n && lane == 0) t[j] = acc;
    }
}

template <typename T>
hipError_t gauss_go(int m, int64_t n, int w, const void* A, int64_t lda, const double* dv, int d_is_d2, uint64_t key,
                    double* B, int ksplit, hipStream_t st) {
    if (ksplit < 1) ksplit = 1;
    int64_t kchunk = (n + ksplit - 1) / ksplit;
    kchunk = ((kchunk + GKS - 1) / GKS) * GKS;
    const int64_t ks = (n + kchunk - 1) / kchunk;
    const dim3 grid((w + GBN - 1) / GBN, (m + GBM - 1) / GBM, (unsigned)ks);
    IPM_LAUNCH((k_sketch_gauss<T>), grid, dim3(GNT), 0, st, m, n, w, reinterpret_cast<const T*>(A), lda, dv, d_is_d2,
               key, 1.0 / sqrt((double)w), B, kchunk, ks > 1 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

uint64_t gauss_key(uint64_t seed, int64_t k) { return mix64((seed ^ mix64((uint64_t)k)) + kGaussDomain); }

int gauss_tiles(int m, int w) { return ((m + GBM - 1) / GBM) * ((w + GBN - 1) / GBN); }

hipError_t launch_sketch_gauss(int dtype, int m, int64_t n, int w, const void* A, int64_t lda, const double* dvals,
                               int dvals_are_d2, uint64_t key, double* B, int ksplit, hipStream_t st) {
    switch (dtype) {
        case 0: return gauss_go<double>(m, n, w, A, lda, dvals, dvals_are_d2, key, B, ksplit, st);
        case 1: return gauss_go<float>(m, n, w, A, lda, dvals, dvals_are_d2, key, B, ksplit, st);
        case 2: return gauss_go<bf16_t>(m, n, w, A, lda, dvals, dvals_are_d2, key, B, ksplit, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gauss_apply(int64_t n, int w, uint64_t key, const double* u, double* t, hipStream_t st) {
    int64_t blocks = (n + AU_NT / 64 - 1) / (AU_NT / 64);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gauss_apply, dim3((unsigned)blocks), dim3(AU_NT), 0, st, n, w, key, 1.0 / sqrt((double)w), u,
                       t);
    return hipGetLastError();
}


}  // namespace ipmsk
