// Learned warm start of the CG solve: features, a three-layer ReLU network in FP32 (forward,
// backward, Adam) and its prediction. Not part of the paper's method; the CG solve starts from
// the M-norm-optimal combination of the previous direction and the prediction (zero start as
// fallback), so the network changes iteration counts only.
//
// Network: h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3, batch-major
// activations (B x width). y is a second warm-start candidate beside the previous direction. Flat parameters: W1 [H x I], b1 [H], W2 [H x H], b2 [H], W3 [O x H],
// b3 [O]. The layers are small (a few MFLOP per sample), so the products run as LDS-tiled FP32
// SIMT tiles; the IPM's own dense contractions use the MFMA kernels in dense.hip.
#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int FNT = 256;          // threads of the feature kernels
constexpr int NBINS = 64;         // histogram bins of log d^2
constexpr int NLEVELS = 12;       // quantile levels i / 13
constexpr double STAT_SCALE = 0.1;

// ---- features --------------------------------------------------------------------------------

// Per-block sum, min and max of l_j = log(x_j / s_j).
__global__ __launch_bounds__(FNT) void k_feat_pass1(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ s, double* __restrict__ part) {
    __shared__ double sh[FNT / 64];
    double sum = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int64_t j = blockIdx.x * (int64_t)FNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * FNT) {
        const double l = log(x[j] / s[j]);
        sum += l;
        lo = fmin(lo, l);
        hi = fmax(hi, l);
    }
    const double t = block_sum(sum, sh);
    const double mn = block_min(lo, sh);
    const double mx = -block_min(-hi, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t;
        part[gridDim.x + blockIdx.x] = mn;
        part[2 * gridDim.x + blockIdx.x] = mx;
    }
}

// sc[0] mean, sc[1] min, sc[2] max; clears the histogram.
__global__ __launch_bounds__(FNT) void k_feat_fin1(int64_t n, const double* __restrict__ part, int g, double* sc,
                                                   int* hist) {
    __shared__ double sh[FNT / 64];
    double sum = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < g; i += FNT) {
        sum += part[i];
        lo = fmin(lo, part[g + i]);
        hi = fmax(hi, part[2 * g + i]);
    }
    const double t = block_sum(sum, sh);
    const double mn = block_min(lo, sh);
    const double mx = -block_min(-hi, sh);
    if (threadIdx.x < NBINS) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        sc[0] = t / (double)n;
        sc[1] = mn;
        sc[2] = mx;
    }
}

// Per-block sum of (l - mean)^2 and the 64-bin histogram of l on [min, max] (integer counts,
// so the result does not depend on the order of the atomic additions).
__global__ __launch_bounds__(FNT) void k_feat_pass2(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ s, const double* __restrict__ sc,
                                                    double* __restrict__ part2, int* hist) {
    __shared__ double sh[FNT / 64];
    __shared__ int hb[NBINS];
    if (threadIdx.x < NBINS) hb[threadIdx.x] = 0;
    __syncthreads();
    const double mean = sc[0], lo = sc[1], hi = sc[2];
    const double span = hi - lo;
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)FNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * FNT) {
        const double l = log(x[j] / s[j]);
        const double dl = l - mean;
        acc += dl * dl;
        int b = 0;
        if (span > 0.0) {
            const double t = (l - lo) / span * (double)NBINS;
            b = (int)floor(t);
            b = b < 0 ? 0 : (b > NBINS - 1 ? NBINS - 1 : b);
        }
        atomicAdd(&hb[b], 1);
    }
    const double t = block_sum(acc, sh);
    __syncthreads();
    if (threadIdx.x < NBINS && hb[threadIdx.x]) atomicAdd(&hist[threadIdx.x], hb[threadIdx.x]);
    if (threadIdx.x == 0) part2[blockIdx.x] = t;
}

// Assembles the feature vector (FP32) and writes ||dy_prev|| to nrm_out.
__global__ __launch_bounds__(FNT) void k_feat_fin2(int m, int64_t n, const double* __restrict__ dy_prev,
                                                   const double* __restrict__ sc, const double* __restrict__ part2,
                                                   int g, const int* __restrict__ hist, double kfrac,
                                                   float* __restrict__ feat, double* nrm_out) {
    __shared__ double sh[FNT / 64];
    __shared__ double q[NLEVELS];
    double a = 0.0;
    for (int i = threadIdx.x; i < g; i += FNT) a += part2[i];
    const double var = block_sum(a, sh) / (double)n;
    double d = 0.0;
    for (int i = threadIdx.x; i < m; i += FNT) d += dy_prev[i] * dy_prev[i];
    const double nrm = sqrt(block_sum(d, sh));
    const double lo = sc[1], hi = sc[2];
    if (threadIdx.x < NLEVELS) {
        const double level = (double)(threadIdx.x + 1) / 13.0;
        double val = lo;
        if (hi > lo) {
            const double target = level * (double)n;
            const double width = (hi - lo) / (double)NBINS;
            double below = 0.0;
            val = hi;
            for (int b = 0; b < NBINS; ++b) {
                const double c = (double)hist[b];
                if (c > 0.0 && below + c >= target) {
                    val = lo + ((double)b + (target - below) / c) * width;
                    break;
                }
                below += c;
            }
        }
        q[threadIdx.x] = val;
    }
    __syncthreads();
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = threadIdx.x; i < m; i += FNT) feat[i] = (float)(dy_prev[i] * inv);
    if (threadIdx.x == 0) {
        feat[m] = (float)(STAT_SCALE * (nrm > 0.0 ? log(nrm) : 0.0));
        feat[m + 1] = (float)(STAT_SCALE * sc[0]);
        feat[m + 2] = (float)(STAT_SCALE * sqrt(var));
        feat[m + 3] = (float)(STAT_SCALE * lo);
        feat[m + 4] = (float)(STAT_SCALE * hi);
        for (int i = 0; i < NLEVELS; ++i) feat[m + 5 + i] = (float)(STAT_SCALE * q[i]);
        feat[m + 17] = (float)kfrac;
        if (nrm_out) *nrm_out = nrm;
    }
}

// ---- strided FP32 product with fused epilogues ---------------------------------------------

enum Epi { EPI_PLAIN = 0, EPI_BIAS_RELU = 1, EPI_BIAS = 2, EPI_MASK = 3 };

struct GemmArgs {
    int M, N, K;
    const float* A;    // A(i, k) = A[i * sam + k * sak]
    int64_t sam, sak;
    const float* B;    // B(k, j) = B[k * sbk + j * sbn]
    int64_t sbk, sbn;
    float* C;          // C(i, j) = C[i * ldc + j]
    int64_t ldc;
    const float* bias; // [N]
    const float* aux;  // mask source (EPI_MASK): aux[i * ldaux + j] > 0
    int64_t ldaux;
    int epi;
};

constexpr int TM = 64, TN = 64, TK = 16, GT = 256;

// 64 x 64 output tile per block, 4 x 4 per thread, K in steps of 16 through LDS.
__global__ __launch_bounds__(GT) void k_sgemm(GemmArgs g) {
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int tid = threadIdx.x;
    const int tr = tid / 16, tc = tid % 16;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < g.K; k0 += TK) {
        for (int e = tid; e < TK * TM; e += GT) {
            const int kk = e / TM, ii = e % TM;
            const int i = i0 + ii, k = k0 + kk;
            As[kk][ii] = (i < g.M && k < g.K) ? g.A[(int64_t)i * g.sam + (int64_t)k * g.sak] : 0.f;
        }
        for (int e = tid; e < TK * TN; e += GT) {
            const int kk = e / TN, jj = e % TN;
            const int j = j0 + jj, k = k0 + kk;
            Bs[kk][jj] = (j < g.N && k < g.K) ? g.B[(int64_t)k * g.sbk + (int64_t)j * g.sbn] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = As[kk][tr + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][tc + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + tr + 16 * r;
        if (i >= g.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tc + 16 * c;
            if (j >= g.N) continue;
            float v = acc[r][c];
            switch (g.epi) {
                case EPI_BIAS_RELU: v = fmaxf(v + g.bias[j], 0.f); break;
                case EPI_BIAS: v = v + g.bias[j]; break;
                case EPI_MASK: v = g.aux[(int64_t)i * g.ldaux + j] > 0.f ? v : 0.f; break;
                default: break;
            }
            g.C[(int64_t)i * g.ldc + j] = v;
        }
    }
}

hipError_t gemm(const GemmArgs& g, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM);
    hipLaunchKernelGGL(k_sgemm, grid, dim3(GT), 0, st, g);
    return hipGetLastError();
}

// Per-sample loss log(e + LOSS_EPS) with e = 1 - (y^T t)^2 / (||y||^2 ||t||^2), the squared
// sine of the angle between output and target (the CG solve rescales the iterate, so only its
// direction counts; the iterations a warm start saves grow like log(1 / e)). Gradient divided
// by the batch: dY = 2 a / (B yy tt (e + LOSS_EPS)) (a / yy y - t), a = y^T t. One block per
// sample.
constexpr double LOSS_EPS = 1e-10;

__global__ __launch_bounds__(FNT) void k_loss(int B, int O, const float* __restrict__ Y, const float* __restrict__ T,
                                              float* __restrict__ dY, double* __restrict__ ratio) {
    __shared__ double sh[FNT / 64];
    const int b = blockIdx.x;
    const float* y = Y + (int64_t)b * O;
    const float* t = T + (int64_t)b * O;
    double ya = 0.0, y2 = 0.0, t2 = 0.0;
    for (int j = threadIdx.x; j < O; j += FNT) {
        const double yj = y[j], tj = t[j];
        ya += yj * tj;
        y2 += yj * yj;
        t2 += tj * tj;
    }
    const double a = block_sum(ya, sh);
    const double yy = block_sum(y2, sh);
    const double tt = block_sum(t2, sh);
    const bool ok = yy > 0.0 && tt > 0.0;
    const double e = ok ? 1.0 - a * a / (yy * tt) : 1.0;
    const double c = ok ? 2.0 * a / ((double)B * yy * tt * (e + LOSS_EPS)) : 0.0;
    const double r = ok ? a / yy : 0.0;
    for (int j = threadIdx.x; j < O; j += FNT)
        dY[(int64_t)b * O + j] = (float)(c * (r * (double)y[j] - (double)t[j]));
    if (threadIdx.x == 0) ratio[b] = log(e + LOSS_EPS);
}

__global__ __launch_bounds__(FNT) void k_loss_fin(int B, const double* __restrict__ ratio, double* out) {
    __shared__ double sh[FNT / 64];
    double a = 0.0;
    for (int b = threadIdx.x; b < B; b += FNT) a += ratio[b];
    const double t = block_sum(a, sh);
    if (threadIdx.x == 0) *out = t / (double)B;
}

// db[j] = sum_b dZ[b][j]
__global__ __launch_bounds__(FNT) void k_colsum(int B, int N, const float* __restrict__ dZ, float* __restrict__ db) {
    const int j = blockIdx.x * FNT + threadIdx.x;
    if (j >= N) return;
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += dZ[(int64_t)b * N + j];
    db[j] = a;
}

__global__ __launch_bounds__(FNT) void k_adam(int64_t count, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m1, float* __restrict__ m2, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)FNT + threadIdx.x; i < count; i += (int64_t)gridDim.x * FNT) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.f - b1) * gi;
        const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = v;
        p[i] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
    }
}

// dy0 = nrm * y (FP64 output of the batch-1 forward)
__global__ __launch_bounds__(FNT) void k_scale_out(int m, const float* __restrict__ y, const double* __restrict__ nrm,
                                                   double* __restrict__ dy0) {
    const int i = blockIdx.x * FNT + threadIdx.x;
    if (i < m) dy0[i] = nrm[0] * (double)y[i];
}

// Training target of one sample (FP32): t = (dy - (u^T dy) u) / ||dy_prev||, u = dy_prev / ||dy_prev||,
// the part of the new direction that the previous one misses. One block.
__global__ __launch_bounds__(FNT) void k_target(int m, const double* __restrict__ dy_prev, const double* __restrict__ dy,
                                                float* __restrict__ t) {
    __shared__ double sh[FNT / 64];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < m; i += FNT) {
        a += dy_prev[i] * dy_prev[i];
        c += dy_prev[i] * dy[i];
    }
    const double n2 = block_sum(a, sh);
    const double pd = block_sum(c, sh);
    const double nrm = sqrt(n2);
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    const double proj = n2 > 0.0 ? pd / n2 : 0.0;   // (u^T dy) / ||dy_prev||
    for (int i = threadIdx.x; i < m; i += FNT) t[i] = (float)((dy[i] - proj * dy_prev[i]) * inv);
}

struct Layout {
    int64_t W1, b1, W2, b2, W3, b3, total;
};

Layout layout(int I, int H, int O) {
    Layout L{};
    L.W1 = 0;
    L.b1 = L.W1 + (int64_t)H * I;
    L.W2 = L.b1 + H;
    L.b2 = L.W2 + (int64_t)H * H;
    L.W3 = L.b2 + H;
    L.b3 = L.W3 + (int64_t)O * H;
    L.total = L.b3 + O;
    return L;
}

}  // namespace

int64_t mlp_param_count(int I, int H, int O) { return layout(I, H, O).total; }

int feat_blocks(int64_t n) {
    int64_t g = (n + FNT - 1) / FNT;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_mlp_features(int m, int64_t n, const double* dy_prev, const double* x, const double* s,
                               double kfrac, double* work, int* hist, float* feat, double* nrm_out, hipStream_t st) {
    const int g = feat_blocks(n);
    double* part = work;             // [3 g]
    double* part2 = work + 3 * g;    // [g]
    double* sc = work + 4 * g;       // [4]
    hipLaunchKernelGGL(k_feat_pass1, dim3(g), dim3(FNT), 0, st, n, x, s, part);
    hipLaunchKernelGGL(k_feat_fin1, dim3(1), dim3(FNT), 0, st, n, part, g, sc, hist);
    hipLaunchKernelGGL(k_feat_pass2, dim3(g), dim3(FNT), 0, st, n, x, s, sc, part2, hist);
    hipLaunchKernelGGL(k_feat_fin2, dim3(1), dim3(FNT), 0, st, m, n, dy_prev, sc, part2, g, hist, kfrac, feat,
                       nrm_out);
    return hipGetLastError();
}

// Forward pass for a batch: act1 = h1 [B x H], act2 = h2 [B x H], Y [B x O].
hipError_t launch_mlp_forward(int I, int H, int O, const float* theta, int B, const float* X, float* act1,
                              float* act2, float* Y, hipStream_t st) {
    const Layout L = layout(I, H, O);
    GemmArgs g{};
    g.M = B; g.N = H; g.K = I;
    g.A = X; g.sam = I; g.sak = 1;
    g.B = theta + L.W1; g.sbk = 1; g.sbn = I;
    g.C = act1; g.ldc = H;
    g.bias = theta + L.b1; g.epi = EPI_BIAS_RELU;
    hipError_t e = gemm(g, st);
    if (e != hipSuccess) return e;
    g.K = H;
    g.A = act1; g.sam = H;
    g.B = theta + L.W2; g.sbn = H;
    g.C = act2;
    g.bias = theta + L.b2;
    e = gemm(g, st);
    if (e != hipSuccess) return e;
    g.N = O;
    g.A = act2;
    g.B = theta + L.W3;
    g.C = Y; g.ldc = O;
    g.bias = theta + L.b3; g.epi = EPI_BIAS;
    return gemm(g, st);
}

// Backward pass after launch_mlp_forward on the same X: gradient of the mean relative squared
// error into grad (flat, same layout as theta) and the loss into *loss (device).
hipError_t launch_mlp_backward(int I, int H, int O, const float* theta, int B, const float* X, const float* T,
                               const float* act1, const float* act2, const float* Y, float* dY, float* dZ2,
                               float* dZ1, double* ratio, float* grad, double* loss, hipStream_t st) {
    const Layout L = layout(I, H, O);
    hipLaunchKernelGGL(k_loss, dim3(B), dim3(FNT), 0, st, B, O, Y, T, dY, ratio);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(FNT), 0, st, B, ratio, loss);
    GemmArgs g{};
    // dW3 = dY^T h2   [O x H]
    g.M = O; g.N = H; g.K = B;
    g.A = dY; g.sam = 1; g.sak = O;
    g.B = act2; g.sbk = H; g.sbn = 1;
    g.C = grad + L.W3; g.ldc = H; g.epi = EPI_PLAIN;
    hipError_t e = gemm(g, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((O + FNT - 1) / FNT), dim3(FNT), 0, st, B, O, dY, grad + L.b3);
    // dZ2 = (dY W3) * (h2 > 0)   [B x H]
    g = GemmArgs{};
    g.M = B; g.N = H; g.K = O;
    g.A = dY; g.sam = O; g.sak = 1;
    g.B = theta + L.W3; g.sbk = H; g.sbn = 1;
    g.C = dZ2; g.ldc = H;
    g.aux = act2; g.ldaux = H; g.epi = EPI_MASK;
    if ((e = gemm(g, st)) != hipSuccess) return e;
    // dW2 = dZ2^T h1, db2
    g = GemmArgs{};
    g.M = H; g.N = H; g.K = B;
    g.A = dZ2; g.sam = 1; g.sak = H;
    g.B = act1; g.sbk = H; g.sbn = 1;
    g.C = grad + L.W2; g.ldc = H; g.epi = EPI_PLAIN;
    if ((e = gemm(g, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((H + FNT - 1) / FNT), dim3(FNT), 0, st, B, H, dZ2, grad + L.b2);
    // dZ1 = (dZ2 W2) * (h1 > 0)
    g = GemmArgs{};
    g.M = B; g.N = H; g.K = H;
    g.A = dZ2; g.sam = H; g.sak = 1;
    g.B = theta + L.W2; g.sbk = H; g.sbn = 1;
    g.C = dZ1; g.ldc = H;
    g.aux = act1; g.ldaux = H; g.epi = EPI_MASK;
    if ((e = gemm(g, st)) != hipSuccess) return e;
    // dW1 = dZ1^T X, db1
    g = GemmArgs{};
    g.M = H; g.N = I; g.K = B;
    g.A = dZ1; g.sam = 1; g.sak = H;
    g.B = X; g.sbk = I; g.sbn = 1;
    g.C = grad + L.W1; g.ldc = I; g.epi = EPI_PLAIN;
    if ((e = gemm(g, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((H + FNT - 1) / FNT), dim3(FNT), 0, st, B, H, dZ1, grad + L.b1);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(int64_t count, float* p, const float* g, float* m1, float* m2, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st) {
    int64_t blocks = (count + FNT - 1) / FNT;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(FNT), 0, st, count, p, g, m1, m2, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_target(int m, const double* dy_prev, const double* dy, float* t, hipStream_t st) {
    hipLaunchKernelGGL(k_target, dim3(1), dim3(FNT), 0, st, m, dy_prev, dy, t);
    return hipGetLastError();
}

hipError_t launch_mlp_scale_out(int m, const float* y, const double* nrm, double* dy0, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_out, dim3((m + FNT - 1) / FNT), dim3(FNT), 0, st, m, y, nrm, dy0);
    return hipGetLastError();
}

}  // namespace ipmsk
