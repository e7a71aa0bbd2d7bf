// Preconditioned CG for A D^2 A^T dy = p with preconditioner Q = L L^T (Algorithm 1, step 3;
// CG on the system of eq. precond_alt written in its preconditioned form, eq. precond).
//
// The preconditioner is applied as two triangular GEMVs with X = L^{-1} and X^T, computed once
// per IPM iteration: z = X^T (X r). The paper's residual norm ||Q^{-1/2} r|| equals ||X r||,
// which is the CG scalar rho = r^T z.
//
// All CG scalars live on the device. One iteration is four launches:
//   matvec pass (strip kernel, then the row reduction of its per-block partials: q = A D^2 A^T d)
//   -> gemv1: d^T q, alpha, dy += alpha d, r -= alpha q, w = X r, partial ||w||^2
//   -> gemv2: rho', beta, d = X^T w + beta d, stop tests.
// A device flag ends the iteration; kernels of later, already queued iterations return at once,
// so the host queues iterations in batches and reads the flag once per batch. dy and r are
// double-buffered by iteration parity because block 0 writes the new values while other blocks
// still read the old ones.
#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int GNT = 256;       // threads per GEMV block
constexpr int GNW = GNT / 64;  // rows in flight per block (one wave per row)

// Row dots of the triangular factors: a lane loads eight of its entries together (predicated),
// then adds them in ascending order, the same sum as one entry at a time.
__device__ __forceinline__ double row_dot_lower(const double* __restrict__ M, int m, int row, const double* xs,
                                                int lane) {
    const double* mr = M + (int64_t)row * m;
    double acc = 0.0;
    for (int l0 = lane; l0 <= row; l0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = l0 + 64 * u <= row ? mr[l0 + 64 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (l0 + 64 * u <= row) acc += v[u] * xs[l0 + 64 * u];
    }
    return wave_sum(acc);
}

__device__ __forceinline__ double row_dot_upper(const double* __restrict__ M, int m, int row, const double* xs,
                                                int lane) {
    const double* mr = M + (int64_t)row * m;
    double acc = 0.0;
    for (int l0 = row + lane; l0 < m; l0 += 64 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = l0 + 64 * u < m ? mr[l0 + 64 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (l0 + 64 * u < m) acc += v[u] * xs[l0 + 64 * u];
    }
    return wave_sum(acc);
}

// The first 512 entries of a wave's row are loaded into registers before the block-wide
// reductions and the staging of the vector, so their latency overlaps that work.
constexpr int PRE = 8;

__device__ __forceinline__ void preload_lower(const double* __restrict__ M, int m, int row, int lane, double* mv) {
    const double* mr = M + (int64_t)row * m;
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        const int l = lane + 64 * u;
        mv[u] = (row < m && l <= row) ? mr[l] : 0.0;
    }
}

// Beyond the preloaded entries a lane loads RU entries of its row together (predicated), then
// adds them in ascending order: the same sums as one entry at a time, with one round trip per
// RU entries instead of one per entry (rows of thousands of entries at m = 2000 and 5000).
constexpr int RU = 8;

__device__ __forceinline__ double finish_lower(const double* __restrict__ M, int m, int row, const double* xs,
                                               int lane, const double* mv) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        const int l = lane + 64 * u;
        if (l <= row) acc += mv[u] * xs[l];
    }
    const double* mr = M + (int64_t)row * m;
    for (int l0 = lane + 64 * PRE; l0 <= row; l0 += 64 * RU) {
        double v[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + 64 * u;
            v[u] = l <= row ? mr[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + 64 * u;
            if (l <= row) acc += v[u] * xs[l];
        }
    }
    return wave_sum(acc);
}

__device__ __forceinline__ void preload_upper(const double* __restrict__ M, int m, int row, int lane, double* mv) {
    const double* mr = M + (int64_t)row * m;
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        const int l = row + lane + 64 * u;
        mv[u] = (row < m && l < m) ? mr[l] : 0.0;
    }
}

__device__ __forceinline__ double finish_upper(const double* __restrict__ M, int m, int row, const double* xs,
                                               int lane, const double* mv) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < PRE; ++u) {
        const int l = row + lane + 64 * u;
        if (l < m) acc += mv[u] * xs[l];
    }
    const double* mr = M + (int64_t)row * m;
    for (int l0 = row + lane + 64 * PRE; l0 < m; l0 += 64 * RU) {
        double v[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + 64 * u;
            v[u] = l < m ? mr[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + 64 * u;
            if (l < m) acc += v[u] * xs[l];
        }
    }
    return wave_sum(acc);
}

// Warm start from up to two candidate vectors v1, v2 with q_i = M v_i: the combination
// alpha v1 + beta v2 closest to the solution in the M-norm (Galerkin condition on the span:
// [v1'q1 v1'q2; v1'q2 v2'q2] [alpha; beta] = [v1'p; v2'p]). When the candidates are nearly
// parallel in the M-norm (det <= 1e-8 a11 a22) or one of them has a non-positive M-norm, the
// single-vector rule alpha = v1'p / v1'q1 (or the same for v2) is used. Writes
// dy_out = alpha v1 + beta v2 (may alias v1), q_out = alpha q1 + beta q2 (may alias q1) and, if
// r_out is given, r_out = p - q_out. One block: the vectors have m entries.
__global__ __launch_bounds__(GNT) void k_warm_galerkin(int m, int nc, const double* v1, const double* v2,
                                                        const double* __restrict__ p, const double* q1,
                                                        const double* q2, double* dy_out, double* q_out,
                                                        double* r_out) {
    __shared__ double sh[GNW];
    double s11 = 0.0, s12 = 0.0, s22 = 0.0, s1p = 0.0, s2p = 0.0;
    for (int l = threadIdx.x; l < m; l += GNT) {
        s11 += v1[l] * q1[l];
        s1p += v1[l] * p[l];
        if (nc > 1) {
            s12 += v1[l] * q2[l];
            s22 += v2[l] * q2[l];
            s2p += v2[l] * p[l];
        }
    }
    const double a11 = block_sum(s11, sh), b1 = block_sum(s1p, sh);
    const double a12 = block_sum(s12, sh), a22 = block_sum(s22, sh), b2 = block_sum(s2p, sh);
    double alpha = 0.0, beta = 0.0;
    const double det = a11 * a22 - a12 * a12;
    if (nc > 1 && a11 > 0.0 && a22 > 0.0 && det > 1e-8 * a11 * a22) {
        alpha = (b1 * a22 - b2 * a12) / det;
        beta = (a11 * b2 - a12 * b1) / det;
    } else if (a11 > 0.0) {
        alpha = b1 / a11;
    } else if (nc > 1 && a22 > 0.0) {
        beta = b2 / a22;
    }
    if (!isfinite(alpha) || !isfinite(beta)) alpha = beta = 0.0;
    for (int l = threadIdx.x; l < m; l += GNT) {
        const double ql = nc > 1 ? alpha * q1[l] + beta * q2[l] : alpha * q1[l];
        const double dl = nc > 1 ? alpha * v1[l] + beta * v2[l] : alpha * v1[l];
        q_out[l] = ql;
        dy_out[l] = dl;
        if (r_out) r_out[l] = p[l] - ql;
    }
}

__global__ __launch_bounds__(GNT) void k_pcg_init1(PcgBufs b, int warm) {
    extern __shared__ double xs[];   // [2][m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int l = tid; l < m; l += GNT) {
        xs[l] = b.p[l];
        if (warm) xs[m + l] = b.p[l] - b.q[l];
    }
    __syncthreads();
    double s1 = 0.0, s2 = 0.0;
    for (int row = blockIdx.x * GNW + wid; row < m; row += gridDim.x * GNW) {
        const double w1 = row_dot_lower(b.X, m, row, xs, lane);
        if (lane == 0) { b.wv[row] = w1; s1 += w1 * w1; }
        if (warm) {
            const double w2 = row_dot_lower(b.X, m, row, xs + m, lane);
            if (lane == 0) { b.wv2[row] = w2; s2 += w2 * w2; }
        }
    }
    const double t1 = block_sum(s1, sh);
    const double t2 = block_sum(s2, sh);
    if (tid == 0) { b.rho_part[2 * blockIdx.x] = t1; b.rho_part[2 * blockIdx.x + 1] = t2; }
}

__global__ __launch_bounds__(GNT) void k_pcg_init2(PcgBufs b, int warm, const double* __restrict__ dy_in) {
    extern __shared__ double xs[];   // [m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const double rs = sum_partials(b.rho_part, b.n_rho, 2, sh);
    const double rr = warm ? sum_partials(b.rho_part + 1, b.n_rho, 2, sh) : 0.0;
    const bool use_warm = warm && (rr < rs);
    const double rho0 = use_warm ? rr : rs;
    for (int l = tid; l < m; l += GNT) {
        xs[l] = use_warm ? b.wv2[l] : b.wv[l];
        if (blockIdx.x == 0) {
            b.r[0][l] = use_warm ? b.p[l] - b.q[l] : b.p[l];
            b.dy[0][l] = use_warm ? dy_in[l] : 0.0;
        }
    }
    __syncthreads();
    for (int row = blockIdx.x * GNW + wid; row < m; row += gridDim.x * GNW) {
        const double z = row_dot_upper(b.XT, m, row, xs, lane);
        if (lane == 0) b.dv[row] = z;
    }
    if (blockIdx.x == 0 && tid == 0) {
        b.cd[PD_RHO0] = rho0;
        b.cd[PD_RHOSTAR] = rs;
        b.cd[PD_HIST] = sqrt(rho0);
        b.ci[PI_WARM] = use_warm ? 1 : 0;
        b.ci[PI_ITERS] = 0;
        b.ci[PI_STATUS] = 0;
        b.ci[PI_DONE] = (sqrt(rho0) <= b.tol * sqrt(rs)) ? 1 : 0;
    }
}

__global__ __launch_bounds__(GNT) void k_pcg_gemv1(PcgBufs b, int j) {
    if (b.ci[PI_DONE]) return;
    extern __shared__ double xs[];   // [m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int par = j & 1;
    const int row0 = blockIdx.x * GNW + wid;
    double mv[PRE];
    preload_lower(b.X, m, row0, lane, mv);
    double dqp = 0.0;
    for (int l0 = tid; l0 < m; l0 += GNT * RU) {   // loads RU at a time, added in ascending order
        double dvv[RU], qv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int l = l0 + GNT * u;
            dvv[u] = l < m ? b.dv[l] : 0.0;
            qv[u] = l < m ? b.q[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (l0 + GNT * u < m) dqp += dvv[u] * qv[u];
    }
    const double dq = block_sum(dqp, sh);
    if (!(dq > 0.0)) {
        if (blockIdx.x == 0 && tid == 0) {
            b.ci[PI_STATUS] = -4;   // IPM_ERR_BREAKDOWN
            b.ci[PI_ITERS] = j;
            b.ci[PI_DONE] = 1;
        }
        return;
    }
    const double alpha = b.cd[PD_RHO0 + par] / dq;
    if (b.ahist != nullptr && blockIdx.x == 0 && tid == 0) b.ahist[j] = alpha;
    const double* __restrict__ rin = b.r[par];
    constexpr int VU = 4;
    for (int l0 = tid; l0 < m; l0 += GNT * VU) {
        double rv[VU], qv[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
            const int l = l0 + GNT * u;
            rv[u] = l < m ? rin[l] : 0.0;
            qv[u] = l < m ? b.q[l] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
            const int l = l0 + GNT * u;
            if (l < m) xs[l] = rv[u] - alpha * qv[u];
        }
        if (blockIdx.x == 0) {
            double yv[VU], dvv[VU];
#pragma unroll
            for (int u = 0; u < VU; ++u) {
                const int l = l0 + GNT * u;
                yv[u] = l < m ? b.dy[par][l] : 0.0;
                dvv[u] = l < m ? b.dv[l] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < VU; ++u) {
                const int l = l0 + GNT * u;
                if (l < m) {
                    b.r[par ^ 1][l] = rv[u] - alpha * qv[u];
                    b.dy[par ^ 1][l] = yv[u] + alpha * dvv[u];
                }
            }
        }
    }
    __syncthreads();
    double s = 0.0;
    for (int row = row0; row < m; row += gridDim.x * GNW) {
        if (row != row0) preload_lower(b.X, m, row, lane, mv);
        const double w = finish_lower(b.X, m, row, xs, lane, mv);
        if (lane == 0) { b.wv[row] = w; s += w * w; }
    }
    const double tt = block_sum(s, sh);
    if (tid == 0) b.rho_part[blockIdx.x] = tt;
}

__global__ __launch_bounds__(GNT) void k_pcg_gemv2(PcgBufs b, int j) {
    if (b.ci[PI_DONE]) return;
    extern __shared__ double xs[];   // [m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int par = j & 1;
    const int row0 = blockIdx.x * GNW + wid;
    double mv[PRE];
    preload_upper(b.XT, m, row0, lane, mv);
    const double rho_new = sum_partials(b.rho_part, b.n_rho, 1, sh);
    const double beta = rho_new / b.cd[PD_RHO0 + par];
    for (int l0 = tid; l0 < m; l0 += GNT * RU) {
        double wv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) wv[u] = l0 + GNT * u < m ? b.wv[l0 + GNT * u] : 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (l0 + GNT * u < m) xs[l0 + GNT * u] = wv[u];
    }
    __syncthreads();
    for (int row = row0; row < m; row += gridDim.x * GNW) {
        if (row != row0) preload_upper(b.XT, m, row, lane, mv);
        const double z = finish_upper(b.XT, m, row, xs, lane, mv);
        if (lane == 0) b.dv[row] = z + beta * b.dv[row];
    }
    if (blockIdx.x == 0 && tid == 0) {
        const double res = sqrt(rho_new);
        double* hist = b.cd + PD_HIST;
        hist[j + 1] = res;
        b.cd[PD_RHO0 + (par ^ 1)] = rho_new;
        const int it = j + 1;
        int stop = 0, status = 0;
        if (res <= b.tol * sqrt(b.cd[PD_RHOSTAR])) {
            stop = 1;
        } else if (it >= b.stag_window && res > b.stag_ratio * hist[it - b.stag_window]) {
            stop = 1; status = 3;   // IPM_PCG_STAGNATED
        } else if (it >= b.maxit) {
            stop = 1; status = 2;   // IPM_PCG_MAXIT
        }
        if (stop) {
            b.ci[PI_STATUS] = status;
            b.ci[PI_ITERS] = it;
            b.ci[PI_DONE] = 1;
        }
    }
}

// Chebyshev, first GEMV: g = X r, per-block ||g||^2 into rho_part.
__global__ __launch_bounds__(GNT) void k_cheb1(PcgBufs b, const double* __restrict__ r, double* __restrict__ g) {
    if (b.ci[PI_DONE]) return;
    extern __shared__ double xs[];   // [m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int row0 = blockIdx.x * GNW + wid;
    double mv[PRE];
    preload_lower(b.X, m, row0, lane, mv);
    for (int l = tid; l < m; l += GNT) xs[l] = r[l];
    __syncthreads();
    double s = 0.0;
    for (int row = row0; row < m; row += gridDim.x * GNW) {
        if (row != row0) preload_lower(b.X, m, row, lane, mv);
        const double w = finish_lower(b.X, m, row, xs, lane, mv);
        if (lane == 0) { g[row] = w; s += w * w; }
    }
    const double tt = block_sum(s, sh);
    if (tid == 0) b.rho_part[blockIdx.x] = tt;
}

// Chebyshev, second GEMV: every block evaluates the stop test from the partials (so all blocks
// take the same decision); unless it stops, z = X^T g, dx = c1 z + c2 dx and dy += dx for the
// block's rows. jt is the total iteration count (CG probe + Chebyshev steps), t the Chebyshev
// step (the residual of step 0 is CG's last one, already in the history).
__global__ __launch_bounds__(GNT) void k_cheb2(PcgBufs b, const double* __restrict__ g, double* __restrict__ dx,
                                               double* __restrict__ dy, double c1, double c2, int jt, int t) {
    if (b.ci[PI_DONE]) return;
    extern __shared__ double xs[];   // [m]
    __shared__ double sh[GNW];
    const int m = b.m, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int row0 = blockIdx.x * GNW + wid;
    double mv[PRE];
    preload_upper(b.XT, m, row0, lane, mv);
    const double res = sqrt(sum_partials(b.rho_part, b.n_rho, 1, sh));
    double* hist = b.cd + PD_HIST;
    int stop = 0, status = 0;
    if (res <= b.tol * sqrt(b.cd[PD_RHOSTAR])) {
        stop = 1;
    } else if (t > 0 && jt >= b.stag_window && res > b.stag_ratio * hist[jt - b.stag_window]) {
        stop = 1; status = 3;   // IPM_PCG_STAGNATED
    } else if (jt >= b.maxit) {
        stop = 1; status = 2;   // IPM_PCG_MAXIT
    }
    if (blockIdx.x == 0 && tid == 0) {
        if (t > 0) hist[jt] = res;
        if (stop) {
            b.ci[PI_STATUS] = status;
            b.ci[PI_ITERS] = jt;
            b.ci[PI_DONE] = 1;
        }
    }
    if (stop) return;
    for (int l = tid; l < m; l += GNT) xs[l] = g[l];
    __syncthreads();
    for (int row = row0; row < m; row += gridDim.x * GNW) {
        if (row != row0) preload_upper(b.XT, m, row, lane, mv);
        const double z = finish_upper(b.XT, m, row, xs, lane, mv);
        if (lane == 0) {
            const double d = c1 * z + c2 * dx[row];
            dx[row] = d;
            dy[row] += d;
        }
    }
}

__global__ __launch_bounds__(GNT) void k_pcg_finish(PcgBufs b, double* __restrict__ dy_out,
                                                    double* __restrict__ info) {
    const int it = b.ci[PI_ITERS];
    const double* src = b.dy[it & 1];
    for (int l = blockIdx.x * GNT + threadIdx.x; l < b.m; l += gridDim.x * GNT) dy_out[l] = src[l];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double rs = b.cd[PD_RHOSTAR];
        info[0] = (double)it;
        info[1] = (double)b.ci[PI_STATUS];
        info[2] = (double)b.ci[PI_WARM];
        info[3] = rs > 0.0 ? b.cd[PD_HIST + it] / sqrt(rs) : 0.0;
        info[4] = rs;
        info[5] = (double)b.ci[PI_DONE];
    }
}

__global__ __launch_bounds__(GNT) void k_trigemv(const double* __restrict__ M, int m, int lower,
                                                 const double* __restrict__ xin, double* __restrict__ yout) {
    extern __shared__ double xs[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int l = tid; l < m; l += GNT) xs[l] = xin[l];
    __syncthreads();
    for (int row = blockIdx.x * GNW + wid; row < m; row += gridDim.x * GNW) {
        const double v = lower ? row_dot_lower(M, m, row, xs, lane) : row_dot_upper(M, m, row, xs, lane);
        if (lane == 0) yout[row] = v;
    }
}

}  // namespace

int gemv_blocks(int m) {
    int g = (m + GNW - 1) / GNW;
    return g > 1024 ? 1024 : g;
}

hipError_t launch_warm_galerkin(int m, int nc, const double* v1, const double* v2, const double* p, const double* q1,
                                const double* q2, double* dy_out, double* q_out, double* r_out, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_galerkin, dim3(1), dim3(GNT), 0, st, m, nc, v1, v2, p, q1, q2, dy_out, q_out, r_out);
    return hipGetLastError();
}

hipError_t launch_pcg_init1(const PcgBufs& b, int warm, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_init1, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * 2 * b.m, st, b, warm);
    return hipGetLastError();
}

hipError_t launch_pcg_init2(const PcgBufs& b, int warm, const double* dy_in, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_init2, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * b.m, st, b, warm, dy_in);
    return hipGetLastError();
}

hipError_t launch_pcg_gemv1(const PcgBufs& b, int j, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_gemv1, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * b.m, st, b, j);
    return hipGetLastError();
}

hipError_t launch_pcg_gemv2(const PcgBufs& b, int j, hipStream_t st) {
    hipLaunchKernelGGL(k_pcg_gemv2, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * b.m, st, b, j);
    return hipGetLastError();
}

hipError_t launch_cheb1(const PcgBufs& b, const double* r, double* g, hipStream_t st) {
    hipLaunchKernelGGL(k_cheb1, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * b.m, st, b, r, g);
    return hipGetLastError();
}

hipError_t launch_cheb2(const PcgBufs& b, const double* g, double* dx, double* dy, double c1, double c2, int jt,
                        int t, hipStream_t st) {
    hipLaunchKernelGGL(k_cheb2, dim3(gemv_blocks(b.m)), dim3(GNT), sizeof(double) * b.m, st, b, g, dx, dy, c1, c2,
                       jt, t);
    return hipGetLastError();
}

hipError_t launch_pcg_finish(const PcgBufs& b, double* dy_out, double* info_out, hipStream_t st) {
    int g = (b.m + GNT - 1) / GNT;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_pcg_finish, dim3(g), dim3(GNT), 0, st, b, dy_out, info_out);
    return hipGetLastError();
}

hipError_t launch_trigemv(const double* M, int m, int lower, const double* xin, double* yout, hipStream_t st) {
    hipLaunchKernelGGL(k_trigemv, dim3(gemv_blocks(m)), dim3(GNT), sizeof(double) * m, st, M, m, lower, xin, yout);
    return hipGetLastError();
}

}  // namespace ipmsk
