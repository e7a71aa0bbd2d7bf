// Pointwise and scalar kernels of one IPM iteration (Algorithm 3, Section 5): duality measure,
// stop-test metrics, step lengths alpha_max / alpha_bar and the update.
#include <cfloat>

#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int PNT = 256;

// d2 = x / s and per-block sums of x^T s, c^T x, c^T c.
__global__ __launch_bounds__(PNT) void k_stats(int64_t n, const double* __restrict__ x, const double* __restrict__ s,
                                               const double* __restrict__ c, double* __restrict__ d2,
                                               double* __restrict__ part3) {
    __shared__ double sh[4];
    double xs = 0.0, cx = 0.0, cc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * PNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * PNT) {
        const double xj = x[j], sj = s[j], cj = c[j];
        d2[j] = xj / sj;
        xs += xj * sj;
        cx += cj * xj;
        cc += cj * cj;
    }
    const double t1 = block_sum(xs, sh), t2 = block_sum(cx, sh), t3 = block_sum(cc, sh);
    if (threadIdx.x == 0) {
        part3[3 * blockIdx.x] = t1;
        part3[3 * blockIdx.x + 1] = t2;
        part3[3 * blockIdx.x + 2] = t3;
    }
}

__global__ __launch_bounds__(PNT) void k_fin_stats(int64_t n, int m, const double* __restrict__ part3, int G,
                                                   const double* __restrict__ b, const double* __restrict__ y,
                                                   double sigma, double* __restrict__ scal) {
    __shared__ double sh[4];
    const double xs = sum_partials(part3, G, 3, sh);
    const double cx = sum_partials(part3 + 1, G, 3, sh);
    const double cc = sum_partials(part3 + 2, G, 3, sh);
    double by = 0.0, bb = 0.0;
    for (int i = threadIdx.x; i < m; i += PNT) { by += b[i] * y[i]; bb += b[i] * b[i]; }
    by = block_sum(by, sh);
    bb = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        const double mu = xs / (double)n;
        scal[SC_XS] = xs;
        scal[SC_CTX] = cx;
        scal[SC_C2] = cc;
        scal[SC_MU] = mu;
        scal[SC_SMU] = sigma * mu;
        scal[SC_BTY] = by;
        scal[SC_B2] = bb;
    }
}

// Stop-test quantities at the current point; on the first call (set_ref) also mu0 and ||r0||.
__global__ __launch_bounds__(PNT) void k_metrics(int64_t n, int m, const double* __restrict__ rp2part, int Grp,
                                                 const double* __restrict__ rd2p, int set_ref, double mu0_in,
                                                 double r0_in, int feasible, double* __restrict__ scal) {
    __shared__ double sh[4];
    const double rp2 = sum_partials(rp2part, Grp, 1, sh);
    const double rd2 = *rd2p;
    if (threadIdx.x == 0) {
        const double ctx = scal[SC_CTX], bty = scal[SC_BTY];
        const double gap = ctx - bty;
        scal[SC_RP2] = rp2;
        scal[SC_RD2] = rd2;
        scal[SC_GAP] = gap;
        scal[SC_OBJ] = ctx;
        scal[SC_RELGAP] = fabs(gap) / (1.0 + fabs(ctx));
        scal[SC_RPREL] = sqrt(rp2) / (1.0 + sqrt(scal[SC_B2]));
        scal[SC_RDREL] = sqrt(rd2) / (1.0 + sqrt(scal[SC_C2]));
        const double rn = sqrt(rp2 + rd2);
        scal[SC_RNORM] = rn;
        scal[SC_MU0] = set_ref ? scal[SC_MU] : mu0_in;
        // the feasible N(gamma) has no residual term: a zero reference switches it off
        scal[SC_R0NORM] = feasible ? 0.0 : (set_ref ? rn : r0_in);
    }
}

__global__ __launch_bounds__(PNT) void k_fin_dx(const double* __restrict__ part3, int G, double* __restrict__ scal) {
    __shared__ double sh[4];
    const double a1 = sum_partials(part3, G, 3, sh);
    const double a2 = sum_partials(part3 + 1, G, 3, sh);
    const double v2 = sum_partials(part3 + 2, G, 3, sh);
    if (threadIdx.x == 0) {
        scal[SC_A1] = a1;
        scal[SC_A2] = a2;
        scal[SC_V2] = v2;
    }
}

// Smallest alpha > 0 at which c + b*alpha + a*alpha^2 falls below min(c, 0); DBL_MAX if never.
// A value already negative at 0 (rounding) is measured against its value at 0.
__device__ double first_exit(double c, double b, double a) {
    const double inf = DBL_MAX;
    if (!(c > 0.0)) {   // c <= 0: treated as 0 after the shift
        if (b < 0.0 || (b == 0.0 && a < 0.0)) return 0.0;
        if (a < 0.0) return -b / a;
        return inf;
    }
    if (a == 0.0) return (b < 0.0) ? -c / b : inf;
    const double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return inf;
    const double sq = sqrt(disc);
    const double qq = -0.5 * (b + copysign(sq, b));
    double best = inf;
    const double r1 = qq / a;
    if (r1 > 0.0) best = r1;
    if (qq != 0.0) {
        const double r2 = c / qq;
        if (r2 > 0.0 && r2 < best) best = r2;
    }
    return best;
}

// Per-block minimum over coordinates of the exits of x_i(a) s_i(a) >= (1-gamma) mu(a),
// x_i(a) > 0 and s_i(a) > 0.
__global__ __launch_bounds__(PNT) void k_roots(int64_t n, const double* __restrict__ x, const double* __restrict__ s,
                                               const double* __restrict__ dx, const double* __restrict__ ds,
                                               double gamma, const double* __restrict__ scal,
                                               double* __restrict__ partmin) {
    __shared__ double sh[4];
    const double g1 = 1.0 - gamma;
    const double mu = scal[SC_MU];
    const double a1n = scal[SC_A1] / (double)n, a2n = scal[SC_A2] / (double)n;
    double best = DBL_MAX;
    for (int64_t j = (int64_t)blockIdx.x * PNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * PNT) {
        const double xj = x[j], sj = s[j], dxj = dx[j], dsj = ds[j];
        double r = first_exit(xj * sj - g1 * mu, xj * dsj + sj * dxj - g1 * a1n, dxj * dsj - g1 * a2n);
        r = fmin(r, first_exit(xj, dxj, 0.0));
        r = fmin(r, first_exit(sj, dsj, 0.0));
        best = fmin(best, r);
    }
    const double t = block_min(best, sh);
    if (threadIdx.x == 0) partmin[blockIdx.x] = t;
}

// alpha_max (with the residual term of N(gamma) and the theta backoff) and alpha_bar.
__global__ __launch_bounds__(PNT) void k_alpha(int64_t n, const double* __restrict__ partmin, int G, double gamma,
                                               double theta, double min_step, double* __restrict__ scal) {
    __shared__ double sh[4];
    double best = DBL_MAX;
    for (int i = threadIdx.x; i < G; i += PNT) best = fmin(best, partmin[i]);
    best = block_min(best, sh);
    if (threadIdx.x == 0) {
        const double xs = scal[SC_XS], a1 = scal[SC_A1], a2 = scal[SC_A2];
        const double mu0 = scal[SC_MU0], r0 = scal[SC_R0NORM];
        double amax = fmin(1.0, best);
        if (r0 > 0.0) {
            const double rho = scal[SC_RNORM] / r0;
            const double nm = (double)n * mu0;
            amax = fmin(amax, first_exit(xs / nm - rho, a1 / nm + rho, a2 / nm));
        }
        scal[SC_ROOT] = amax;
        if (amax < 1.0) amax *= theta;
        double abar;
        if (a2 > 0.0) abar = fmin(fmax(-a1 / (2.0 * a2), 0.0), amax);
        else abar = (a1 * amax + a2 * amax * amax <= 0.0) ? amax : 0.0;
        scal[SC_AMAX] = amax;
        scal[SC_ABAR] = abar;
        scal[SC_STALL] = (abar < min_step) ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(PNT) void k_update(int64_t n, int m, double* __restrict__ x, double* __restrict__ y,
                                                double* __restrict__ s, const double* __restrict__ dx,
                                                const double* __restrict__ dy, const double* __restrict__ ds,
                                                const double* __restrict__ scal) {
    if (scal[SC_STALL] != 0.0) return;
    const double a = scal[SC_ABAR];
    for (int64_t j = (int64_t)blockIdx.x * PNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * PNT) {
        x[j] += a * dx[j];
        s[j] += a * ds[j];
    }
    for (int64_t i = (int64_t)blockIdx.x * PNT + threadIdx.x; i < m; i += (int64_t)gridDim.x * PNT) y[i] += a * dy[i];
}

__global__ __launch_bounds__(PNT) void k_axpy(int m, double alpha, const double* __restrict__ x,
                                              double* __restrict__ y) {
    for (int i = blockIdx.x * PNT + threadIdx.x; i < m; i += gridDim.x * PNT) y[i] += alpha * x[i];
}

__global__ __launch_bounds__(PNT) void k_dot(int m, const double* __restrict__ x, const double* __restrict__ y,
                                             double* __restrict__ out) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += PNT) s += x[i] * y[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

hipError_t launch_axpy(int m, double alpha, const double* x, double* y, hipStream_t st) {
    int g = (m + PNT - 1) / PNT;
    if (g > 64) g = 64;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_axpy, dim3(g), dim3(PNT), 0, st, m, alpha, x, y);
    return hipGetLastError();
}

hipError_t launch_dot(int m, const double* x, const double* y, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(PNT), 0, st, m, x, y, out);
    return hipGetLastError();
}

hipError_t launch_stats(int64_t n, const double* x, const double* s, const double* c, double* d2, double* part3,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_stats, dim3(pointwise_blocks(n)), dim3(PNT), 0, st, n, x, s, c, d2, part3);
    return hipGetLastError();
}

hipError_t launch_fin_stats(int64_t n, int m, const double* part3, int G, const double* b, const double* y,
                            double sigma, double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_stats, dim3(1), dim3(PNT), 0, st, n, m, part3, G, b, y, sigma, scal);
    return hipGetLastError();
}

hipError_t launch_metrics(int64_t n, int m, const double* rp2part, int Grp, const double* rd2, int set_ref,
                          double mu0_in, double r0_in, int feasible, double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_metrics, dim3(1), dim3(PNT), 0, st, n, m, rp2part, Grp, rd2, set_ref, mu0_in, r0_in,
                       feasible, scal);
    return hipGetLastError();
}

hipError_t launch_fin_dx(const double* part3, int G, double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_dx, dim3(1), dim3(PNT), 0, st, part3, G, scal);
    return hipGetLastError();
}

hipError_t launch_roots(int64_t n, const double* x, const double* s, const double* dx, const double* ds,
                        double gamma, const double* scal, double* partmin, hipStream_t st) {
    hipLaunchKernelGGL(k_roots, dim3(pointwise_blocks(n)), dim3(PNT), 0, st, n, x, s, dx, ds, gamma, scal, partmin);
    return hipGetLastError();
}

hipError_t launch_alpha(int64_t n, const double* partmin, int G, double gamma, double theta, double min_step,
                        double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_alpha, dim3(1), dim3(PNT), 0, st, n, partmin, G, gamma, theta, min_step, scal);
    return hipGetLastError();
}

hipError_t launch_update(int64_t n, int m, double* x, double* y, double* s, const double* dx, const double* dy,
                         const double* ds, const double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(pointwise_blocks(n)), dim3(PNT), 0, st, n, m, x, y, s, dx, dy, ds, scal);
    return hipGetLastError();
}

}  // namespace ipmsk
