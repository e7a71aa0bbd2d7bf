// Single-pass column-strip kernels over row-major A (m x n, row stride ld).
//
// Every pass here has the shape "per column j: dot a_j with one m-vector, turn the dots into
// per-column coefficients; per row i: accumulate sum_j A[i][j] * coef_j". Reading A once per
// pass requires each column strip to stay on chip between the dot and the accumulation, so a
// block owns a strip of SW columns across all m rows, held in registers:
//   - lanes: 8 lanes per row, 16-byte vector loads -> 128 contiguous bytes per row segment;
//   - thread (c, g) holds rows g, g+RG, ... (RG = blockDim/8 row groups) of columns
//     [strip*SW + c*VEC, +VEC);
//   - column dots: per-thread partials, then wave shuffles over the 8 row groups of a wave,
//     then one LDS exchange across waves (double-buffered, one barrier per strip);
//   - row sums: per-thread register accumulators, reduced over the 8 column lanes once at the
//     end of the persistent loop and written as one partial m-vector per block.
// The CG matvec q = A D^2 A^T v (Algorithm 1, step 3) is one such pass; so are the residual
// pass (r_d = A^T y + s - c, then A x and A u for r_p and p, Section 5 / Algorithm 3 step 3) and
// the direction pass (ds = -r_d - A^T dy, then A D^2 A^T dy for the true residual).
#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int LPR = 8;   // lanes per row segment

struct OpMatvec {
    static constexpr int NDOT = 1, NACC = 1, NCR = 0;
    struct S {};
    __device__ static S init(const StripCall&) { return {}; }
    template <typename ACC>
    __device__ static void column(const StripCall& a, const S&, int64_t j, bool valid, bool,
                                  const ACC* dots, ACC* coef, double*) {
        coef[0] = valid ? (ACC)a.d2[j] * dots[0] : (ACC)0;
    }
};

struct OpResid {
    static constexpr int NDOT = 1, NACC = 2, NCR = 1;
    struct S { double smu; };
    __device__ static S init(const StripCall& a) { return S{a.scal[SC_SMU]}; }
    template <typename ACC>
    __device__ static void column(const StripCall& a, const S& st, int64_t j, bool valid, bool writer,
                                  const ACC* dots, ACC* coef, double* cr) {
        if (!valid) { coef[0] = coef[1] = (ACC)0; return; }
        const double sj = a.s[j];
        const double rdj = (double)dots[0] + sj - a.c[j];
        if (writer) { a.rd_out[j] = rdj; cr[0] += rdj * rdj; }
        coef[0] = (ACC)a.x[j];
        coef[1] = (ACC)(st.smu / sj + a.d2[j] * rdj);
    }
};

struct OpDir {
    static constexpr int NDOT = 1, NACC = 1, NCR = 0;
    struct S {};
    __device__ static S init(const StripCall&) { return {}; }
    template <typename ACC>
    __device__ static void column(const StripCall& a, const S&, int64_t j, bool valid, bool writer,
                                  const ACC* dots, ACC* coef, double*) {
        if (!valid) { coef[0] = (ACC)0; return; }
        const double t = (double)dots[0];
        if (writer) a.ds_out[j] = -a.rd[j] - t;
        coef[0] = (ACC)(a.d2[j] * t);
    }
};

template <typename T, typename ACC, int NT, int RPT, class Op>
__global__ __launch_bounds__(NT) void k_strip(StripCall a, int nstrips) {
    constexpr int VEC = Elem<T>::VEC;
    constexpr int SW = LPR * VEC;
    constexpr int RG = NT / LPR;
    constexpr int NW = NT / 64;
    constexpr int ND = Op::NDOT, NA = Op::NACC, NCR = Op::NCR;
    constexpr int MPAD = RG * RPT;

    if (a.done != nullptr && *a.done) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    ACC* vs = reinterpret_cast<ACC*>(smem_raw);          // [MPAD]   vector dotted with columns
    ACC* red = vs + ND * MPAD;                              // [2][NW][SW][ND]
    __shared__ double shr[NW];

    const int tid = threadIdx.x;
    const int c = tid % LPR, g = tid / LPR, lane = tid & 63, wid = tid >> 6;
    const int m = a.m;
    const T* __restrict__ A = reinterpret_cast<const T*>(a.A);

    for (int i = tid; i < MPAD; i += NT) vs[i] = (i < m) ? (ACC)a.vec0[i] : (ACC)0;
    __syncthreads();
    const typename Op::S st = Op::init(a);

    ACC q[NA][RPT];
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
        for (int k = 0; k < RPT; ++k) q[aa][k] = (ACC)0;
    double cr[NCR > 0 ? NCR : 1] = {0.0};

    int buf = 0;
    for (int strip = blockIdx.x; strip < nstrips; strip += gridDim.x) {
        const int64_t j0 = (int64_t)strip * SW + c * VEC;
        const bool full = (j0 + VEC <= a.n);
        ACC av[RPT][VEC];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = g + RG * k;
            if (i < m) {
                const T* ptr = A + (int64_t)i * a.ld + j0;
                if (full) {
                    Elem<T>::template load16<ACC>(ptr, av[k]);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        av[k][e] = (j0 + e < a.n) ? (ACC)Elem<T>::load1(ptr + e) : (ACC)0;
                }
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) av[k][e] = (ACC)0;
            }
        }
        // column dots over this thread's rows
        ACC pd[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) pd[e] = (ACC)0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const ACC vv = vs[g + RG * k];
#pragma unroll
            for (int e = 0; e < VEC; ++e) pd[e] += av[k][e] * vv;
        }
        // over the 8 row groups of this wave (lane bits 3..5)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            ACC v = pd[e];
            v += __shfl_xor(v, 8, 64);
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            pd[e] = v;
        }
        ACC* rb = red + buf * NW * SW;
        if (lane < LPR) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) rb[wid * SW + c * VEC + e] = pd[e];
        }
        __syncthreads();
        ACC coef[NA][VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            ACC t = (ACC)0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += rb[w * SW + c * VEC + e];
            ACC cf[NA];
            const int64_t j = j0 + e;
            Op::template column<ACC>(a, st, j, j < a.n, g == 0, &t, cf, cr);
#pragma unroll
            for (int aa = 0; aa < NA; ++aa) coef[aa][e] = cf[aa];
        }
#pragma unroll
        for (int k = 0; k < RPT; ++k)
#pragma unroll
            for (int aa = 0; aa < NA; ++aa) {
                ACC sacc = (ACC)0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) sacc += av[k][e] * coef[aa][e];
                q[aa][k] += sacc;
            }
        buf ^= 1;
    }

    // row sums over the 8 column lanes of each row group
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            ACC v = q[aa][k];
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            q[aa][k] = v;
        }
    if (c == 0) {
#pragma unroll
        for (int aa = 0; aa < NA; ++aa)
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int i = g + RG * k;
                if (i < m) a.part[((int64_t)aa * gridDim.x + blockIdx.x) * m + i] = (double)q[aa][k];
            }
    }
    if constexpr (NCR > 0) {
#pragma unroll
        for (int r = 0; r < NCR; ++r) {
            const double t = block_sum(cr[r], shr);
            if (tid == 0) a.colpart[(int64_t)blockIdx.x * NCR + r] = t;
        }
    }
}

template <typename T, typename ACC, int NT, class Op>
hipError_t dispatch_rpt(const StripCall& c, const StripPlan& p, hipStream_t st) {
    switch (p.rpt) {
#define IPM_RPT_CASE(R)                                                                          \
    case R:                                                                                      \
        hipLaunchKernelGGL((k_strip<T, ACC, NT, R, Op>), dim3(p.grid), dim3(NT), p.lds, st, c,  \
                           p.nstrips);                                                           \
        break;
        IPM_RPT_CASE(1)
        IPM_RPT_CASE(2)
        IPM_RPT_CASE(4)
        IPM_RPT_CASE(8)
        IPM_RPT_CASE(12)
        IPM_RPT_CASE(16)
#undef IPM_RPT_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, typename ACC, class Op>
hipError_t dispatch_nt(const StripCall& c, const StripPlan& p, hipStream_t st) {
    if (p.nt == 256) return dispatch_rpt<T, ACC, 256, Op>(c, p, st);
    if (p.nt == 1024) return dispatch_rpt<T, ACC, 1024, Op>(c, p, st);
    return hipErrorInvalidValue;
}

template <class Op>
hipError_t dispatch_type(const StripCall& c, const StripPlan& p, hipStream_t st) {
    switch (c.dtype) {
        case 0: return dispatch_nt<double, double, Op>(c, p, st);
        case 1: return c.acc64 ? dispatch_nt<float, double, Op>(c, p, st) : dispatch_nt<float, float, Op>(c, p, st);
        case 2: return c.acc64 ? dispatch_nt<bf16_t, double, Op>(c, p, st) : dispatch_nt<bf16_t, float, Op>(c, p, st);
        default: return hipErrorInvalidValue;
    }
}

// ---- row reduction of the partials ------------------------------------------------------------
constexpr int RR_ROWS = 16, RR_SLICES = 16;

template <int POST>
__global__ __launch_bounds__(256) void k_reduce_rows(const double* __restrict__ part, int G, int m, int nacc,
                                                     const double* __restrict__ b, const double* __restrict__ pvec,
                                                     const double* __restrict__ dvec, double* __restrict__ out0,
                                                     double* __restrict__ out1, double* __restrict__ blockpart,
                                                     const int* __restrict__ done) {
    if (done != nullptr && *done) return;
    __shared__ double sh[2][RR_SLICES][RR_ROWS + 1];
    __shared__ double shr[4];
    const int tr = threadIdx.x % RR_ROWS, sl = threadIdx.x / RR_ROWS;
    const int i = blockIdx.x * RR_ROWS + tr;
    double s0 = 0.0, s1 = 0.0;
    if (i < m) {
        for (int g = sl; g < G; g += RR_SLICES) {
            s0 += part[(int64_t)g * m + i];
            if (nacc > 1) s1 += part[((int64_t)G + g) * m + i];
        }
    }
    sh[0][sl][tr] = s0;
    sh[1][sl][tr] = s1;
    __syncthreads();
    double contrib = 0.0;
    if (sl == 0 && i < m) {
        double t0 = 0.0, t1 = 0.0;
        for (int k = 0; k < RR_SLICES; ++k) { t0 += sh[0][k][tr]; t1 += sh[1][k][tr]; }
        if (POST == POST_PLAIN) {
            out0[i] = t0;
        } else if (POST == POST_MATVEC) {
            out0[i] = t0;
            contrib = dvec[i] * t0;
        } else if (POST == POST_RESID) {
            const double rp = t0 - b[i];
            out0[i] = rp;
            out1[i] = b[i] - t1;
            contrib = rp * rp;
        } else if (POST == POST_RHAT) {
            out0[i] = t0 - pvec[i];
        }
    }
    if (POST == POST_MATVEC || POST == POST_RESID) {
        const double t = block_sum(contrib, shr);
        if (threadIdx.x == 0) blockpart[blockIdx.x] = t;
    }
}

}  // namespace

StripPlan strip_plan(int dtype, int m, int64_t n, int num_cu, int kind) {
    StripPlan p{};
    const int vec = dtype == 0 ? 2 : (dtype == 1 ? 4 : 8);
    p.sw = LPR * vec;
    p.nstrips = (int)((n + p.sw - 1) / p.sw);
    // rows per thread: smallest instance covering m with 256 threads, else 1024 threads
    static const int rpts[] = {1, 2, 4, 8, 12, 16};
    p.nt = 0;
    for (int nt : {256, 1024}) {
        const int rg = nt / LPR;
        for (int r : rpts)
            if (r * rg >= m) { p.nt = nt; p.rpt = r; break; }
        if (p.nt) break;
    }
    if (!p.nt) { p.nt = -1; return p; }   // m too large for the dense strip pass
    const int per_cu = p.nt == 256 ? 4 : 1;
    int grid = num_cu * per_cu;
    if (grid > p.nstrips) grid = p.nstrips;
    if (grid < 1) grid = 1;
    p.grid = grid;
    const int rg = p.nt / LPR;
    const int nw = p.nt / 64;
    const size_t acc = 8;   // sized for FP64 accumulation (enough for FP32 too)
    (void)kind;
    p.lds = acc * ((size_t)rg * p.rpt + 2 * (size_t)nw * p.sw);
    return p;
}

hipError_t launch_strip(const StripCall& c, const StripPlan& p, hipStream_t st) {
    if (p.nt <= 0) return hipErrorInvalidValue;
    switch (c.kind) {
        case STRIP_MATVEC: return dispatch_type<OpMatvec>(c, p, st);
        case STRIP_RESID: return dispatch_type<OpResid>(c, p, st);
        case STRIP_DIR: return dispatch_type<OpDir>(c, p, st);
        default: return hipErrorInvalidValue;
    }
}

int reduce_rows_blocks(int m) { return (m + RR_ROWS - 1) / RR_ROWS; }

hipError_t launch_reduce_rows(int post, const double* part, int G, int m, int nacc, const double* b,
                              const double* pvec, const double* dvec, double* out0, double* out1,
                              double* blockpart, const int* done, hipStream_t st) {
    const dim3 grid(reduce_rows_blocks(m)), block(256);
    switch (post) {
        case POST_PLAIN:
            hipLaunchKernelGGL(k_reduce_rows<POST_PLAIN>, grid, block, 0, st, part, G, m, nacc, b, pvec, dvec, out0,
                               out1, blockpart, done);
            break;
        case POST_MATVEC:
            hipLaunchKernelGGL(k_reduce_rows<POST_MATVEC>, grid, block, 0, st, part, G, m, nacc, b, pvec, dvec,
                               out0, out1, blockpart, done);
            break;
        case POST_RESID:
            hipLaunchKernelGGL(k_reduce_rows<POST_RESID>, grid, block, 0, st, part, G, m, nacc, b, pvec, dvec,
                               out0, out1, blockpart, done);
            break;
        case POST_RHAT:
            hipLaunchKernelGGL(k_reduce_rows<POST_RHAT>, grid, block, 0, st, part, G, m, nacc, b, pvec, dvec, out0,
                               out1, blockpart, done);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ipmsk
