// Passes over a sparse A stored in CSR with a CSC mirror of the same nonzeros (the sparse
// configurations: a few nonzeros per column, about a thousand per row).
//
// Every pass over A has the two halves of the dense strip pass (strip.hip), here as two kernels:
//   column pass (CSC): t_j = a_j^T vec0 (and a_j^T vec1 for the paired matvec), then the
//                      per-column step of the pass (strip_ops.hpp),
//                      writing the column coefficients to an n-vector workspace;
//   row pass (CSR):    q_i = sum_j a_ij coef_j, then the row post step (plain, residual, true
//                      residual, p - q), one wave per row.
// Values may be FP64, FP32 or BF16; accumulation is FP64. The sketch scatters each row's
// nonzeros into LDS buckets, one block per (row, bucket range of one copy of W).
#include "strip_ops.hpp"

namespace ipmsk {

namespace {

constexpr int CNT = 256;            // column pass threads (one column per thread)
constexpr int RNT_S = 256;          // row pass threads (one wave per row)
constexpr int SKT = 256;            // sketch threads

template <typename T>
__device__ __forceinline__ double elem(const void* v, int64_t k) {
    return (double)Elem<T>::load1(reinterpret_cast<const T*>(v) + k);
}

template <typename T, class Op>
__global__ __launch_bounds__(CNT) void k_csc_cols(StripCall a) {
    if (a.done != nullptr && *a.done) return;
    constexpr int NA = Op::NACC, NCR = Op::NCR, ND = Op::ND;
    __shared__ double sh[CNT / 64];
    const typename Op::S st = Op::init(a);
    double cr[NCR > 0 ? NCR : 1] = {0.0};
    for (int64_t j = (int64_t)blockIdx.x * CNT + threadIdx.x; j < a.n; j += (int64_t)gridDim.x * CNT) {
        const int64_t k0 = a.col_ptr[j], k1 = a.col_ptr[j + 1];
        double t[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) t[d] = 0.0;
        for (int64_t k = k0; k < k1; ++k) {
            const double v = elem<T>(a.csc_val, k);
            const int32_t i = a.row_idx[k];
            t[0] += v * a.vec0[i];
            if constexpr (ND > 1) t[1] += v * a.vec1[i];
        }
        double cf[NA];
        Op::template column<double>(a, st, j, true, true, t, cf, cr, Op::PF ? Op::pre(a, j, true) : 0.0);
#pragma unroll
        for (int aa = 0; aa < NA; ++aa) a.coefs[(int64_t)aa * a.n + j] = cf[aa];
    }
    if constexpr (NCR > 0) {
#pragma unroll
        for (int r = 0; r < NCR; ++r) {
            const double tt = block_sum(cr[r], sh);
            if (threadIdx.x == 0) a.colpart[(int64_t)blockIdx.x * NCR + r] = tt;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(RNT_S) void k_csr_rows(StripCall a, int nacc, int ncolblocks) {
    if (a.done != nullptr && *a.done) return;
    __shared__ double shr[RNT_S / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = a.m;
    const int i = blockIdx.x * (RNT_S / 64) + wid;
    double contrib = 0.0;
    if (i < m) {
        const int64_t k0 = a.row_ptr[i], k1 = a.row_ptr[i + 1];
        const double* c0 = a.coefs;
        const double* c1 = a.coefs + a.n;
        double t0 = 0.0, t1 = 0.0;
        for (int64_t k = k0 + lane; k < k1; k += 64) {
            const double v = elem<T>(a.A, k);
            const int32_t j = a.col_idx[k];
            t0 += v * c0[j];
            if (nacc > 1) t1 += v * c1[j];
        }
        t0 = wave_sum(t0);
        if (nacc > 1) t1 = wave_sum(t1);
        if (lane == 0) {
            switch (a.post) {
                case POST_PLAIN:
                case POST_MATVEC: a.out0[i] = t0; break;
                case POST_RESID: {
                    const double rp = t0 - a.b[i];
                    a.out0[i] = rp;
                    a.out1[i] = a.feasible ? t0 - t1 : a.b[i] - t1;   // p (eqn. pdef when feasible)
                    contrib = rp * rp;
                    break;
                }
                case POST_RHAT: a.out0[i] = t0 - a.pvec[i]; break;
                case POST_RESP: a.out0[i] = a.pvec[i] - t0; break;
                case POST_SUBR: a.out0[i] -= t0; break;   // r -= M dx (Chebyshev)
                case POST_PAIR: a.out0[i] = t0; a.out1[i] = t1; break;
                default: break;
            }
        }
    }
    if (a.post == POST_RESID) {
        const double tot = block_sum(contrib, shr);
        if (threadIdx.x == 0) a.gpart[blockIdx.x] = tot;   // per-block sums of r_p^2
        if (blockIdx.x == 0) {
            double sacc = 0.0;
            for (int g = threadIdx.x; g < ncolblocks; g += RNT_S) sacc += a.colpart[g];
            sacc = block_sum(sacc, shr);
            if (threadIdx.x == 0) a.outsc[1] = sacc;   // sum of r_d^2
        }
    }
}

template <typename T, class Op>
hipError_t sparse_go(const StripCall& c, hipStream_t st) {
    const int gc = sparse_col_blocks(c.n);
    hipLaunchKernelGGL((k_csc_cols<T, Op>), dim3(gc), dim3(CNT), 0, st, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nacc = Op::NACC;
    hipLaunchKernelGGL(k_csr_rows<T>, dim3(rowsum_blocks(c.m)), dim3(RNT_S), 0, st, c, nacc, gc);
    return hipGetLastError();
}

template <class Op>
hipError_t sparse_type(const StripCall& c, hipStream_t st) {
    switch (c.dtype) {
        case 0: return sparse_go<double, Op>(c, st);
        case 1: return sparse_go<float, Op>(c, st);
        case 2: return sparse_go<bf16_t, Op>(c, st);
        default: return hipErrorInvalidValue;
    }
}

// One block per (row i, bucket range [b0, b1) of copy r): the row's nonzeros scattered into LDS.
template <typename T, typename BT>
__global__ __launch_bounds__(SKT) void k_sketch_csr(const T* __restrict__ val, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx, const double* __restrict__ dv,
                                                    int d_is_d2, HashKeys hk, int w, int wb, int ranges_per_copy,
                                                    BT* __restrict__ B) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* bk = reinterpret_cast<double*>(smem_raw);   // [wb]
    const int i = blockIdx.x;
    const int r = blockIdx.y / ranges_per_copy;
    const int b0 = r * hk.blk + (blockIdx.y % ranges_per_copy) * wb;
    const int b1 = min(b0 + wb, (r + 1) * hk.blk);
    for (int b = threadIdx.x; b < b1 - b0; b += SKT) bk[b] = 0.0;
    __syncthreads();
    const int64_t k0 = row_ptr[i], k1 = row_ptr[i + 1];
    for (int64_t k = k0 + threadIdx.x; k < k1; k += SKT) {
        const int32_t j = col_idx[k];
        int bucket;
        double sign;
        w_entry(hk, r, (uint64_t)j, bucket, sign);
        if (bucket >= b0 && bucket < b1) {
            const double dd = dv[j];
            const double dj = d_is_d2 ? sqrt(dd) : dd;
            atomicAdd(&bk[bucket - b0], sign * dj * hk.scale * (double)Elem<T>::load1(val + k));
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < b1 - b0; b += SKT) B[(int64_t)i * w + b0 + b] = (BT)bk[b];
}

template <typename T, typename BT>
hipError_t sketch_csr_go(const void* val, const int64_t* row_ptr, const int32_t* col_idx, int m, const double* dv,
                         int d2, const HashKeys& hk, int w, void* B, hipStream_t st) {
    const int blk = w / hk.s;
    const int wb = blk < 20480 ? blk : 20480;   // at most 160 KB of FP64 buckets
    const int rpc = (blk + wb - 1) / wb;
    IPM_LAUNCH((k_sketch_csr<T, BT>), dim3(m, hk.s * rpc), dim3(SKT), (size_t)wb * 8, st,
               reinterpret_cast<const T*>(val), row_ptr, col_idx, dv, d2, hk, w, wb, rpc, reinterpret_cast<BT*>(B));
    return hipGetLastError();
}

}  // namespace

int sparse_col_blocks(int64_t n) {
    int64_t g = (n + CNT - 1) / CNT;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_sparse_pass(const StripCall& c, hipStream_t st) {
    switch (c.kind) {
        case STRIP_MATVEC: return sparse_type<OpMatvec>(c, st);
        case STRIP_RESID: return sparse_type<OpResid>(c, st);
        case STRIP_DIR: return sparse_type<OpDir>(c, st);
        case STRIP_MATVEC2: return sparse_type<OpMatvec2>(c, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sketch_csr(int dtype, const void* val, const int64_t* row_ptr, const int32_t* col_idx, int m,
                             const double* dvals, int dvals_are_d2, const HashKeys& hk, int w, int out_f64, void* B,
                             hipStream_t st) {
    if (out_f64) {
        switch (dtype) {
            case 0: return sketch_csr_go<double, double>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
            case 1: return sketch_csr_go<float, double>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
            case 2: return sketch_csr_go<bf16_t, double>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
        }
    } else {
        switch (dtype) {
            case 0: return sketch_csr_go<double, float>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
            case 1: return sketch_csr_go<float, float>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
            case 2: return sketch_csr_go<bf16_t, float>(val, row_ptr, col_idx, m, dvals, dvals_are_d2, hk, w, B, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace ipmsk
