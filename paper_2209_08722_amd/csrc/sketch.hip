// The sparse-embedding sketch B = A D W (Algorithm 1, step 1; W from Section 2) and the
// perturbation v = (XS)^{1/2} W (ADW)^+ r of eq. compv (Section 4), which reuses the same W.
//
// Sketch: a block owns R rows of A and a range of columns. Its threads stream along the rows
// (consecutive threads read consecutive columns, so every load is coalesced), hash each column
// once into its s buckets and signs, and scatter-add sign * d_j * A[i][j] / sqrt(s) into an
// LDS-resident R x w bucket array with LDS atomics. The buckets accumulate in FP64 whatever the
// type of B (FP64 LDS atomics measured several times faster than FP32 ones on gfx950 for this
// random scatter). When one block covers all columns of its rows the bucket array is stored to B
// (converted to B's type); otherwise blocks add their arrays into B with global atomics. W is
// never stored as a matrix: the hash is recomputed wherever W is applied. A sketch whose blocks
// hold one or two rows (a wide bucket array) first forms, once per call (k_sketch_prep), d_j /
// sqrt(s) and, for s <= 2, every column's buckets and signs packed into 32 bits, so that neither
// the square root nor the hash is computed again for every row.
#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int SNT = 1024;     // 16 waves per block: the LDS bucket array limits blocks per CU, so
                              // the block itself must carry enough waves to hide load latency
constexpr int SUNROLL = 4;    // columns per thread per pass (independent loads in flight)

// Columns per thread per pass of the bucket kernel: R rows x U columns of A in flight per thread,
// at most 8 values, so the kernel stays within 64 VGPRs (eight waves per SIMD: two 16-wave blocks
// per CU whenever two bucket arrays fit in LDS). One row per block takes 8 columns of FP32 or FP64
// A (2000 x 2*10^6 FP64: 9.4 -> 8.9 ms against 4) but 4 of BF16 (11.7 against 11.9 ms). With the
// packed bucket table (TAB) each column also carries its table entry, and 8 columns of FP32 or
// FP64 A no longer fit 64 VGPRs: 4.
template <int R, int ESZ, bool TAB = false>
constexpr int sketch_unroll() { return R >= 8 ? 1 : (R >= 4 ? 2 : (R >= 2 || ESZ < 4 || TAB ? 4 : 8)); }

// d_j / sqrt(s) for every column, once per call, for the sketch with one or two rows per block
// (which would otherwise take the square root of d2_j for every row). With tab, also the column's
// buckets and signs for up to two copies of W, packed as 16-bit entries (bucket within the copy's
// block in bits 0-14, bit 15 set for a negative sign; copy r in bits 16r..16r+15), so that the
// row blocks read them instead of hashing every column again.
__global__ __launch_bounds__(256) void k_sketch_prep(int64_t n, const double* __restrict__ dv, int d_is_d2,
                                                     double scale, double* __restrict__ dsc, HashKeys hk,
                                                     uint32_t* __restrict__ tab) {
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const double dd = dv[j];
        dsc[j] = (d_is_d2 ? sqrt(dd) : dd) * scale;
        if (tab != nullptr) {
            uint32_t e = 0;
            for (int r = 0; r < hk.s; ++r) {
                int bucket;
                double sign;
                w_entry(hk, r, (uint64_t)j, bucket, sign);
                e |= ((uint32_t)(bucket - r * hk.blk) | (sign < 0.0 ? 0x8000u : 0u)) << (16 * r);
            }
            tab[j] = e;
        }
    }
}

// DSC: d_j / sqrt(s) read from k_sketch_prep's vector; sign * (d_j / sqrt(s)) equals
// (sign * d_j) / sqrt(s) exactly, so B is the same either way. A thread's columns advance by
// fixed strides, so (j + 1) kPhi of the hash advances by additions. TAB (with DSC; s <= 2): the
// buckets and signs come from k_sketch_prep's packed table instead of the hash; a negative sign
// negates the coefficient, which is exactly the product with -1.
template <typename T, typename BT, int R, bool DSC, bool TAB = false>
__global__ __launch_bounds__(SNT) __attribute__((amdgpu_waves_per_eu(8))) void k_sketch_lds(const T* __restrict__ A, int m, int64_t n, int64_t ld,
                                                    const double* __restrict__ dv, int d_is_d2, HashKeys hk, int w,
                                                    int64_t cpc, BT* __restrict__ B, int atomic,
                                                    const double* __restrict__ dsc, const uint32_t* __restrict__ tab) {
    static_assert(!TAB || DSC, "the table path reads d_j / sqrt(s) from the prep vector");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* bk = reinterpret_cast<double*>(smem_raw);   // [R][w]
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * R;
    const int64_t jb = (int64_t)blockIdx.y * cpc;
    const int64_t je = (jb + cpc < n) ? jb + cpc : n;
    for (int i = tid; i < R * w; i += SNT) bk[i] = 0.0;
    __syncthreads();
    const int s = hk.s;
    constexpr int U = sketch_unroll<R, (int)sizeof(T), TAB>();
    uint64_t zj0 = ((uint64_t)(jb + tid) + 1ull) * kPhi;   // (j + 1) kPhi for this pass's first column
    for (int64_t jj = jb + tid; jj < je; jj += (int64_t)SNT * U, zj0 += (uint64_t)SNT * U * kPhi) {
        double av[U][R];
        double dj[U];
        uint32_t te[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = jj + (int64_t)u * SNT;
            const bool ok = j < je;
            if constexpr (TAB) te[u] = ok ? tab[j] : 0u;
            if constexpr (DSC) {
                dj[u] = ok ? dsc[j] : 0.0;
            } else {
                double dd = ok ? dv[ok ? j : 0] : 0.0;
                dj[u] = d_is_d2 ? sqrt(dd) : dd;
            }
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int i = row0 + rr;
                av[u][rr] = (ok && i < m) ? (double)Elem<T>::load1_stream(A + (int64_t)i * ld + j) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = jj + (int64_t)u * SNT;
            if (j >= je) continue;
            if constexpr (TAB) {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (r >= s) break;
                    const uint32_t e = te[u] >> (16 * r);
                    const int bucket = r * hk.blk + (int)(e & 0x7fffu);
                    const double coef = (e & 0x8000u) ? -dj[u] : dj[u];
#pragma unroll
                    for (int rr = 0; rr < R; ++rr) atomicAdd(&bk[rr * w + bucket], coef * av[u][rr]);
                }
                continue;
            }
            const uint64_t zj = zj0 + (uint64_t)u * SNT * kPhi;
            for (int r = 0; r < s; ++r) {
                int bucket;
                double sign;
                w_entry_z(hk, r, zj, bucket, sign);
                const double coef = DSC ? sign * dj[u] : sign * dj[u] * hk.scale;
#pragma unroll
                for (int rr = 0; rr < R; ++rr) atomicAdd(&bk[rr * w + bucket], coef * av[u][rr]);
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < R * w; idx += SNT) {
        const int rr = idx / w, bcol = idx - rr * w;
        const int i = row0 + rr;
        if (i < m) {
            BT* dst = B + (int64_t)i * w + bcol;
            if (atomic) unsafeAtomicAdd(dst, (BT)bk[idx]);
            else *dst = (BT)bk[idx];
        }
    }
}

// Packed-table form of the bucket kernel for one row per block (a bucket array too wide for two
// rows): the buckets and signs come from k_sketch_prep's table. A thread takes CPL consecutive
// columns per step (CPL elements of A, their CPL table entries and CPL values of d_j / sqrt(s),
// each read with one or two vector loads), and issues the next step's loads before this step's
// LDS atomics, so that they stream in while the atomics run. Requires ld and the chunk start to be
// multiples of CPL columns and A, dsc and tab aligned to CPL elements (checked by the host).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

// NW consecutive 32-bit words from p (NW = 1, 2, 4 or 8), with the non-temporal hint if NT.
template <int NW, bool NT>
__device__ __forceinline__ void load_words(const void* p, uint32_t* out) {
    if constexpr (NW == 1) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
        out[0] = NT ? __builtin_nontemporal_load(q) : *q;
    } else if constexpr (NW == 2) {
        const u32x2_t* q = reinterpret_cast<const u32x2_t*>(p);
        const u32x2_t v = NT ? __builtin_nontemporal_load(q) : *q;
        out[0] = v.x; out[1] = v.y;
    } else {
#pragma unroll
        for (int h = 0; h < NW / 4; ++h) {
            const u32x4_t* q = reinterpret_cast<const u32x4_t*>(p) + h;
            const u32x4_t v = NT ? __builtin_nontemporal_load(q) : *q;
            out[4 * h] = v.x; out[4 * h + 1] = v.y; out[4 * h + 2] = v.z; out[4 * h + 3] = v.w;
        }
    }
}

// The first cnt of CPL consecutive elements of type E as 32-bit words, the rest zero.
template <typename E, int CPL>
__device__ __forceinline__ void load_partial(const E* p, int cnt, uint32_t* out) {
    union { uint32_t w[(CPL * sizeof(E) + 3) / 4]; E e[CPL]; } u;
#pragma unroll
    for (int k = 0; k < (int)((CPL * sizeof(E) + 3) / 4); ++k) u.w[k] = 0u;
#pragma unroll
    for (int k = 0; k < CPL; ++k)
        if (k < cnt) u.e[k] = p[k];
#pragma unroll
    for (int k = 0; k < (int)((CPL * sizeof(E) + 3) / 4); ++k) out[k] = u.w[k];
}

template <typename T, int CPL>
struct SketchCols {
    static constexpr int NA = CPL * (int)sizeof(T) / 4;   // words of A
    uint32_t a[NA];
    uint32_t t[CPL];       // packed table entries
    uint32_t d[2 * CPL];   // FP64 d_j / sqrt(s)
};

template <typename T, int CPL>
__device__ __forceinline__ double col_value(const SketchCols<T, CPL>& q, int k) {
    if constexpr (sizeof(T) == 2) {
        const uint32_t wd = q.a[k >> 1];
        return (double)__uint_as_float((k & 1) ? (wd & 0xFFFF0000u) : (wd << 16));
    } else if constexpr (sizeof(T) == 4) {
        return (double)__uint_as_float(q.a[k]);
    } else {
        return __hiloint2double((int)q.a[2 * k + 1], (int)q.a[2 * k]);
    }
}

template <typename T, int CPL>
__device__ __forceinline__ void cols_fetch(const T* __restrict__ row, const double* __restrict__ dsc,
                                           const uint32_t* __restrict__ tab, int64_t j, int64_t left, bool row_ok,
                                           SketchCols<T, CPL>& q) {
    constexpr int NA = SketchCols<T, CPL>::NA;
    if (left >= CPL) {
        load_words<CPL, false>(tab + j, q.t);
        load_words<2 * CPL, false>(dsc + j, q.d);
        if (row_ok) {
            load_words<NA, true>(row + j, q.a);
        } else {
#pragma unroll
            for (int k = 0; k < NA; ++k) q.a[k] = 0u;
        }
    } else {
        const int cnt = left > 0 ? (int)left : 0;
        load_partial<uint32_t, CPL>(tab + j, cnt, q.t);
        load_partial<double, CPL>(dsc + j, cnt, q.d);
        load_partial<T, CPL>(row + j, row_ok ? cnt : 0, q.a);
    }
}

template <typename T, typename BT, int CPL>
__global__ __launch_bounds__(SNT) __attribute__((amdgpu_waves_per_eu(8))) void k_sketch_tab(
        const T* __restrict__ A, int m, int64_t n, int64_t ld, HashKeys hk, int w, int64_t cpc, BT* __restrict__ B,
        int atomic, const double* __restrict__ dsc, const uint32_t* __restrict__ tab) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* bk = reinterpret_cast<double*>(smem_raw);   // [w]
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    const int64_t jb = (int64_t)blockIdx.y * cpc;
    const int64_t je = (jb + cpc < n) ? jb + cpc : n;
    for (int b = tid; b < w; b += SNT) bk[b] = 0.0;
    __syncthreads();
    const int s = hk.s;
    const bool row_ok = i < m;
    const T* row = A + (int64_t)(row_ok ? i : 0) * ld;
    SketchCols<T, CPL> cur, nxt;
    int64_t j = jb + CPL * (int64_t)tid;
    cols_fetch<T, CPL>(row, dsc, tab, j, je - j, row_ok, cur);
    for (; j < je; j += CPL * (int64_t)SNT) {
        const int64_t jn = j + CPL * (int64_t)SNT;
        cols_fetch<T, CPL>(row, dsc, tab, jn < je ? jn : j, jn < je ? je - jn : 0, row_ok, nxt);
        const int64_t left = je - j;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (k >= left) break;
            const double a = col_value<T, CPL>(cur, k);
            const double dk = __hiloint2double((int)cur.d[2 * k + 1], (int)cur.d[2 * k]);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (r >= s) break;
                const uint32_t e = cur.t[k] >> (16 * r);
                const int bucket = r * hk.blk + (int)(e & 0x7fffu);
                const double coef = (e & 0x8000u) ? -dk : dk;
                atomicAdd(&bk[bucket], coef * a);
            }
        }
        cur = nxt;
    }
    __syncthreads();
    if (row_ok) {
        for (int b = tid; b < w; b += SNT) {
            BT* dst = B + (int64_t)i * w + b;
            if (atomic) unsafeAtomicAdd(dst, (BT)bk[b]);
            else *dst = (BT)bk[b];
        }
    }
}

// Wide sketches (a row of buckets larger than LDS): a block owns one row of A and one range of
// at most `wb` buckets inside the bucket block of one copy r (copy r only ever lands in
// [r w/s, (r+1) w/s)). It streams the whole row, hashes copy r of each column and keeps the
// columns whose bucket falls in its range, accumulating them in LDS (FP64); the range is then
// stored to B. Each row is read once per range.
template <typename T, typename BT>
__global__ __launch_bounds__(SNT) void k_sketch_range(const T* __restrict__ A, int m, int64_t n, int64_t ld,
                                                      const double* __restrict__ dv, int d_is_d2, HashKeys hk,
                                                      int w, int wb, int ranges_per_copy, BT* __restrict__ B) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* bk = reinterpret_cast<double*>(smem_raw);   // [wb]
    const int i = blockIdx.x;
    const int r = blockIdx.y / ranges_per_copy;
    const int b0 = r * hk.blk + (blockIdx.y % ranges_per_copy) * wb;
    const int b1 = min(b0 + wb, (r + 1) * hk.blk);
    for (int b = threadIdx.x; b < b1 - b0; b += SNT) bk[b] = 0.0;
    __syncthreads();
    const T* row = A + (int64_t)i * ld;
    for (int64_t jj = threadIdx.x; jj < n; jj += (int64_t)SNT * SUNROLL) {
        double av[SUNROLL], dj[SUNROLL];
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u) {
            const int64_t j = jj + (int64_t)u * SNT;
            const bool ok = j < n;
            const double dd = ok ? dv[j] : 0.0;
            dj[u] = d_is_d2 ? sqrt(dd) : dd;
            av[u] = ok ? (double)Elem<T>::load1_stream(row + j) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u) {
            const int64_t j = jj + (int64_t)u * SNT;
            if (j >= n) continue;
            int bucket;
            double sign;
            w_entry(hk, r, (uint64_t)j, bucket, sign);
            if (bucket >= b0 && bucket < b1) atomicAdd(&bk[bucket - b0], sign * dj[u] * hk.scale * av[u]);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < b1 - b0; b += SNT) B[(int64_t)i * w + b0 + b] = (BT)bk[b];
}

template <typename T, typename BT, int R>
void sketch_go(const T* A, int m, int64_t n, int64_t ld, const double* dv, int d2, const HashKeys& hk, int w,
               BT* B, const SketchPlan& sp, const double* dsc, const uint32_t* tab, hipStream_t st) {
    const dim3 grid((m + R - 1) / R, sp.chunks);
    // BF16 and FP32 A: four columns per lane, loads one step ahead (2000 x 2*10^6 BF16: 9.2 -> 6.0
    // ms); FP64 A stays with the per-column kernel (7.2 ms against 7.4, 8.7 and 10.0 with two,
    // four and one columns per lane in the pipelined one)
    if constexpr (R == 1 && sizeof(T) <= 4) {
        constexpr int CPL = 4;
        if (sp.table && tab != nullptr && ld % CPL == 0 && reinterpret_cast<uintptr_t>(A) % (CPL * sizeof(T)) == 0 &&
            reinterpret_cast<uintptr_t>(tab) % (CPL * 4) == 0 && reinterpret_cast<uintptr_t>(dsc) % (CPL * 8) == 0 &&
            (sp.chunks == 1 || sp.cols_per_chunk % CPL == 0)) {
            IPM_LAUNCH((k_sketch_tab<T, BT, CPL>), grid, dim3(SNT), sp.lds, st, A, m, n, ld, hk, w, sp.cols_per_chunk,
                       B, sp.atomic ? 1 : 0, dsc, tab);
            return;
        }
    }
    if constexpr (R <= 2) {
        if (sp.table && tab != nullptr) {
            IPM_LAUNCH((k_sketch_lds<T, BT, R, true, true>), grid, dim3(SNT), sp.lds, st, A, m, n, ld, dv, d2, hk, w,
                       sp.cols_per_chunk, B, sp.atomic ? 1 : 0, dsc, tab);
            return;
        }
        if (sp.table) {
            IPM_LAUNCH((k_sketch_lds<T, BT, R, true>), grid, dim3(SNT), sp.lds, st, A, m, n, ld, dv, d2, hk, w,
                       sp.cols_per_chunk, B, sp.atomic ? 1 : 0, dsc, nullptr);
            return;
        }
    }
    IPM_LAUNCH((k_sketch_lds<T, BT, R, false>), grid, dim3(SNT), sp.lds, st, A, m, n, ld, dv, d2, hk, w,
               sp.cols_per_chunk, B, sp.atomic ? 1 : 0, nullptr, nullptr);
}

template <typename T, typename BT>
hipError_t sketch_type(const void* Av, int m, int64_t n, int64_t ld, const double* dv, int d2, const HashKeys& hk,
                       int w, void* Bv, const SketchPlan& sp, const double* dsc, const uint32_t* tab,
                       hipStream_t st) {
    const T* A = reinterpret_cast<const T*>(Av);
    BT* B = reinterpret_cast<BT*>(Bv);
    if (sp.global_only) {
        const int blk = w / hk.s;
        const int rpc = (blk + sp.range_width - 1) / sp.range_width;
        IPM_LAUNCH((k_sketch_range<T, BT>), dim3(m, hk.s * rpc), dim3(SNT), sp.lds, st, A, m, n, ld, dv, d2, hk, w,
                   sp.range_width, rpc, B);
        return hipGetLastError();
    }
    switch (sp.rows_per_block) {
        case 1: sketch_go<T, BT, 1>(A, m, n, ld, dv, d2, hk, w, B, sp, dsc, tab, st); break;
        case 2: sketch_go<T, BT, 2>(A, m, n, ld, dv, d2, hk, w, B, sp, dsc, tab, st); break;
        case 4: sketch_go<T, BT, 4>(A, m, n, ld, dv, d2, hk, w, B, sp, dsc, tab, st); break;
        case 8: sketch_go<T, BT, 8>(A, m, n, ld, dv, d2, hk, w, B, sp, dsc, tab, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// u = B^T g: thread per bucket column, block rows chunked; partial sums added atomically.
template <typename BT>
__global__ __launch_bounds__(256) void k_btg(const BT* __restrict__ B, int m, int w, int rows_per_chunk,
                                             const double* __restrict__ g, double* __restrict__ u) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int i0 = blockIdx.y * rows_per_chunk;
    const int i1 = min(m, i0 + rows_per_chunk);
    if (b >= w) return;
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) acc += (double)B[(int64_t)i * w + b] * g[i];
    unsafeAtomicAdd(&u[b], acc);
}

// dx_j = -x_j + sigma mu / s_j - d2_j ds_j - v_j / s_j with
// v_j = sqrt(x_j s_j) * sum_r sign_r(j) u[bucket_r(j)] / sqrt(s)   (eq. compv; eq. delxhat_i)
// plus per-block sums of x ds + s dx, dx ds and v^2.
__global__ __launch_bounds__(256) void k_dx(int64_t n, const double* __restrict__ x, const double* __restrict__ s,
                                            const double* __restrict__ d2, const double* __restrict__ ds,
                                            const double* __restrict__ u, int vcorr, HashKeys hk,
                                            const double* __restrict__ wu, const double* __restrict__ scal,
                                            double* __restrict__ dx, double* __restrict__ part3) {
    __shared__ double sh[4];
    const double smu = scal[SC_SMU];
    double a1 = 0.0, a2 = 0.0, v2 = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const double xj = x[j], sj = s[j], dsj = ds[j];
        double v = 0.0;
        if (vcorr && wu != nullptr) {
            v = sqrt(xj * sj) * wu[j];   // (W u)_j computed beforehand (Gaussian W)
        } else if (vcorr) {
            double acc = 0.0;
            for (int r = 0; r < hk.s; ++r) {
                int bucket;
                double sign;
                w_entry(hk, r, (uint64_t)j, bucket, sign);
                acc += sign * u[bucket];
            }
            v = sqrt(xj * sj) * acc * hk.scale;
        }
        const double dxj = -xj + smu / sj - d2[j] * dsj - v / sj;
        dx[j] = dxj;
        a1 += xj * dsj + sj * dxj;
        a2 += dxj * dsj;
        v2 += v * v;
    }
    const double t1 = block_sum(a1, sh);
    const double t2 = block_sum(a2, sh);
    const double t3 = block_sum(v2, sh);
    if (threadIdx.x == 0) {
        part3[3 * blockIdx.x] = t1;
        part3[3 * blockIdx.x + 1] = t2;
        part3[3 * blockIdx.x + 2] = t3;
    }
}

}  // namespace

SketchPlan sketch_plan(int m, int64_t n, int w, int out_f64, int num_cu) {
    SketchPlan sp{};
    (void)out_f64;
    const size_t esz = 8;   // LDS buckets accumulate in FP64 for either type of B
    const size_t budget_small = 64 * 1024, budget_max = 160 * 1024;
    int R = 0;
    for (int r : {8, 4, 2, 1})
        if ((size_t)r * w * esz <= budget_small && r <= m) { R = r; break; }
    if (R == 0 && (size_t)w * esz <= budget_max) R = 1;
    if (R == 0) {
        // one row per block and a bucket range of at most 160 KB of FP64 buckets
        sp.global_only = true;
        sp.atomic = false;
        sp.chunks = 1;
        sp.cols_per_chunk = n;
        sp.range_width = (int)(budget_max / esz);
        sp.lds = (size_t)sp.range_width * esz;
        return sp;
    }
    sp.rows_per_block = R;
    sp.lds = (size_t)R * w * esz;
    // one or two rows per block: sqrt(d2_j) would be taken again for every row
    sp.table = R <= 2;
    // Blocks resident at once: two per CU when two bucket arrays fit in LDS (the kernel is held to
    // eight waves per SIMD), else one. With the column range split into c chunks the grid runs in
    // ceil(row_blocks c / slots) rounds; per row a block streams n / c columns and clears, then
    // adds back, its w buckets (weighted as 2 w columns), and c minimises rounds x that sum (the
    // fewest chunks among equals).
    const int row_blocks = (m + R - 1) / R;
    const int slots = num_cu * (2 * sp.lds <= budget_max ? 2 : 1);
    const int64_t by_cols = (n + 4095) / 4096;   // keep at least 4096 columns per block
    const int64_t max_chunks = by_cols < 64 ? by_cols : 64;
    int chunks = 1;
    double best = 0.0;
    for (int c = 1; c <= max_chunks; ++c) {
        const double rounds = (double)(((int64_t)row_blocks * c + slots - 1) / slots);
        const double cost = rounds * ((double)n / c + 2.0 * w);
        if (c == 1 || cost < best - 1e-12) { best = cost; chunks = c; }
    }
    sp.chunks = chunks;
    // a multiple of four columns, so that every chunk of the packed-table kernel starts aligned
    sp.cols_per_chunk = (((n + chunks - 1) / chunks) + 3) & ~(int64_t)3;
    sp.atomic = chunks > 1;
    return sp;
}

bool sketch_table_fits(const HashKeys& hk) { return hk.s <= 2 && hk.blk <= 0x8000; }

hipError_t launch_sketch_prep(int64_t n, const double* dvals, int dvals_are_d2, double scale, double* dsc,
                              const HashKeys& hk, uint32_t* tab, hipStream_t st) {
    if (tab != nullptr && !sketch_table_fits(hk)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sketch_prep, dim3(pointwise_blocks(n)), dim3(256), 0, st, n, dvals, dvals_are_d2, scale, dsc,
                       hk, tab);
    return hipGetLastError();
}

hipError_t launch_sketch(int dtype, const void* A, int m, int64_t n, int64_t ld, const double* dvals,
                         int dvals_are_d2, const HashKeys& hk, int w, int out_f64, void* B, const SketchPlan& sp,
                         const double* dsc, const uint32_t* tab, hipStream_t st) {
    if (sp.table && dsc == nullptr) return hipErrorInvalidValue;
    if (tab != nullptr && !sketch_table_fits(hk)) return hipErrorInvalidValue;
    if (out_f64) {
        switch (dtype) {
            case 0: return sketch_type<double, double>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
            case 1: return sketch_type<float, double>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
            case 2: return sketch_type<bf16_t, double>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
        }
    } else {
        switch (dtype) {
            case 0: return sketch_type<double, float>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
            case 1: return sketch_type<float, float>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
            case 2: return sketch_type<bf16_t, float>(A, m, n, ld, dvals, dvals_are_d2, hk, w, B, sp, dsc, tab, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_btg(const void* B, int b_f64, int m, int w, const double* g, double* u, hipStream_t st) {
    hipError_t e = launch_fill(u, w, 0.0, st);
    if (e != hipSuccess) return e;
    const int bx = (w + 255) / 256;
    int chunks = (512 + bx - 1) / bx;
    int rpc = (m + chunks - 1) / chunks;
    if (rpc < 16) rpc = 16;
    chunks = (m + rpc - 1) / rpc;
    if (b_f64)
        hipLaunchKernelGGL(k_btg<double>, dim3(bx, chunks), dim3(256), 0, st, reinterpret_cast<const double*>(B), m, w,
                           rpc, g, u);
    else
        hipLaunchKernelGGL(k_btg<float>, dim3(bx, chunks), dim3(256), 0, st, reinterpret_cast<const float*>(B), m, w,
                           rpc, g, u);
    return hipGetLastError();
}

int pointwise_blocks(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_dx(int64_t n, const double* x, const double* s, const double* d2, const double* ds,
                     const double* u, int vcorr, const HashKeys& hk, const double* wu, const double* scal, double* dx,
                     double* part3, hipStream_t st) {
    hipLaunchKernelGGL(k_dx, dim3(pointwise_blocks(n)), dim3(256), 0, st, n, x, s, d2, ds, u, vcorr, hk, wu, scal,
                       dx, part3);
    return hipGetLastError();
}

}  // namespace ipmsk
