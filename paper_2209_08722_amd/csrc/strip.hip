// Single-pass column-strip kernels over row-major A (m x n, row stride ld).
//
// Every pass here has the shape "per column j: dot a_j with one m-vector (two for the paired
// matvec), turn the dots into per-column coefficients; per row i: accumulate
// sum_j A[i][j] * coef_j" (one or two accumulations). Reading A once per
// pass requires each column strip to stay on chip between the dot and the accumulation, so a
// block owns a strip of SW columns across all m rows, held in registers:
//   - lanes: LPR lanes per row, 16-byte vector loads -> LPR*16 contiguous bytes per row segment;
//   - thread (c, g) holds rows g, g+RG, ... (RG = blockDim/LPR row groups) of columns
//     [strip*SW + c*VEC, +VEC);
//   - column dots: per-thread partials, then wave shuffles over the row groups of a wave, then
//     one LDS exchange across waves (double-buffered, one barrier per strip);
//   - the strip stays in registers as raw 16-byte words, converted to the accumulation type at use;
//   - row sums: per-thread register accumulators reduced over the column lanes once at the end
//     of the persistent loop, or (more than 16 rows per thread) reduce-scattered over the eight
//     column lanes every strip (lane c keeps every eighth row's running sum in registers);
//   - each block writes its partial row sums as part[acc][row][block]; a second kernel reduces
//     them with one wave per row (coalesced over blocks) in a fixed order and applies the
//     post-processing step (r_p, p, the true residual, ...).
// The CG matvec q = A D^2 A^T v (Algorithm 1, step 3) is one such pass; so are the residual
// pass (r_d = A^T y + s - c, then A x and A u for r_p and p, Section 5 / Algorithm 3 step 3) and
// the direction pass (ds = -r_d - A^T dy, then A D^2 A^T dy for the true residual); the paired
// matvec A D^2 A^T [v0 v1] (the warm start's two candidate products) reads A once for both.
#include "strip_ops.hpp"

#include <type_traits>

namespace ipmsk {

namespace {

constexpr int kLpr = 8;      // lanes per row segment (8 x 16 B = 128 B)
constexpr int kRrNt = 512;   // re-read form: threads per block
constexpr int kRrCh = 4;     // re-read form: rows per thread per chunk

// Sum of the per-block partials part[acc][row][block] and the RowPost step: one wave per row.
// R 16-byte words of one column segment, rows g + RG k (k < R), rows >= m read as zero. seg is
// the segment's address in row g and seg0 its address in row 0. A segment inside A (left >=
// VEC elements) is read without branches: rows past the end read row 0 and are masked, so all
// R loads are in flight together (per-row branches made the compiler wait for each load before
// the next). A segment crossing the end of the row (last strip only) is read element by element.
template <typename T, int R, bool STREAM>
__device__ __forceinline__ void load_segment(const T* seg, const T* seg0, int64_t rowstride, int g, int RG, int m,
                                             int64_t left, uint4* av) {
    constexpr int VEC = Elem<T>::VEC;
    if (left >= VEC) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const bool ok = g + RG * k < m;
            const T* p = ok ? seg + (int64_t)k * rowstride : seg0;
            const uint4 w = STREAM ? raw16_stream(p) : Elem<T>::raw16(p);
            const uint32_t msk = ok ? 0xffffffffu : 0u;
            av[k] = make_uint4(w.x & msk, w.y & msk, w.z & msk, w.w & msk);
        }
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const bool ok = g + RG * k < m && left > 0;
            av[k] = ok ? raw_partial<T>(seg + (int64_t)k * rowstride, (int)left) : make_uint4(0u, 0u, 0u, 0u);
        }
    }
}

// 16 bytes at byte offset voff of one row group of a strip: base is the group's row-0 segment
// (block-uniform) and nrec the bytes of the group's rows that lie inside A. A buffer load returns
// zero at offsets >= nrec, so rows past m read as zero with neither a branch nor a mask (both of
// which made the compiler wait on each load as it was issued). Non-temporal.
__device__ __forceinline__ uint4 load_group_row(const void* base, uint32_t nrec, uint32_t voff) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                                                       (int)nrec, 0x00020000);
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 2);
    return make_uint4(v[0], v[1], v[2], v[3]);
}

constexpr int RNT = 256;
__global__ __launch_bounds__(RNT) void k_rowsum(StripCall a, int G, int nacc, int ncr) {
    if (a.done != nullptr && *a.done) return;
    __shared__ double shr[RNT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = a.m;
    const int i = blockIdx.x * (RNT / 64) + wid;
    double contrib = 0.0;
    if (i < m) {
        double t0 = 0.0, t1 = 0.0;
        const double* p0 = a.part + (int64_t)i * G;
        const double* p1 = a.part + ((int64_t)m + i) * G;
        for (int g = lane; g < G; g += 64) {
            t0 += p0[g];
            if (nacc > 1) t1 += p1[g];
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
        if (blockIdx.x == 0 && ncr > 0) {
            double s = 0.0;
            for (int g = threadIdx.x; g < G; g += RNT) s += a.colpart[g];
            s = block_sum(s, shr);
            if (threadIdx.x == 0) a.outsc[1] = s;   // sum of r_d^2
        }
    }
}

template <typename T, typename ACC, int NT, int RPT, int LPR, bool QL, class Op, bool RL = false>
__global__ __launch_bounds__(NT) void k_strip(StripCall a, int nstrips) {
    static_assert(LPR == 4 || LPR == 8 || LPR == 16 || LPR == 32 || LPR == 64, "LPR");
    constexpr int VEC = Elem<T>::VEC;
    constexpr int SW = LPR * VEC;
    constexpr int RG = NT / LPR;
    constexpr int NW = NT / 64;
    constexpr int NA = Op::NACC, NCR = Op::NCR, ND = Op::ND;
    constexpr int MPAD = RG * RPT;

    if (a.done != nullptr && *a.done) return;

    extern __shared__ __align__(16) unsigned char smem_raw[];
    ACC* vs = reinterpret_cast<ACC*>(smem_raw);   // [ND][MPAD]        vectors dotted with columns
    ACC* red = vs + ND * MPAD;                       // [2][ND][NW][SW]   per-wave column dots
    // QL row sums [NA][RPT][RG + 8]: row g + RG k at k (RG + 8) + g; the padding puts the eight
    // rows a wave's lane c of eight row groups add at once into distinct bank pairs but for c
    // and c + 4
    constexpr int QS_K = RG + 8, QS_A = RPT * QS_K;
    // FP32 storage with FP64 accumulation (four conversions per word) has no registers left for
    // the reduce-scatter's partial sums at 32 rows per thread in the residual and direction
    // passes; there it sums each row on its own (the matvec passes, whose strips are read with
    // buffer loads, keep the reduce-scatter)
    constexpr bool RS = (QL && Op::PF) || !(sizeof(T) == 4 && sizeof(ACC) == 8 && RPT > 24);
    // the paired pass over FP32 storage reads whole strips with buffer loads: per-row 64-bit
    // addresses held across the strip loop spill at this register count (FP64 and BF16 storage
    // are faster with the per-row loads)
    constexpr bool BUFLD = QL && ND > 1 && sizeof(T) == 4 && sizeof(ACC) == 8;
    double* qs = reinterpret_cast<double*>(red + 2 * ND * NW * SW);
    __shared__ double shr[NW];

    const int tid = threadIdx.x;
    const int c = tid % LPR, g = tid / LPR, lane = tid & 63, wid = tid >> 6;
    const int m = a.m;
    const int G = gridDim.x;
    const T* __restrict__ A = reinterpret_cast<const T*>(a.A);

    for (int i = tid; i < MPAD; i += NT) {
        vs[i] = (i < m) ? (ACC)a.vec0[i] : (ACC)0;
        if constexpr (ND > 1) vs[MPAD + i] = (i < m) ? (ACC)a.vec1[i] : (ACC)0;
    }
    if constexpr (QL) {
        for (int i = tid; i < NA * QS_A; i += NT) qs[i] = 0.0;
    }
    __syncthreads();
    const typename Op::S st = Op::init(a);

    // Address of (row g + RG*k, column strip*SW + c*VEC): a uniform part (strip, k) plus a
    // per-thread offset that stays the same for every strip and row block, so the loads use a
    // scalar base and one 32-bit VGPR offset.
    const uint32_t lane_off = (uint32_t)g * (uint32_t)a.ld + (uint32_t)(c * VEC);

    // row sums: with QL, per strip the eight column lanes of a row group reduce-scatter the sums
    // of eight rows, and lane c adds row g + RG (8 t + c) into the LDS row-sum array qs (one
    // LDS atomic per lane per eight rows, all lanes of a wave on distinct rows); without QL each
    // thread keeps its own rows' column-lane partials in q and reduces them at the end
    static_assert(!QL || RPT % 8 == 0, "QL needs a multiple of 8 rows per thread");
    ACC q[NA][QL ? 1 : RPT];
#pragma unroll
    for (int aa = 0; aa < NA; ++aa)
#pragma unroll
        for (int k = 0; k < (QL ? 1 : RPT); ++k) q[aa][k] = (ACC)0;
    double cr[NCR > 0 ? NCR : 1] = {0.0};

    // ROLL (the CG matvec): the next strip's rows are loaded into the registers of this strip's
    // rows as soon as the accumulation phase has used them, so the next strip streams in during
    // this strip's accumulation and the next strip's column dots. Whole strips are read with
    // buffer loads (load_group_row), whose byte offsets within a row group must stay below 2^32:
    // the host guarantees it for the many-rows instances (QL) and selects RL (the same for the
    // per-thread row sums, FP64 storage) only where it holds.
    constexpr bool ROLL = (QL ? RS : RL) && Op::PF && ND == 1;
    const int64_t rowstride = (int64_t)RG * a.ld;
    const uint32_t lane_bytes = lane_off * (uint32_t)sizeof(T);
    const uint32_t group_bytes = (uint32_t)((int64_t)RG * a.ld * (int64_t)sizeof(T));
    // bytes of row group k's rows inside A: all RG rows, fewer for the last group, none past it
    auto group_nrec = [&](int k) -> uint32_t {
        const int rows = m - RG * k;
        return rows >= RG ? group_bytes : (rows > 0 ? (uint32_t)((int64_t)rows * a.ld * (int64_t)sizeof(T)) : 0u);
    };
    auto whole = [&](int sidx) { return (int64_t)(sidx + 1) * SW <= a.n; };
    int buf = 0;
    double pfv[VEC];
    uint4 av[RPT];
    if constexpr (ROLL) {
        const int strip = blockIdx.x;
        const int64_t j0 = (int64_t)strip * SW + c * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) pfv[e] = Op::PF ? Op::pre(a, j0 + e, j0 + e < a.n) : 0.0;
        if (strip < nstrips) {
            if (whole(strip)) {
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    av[k] = load_group_row(A + (int64_t)strip * SW + (int64_t)k * rowstride, group_nrec(k), lane_bytes);
            } else {
                load_segment<T, RPT, true>(A + (int64_t)strip * SW + lane_off, A + (int64_t)strip * SW + c * VEC,
                                           rowstride, g, RG, m, a.n - j0, av);
            }
        }
    }
    for (int strip = blockIdx.x; strip < nstrips; strip += G) {
        const int64_t j0 = (int64_t)strip * SW + c * VEC;
        if constexpr (!ROLL) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) pfv[e] = Op::PF ? Op::pre(a, j0 + e, j0 + e < a.n) : 0.0;
            if (BUFLD && whole(strip)) {
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    av[k] = load_group_row(A + (int64_t)strip * SW + (int64_t)k * rowstride, group_nrec(k), lane_bytes);
            } else {
                load_segment<T, RPT, true>(A + (int64_t)strip * SW + lane_off, A + (int64_t)strip * SW + c * VEC,
                                           rowstride, g, RG, m, a.n - j0, av);
            }
        }
        // column dots over this thread's rows, one vector after the other, then over the 64/LPR
        // row groups of this wave (lane bits log2(LPR)..5)
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            ACC pd[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) pd[e] = (ACC)0;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const ACC vv = vs[d * MPAD + g + RG * k];
#pragma unroll
                for (int e = 0; e < VEC; ++e) pd[e] += Elem<T>::template get<ACC>(av[k], e) * vv;
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                ACC v = pd[e];
#pragma unroll
                for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                pd[e] = v;
            }
            if (lane < LPR) {
                ACC* rw = red + (buf * ND + d) * NW * SW;
#pragma unroll
                for (int e = 0; e < VEC; ++e) rw[wid * SW + c * VEC + e] = pd[e];
            }
            if constexpr (ND > 1) {
                // the next vector converts the raw words again (see below)
#pragma unroll
                for (int k = 0; k < RPT; ++k)
                    asm volatile("" : "+v"(av[k].x), "+v"(av[k].y), "+v"(av[k].z), "+v"(av[k].w));
            }
        }
        __syncthreads();
        const ACC* rb = red + buf * ND * NW * SW;
        ACC coef[NA][VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            ACC t[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                t[d] = (ACC)0;
#pragma unroll
                for (int w = 0; w < NW; ++w) t[d] += rb[(d * NW + w) * SW + c * VEC + e];
            }
            ACC cf[NA];
            const int64_t j = j0 + e;
            Op::template column<ACC>(a, st, j, j < a.n, g == 0, t, cf, cr, pfv[e]);
#pragma unroll
            for (int aa = 0; aa < NA; ++aa) coef[aa][e] = cf[aa];
        }
        // Keep the strip as raw words across the barrier: without this the compiler holds the
        // already converted elements of the dot phase live (up to 4x the registers) instead of
        // converting again. The empty asm emits no instruction.
#pragma unroll
        for (int k = 0; k < RPT; ++k) asm volatile("" : "+v"(av[k].x), "+v"(av[k].y), "+v"(av[k].z), "+v"(av[k].w));
        if constexpr (QL && !RS) {
            // one group sum per row, added by the row's first column lane
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int aa = 0; aa < NA; ++aa) {
                    ACC sacc = (ACC)0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sacc += Elem<T>::template get<ACC>(av[k], e) * coef[aa][e];
                    sacc = group_sum<LPR>(sacc);
                    if (c == 0) atomicAdd(&qs[aa * QS_A + k * QS_K + g], (double)sacc);
                }
        } else if constexpr (QL) {
            const int nxt = strip + G;
            const int64_t jn = (int64_t)nxt * SW + c * VEC;
            // the next strip's rows stream in during this accumulation when it is a whole strip
            // (block-uniform); otherwise strip 0 (whole: these instances need n >= m > 1024) is
            // read and dropped, and a last, partial strip is read after the accumulation
            const bool roll_rows = ROLL && nxt < nstrips && whole(nxt);
            const T* nbase = A + (int64_t)(roll_rows ? nxt : 0) * SW;
#pragma unroll
            for (int t = 0; t < RPT / 8; ++t) {
                // rows 8t + j and 8t + j + 4 together, straight into the first stage
                ACC k4[NA][4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ACC lo[NA], hi[NA];
#pragma unroll
                    for (int aa = 0; aa < NA; ++aa) lo[aa] = hi[aa] = (ACC)0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const ACC xl = Elem<T>::template get<ACC>(av[8 * t + j], e);
                        const ACC xh = Elem<T>::template get<ACC>(av[8 * t + j + 4], e);
#pragma unroll
                        for (int aa = 0; aa < NA; ++aa) {
                            lo[aa] += xl * coef[aa][e];
                            hi[aa] += xh * coef[aa][e];
                        }
                    }
#pragma unroll
                    for (int aa = 0; aa < NA; ++aa) k4[aa][j] = reduce_scatter8_first(lo[aa], hi[aa], c);
                }
#pragma unroll
                for (int aa = 0; aa < NA; ++aa)
                    atomicAdd(&qs[aa * QS_A + (8 * t + c) * QS_K + g], (double)reduce_scatter8_rest(k4[aa], c));
                if constexpr (ROLL) {
                    // this group of rows is used: its registers take the next strip's rows
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int k = 8 * t + r;
                        av[k] = load_group_row(nbase + (int64_t)k * rowstride, group_nrec(k), lane_bytes);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if constexpr (ROLL) {
                if (nxt < nstrips) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) pfv[e] = Op::PF ? Op::pre(a, jn + e, jn + e < a.n) : 0.0;
                    if (!roll_rows)
                        load_segment<T, RPT, true>(A + (int64_t)nxt * SW + lane_off, A + (int64_t)nxt * SW + c * VEC,
                                                   rowstride, g, RG, m, a.n - jn, av);
                }
            }
        } else {
            // rolling form: the next whole strip's row k is loaded as soon as row k is summed
            const int nxt = strip + G;
            const int64_t jn = (int64_t)nxt * SW + c * VEC;
            const bool roll_rows = ROLL && nxt < nstrips && whole(nxt);
            const T* nbase = A + (int64_t)(roll_rows ? nxt : 0) * SW;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
#pragma unroll
                for (int aa = 0; aa < NA; ++aa) {
                    ACC sacc = (ACC)0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sacc += Elem<T>::template get<ACC>(av[k], e) * coef[aa][e];
                    q[aa][k] += sacc;
                }
                if constexpr (ROLL) {
                    if (roll_rows) av[k] = load_group_row(nbase + (int64_t)k * rowstride, group_nrec(k), lane_bytes);
                    if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
            }
            if constexpr (ROLL) {
                if (nxt < nstrips) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) pfv[e] = Op::PF ? Op::pre(a, jn + e, jn + e < a.n) : 0.0;
                    if (!roll_rows)
                        load_segment<T, RPT, true>(A + (int64_t)nxt * SW + lane_off, A + (int64_t)nxt * SW + c * VEC,
                                                   rowstride, g, RG, m, a.n - jn, av);
                }
            }
        }
        buf ^= 1;
    }

    if constexpr (QL) {
        static_assert(LPR == 8, "QL reduce-scatters over eight column lanes");
        __syncthreads();
        for (int i = tid; i < m; i += NT)
#pragma unroll
            for (int aa = 0; aa < NA; ++aa)
                a.part[((int64_t)aa * m + i) * G + blockIdx.x] = qs[aa * QS_A + (i / RG) * QS_K + i % RG];
    } else {
        // row sums over the LPR column lanes of each row group
#pragma unroll
        for (int aa = 0; aa < NA; ++aa)
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                ACC v = q[aa][k];
                v = group_sum<LPR>(v);
                q[aa][k] = v;
            }
        if (c == 0) {
#pragma unroll
            for (int aa = 0; aa < NA; ++aa)
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int i = g + RG * k;
                    if (i < m) a.part[((int64_t)aa * m + i) * G + blockIdx.x] = (double)q[aa][k];
                }
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

// Re-read form for BF16 storage beyond 2048 rows: rows are processed in chunks of CH per thread;
// the column-dot phase streams all chunks, then the accumulation phase streams them again, so the
// strip does not have to stay in registers. The second read misses L2 at these strip sizes
// (FETCH_SIZE shows twice the bytes of A), so up to 2048 rows the register-resident form, which
// reads A once, is used instead (2000 x 2*10^6: 1.89 ms against 2.35 ms).
template <typename T, typename ACC, int NT, int CH, int LPR, class Op>
__global__ __launch_bounds__(NT) void k_strip_rr(StripCall a, int nstrips, int K) {
    constexpr int VEC = Elem<T>::VEC;
    constexpr int SW = LPR * VEC;
    constexpr int RG = NT / LPR;
    constexpr int NW = NT / 64;
    constexpr int NA = Op::NACC, NCR = Op::NCR, ND = Op::ND;
    if (a.done != nullptr && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int MPAD = RG * K;
    ACC* vs = reinterpret_cast<ACC*>(smem_raw);                        // [ND][MPAD]
    ACC* red = vs + ND * MPAD;                                          // [2][ND][NW][SW]
    double* qs = reinterpret_cast<double*>(red + 2 * ND * NW * SW);    // [NA][MPAD]
    __shared__ double shr[NW];
    const int tid = threadIdx.x;
    const int c = tid % LPR, g = tid / LPR, lane = tid & 63, wid = tid >> 6;
    const int m = a.m;
    const int G = gridDim.x;
    const T* __restrict__ A = reinterpret_cast<const T*>(a.A);
    for (int i = tid; i < MPAD; i += NT) {
        vs[i] = (i < m) ? (ACC)a.vec0[i] : (ACC)0;
        if constexpr (ND > 1) vs[MPAD + i] = (i < m) ? (ACC)a.vec1[i] : (ACC)0;
    }
    for (int i = tid; i < NA * MPAD; i += NT) qs[i] = 0.0;
    __syncthreads();
    const typename Op::S st = Op::init(a);
    const uint32_t lane_off = (uint32_t)g * (uint32_t)a.ld + (uint32_t)(c * VEC);
    double cr[NCR > 0 ? NCR : 1] = {0.0};
    int buf = 0;
    for (int strip = blockIdx.x; strip < nstrips; strip += G) {
        const int64_t j0 = (int64_t)strip * SW + c * VEC;
        const int64_t left = a.n - j0;
        double pfv[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) pfv[e] = Op::PF ? Op::pre(a, j0 + e, j0 + e < a.n) : 0.0;
        ACC pd[ND][VEC];
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int e = 0; e < VEC; ++e) pd[d][e] = (ACC)0;
        for (int k0 = 0; k0 < K; k0 += CH) {
            uint4 av[CH];
            load_segment<T, CH, false>(A + (int64_t)strip * SW + (int64_t)(RG * k0) * a.ld + lane_off,
                                       A + (int64_t)strip * SW + c * VEC, (int64_t)RG * a.ld, g + RG * k0, RG, m,
                                       left, av);
#pragma unroll
            for (int kk = 0; kk < CH; ++kk)
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    const ACC vv = vs[d * MPAD + g + RG * (k0 + kk)];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) pd[d][e] += Elem<T>::template get<ACC>(av[kk], e) * vv;
                }
        }
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                ACC v = pd[d][e];
#pragma unroll
                for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                pd[d][e] = v;
            }
        ACC* rb = red + buf * ND * NW * SW;
        if (lane < LPR) {
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int e = 0; e < VEC; ++e) rb[(d * NW + wid) * SW + c * VEC + e] = pd[d][e];
        }
        __syncthreads();
        ACC coef[NA][VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            ACC t[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                t[d] = (ACC)0;
#pragma unroll
                for (int w = 0; w < NW; ++w) t[d] += rb[(d * NW + w) * SW + c * VEC + e];
            }
            ACC cf[NA];
            const int64_t j = j0 + e;
            Op::template column<ACC>(a, st, j, j < a.n, g == 0, t, cf, cr, pfv[e]);
#pragma unroll
            for (int aa = 0; aa < NA; ++aa) coef[aa][e] = cf[aa];
        }
        for (int k0 = 0; k0 < K; k0 += CH) {
            uint4 av[CH];
            load_segment<T, CH, false>(A + (int64_t)strip * SW + (int64_t)(RG * k0) * a.ld + lane_off,
                                       A + (int64_t)strip * SW + c * VEC, (int64_t)RG * a.ld, g + RG * k0, RG, m,
                                       left, av);
#pragma unroll
            for (int kk = 0; kk < CH; ++kk)
#pragma unroll
                for (int aa = 0; aa < NA; ++aa) {
                    ACC sacc = (ACC)0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sacc += Elem<T>::template get<ACC>(av[kk], e) * coef[aa][e];
                    sacc = group_sum<LPR>(sacc);
                    if (c == 0) qs[aa * MPAD + g + RG * (k0 + kk)] += (double)sacc;
                }
        }
        buf ^= 1;
    }
    __syncthreads();
    for (int i = tid; i < m; i += NT)
#pragma unroll
        for (int aa = 0; aa < NA; ++aa) a.part[((int64_t)aa * m + i) * G + blockIdx.x] = qs[aa * MPAD + i];
    if constexpr (NCR > 0) {
#pragma unroll
        for (int r = 0; r < NCR; ++r) {
            const double t = block_sum(cr[r], shr);
            if (tid == 0) a.colpart[(int64_t)blockIdx.x * NCR + r] = t;
        }
    }
}

// R <= 16 rows per thread with FP64 storage: the rolling form of the CG matvec when a row group's
// byte offsets fit 32 bits (100 x 2*10^6 FP64: 545 -> 345 us; 300 x 400000: 191 -> 166 us; equal
// at 500 x 100000 and at 512 threads). FP32 and BF16 storage keep the plain form: the rolling
// form pushes their register use past two waves per SIMD.
#define IPM_RPT_CASE(NTV, R)                                                                               \
    case R:                                                                                                \
        if constexpr (std::is_same<T, double>::value && R <= 16 && Op::PF && Op::ND == 1) {               \
            if (roll_fits(c, NTV)) {                                                                       \
                IPM_LAUNCH((k_strip<T, ACC, NTV, R, kLpr, false, Op, true>), dim3(p.grid), dim3(NTV), p.lds, \
                           st, c, p.nstrips);                                                              \
                break;                                                                                     \
            }                                                                                              \
        }                                                                                                  \
        IPM_LAUNCH((k_strip<T, ACC, NTV, R, kLpr, (R > 16), Op>), dim3(p.grid), dim3(NTV), p.lds, st, c,   \
                   p.nstrips);                                                                             \
        break;

// A row group's bytes (NT / lanes-per-row rows of ld elements) within 32-bit buffer offsets.
inline bool roll_fits(const StripCall& c, int nt) {
    const int es = c.dtype == 0 ? 8 : (c.dtype == 1 ? 4 : 2);
    return (uint64_t)(nt / kLpr) * (uint64_t)c.ld * (uint64_t)es <= (uint64_t)UINT32_MAX;
}

template <typename T, typename ACC, class Op>
hipError_t dispatch_nt(const StripCall& c, const StripPlan& p, hipStream_t st) {
    if (p.rr) {
        if (p.nt != kRrNt || p.rpt != kRrCh || p.lpr != kLpr) return hipErrorInvalidValue;
        IPM_LAUNCH((k_strip_rr<T, ACC, kRrNt, kRrCh, kLpr, Op>), dim3(p.grid), dim3(kRrNt), p.lds, st, c, p.nstrips,
                   p.kk);
        return hipGetLastError();
    }
    if (p.nt == 256) {
        switch (p.rpt) {
            IPM_RPT_CASE(256, 1)
            IPM_RPT_CASE(256, 2)
            IPM_RPT_CASE(256, 4)
            IPM_RPT_CASE(256, 8)
            IPM_RPT_CASE(256, 12)
            IPM_RPT_CASE(256, 16)
            default: return hipErrorInvalidValue;
        }
    } else if (p.nt == 512) {
        switch (p.rpt) {
            IPM_RPT_CASE(512, 12)
            IPM_RPT_CASE(512, 16)
            IPM_RPT_CASE(512, 24)
            IPM_RPT_CASE(512, 32)
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef IPM_RPT_CASE

template <class Op>
hipError_t dispatch_type(const StripCall& c, const StripPlan& p, hipStream_t st) {
    if constexpr (Op::ND > 1) {
        // the paired pass (the warm start's products) accumulates in FP64 only
        if (!c.acc64) return hipErrorInvalidValue;
        switch (c.dtype) {
            case 0: return dispatch_nt<double, double, Op>(c, p, st);
            case 1: return dispatch_nt<float, double, Op>(c, p, st);
            case 2: return dispatch_nt<bf16_t, double, Op>(c, p, st);
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (c.dtype) {
            case 0: return dispatch_nt<double, double, Op>(c, p, st);
            case 1:
                return c.acc64 ? dispatch_nt<float, double, Op>(c, p, st) : dispatch_nt<float, float, Op>(c, p, st);
            case 2:
                return c.acc64 ? dispatch_nt<bf16_t, double, Op>(c, p, st) : dispatch_nt<bf16_t, float, Op>(c, p, st);
            default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace

int rowsum_blocks(int m) { return (m + RNT / 64 - 1) / (RNT / 64); }

// Strip s goes to block s mod G and consecutive blocks to the 8 XCDs in turn, so with G a
// multiple of 8 every strip s lands on XCD s mod 8, round after round, and each XCD streams the
// same column offsets of every row. An odd G rotates the strips over the XCDs from one round to
// the next; the last block slot left idle costs less than that aliasing (measured: 500 x 10^6
// FP64 622 us at G = 511 against 658 us at 512; 2000 x 200000 FP64 583-595 us at 251-255 against
// 603-622 us at 256).
static int odd_grid(int grid) { return (grid > 1 && grid % 2 == 0) ? grid - 1 : grid; }

StripPlan strip_plan(int dtype, int m, int64_t n, int num_cu, int kind) {
    StripPlan p{};
    const size_t nd = kind == STRIP_MATVEC2 ? 2 : 1;   // vectors dotted with each column
    const int vec = dtype == 0 ? 2 : (dtype == 1 ? 4 : 8);
    p.lpr = kLpr;
    p.sw = kLpr * vec;
    p.nstrips = (int)((n + p.sw - 1) / p.sw);
    // rows per thread: the smallest instance covering m; 256-thread blocks (2 per CU, measured
    // best for m <= 512), then 512-thread blocks with up to 32 rows per thread (one per CU)
    struct Inst { int nt, rpt; };
    static const Inst insts[] = {{256, 1}, {256, 2}, {256, 4}, {256, 8}, {256, 12}, {256, 16},
                                 {512, 12}, {512, 16}, {512, 24}, {512, 32}};
    p.nt = 0;
    p.rr = 0;
    if (dtype == 2 && m > 2048) {
        // BF16 beyond the register-resident instances (more than 32 rows per thread): the re-read
        // form, rows padded to whole chunks
        const int rg = kRrNt / kLpr;
        int K = (m + rg - 1) / rg;
        K = (K + kRrCh - 1) / kRrCh * kRrCh;
        p.rr = 1;
        p.nt = kRrNt;
        p.rpt = kRrCh;
        p.kk = K;
        int grid = num_cu * 2;
        if (grid > p.nstrips) grid = p.nstrips;
        if (grid > kStripMaxGrid) grid = kStripMaxGrid;
        p.grid = odd_grid(grid < 1 ? 1 : grid);
        const int nw = kRrNt / 64;
        p.lds = 8 * nd * ((size_t)rg * K + 2 * (size_t)nw * p.sw) + 8 * 2 * (size_t)rg * K;
        if (p.lds > 160 * 1024) { p.nt = -1; return p; }
        return p;
    }
    for (const Inst& in : insts)
        if (in.rpt * (in.nt / kLpr) >= m) { p.nt = in.nt; p.rpt = in.rpt; break; }
    if (!p.nt) { p.nt = -1; return p; }   // m too large for the dense strip pass
    const int per_cu = p.nt == 256 ? 2 : 1;
    int grid = num_cu * per_cu;
    if (grid > p.nstrips) grid = p.nstrips;
    if (grid > kStripMaxGrid) grid = kStripMaxGrid;
    if (grid < 1) grid = 1;
    p.grid = odd_grid(grid);
    const int rg = p.nt / kLpr;
    const int nw = p.nt / 64;
    const size_t acc = 8;   // sized for FP64 accumulation (enough for FP32 too)
    p.lds = acc * nd * ((size_t)rg * p.rpt + 2 * (size_t)nw * p.sw);
    if (p.rpt > 16) p.lds += 8 * 2 * (size_t)p.rpt * (rg + 8);   // QL row sums (up to 2 accumulators)
    return p;
}

hipError_t launch_strip_pass(const StripCall& c, const StripPlan& p, hipStream_t st) {
    if (p.nt <= 0 || p.grid > kStripMaxGrid) return hipErrorInvalidValue;
    switch (c.kind) {
        case STRIP_MATVEC: return dispatch_type<OpMatvec>(c, p, st);
        case STRIP_RESID: return dispatch_type<OpResid>(c, p, st);
        case STRIP_DIR: return dispatch_type<OpDir>(c, p, st);
        case STRIP_MATVEC2: return dispatch_type<OpMatvec2>(c, p, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_strip_rowsum(const StripCall& c, const StripPlan& p, hipStream_t st) {
    const int nacc = strip_nacc(c.kind);
    const int ncr = c.kind == STRIP_RESID ? 1 : 0;
    hipLaunchKernelGGL(k_rowsum, dim3(rowsum_blocks(c.m)), dim3(RNT), 0, st, c, p.grid, nacc, ncr);
    return hipGetLastError();
}

hipError_t launch_strip(const StripCall& c, const StripPlan& p, hipStream_t st) {
    hipError_t e = launch_strip_pass(c, p, st);
    if (e != hipSuccess) return e;
    return launch_strip_rowsum(c, p, st);
}

}  // namespace ipmsk
