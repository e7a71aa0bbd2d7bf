// Attainable-bandwidth probes: one read-only pass and one copy over device buffers. They are the
// measured denominators beside the vendor's 8 TB/s against which the streaming passes (matvec,
// sketch, residual and direction passes) are judged; they are not steps of the method.
//
// Both kernels give each block one contiguous range of 16-byte words and keep PU non-temporal
// 16-byte loads in flight per thread, as the strip passes do, so they measure the access pattern
// those passes use. The read pass sums the words (FP64) so that no load is dead and its result can
// be checked; per-block partials are added in a fixed order by one block.
#include "kernels.hpp"

namespace ipmsk {

namespace {

constexpr int PNT = 512;   // threads per block (8 waves)
constexpr int PU = 4;      // 16-byte loads in flight per thread per pass

typedef double f64x2_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(PNT) void k_stream_read(const double* __restrict__ x, int64_t pairs, int64_t per_block,
                                                     double* __restrict__ part) {
    __shared__ double sh[PNT / 64];
    const f64x2_t* x2 = reinterpret_cast<const f64x2_t*>(x);
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = (b0 + per_block < pairs) ? b0 + per_block : pairs;
    double acc = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += (int64_t)PNT * PU) {
        f64x2_t v[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int64_t j = i + (int64_t)u * PNT;
            v[u] = __builtin_nontemporal_load(x2 + (j < b1 ? j : b0));
            if (j >= b1) v[u] = f64x2_t{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < PU; ++u) acc += v[u].x + v[u].y;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out = sum of the partials in order, plus the odd last word when the count is odd.
__global__ __launch_bounds__(256) void k_stream_read_fin(const double* __restrict__ part, int nparts,
                                                         const double* __restrict__ tail, double* __restrict__ out) {
    __shared__ double sh[4];
    const double t = sum_partials(part, nparts, 1, sh);
    if (threadIdx.x == 0) out[0] = t + (tail != nullptr ? tail[0] : 0.0);
}

__global__ __launch_bounds__(PNT) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     int64_t words, int64_t per_block,
                                                     const unsigned char* __restrict__ src_tail,
                                                     unsigned char* __restrict__ dst_tail, int tail_bytes) {
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = (b0 + per_block < words) ? b0 + per_block : words;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += (int64_t)PNT * PU) {
        uint4 v[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int64_t j = i + (int64_t)u * PNT;
            v[u] = (j < b1) ? raw16_stream(src + j) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const int64_t j = i + (int64_t)u * PNT;
            if (j < b1) {
                u32x4_t w = {v[u].x, v[u].y, v[u].z, v[u].w};
                __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t*>(dst + j));
            }
        }
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < tail_bytes) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

// Blocks and the per-block range (a whole number of passes) for `units` 16-byte words.
void stream_grid(int64_t units, int num_cu, int* blocks, int64_t* per_block) {
    const int64_t pass = (int64_t)PNT * PU;
    const int64_t passes = units > 0 ? (units + pass - 1) / pass : 1;
    int64_t b = (int64_t)num_cu * 4;   // four 8-wave blocks per CU
    if (b > passes) b = passes;
    if (b < 1) b = 1;
    const int64_t per = (passes + b - 1) / b;
    *per_block = per * pass;
    *blocks = (int)((units + *per_block - 1) / *per_block);
    if (*blocks < 1) *blocks = 1;
}

}  // namespace

int stream_read_parts(int64_t count, int num_cu) {
    int blocks;
    int64_t per;
    stream_grid(count / 2, num_cu, &blocks, &per);
    return blocks;
}

hipError_t launch_stream_read(const double* x, int64_t count, double* part, double* out, int num_cu,
                              hipStream_t st) {
    int blocks;
    int64_t per;
    const int64_t pairs = count / 2;
    stream_grid(pairs, num_cu, &blocks, &per);
    IPM_LAUNCH(k_stream_read, dim3(blocks), dim3(PNT), 0, st, x, pairs, per, part);
    hipLaunchKernelGGL(k_stream_read_fin, dim3(1), dim3(256), 0, st, part, blocks,
                       (count & 1) ? x + (count - 1) : nullptr, out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, int num_cu, hipStream_t st) {
    int blocks;
    int64_t per;
    const int64_t words = bytes / 16;
    const int tail = (int)(bytes - words * 16);
    stream_grid(words, num_cu, &blocks, &per);
    const unsigned char* s = reinterpret_cast<const unsigned char*>(src);
    unsigned char* d = reinterpret_cast<unsigned char*>(dst);
    IPM_LAUNCH(k_stream_copy, dim3(blocks), dim3(PNT), 0, st, reinterpret_cast<const uint4*>(src),
               reinterpret_cast<uint4*>(dst), words, per, s + words * 16, d + words * 16, tail);
    return hipGetLastError();
}

}  // namespace ipmsk
