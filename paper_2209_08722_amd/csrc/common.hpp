// Shared device helpers for the ipmsk HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipmsk {

// Events for the next measured launch. When set, IPM_LAUNCH launches through
// hipExtLaunchKernelGGL, which records them at the kernel's own start and end, and clears them.
struct LaunchTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
extern thread_local LaunchTiming g_launch_timing;

#define IPM_LAUNCH(kernel, grid, block, shmem, stream, ...)                                            \
    do {                                                                                              \
        if (::ipmsk::g_launch_timing.start != nullptr) {                                              \
            hipEvent_t ev0_ = ::ipmsk::g_launch_timing.start, ev1_ = ::ipmsk::g_launch_timing.stop;    \
            ::ipmsk::g_launch_timing = ::ipmsk::LaunchTiming{};                                       \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev0_, ev1_, 0, __VA_ARGS__);     \
        } else {                                                                                      \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                       \
        }                                                                                             \
    } while (0)

constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kGaussDomain = 0xD1B54A32D192ED03ull;   // offset of the Gaussian sketch's key

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per-iteration description of the sparse embedding W (n x w, s nonzeros per row).
struct HashKeys {
    uint64_t key[8];   // stream start state of copy r
    int32_t s;         // nonzeros per row
    int32_t blk;       // w / s, width of each copy's bucket block
    double scale;      // 1 / sqrt(s)
};

// Bucket and sign of copy r of row j of W, from zj = (j + 1) * kPhi (mod 2^64), which a loop
// over j can advance by additions.
__device__ __forceinline__ void w_entry_z(const HashKeys& hk, int r, uint64_t zj, int& bucket, double& sign) {
    const uint64_t h = mix64(hk.key[r] + zj);
    const uint64_t hi = h >> 32;
    bucket = r * hk.blk + (int)((hi * (uint64_t)hk.blk) >> 32);
    sign = (h & 1ull) ? -1.0 : 1.0;
}

// Bucket and sign of copy r of row j of W.
__device__ __forceinline__ void w_entry(const HashKeys& hk, int r, uint64_t j, int& bucket, double& sign) {
    w_entry_z(hk, r, (j + 1ull) * kPhi, bucket, sign);
}

// ---- reductions -----------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over each group of eight consecutive lanes, left in every lane of the group; all 64 lanes
// must be active. Three DPP moves: quad permutations [1,0,3,2] and [2,3,0,1] (partners lane^1,
// lane^2), then the half-row mirror (lane i of eight reads lane 7-i, which holds the other quad's
// sum). No LDS traffic, unlike a shuffle, and the same pairings as the xor-1/2/4 butterfly.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <typename V>
__device__ __forceinline__ V sum8_lanes(V v) {
    v += dpp_mov<kDppQuadXor1>(v);
    v += dpp_mov<kDppQuadXor2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    return v;
}

// Eight sums over each group of eight consecutive lanes at once, scattered: lane c of the group
// returns the group's sum of v[c]. A reduce-scatter: the half-row mirror pairs lane c with 7-c
// (different halves of the index range), then quad xor 2 and quad xor 1; each stage sends the
// half of the values the partner keeps. 7 DPP moves and 7 adds, against 24 of each for eight
// separate group sums. All 64 lanes must be active.
// First stage alone, for values j and j + 4 (so a caller can produce the eight values in pairs
// and keep four partial sums live instead of eight values): lane c keeps value j + 4 (c & 4) summed
// with lane 7 - c's.
template <typename V>
__device__ __forceinline__ V reduce_scatter8_first(V lo, V hi, int c) {
    const bool b2 = (c & 4) != 0;
    return (b2 ? hi : lo) + dpp_mov<kDppHalfMirror>(b2 ? lo : hi);
}

// The remaining two stages on the four partial sums of reduce_scatter8_first.
template <typename V>
__device__ __forceinline__ V reduce_scatter8_rest(const V (&k4)[4], int c) {
    const bool b1 = (c & 2) != 0, b0 = (c & 1) != 0;
    V k2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const V send = b1 ? k4[j] : k4[j + 2];
        const V keep = b1 ? k4[j + 2] : k4[j];
        k2[j] = keep + dpp_mov<kDppQuadXor2>(send);
    }
    const V send = b0 ? k2[0] : k2[1];
    const V keep = b0 ? k2[1] : k2[0];
    return keep + dpp_mov<kDppQuadXor1>(send);
}

template <typename V>
__device__ __forceinline__ V reduce_scatter8(const V (&v)[8], int c) {
    const bool b2 = (c & 4) != 0, b1 = (c & 2) != 0, b0 = (c & 1) != 0;
    V k4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const V send = b2 ? v[j] : v[j + 4];
        const V keep = b2 ? v[j + 4] : v[j];
        k4[j] = keep + dpp_mov<kDppHalfMirror>(send);
    }
    V k2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const V send = b1 ? k4[j] : k4[j + 2];
        const V keep = b1 ? k4[j + 2] : k4[j];
        k2[j] = keep + dpp_mov<kDppQuadXor2>(send);
    }
    const V send = b0 ? k2[0] : k2[1];
    const V keep = b0 ? k2[1] : k2[0];
    return keep + dpp_mov<kDppQuadXor1>(send);
}

// Sum over each group of W consecutive lanes (W = 1, 2, 4, 8, 16, 32 or 64).
template <int W, typename V>
__device__ __forceinline__ V group_sum(V v) {
    if constexpr (W == 8) {
        return sum8_lanes(v);
    } else {
#pragma unroll
        for (int o = 1; o < W; o <<= 1) v += __shfl_xor(v, o, 64);
        return v;
    }
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide sum; every thread gets the result. `sh` needs blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += sh[i];
    return t;
}

__device__ __forceinline__ double block_min(double v, double* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_min(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < nw; ++i) t = fmin(t, sh[i]);
    return t;
}

// Sum of `cnt` partial values with stride `stride`, in a fixed order, computed by the whole
// block (deterministic: every block that calls it gets the same bits).
__device__ __forceinline__ double sum_partials(const double* p, int cnt, int stride, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) v += p[(int64_t)i * stride];
    return block_sum(v, sh);
}

// ---- element types ----------------------------------------------------------------------------

typedef uint16_t bf16_t;

__device__ __forceinline__ float bf16_to_float(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

template <typename T> struct Elem;

// 16-byte raw loads (kept as 4 dwords in registers) and conversion of element e to the
// accumulation type ACC (float or double) at the point of use.
template <> struct Elem<double> {
    static constexpr int VEC = 2;   // elements per 16-byte load
    __device__ __forceinline__ static uint4 raw16(const double* p) { return *reinterpret_cast<const uint4*>(p); }
    template <typename ACC>
    __device__ __forceinline__ static ACC get(const uint4& v, int e) {
        const uint32_t lo = e == 0 ? v.x : v.z, hi = e == 0 ? v.y : v.w;
        return (ACC)__hiloint2double((int)hi, (int)lo);
    }
    __device__ __forceinline__ static double load1(const double* p) { return *p; }
    __device__ __forceinline__ static double load1_stream(const double* p) { return __builtin_nontemporal_load(p); }
};

template <> struct Elem<float> {
    static constexpr int VEC = 4;
    __device__ __forceinline__ static uint4 raw16(const float* p) { return *reinterpret_cast<const uint4*>(p); }
    template <typename ACC>
    __device__ __forceinline__ static ACC get(const uint4& v, int e) {
        const uint32_t w = e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
        return (ACC)__uint_as_float(w);
    }
    __device__ __forceinline__ static float load1(const float* p) { return *p; }
    __device__ __forceinline__ static float load1_stream(const float* p) { return __builtin_nontemporal_load(p); }
};

template <> struct Elem<bf16_t> {
    static constexpr int VEC = 8;
    __device__ __forceinline__ static uint4 raw16(const bf16_t* p) { return *reinterpret_cast<const uint4*>(p); }
    template <typename ACC>
    __device__ __forceinline__ static ACC get(const uint4& v, int e) {
        const uint32_t w = (e >> 1) == 0 ? v.x : ((e >> 1) == 1 ? v.y : ((e >> 1) == 2 ? v.z : v.w));
        return (ACC)__uint_as_float((e & 1) ? (w & 0xFFFF0000u) : (w << 16));
    }
    __device__ __forceinline__ static float load1(const bf16_t* p) { return bf16_to_float(*p); }
    __device__ __forceinline__ static float load1_stream(const bf16_t* p) {
        return bf16_to_float(__builtin_nontemporal_load(p));
    }
};

// 16-byte load with the non-temporal hint, for data read once per pass (A in the single-read
// strip pass): streaming it without keeping it in the caches measured 12 % faster on a
// 400 MB FP64 A than plain loads.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 raw16_stream(const void* p) {
    const u32x4_t w = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(w.x, w.y, w.z, w.w);
}

// Raw 16-byte word holding elements [0, cnt) read one by one (tail of a row), zero elsewhere.
template <typename T>
__device__ __forceinline__ uint4 raw_partial(const T* p, int cnt) {
    union { uint4 v; T e[16 / sizeof(T)]; } u;
    u.v = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int e = 0; e < (int)(16 / sizeof(T)); ++e)
        if (e < cnt) u.e[e] = p[e];
    return u.v;
}

}  // namespace ipmsk
