// Shared device helpers for the ipmsk HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipmsk {

constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;

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

// Bucket and sign of copy r of row j of W.
__device__ __forceinline__ void w_entry(const HashKeys& hk, int r, uint64_t j, int& bucket, double& sign) {
    const uint64_t h = mix64(hk.key[r] + (j + 1ull) * kPhi);
    const uint64_t hi = h >> 32;
    bucket = r * hk.blk + (int)((hi * (uint64_t)hk.blk) >> 32);
    sign = (h & 1ull) ? -1.0 : 1.0;
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

// 16-byte vector loads converted to the accumulation type ACC (float or double).
template <> struct Elem<double> {
    static constexpr int VEC = 2;   // elements per 16-byte load
    template <typename ACC>
    __device__ __forceinline__ static void load16(const double* p, ACC* o) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = (ACC)v.x; o[1] = (ACC)v.y;
    }
    __device__ __forceinline__ static double load1(const double* p) { return *p; }
};

template <> struct Elem<float> {
    static constexpr int VEC = 4;
    template <typename ACC>
    __device__ __forceinline__ static void load16(const float* p, ACC* o) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = (ACC)v.x; o[1] = (ACC)v.y; o[2] = (ACC)v.z; o[3] = (ACC)v.w;
    }
    __device__ __forceinline__ static float load1(const float* p) { return *p; }
};

template <> struct Elem<bf16_t> {
    static constexpr int VEC = 8;
    template <typename ACC>
    __device__ __forceinline__ static void load16(const bf16_t* p, ACC* o) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            o[2 * q] = (ACC)__uint_as_float(w[q] << 16);
            o[2 * q + 1] = (ACC)__uint_as_float(w[q] & 0xFFFF0000u);
        }
    }
    __device__ __forceinline__ static float load1(const bf16_t* p) { return bf16_to_float(*p); }
};

}  // namespace ipmsk
