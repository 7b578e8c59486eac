// Internal helpers shared by the gfx950 HIP sources of the D-VQLS library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "dvq.h"

namespace dvq {

// Records a one-line message for dvq_last_error() and returns `s`.
dvq_status fail(dvq_status s, const char* fmt, ...);

inline hipStream_t stream_of(dvq_stream s) { return reinterpret_cast<hipStream_t>(s); }

#define DVQ_TRY_HIP(call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::dvq::fail(DVQ_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define DVQ_CHECK_LAUNCH(name)                                                         \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return ::dvq::fail(DVQ_EDEVICE, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

#define DVQ_REQUIRE(cond, ...)                                                         \
    do {                                                                               \
        if (!(cond)) return ::dvq::fail(DVQ_EINVAL, __VA_ARGS__);                      \
    } while (0)

// Sets the dynamic-LDS limit of a kernel once; returns hipSuccess or the error.
hipError_t allow_lds(const void* kernel, size_t bytes);

constexpr size_t kMaxLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup

// --------------------------------------------------------------- device side

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// a * i^p for p in 0..3 (exact: only swaps and sign changes).
template <typename T>
__device__ __forceinline__ cplx<T> mul_ipow(cplx<T> a, int p) {
    switch (p & 3) {
        case 0: return a;
        case 1: return {-a.im, a.re};
        case 2: return {-a.re, -a.im};
        default: return {a.im, -a.re};
    }
}

__device__ __forceinline__ int parity(uint32_t v) { return __popc(v) & 1; }

// Fused multiply-add in the operand's own precision.
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Block-wide sum of one double per thread; every thread gets the result.
// Fixed reduction order (wavefront butterfly, then waves in index order), so
// the result is bit-reproducible for a given block size.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ T block_sum(T v, T* scratch /* >= blockDim.x/64 entries */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < nw; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

}  // namespace dvq
