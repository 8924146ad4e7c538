// Device-side helpers shared by the SpMV kernels.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include <cstdint>
#include <type_traits>

#include "kdefs.h"

namespace csr {

// Storage traits: stored value type V, vector type X (x and y), accumulator A.
template <int S> struct St;
template <> struct St<CSR_VAL_F64> {
    using V = double;
    using X = double;
    using A = double;
    static __device__ __forceinline__ A cvt(V v) { return v; }
};
template <> struct St<CSR_VAL_F32> {
    using V = float;
    using X = float;
    using A = float;
    static __device__ __forceinline__ A cvt(V v) { return v; }
};
template <> struct St<CSR_VAL_BF16> {
    using V = uint16_t;  // raw BF16 bits
    using X = float;
    using A = float;
    static __device__ __forceinline__ A cvt(V v) { return __uint_as_float((uint32_t)v << 16); }
};

__device__ __forceinline__ double fma_acc(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return fmaf(a, b, c); }

// Streaming loads: the nt variant marks val/col as non-temporal so they do not
// evict the x vector from L2 and the Infinity Cache.
template <bool NT, class T> __device__ __forceinline__ T ld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Sum over the G lanes of a lane group (G a power of two <= 64). Butterfly
// order is fixed, so the result is deterministic.
template <int G, class A> __device__ __forceinline__ A group_sum(A v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

template <int G> __device__ __forceinline__ int32_t group_max(int32_t v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, G));
    return v;
}

template <int G> __device__ __forceinline__ int32_t group_isum(int32_t v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Inclusive prefix sum over the G lanes of a lane group.
template <int G> __device__ __forceinline__ int32_t group_scan(int32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        int32_t t = __shfl_up(v, off, G);
        if (lane >= off) v += t;
    }
    return v;
}

// Delta code of entry j: the first entry of a row is a signed offset from the
// row index, later entries unsigned gaps from the previous column.
template <int IDX> __device__ __forceinline__ int32_t load_code(const void *codes, int64_t j,
                                                                bool first) {
    if constexpr (IDX == IDX_D16) {
        uint16_t u = static_cast<const uint16_t *>(codes)[j];
        return first ? (int32_t)(int16_t)u : (int32_t)u;
    } else {
        uint8_t u = static_cast<const uint8_t *>(codes)[j];
        return first ? (int32_t)(int8_t)u : (int32_t)u;
    }
}

}  // namespace csr
