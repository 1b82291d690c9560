// Split-precision helpers: x = hi + lo in BF16 or FP16 (round to nearest
// even), FP16 lo parts scaled by 2^11, and the 16x16x32 matrix-core product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lmmse.h"

namespace lmmse {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <bool FP16>
__device__ __forceinline__ void split2(float v, uint16_t& h, uint16_t& l) {
    if constexpr (FP16) {
        const _Float16 hh = (_Float16)v;
        const _Float16 ll = (_Float16)((v - (float)hh) * 2048.0f);
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    } else {
        const __bf16 hh = (__bf16)v;
        const __bf16 ll = (__bf16)(v - (float)hh);
        h = __builtin_bit_cast(uint16_t, hh);
        l = __builtin_bit_cast(uint16_t, ll);
    }
}

// FP16 hi parts hold magnitudes below 65504 (a larger value rounds to inf,
// NaN stays NaN): false when v leaves that range.
__device__ __forceinline__ bool f16_in_range(float2 v) {
    return fabsf(v.x) < 65504.0f && fabsf(v.y) < 65504.0f;
}

// Records LMMSE_ERR_RANGE (info -1) in a status word [code, info] when any
// lane of the wave saw an out-of-range value; the first error wins.  `bad`
// may differ between lanes.
__device__ __forceinline__ void report_range(bool bad, int* status) {
    if (__any(bad) && (threadIdx.x & 63) == 0 && status)
        if (atomicCAS(status, 0, LMMSE_ERR_RANGE) == 0) status[1] = -1;
}

// hi and lo of one complex value, each as a packed (re, im) pair
template <bool FP16>
__device__ __forceinline__ void split_c(float2 v, uint32_t& hi, uint32_t& lo) {
    uint16_t hr, lr, hi_, li;
    split2<FP16>(v.x, hr, lr);
    split2<FP16>(v.y, hi_, li);
    hi = (uint32_t)hr | ((uint32_t)hi_ << 16);
    lo = (uint32_t)lr | ((uint32_t)li << 16);
}

template <bool FP16>
__device__ __forceinline__ floatx4 mma(const float4& a, const float4& b, floatx4 c) {
    if constexpr (FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// 2^11 hi for the FP16 hi_W hi_X product (exact for |hi| < 32).
__device__ __forceinline__ float4 scale2048_f16(const float4& a) {
    f16x8 h = __builtin_bit_cast(f16x8, a);
    h = h * (_Float16)2048.0f;
    return __builtin_bit_cast(float4, h);
}

// Per-window split filter parts, chunk-major: entry (o, col) of the window
// whose block starts at wbase (window index x B x W16) sits at
// wbase + ((col / 16) B + o) 16 + col % 16, so that the 16 columns of one
// chunk of all B rows are one contiguous block; W16 = Wn rounded up to 16.
__device__ __forceinline__ long long split_w_index(long long wbase, int B, int o, int col) {
    return wbase + ((long long)(col >> 4) * B + o) * 16 + (col & 15);
}

// Entry (o, col) of a window's split filter parts, and at col 0 the zero pad
// entries Wn..W16-1 of row o.
__device__ __forceinline__ void store_split_w(uint32_t* whi, uint32_t* wlo, long long wbase, int B, int o,
                                              int col, int Wn, int W16, double2 w, int fp16) {
    uint32_t h, l;
    const float2 wf = make_float2((float)w.x, (float)w.y);
    if (fp16)
        split_c<true>(wf, h, l);
    else
        split_c<false>(wf, h, l);
    const long long i = split_w_index(wbase, B, o, col);
    whi[i] = h;
    wlo[i] = l;
    if (col == 0)
        for (int c = Wn; c < W16; ++c) {
            const long long k = split_w_index(wbase, B, o, c);
            whi[k] = 0u;
            wlo[k] = 0u;
        }
}

}  // namespace lmmse
