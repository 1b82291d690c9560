// Input side shared by the block-filtering kernels (apply_f32.hip,
// apply_split.hip): 4-wave workgroups over 192 LS columns, the window
// streamed in chunks of 16 complex rows.
//
//  * raw inputs of a chunk (H_LS, or the K pilot symbols y of each antenna on
//    the fused path) are loaded into registers one chunk ahead;
//  * the pilot slice x_k[s0 + 16c + r] of a chunk is loaded two chunks ahead
//    and staged in a double-buffered LDS array;
//  * filter rows go straight from global memory to LDS with the direct
//    global-to-LDS loads of gfx950 (no register staging);
//  * workgroups are remapped so that each XCD takes a contiguous tile range.
//
// Addresses are a workgroup-uniform base (scalar registers) plus a 32-bit
// per-lane offset, which keeps the per-lane address state to one register
// per stream.
#pragma once

#include "internal.h"

namespace lmmse {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kCT = 3;                     // 16-column MFMA tiles per wave
constexpr int kCols = 16 * kCT * kWaves;   // 192 LS columns per workgroup
// Row stride, in 16-byte slots, of an LS chunk in LDS (slot-major [slot][col]):
// a lane group reads 16 consecutive columns of one slot (256 contiguous
// bytes), the odd stride spreads the slots a writing lane group touches over
// distinct banks, and the columns of one thread's users differ by constant
// offsets.
constexpr int kXP = kCols + 1;

__device__ __forceinline__ long long xcd_remap(long long id, long long total) {
    const long long NX = 8;
    const long long q = total / NX, r = total % NX;
    const long long x = id % NX, k = id / NX;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Raw LS-path inputs one thread holds for one chunk (window rows [16c, 16c+16)):
// KF == 0: H_LS values of (column, row) pairs; KF > 0: the KF pilot symbols
// of (antenna, row) pairs.
template <int KF>
struct RawRegs {
    static constexpr int NPAIR = KF == 0 ? kCols * 16 : (kCols / KF) * 16;
    static constexpr int TX = (NPAIR + kThreads - 1) / kThreads;
    static constexpr int KV = KF == 0 ? 1 : KF;
    float2 v[TX][KV];
};

// Args: x, ncols, N, Wn as in the kernels' argument blocks.
template <int KF, typename Args>
__device__ __forceinline__ void load_raw(const Args& a, int tid, int cc, int s0, long long c0,
                                         RawRegs<KF>& R) {
    using CR = RawRegs<KF>;
#pragma unroll
    for (int u = 0; u < CR::TX; ++u) {
        const int i = tid + u * kThreads;
        const int cq = i >> 4, r = i & 15;
        const int j = cc * 16 + r;
        if constexpr (KF == 0) {
            const float2* xb = a.x + c0 * a.N + s0;
            const bool live = i < CR::NPAIR && j < a.Wn && c0 + cq < a.ncols;
            const unsigned o = (unsigned)(cq * a.N + j);
            R.v[u][0] = live ? xb[o] : make_float2(0.f, 0.f);
        } else {
            const long long ant0 = c0 / KF;
            const bool live = i < CR::NPAIR && j < a.Wn && ant0 + cq < a.ncols / KF;
            const unsigned o = (unsigned)(cq * KF * a.N + j);
#pragma unroll
            for (int tt = 0; tt < KF; ++tt) {
                const float2* xb = a.x + (ant0 * KF + tt) * a.N + s0;
                R.v[u][tt] = live ? xb[o] : make_float2(0.f, 0.f);
            }
        }
    }
}

// Pilot slice of one chunk, x_k[s0 + 16c + r] at [k*16 + r] (fused path).
// Rows past the window read a clamped, valid subcarrier; their LS values are
// zeroed when stored.
template <int KF>
struct PilotRegs {
    static constexpr int NS = (KF == 0 ? 1 : KF) * 16;
    static constexpr int TX = (NS + kThreads - 1) / kThreads;
    float2 v[TX];
};

template <int KF, typename Args>
__device__ __forceinline__ void load_pil(const Args& a, int s0, int cc, int tid, PilotRegs<KF>& P) {
#pragma unroll
    for (int u = 0; u < PilotRegs<KF>::TX; ++u) {
        const int i = tid + u * kThreads;
        if (i < PilotRegs<KF>::NS) {
            const int n = min(s0 + cc * 16 + (i & 15), a.N - 1);
            P.v[u] = a.pilots[(unsigned)((i >> 4) * a.N + n)];
        }
    }
}

template <int KF>
__device__ __forceinline__ void store_pil(const PilotRegs<KF>& P, float2* pl, int tid) {
#pragma unroll
    for (int u = 0; u < PilotRegs<KF>::TX; ++u) {
        const int i = tid + u * kThreads;
        if (i < PilotRegs<KF>::NS) pl[i] = P.v[u];
    }
}

// Copies UNITS 16-byte units (a multiple of 64) from global src to LDS dst
// with the direct global-to-LDS loads: each wave instruction moves 64 x 16
// bytes to 1 KB of LDS, wave w taking runs 4u + w.  `wave` must be uniform.
template <int UNITS>
__device__ __forceinline__ void dma_copy(const float4* src, float4* dst, int wave, int lane) {
    static_assert(UNITS % 64 == 0, "whole 1 KB runs");
#pragma unroll
    for (int u = 0; u < (UNITS + kThreads - 1) / kThreads; ++u) {
        const int base = u * kThreads + wave * 64;
        if (base < UNITS) {
            const float4* s = src + base;
            s += lane;
            __builtin_amdgcn_global_load_lds(
                s, (__attribute__((address_space(3))) void*)(dst + base), 16, 0, 0);
        }
    }
}

// vmcnt(0): this wave's global loads, including its LDS copies, have landed.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

}  // namespace lmmse
