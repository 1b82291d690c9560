// Small in-register DFTs used to undo the pilot cover code.
//
// With the K x K DFT cover c[k,t] = exp(-j 2 pi k t / K), user k's pilot is
// isolated by z_k = sum_t exp(+j 2 pi k t / K) y_t (the conjugate cover), so
// every routine here computes the "+" sign transform, unnormalised:
//     out[k] = sum_t in[t] * exp(+j 2 pi k t / K).
// Sizes 1, 2, 3, 4, 8 are written out; 6 = 2*3, 12 = 3*4 and 24 = 3*8 use
// the prime-factor (Good-Thomas) mapping, which needs no twiddles between the
// two stages.  Other sizes fall back to the direct sum with a twiddle table.
#pragma once

#include <hip/hip_runtime.h>

namespace lmmse {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cmulj(float2 a) { return make_float2(-a.y, a.x); }  // j*a

template <int K>
struct Dft {
    // Direct sum; tw[r] = exp(+j 2 pi r / K) (only used for sizes below
    // without a dedicated routine).
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2* tw) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int t = 0; t < K; ++t) {
                float2 w = tw[(k * t) % K];
                acc.x += in[t].x * w.x - in[t].y * w.y;
                acc.y += in[t].x * w.y + in[t].y * w.x;
            }
            out[k] = acc;
        }
    }
};

template <>
struct Dft<1> {
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) { out[0] = in[0]; }
};

template <>
struct Dft<2> {
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) {
        out[0] = cadd(in[0], in[1]);
        out[1] = csub(in[0], in[1]);
    }
};

template <>
struct Dft<3> {
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) {
        // w = exp(+j 2 pi / 3) = -1/2 + j sqrt(3)/2
        const float h = 0.86602540378443864676f;
        float2 s = cadd(in[1], in[2]);
        float2 d = csub(in[1], in[2]);
        float2 m = make_float2(in[0].x - 0.5f * s.x, in[0].y - 0.5f * s.y);
        float2 jd = make_float2(-h * d.y, h * d.x);  // j sqrt(3)/2 (in1 - in2)
        out[0] = cadd(in[0], s);
        out[1] = cadd(m, jd);
        out[2] = csub(m, jd);
    }
};

template <>
struct Dft<4> {
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) {
        float2 a = cadd(in[0], in[2]);
        float2 b = csub(in[0], in[2]);
        float2 c = cadd(in[1], in[3]);
        float2 d = cmulj(csub(in[1], in[3]));
        out[0] = cadd(a, c);
        out[2] = csub(a, c);
        out[1] = cadd(b, d);
        out[3] = csub(b, d);
    }
};

template <>
struct Dft<8> {
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) {
        float2 e[4], o[4], E[4], O[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            e[i] = in[2 * i];
            o[i] = in[2 * i + 1];
        }
        Dft<4>::run(e, E, nullptr);
        Dft<4>::run(o, O, nullptr);
        const float r = 0.70710678118654752440f;
        float2 t0 = O[0];
        float2 t1 = make_float2(r * (O[1].x - O[1].y), r * (O[1].x + O[1].y));    // e^{j pi/4}
        float2 t2 = cmulj(O[2]);                                                  // e^{j pi/2}
        float2 t3 = make_float2(-r * (O[3].x + O[3].y), r * (O[3].x - O[3].y));   // e^{j 3pi/4}
        out[0] = cadd(E[0], t0); out[4] = csub(E[0], t0);
        out[1] = cadd(E[1], t1); out[5] = csub(E[1], t1);
        out[2] = cadd(E[2], t2); out[6] = csub(E[2], t2);
        out[3] = cadd(E[3], t3); out[7] = csub(E[3], t3);
    }
};

// Prime-factor composition for K = N1 * N2, gcd(N1, N2) = 1:
//   input  t = (N2 t1 + N1 t2) mod K,
//   output k = (k1 N2 (N2^-1 mod N1) + k2 N1 (N1^-1 mod N2)) mod K,
// out[k] = sum_t1 w_N1^{k1 t1} sum_t2 w_N2^{k2 t2} in[t].
template <int N1, int N2, int A, int Bi>
struct Pfa {
    static constexpr int K = N1 * N2;
    __device__ __forceinline__ static void run(const float2* in, float2* out, const float2*) {
        float2 u[N1][N2];
#pragma unroll
        for (int t1 = 0; t1 < N1; ++t1) {
            float2 v[N2];
#pragma unroll
            for (int t2 = 0; t2 < N2; ++t2) v[t2] = in[(N2 * t1 + N1 * t2) % K];
            Dft<N2>::run(v, u[t1], nullptr);
        }
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            float2 v[N1], z[N1];
#pragma unroll
            for (int t1 = 0; t1 < N1; ++t1) v[t1] = u[t1][k2];
            Dft<N1>::run(v, z, nullptr);
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) out[(k1 * N2 * A + k2 * N1 * Bi) % K] = z[k1];
        }
    }
};

template <> struct Dft<6> : Pfa<2, 3, 1, 2> {};    // 3^-1 mod 2 = 1, 2^-1 mod 3 = 2
template <> struct Dft<12> : Pfa<3, 4, 1, 3> {};   // 4^-1 mod 3 = 1, 3^-1 mod 4 = 3
template <> struct Dft<24> : Pfa<3, 8, 2, 3> {};   // 8^-1 mod 3 = 2, 3^-1 mod 8 = 3

// Sizes handled without a twiddle table.
__host__ __device__ constexpr bool dft_is_fast(int K) {
    return K == 1 || K == 2 || K == 3 || K == 4 || K == 6 || K == 8 || K == 12 || K == 24;
}

}  // namespace lmmse
