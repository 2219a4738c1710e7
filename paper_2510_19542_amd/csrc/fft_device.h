// Device-side FFT building blocks for gfx950 (wave64).
//
// An M-point complex FFT (M = N1 * N2) is done by a "team" of T threads in two
// register passes with one LDS exchange (the four-step factorisation):
//   input index  n = N2 * n1 + n2,  output index k = k1 + N1 * k2,
//   pass 1: for each n2, Y[k1][n2] = W_M^(n2 k1) * sum_n1 x[N2 n1 + n2] W_N1^(n1 k1)
//   pass 2: for each k1, X[k1 + N1 k2] = sum_n2 Y[k1][n2] W_N2^(n2 k2)
// Teams never straddle a wavefront (T divides 64).  The twiddles W_M^e are read
// from a per-size table of (cos, sin)(2 pi e / M) computed in FP64 on the host.
// DIR = -1 is the forward transform exp(-2 pi i ...), DIR = +1 the inverse
// (unnormalised).
#pragma once
#include <hip/hip_runtime.h>

namespace safr {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * exp(DIR * i pi / 2): DIR = -1 multiplies by -i, DIR = +1 by +i
template <int DIR> __device__ __forceinline__ float2 rot90(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
// twiddle e^(DIR i 2 pi e / M) from the (cos, sin) table
template <int DIR> __device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int e) {
    float2 w = tw[e];
    return make_float2(w.x, DIR < 0 ? -w.y : w.y);
}

constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kCosPi8 = 0.92387953251128675613f;
constexpr float kSinPi8 = 0.38268343236508977173f;

template <int DIR> __device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR> __device__ __forceinline__ void dft4(float2* x) {
    float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    float2 t2 = cadd(x[1], x[3]), t3 = rot90<DIR>(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
}

template <int DIR> __device__ __forceinline__ void dft8(float2* x) {
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    const float d = (float)DIR;
    o[1] = cmul(o[1], make_float2(kSqrtHalf, d * kSqrtHalf));
    o[2] = rot90<DIR>(o[2]);
    o[3] = cmul(o[3], make_float2(-kSqrtHalf, d * kSqrtHalf));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 4] = csub(e[k], o[k]);
    }
}

template <int DIR> __device__ __forceinline__ void dft16(float2* x) {
    float2 e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        e[i] = x[2 * i];
        o[i] = x[2 * i + 1];
    }
    dft8<DIR>(e);
    dft8<DIR>(o);
    const float d = (float)DIR;
    o[1] = cmul(o[1], make_float2(kCosPi8, d * kSinPi8));
    o[2] = cmul(o[2], make_float2(kSqrtHalf, d * kSqrtHalf));
    o[3] = cmul(o[3], make_float2(kSinPi8, d * kCosPi8));
    o[4] = rot90<DIR>(o[4]);
    o[5] = cmul(o[5], make_float2(-kSinPi8, d * kCosPi8));
    o[6] = cmul(o[6], make_float2(-kSqrtHalf, d * kSqrtHalf));
    o[7] = cmul(o[7], make_float2(-kCosPi8, d * kSinPi8));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = cadd(e[k], o[k]);
        x[k + 8] = csub(e[k], o[k]);
    }
}

template <int N, int DIR> __device__ __forceinline__ void dft(float2* x) {
    if constexpr (N == 2) dft2<DIR>(x[0], x[1]);
    else if constexpr (N == 4) dft4<DIR>(x);
    else if constexpr (N == 8) dft8<DIR>(x);
    else if constexpr (N == 16) dft16<DIR>(x);
    else static_assert(N == 2 || N == 4 || N == 8 || N == 16, "unsupported radix");
}

// Orders the LDS accesses of one wavefront.  A team never straddles a wavefront and the DS
// operations of a wavefront are performed in issue order, so the exchanges inside a team's own
// region need no workgroup barrier: the fences and the wave barrier only keep the compiler from
// moving memory operations across this point.
__device__ __forceinline__ void team_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Factorisation and team size per transform length.
template <int M> struct FftShape;
template <> struct FftShape<32>  { static constexpr int N1 = 8,  N2 = 4,  T = 4;  };
template <> struct FftShape<64>  { static constexpr int N1 = 8,  N2 = 8,  T = 8;  };
template <> struct FftShape<128> { static constexpr int N1 = 16, N2 = 8,  T = 8;  };
template <> struct FftShape<256> { static constexpr int N1 = 16, N2 = 16, T = 16; };

// LDS floats2 needed per team for the pass-1 -> pass-2 exchange (rows padded by one).
template <int M> constexpr int team_lds() { return FftShape<M>::N1 * (FftShape<M>::N2 + 1); }

// Pass 1 for team thread t: sub-sequences n2 = t, t + T, ...; load(idx) returns x[idx].
template <int M, int DIR, class Load>
__device__ __forceinline__ void fft_pass1(int t, float2* __restrict__ lds, const float2* __restrict__ tw,
                                          Load load) {
    using S = FftShape<M>;
#pragma unroll
    for (int s = 0; s < S::N2 / S::T; ++s) {
        const int n2 = t + S::T * s;
        float2 x[S::N1];
#pragma unroll
        for (int n1 = 0; n1 < S::N1; ++n1) x[n1] = load(S::N2 * n1 + n2);
        dft<S::N1, DIR>(x);
        lds[n2] = x[0];
#pragma unroll
        for (int k1 = 1; k1 < S::N1; ++k1)
            lds[k1 * (S::N2 + 1) + n2] = cmul(x[k1], twiddle<DIR>(tw, n2 * k1));
    }
}

// Pass 1 from inputs already in registers: x[n1] = input[N2 * n1 + t] (shapes with N2 == T).
template <int M, int DIR>
__device__ __forceinline__ void fft_pass1_regs(int t, float2* __restrict__ lds, const float2* __restrict__ tw,
                                               float2 (&x)[FftShape<M>::N1]) {
    using S = FftShape<M>;
    static_assert(S::N2 == S::T, "one pass-1 sub-transform per thread");
    dft<S::N1, DIR>(x);
    lds[t] = x[0];
#pragma unroll
    for (int k1 = 1; k1 < S::N1; ++k1) lds[k1 * (S::N2 + 1) + t] = cmul(x[k1], twiddle<DIR>(tw, t * k1));
}

// Pass 2 for team thread t: k1 = t, t + T, ...; store(k, value) receives X[k].
template <int M, int DIR, class Store>
__device__ __forceinline__ void fft_pass2(int t, const float2* __restrict__ lds, Store store) {
    using S = FftShape<M>;
#pragma unroll
    for (int s = 0; s < S::N1 / S::T; ++s) {
        const int k1 = t + S::T * s;
        float2 z[S::N2];
#pragma unroll
        for (int n2 = 0; n2 < S::N2; ++n2) z[n2] = lds[k1 * (S::N2 + 1) + n2];
        dft<S::N2, DIR>(z);
#pragma unroll
        for (int k2 = 0; k2 < S::N2; ++k2) store(k1 + S::N1 * k2, z[k2]);
    }
}

// Pass 2 split in two, for transforms whose output overwrites the exchange buffer:
// fft_pass2_load takes every value the thread needs into registers (a barrier may
// then separate it from the stores), fft_pass2_regs transforms and stores.
template <int M>
__device__ __forceinline__ void fft_pass2_load(int t, const float2* __restrict__ lds,
                                               float2 (&z)[FftShape<M>::N1 / FftShape<M>::T][FftShape<M>::N2]) {
    using S = FftShape<M>;
#pragma unroll
    for (int s = 0; s < S::N1 / S::T; ++s)
#pragma unroll
        for (int n2 = 0; n2 < S::N2; ++n2) z[s][n2] = lds[(t + S::T * s) * (S::N2 + 1) + n2];
}

template <int M, int DIR, class Store>
__device__ __forceinline__ void fft_pass2_regs(int t, float2 (&z)[FftShape<M>::N1 / FftShape<M>::T][FftShape<M>::N2],
                                               Store store) {
    using S = FftShape<M>;
#pragma unroll
    for (int s = 0; s < S::N1 / S::T; ++s) {
        dft<S::N2, DIR>(z[s]);
#pragma unroll
        for (int k2 = 0; k2 < S::N2; ++k2) store(t + S::T * s + S::N1 * k2, z[s][k2]);
    }
}

}  // namespace safr
