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

#define SAFR_HD __host__ __device__ __forceinline__

SAFR_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
SAFR_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
SAFR_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
SAFR_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * exp(DIR * i pi / 2): DIR = -1 multiplies by -i, DIR = +1 by +i
template <int DIR> SAFR_HD float2 rot90(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
// x * e^(DIR i theta) for a table entry w = (cos, sin)(theta), as one multiply and one FMA per part written
// out, so that every kernel rounds it the same way whatever the compiler would contract
template <int DIR> SAFR_HD float2 mul_twiddle(float2 x, float2 w) {
    return DIR < 0 ? make_float2(fmaf(x.x, w.x, x.y * w.y), fmaf(x.y, w.x, -(x.x * w.y)))
                   : make_float2(fmaf(x.x, w.x, -(x.y * w.y)), fmaf(x.y, w.x, x.x * w.y));
}

constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kCosPi8 = 0.92387953251128675613f;
constexpr float kTanPi8 = 0.41421356237309504880f;      // sqrt(2) - 1

template <int DIR> SAFR_HD void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR> SAFR_HD void dft4(float2* x) {
    float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    float2 t2 = cadd(x[1], x[3]), t3 = rot90<DIR>(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
}

// Butterflies with a twiddle w = f (a + i b) written as a scale f times a factor with one entry of
// magnitude one: u = o (a + i b) takes two FMAs (or two adds when |a| = |b| = 1), and e + f u, e - f u four
// FMAs, six operations instead of the eight of a complex product followed by an add and a subtract.
SAFR_HD void bfly_scaled(float2& lo, float2& hi, float2 e, float2 u, float f) {
    lo = make_float2(fmaf(f, u.x, e.x), fmaf(f, u.y, e.y));
    hi = make_float2(fmaf(-f, u.x, e.x), fmaf(-f, u.y, e.y));
}
// o (1 + i d) and o (-1 + i d), d = DIR: the twiddles of angle pi/4 and 3 pi/4 without their sqrt(1/2)
template <int DIR> SAFR_HD float2 mul_1p(float2 o) {
    return DIR < 0 ? make_float2(o.x + o.y, o.y - o.x) : make_float2(o.x - o.y, o.y + o.x);
}
template <int DIR> SAFR_HD float2 mul_1m(float2 o) {
    return DIR < 0 ? make_float2(o.y - o.x, -(o.x + o.y)) : make_float2(-(o.x + o.y), o.x - o.y);
}

template <int DIR> SAFR_HD void dft8(float2* x) {
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    // W8^1 = sqrt(1/2) (1 + i d), W8^2 = i d, W8^3 = sqrt(1/2) (-1 + i d)
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    bfly_scaled(x[1], x[5], e[1], mul_1p<DIR>(o[1]), kSqrtHalf);
    const float2 o2 = rot90<DIR>(o[2]);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    bfly_scaled(x[3], x[7], e[3], mul_1m<DIR>(o[3]), kSqrtHalf);
}

template <int DIR> SAFR_HD void dft16(float2* x) {
    float2 e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        e[i] = x[2 * i];
        o[i] = x[2 * i + 1];
    }
    dft8<DIR>(e);
    dft8<DIR>(o);
    // W16^k = (cos k pi/8, d sin k pi/8), d = DIR, with c = cos pi/8 and t = tan pi/8:
    // W^1 = c (1 + i d t), W^3 = c (t + i d), W^5 = c (-t + i d), W^7 = c (-1 + i d t),
    // W^2 = sqrt(1/2) (1 + i d), W^6 = sqrt(1/2) (-1 + i d), W^4 = i d
    constexpr float d = (float)DIR, dt = d * kTanPi8;
    x[0] = cadd(e[0], o[0]);
    x[8] = csub(e[0], o[0]);
    bfly_scaled(x[1], x[9], e[1], make_float2(fmaf(-dt, o[1].y, o[1].x), fmaf(dt, o[1].x, o[1].y)), kCosPi8);
    bfly_scaled(x[2], x[10], e[2], mul_1p<DIR>(o[2]), kSqrtHalf);
    bfly_scaled(x[3], x[11], e[3], make_float2(fmaf(kTanPi8, o[3].x, -d * o[3].y), fmaf(kTanPi8, o[3].y, d * o[3].x)),
                kCosPi8);
    const float2 o4 = rot90<DIR>(o[4]);
    x[4] = cadd(e[4], o4);
    x[12] = csub(e[4], o4);
    bfly_scaled(x[5], x[13], e[5], make_float2(fmaf(-kTanPi8, o[5].x, -d * o[5].y), fmaf(-kTanPi8, o[5].y, d * o[5].x)),
                kCosPi8);
    bfly_scaled(x[6], x[14], e[6], mul_1m<DIR>(o[6]), kSqrtHalf);
    bfly_scaled(x[7], x[15], e[7], make_float2(fmaf(-dt, o[7].y, -o[7].x), fmaf(dt, o[7].x, -o[7].y)), kCosPi8);
}

template <int N, int DIR> SAFR_HD void dft(float2* x) {
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
            lds[k1 * (S::N2 + 1) + n2] = mul_twiddle<DIR>(x[k1], tw[n2 * k1]);
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
    for (int k1 = 1; k1 < S::N1; ++k1) lds[k1 * (S::N2 + 1) + t] = mul_twiddle<DIR>(x[k1], tw[t * k1]);
}

// The thread's pass-1 twiddles in registers: twr[k1] = (cos, sin)(2 pi t k1 / M) for team thread t (shapes
// with N2 == T, where each thread applies the same N1 - 1 twiddles in every transform), read once from the
// table in global memory instead of from LDS in every transform.
template <int M>
__device__ __forceinline__ void load_pass1_twiddles(const float2* __restrict__ tw, int t,
                                                    float2 (&twr)[FftShape<M>::N1]) {
#pragma unroll
    for (int k1 = 0; k1 < FftShape<M>::N1; ++k1) twr[k1] = tw[t * k1];
}

// Pass 1 from inputs in registers with the twiddles in registers (see load_pass1_twiddles).
template <int M, int DIR>
__device__ __forceinline__ void fft_pass1_regs(int t, float2* __restrict__ lds, const float2 (&twr)[FftShape<M>::N1],
                                               float2 (&x)[FftShape<M>::N1]) {
    using S = FftShape<M>;
    static_assert(S::N2 == S::T, "one pass-1 sub-transform per thread");
    dft<S::N1, DIR>(x);
    lds[t] = x[0];
#pragma unroll
    for (int k1 = 1; k1 < S::N1; ++k1)
        lds[k1 * (S::N2 + 1) + t] = mul_twiddle<DIR>(x[k1], twr[k1]);
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
