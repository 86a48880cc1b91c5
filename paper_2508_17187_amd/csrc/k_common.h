// Device helpers shared by the gridding and degridding kernels: complex
// values, vector and streaming loads / stores, kernel-table element decoding,
// complex multiply-adds, the pointing phasor and wavefront sums.
#pragma once

#include <type_traits>

#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

template <typename T>
struct cpx {
    T x, y;
};

// Per-sample records (npol values) moved in 16-byte pieces when their size
// allows: callers pass pointers to whole records, which are 16-byte aligned
// whenever the record size is a multiple of 16.
template <typename E, int N>
__device__ __forceinline__ void vload(const E *p, E (&out)[N]) {
    if constexpr ((N * sizeof(E)) % 16 == 0) {
        const E *q = (const E *)__builtin_assume_aligned(p, 16);
        __builtin_memcpy(out, q, N * sizeof(E));
    } else {
        for (int i = 0; i < N; ++i) out[i] = p[i];
    }
}

template <typename E, int N>
__device__ __forceinline__ void vstore(E *p, const E (&in)[N]) {
    if constexpr ((N * sizeof(E)) % 16 == 0) {
        E *q = (E *)__builtin_assume_aligned(p, 16);
        __builtin_memcpy(q, in, N * sizeof(E));
    } else {
        for (int i = 0; i < N; ++i) p[i] = in[i];
    }
}

// Streaming (nontemporal) moves of FP32 records that are read or written
// once per call (the visibilities and weights in the presum and expand
// passes), so they do not displace the grid, table and group data the
// other kernels reuse from cache.  FP64 records take the ordinary path:
// measured slower with streaming stores on this chip.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename E>
constexpr bool kStream = std::is_same<E, float>::value || std::is_same<E, cpx<float>>::value;

template <typename E, int N>
__device__ __forceinline__ void sload(const E *p, E (&out)[N]) {
    if constexpr ((N * sizeof(E)) % 16 == 0 && kStream<E>) {
        constexpr int K = N * sizeof(E) / 16;
        f32x4 t[K];
        const f32x4 *q = (const f32x4 *)__builtin_assume_aligned(p, 16);
        for (int i = 0; i < K; ++i) t[i] = __builtin_nontemporal_load(q + i);
        __builtin_memcpy(out, t, N * sizeof(E));
    } else {
        vload(p, out);
    }
}

template <typename E, int N>
__device__ __forceinline__ void sstore(E *p, const E (&in)[N]) {
    if constexpr ((N * sizeof(E)) % 16 == 0 && kStream<E>) {
        constexpr int K = N * sizeof(E) / 16;
        f32x4 t[K];
        __builtin_memcpy(t, in, N * sizeof(E));
        f32x4 *q = (f32x4 *)__builtin_assume_aligned(p, 16);
        for (int i = 0; i < K; ++i) __builtin_nontemporal_store(t[i], q + i);
    } else {
        vstore(p, in);
    }
}

// ---------------------------------------------------------------------------
// CF element access; f16 / bf16 pairs are decoded exactly to FP32 and
// multiplied by the plane's 2^-e.
template <int ST>
struct CFElem;
template <>
struct CFElem<LR_F64> {
    typedef double T;
    __device__ static cpx<double> load(const void *t, int64_t i, float) {
        double2 v = ((const double2 *)t)[i];
        return {v.x, v.y};
    }
};
template <>
struct CFElem<LR_F32> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float) {
        float2 v = ((const float2 *)t)[i];
        return {v.x, v.y};
    }
};
template <>
struct CFElem<LR_F32_CF16> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float sc) {
        uint32_t b = ((const uint32_t *)t)[i];
        _Float16 lo, hi;
        uint16_t l16 = (uint16_t)(b & 0xffffu), h16 = (uint16_t)(b >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return {(float)lo * sc, (float)hi * sc};
    }
};
template <>
struct CFElem<LR_F32_CFBF16> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float sc) {
        uint32_t b = ((const uint32_t *)t)[i];
        return {__uint_as_float(b << 16) * sc, __uint_as_float(b & 0xffff0000u) * sc};
    }
};

// Raw storage words of one CF element, loaded from a byte address and
// decoded later, so that a batch of loads is in flight before any value is
// needed.
template <int ST>
struct CFRaw;
template <>
struct CFRaw<LR_F64> {
    typedef double2 R;
    static constexpr int bytes = 16;
    __device__ static cpx<double> decode(R v, float) { return {v.x, v.y}; }
};
template <>
struct CFRaw<LR_F32> {
    typedef float2 R;
    static constexpr int bytes = 8;
    __device__ static cpx<float> decode(R v, float) { return {v.x, v.y}; }
};
template <>
struct CFRaw<LR_F32_CF16> {
    typedef uint32_t R;
    static constexpr int bytes = 4;
    __device__ static cpx<float> decode(R b, float sc) {
        _Float16 lo, hi;
        uint16_t l16 = (uint16_t)(b & 0xffffu), h16 = (uint16_t)(b >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return {(float)lo * sc, (float)hi * sc};
    }
};
template <>
struct CFRaw<LR_F32_CFBF16> {
    typedef uint32_t R;
    static constexpr int bytes = 4;
    __device__ static cpx<float> decode(R b, float sc) {
        return {__uint_as_float(b << 16) * sc, __uint_as_float(b & 0xffff0000u) * sc};
    }
};

// Real tables (no A term, no w-dependence): only the real word of each
// stored pair is loaded, and a tap costs two FMAs per polarisation instead
// of four (the imaginary parts are rounding noise, below 1e-16 relative).
template <int ST>
struct CFReal;
template <>
struct CFReal<LR_F64> {
    typedef double R;
    __device__ static double decode(R v, float) { return v; }
};
template <>
struct CFReal<LR_F32> {
    typedef float R;
    __device__ static float decode(R v, float) { return v; }
};
template <>
struct CFReal<LR_F32_CF16> {
    typedef uint16_t R;
    __device__ static float decode(R b, float sc) {
        _Float16 x;
        __builtin_memcpy(&x, &b, 2);
        return (float)x * sc;
    }
};
template <>
struct CFReal<LR_F32_CFBF16> {
    typedef uint16_t R;
    __device__ static float decode(R b, float sc) { return __uint_as_float((uint32_t)b << 16) * sc; }
};

// Wave-uniform copies of values that are the same in every lane.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)uni((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ void cmac(cpx<T> &acc, const cpx<T> &c, const cpx<T> &a) {
    acc.x = fma(c.x, a.x, acc.x);
    acc.x = fma(-c.y, a.y, acc.x);
    acc.y = fma(c.x, a.y, acc.y);
    acc.y = fma(c.y, a.x, acc.y);
}

// conj(c) * g accumulated
template <typename T>
__device__ __forceinline__ void cmac_conj(cpx<T> &acc, const cpx<T> &c, const cpx<T> &g) {
    acc.x = fma(c.x, g.x, acc.x);
    acc.x = fma(c.y, g.y, acc.x);
    acc.y = fma(c.x, g.y, acc.y);
    acc.y = fma(-c.y, g.x, acc.y);
}

// Pointing phasor of tap (tu, tv): f exp(-2 pi i ((tu O - ou) bu + (tv O - ov) bv)),
// argument formed and reduced modulo 1 in FP64.
template <typename T>
__device__ __forceinline__ cpx<T> phasor(const GroupMeta &gm, int tu, int tv, int O) {
    double a = fma((double)(tu * O - gm.ou), gm.bu, (double)(tv * O - gm.ov) * gm.bv);
    a = a - rint(a);
    cpx<T> r;
    if (sizeof(T) == 8) {
        double s, c;
        sincospi(-2.0 * a, &s, &c);
        r.x = (T)(gm.f * c);
        r.y = (T)(gm.f * s);
    } else {
        float s, c;
        sincospif((float)(-2.0 * a), &s, &c);
        r.x = (T)((float)gm.f * c);
        r.y = (T)((float)gm.f * s);
    }
    return r;
}

template <typename T>
__device__ __forceinline__ cpx<T> cmul(const cpx<T> &a, const cpx<T> &b) {
    cpx<T> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}


// Exact t / S and t % S for 0 <= t < 2^22 through a float reciprocal.
__device__ __forceinline__ void divmod_small(int t, int S, float invS, int &q, int &r) {
    q = (int)(((float)t + 0.5f) * invS);
    r = t - q * S;
    if (r < 0) { --q; r += S; } else if (r >= S) { ++q; r -= S; }
}

// s_waitcnt operand for vmcnt(0) with the other counters left alone
// (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVm0 = 0x0F70;

// Two neighbouring complex64 (or FP16 / BF16 pair) kernel or grid values in
// one load: 8-byte (4-byte) alignment is all the paired loads can promise.
typedef float f32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace lr
