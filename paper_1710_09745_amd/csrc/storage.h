// Storage policies of block vectors and folded links, and their accessors.
//
//   F64 : complex double pairs                    (16 bytes per complex)
//   F32 : complex float pairs                     ( 8 bytes per complex)
//   H16 : FP16 pairs scaled by one FP32 number per (column, site)
//   B16 : BF16 pairs scaled by one FP32 number per (column, site)
//   X16 : 16-bit fixed-point pairs (q / 32767) scaled the same way
//
// A group of K complex numbers that share a scale is one (column, site) entry:
// the 3 colour components of a vector, or the 9 entries of a folded link matrix.
// Data layout [cols][K][Vh] (pairs), scales [cols][Vh] stored right after the
// data in the same allocation; a 16-bit group stores x / s with s = max |re|,|im|
// over the group, so every stored component lies in [-1, 1].
// Arithmetic runs in FP64 for F64 and in FP32 for every other policy.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace bcg {

struct F64 {
    using real = double;
    using pair = double2;
    static constexpr bool scaled = false;
    static constexpr int bytes = 16;
};
struct F32 {
    using real = float;
    using pair = float2;
    static constexpr bool scaled = false;
    static constexpr int bytes = 8;
};
struct H16 {
    using real = float;
    using pair = unsigned int;
    static constexpr bool scaled = true;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ unsigned short enc(float x) {
        return __builtin_bit_cast(unsigned short, (_Float16)x);
    }
    static __device__ __forceinline__ float dec(unsigned short u) {
        return (float)__builtin_bit_cast(_Float16, u);
    }
};
struct B16 {
    using real = float;
    using pair = unsigned int;
    static constexpr bool scaled = true;
    static constexpr int bytes = 4;
    static __device__ __forceinline__ unsigned short enc(float x) {
        return __builtin_bit_cast(unsigned short, (__bf16)x);
    }
    static __device__ __forceinline__ float dec(unsigned short u) {
        return __builtin_bit_cast(float, (unsigned int)u << 16);
    }
};

struct X16 {
    using real = float;
    using pair = unsigned int;
    static constexpr bool scaled = true;
    static constexpr int bytes = 4;
    // x in [-1, 1] (the group is divided by its largest component): q = rint(32767 x)
    static __device__ __forceinline__ unsigned short enc(float x) {
        return (unsigned short)(short)__float2int_rn(x * 32767.0f);
    }
    static __device__ __forceinline__ float dec(unsigned short u) { return (float)(short)u * (1.0f / 32767.0f); }
};

// Buffer-resource loads.  A resource is made from a wave-uniform base address
// (SGPRs); the per-lane byte offset travels in one VGPR and the per-plane byte
// offset in an SGPR, so a gather needs no per-load 64-bit address arithmetic.
// Offsets from a base stay below 4 GiB: bases are re-made per column or per
// folded matrix.  aux = 2 marks a streaming (non-temporal) load.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}
enum { AUX_NONE = 0, AUX_NT = 2 };

template <int AUX> __device__ __forceinline__ C2<double> buf_pair(rsrc_t r, unsigned vo, unsigned so, double) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, AUX);
    const double2 p = __builtin_bit_cast(double2, u);
    return C2<double>{p.x, p.y};
}
template <int AUX> __device__ __forceinline__ C2<float> buf_pair(rsrc_t r, unsigned vo, unsigned so, float) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX);
    const float2 p = __builtin_bit_cast(float2, u);
    return C2<float>{p.x, p.y};
}

// K complex numbers of one group: component c at byte offset vo + c * plane of
// resource d; for scaled policies the scale at byte offset svo of resource sc
template <typename S, int K, int AUX>
__device__ __forceinline__ void buf_group(rsrc_t d, rsrc_t sc, unsigned vo, unsigned svo, unsigned plane,
                                          C2<typename S::real> v[K]) {
    if constexpr (!S::scaled) {
#pragma unroll
        for (int c = 0; c < K; ++c) v[c] = buf_pair<AUX>(d, vo, c * plane, (typename S::real)0);
    } else {
        const float s = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sc, svo, 0, AUX));
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const unsigned int u = __builtin_amdgcn_raw_buffer_load_b32(d, vo, c * plane, AUX);
            v[c] = C2<float>{S::dec((unsigned short)(u & 0xffffu)) * s, S::dec((unsigned short)(u >> 16)) * s};
        }
    }
}

// streaming (non-temporal) loads: data read once, kept out of the way of reused lines
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ unsigned int ld_nt(const unsigned int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }

// load the K complex numbers of group (col, i); NT: non-temporal loads
template <typename S, int K, bool NT = false>
__device__ __forceinline__ void load_group(const typename S::pair* __restrict__ d,
                                           const float* __restrict__ sc, long Vh, long col, long i,
                                           C2<typename S::real> v[K]) {
    if constexpr (!S::scaled) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const typename S::pair* a = d + (col * K + c) * Vh + i;
            const typename S::pair p = NT ? ld_nt(a) : *a;
            v[c] = C2<typename S::real>{p.x, p.y};
        }
    } else {
        const float s = NT ? ld_nt(sc + col * Vh + i) : sc[col * Vh + i];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const unsigned int* a = d + (col * K + c) * Vh + i;
            const unsigned int u = NT ? ld_nt(a) : *a;
            v[c] = C2<float>{S::dec((unsigned short)(u & 0xffffu)) * s, S::dec((unsigned short)(u >> 16)) * s};
        }
    }
}

// one complex number of group (col, i), component c (16-bit: needs the scale)
template <typename S, int K>
__device__ __forceinline__ C2<double> load_one_d(const typename S::pair* __restrict__ d,
                                                 const float* __restrict__ sc, long Vh, long col,
                                                 int c, long i) {
    if constexpr (!S::scaled) {
        const typename S::pair p = d[(col * K + c) * Vh + i];
        return C2<double>{(double)p.x, (double)p.y};
    } else {
        const float s = sc[col * Vh + i];
        const unsigned int u = d[(col * K + c) * Vh + i];
        return C2<double>{(double)(S::dec((unsigned short)(u & 0xffffu)) * s),
                          (double)(S::dec((unsigned short)(u >> 16)) * s)};
    }
}

// store the K complex numbers of group (col, i); R is the arithmetic type of v
template <typename S, int K, typename R>
__device__ __forceinline__ void store_group(typename S::pair* __restrict__ d, float* __restrict__ sc,
                                            long Vh, long col, long i, const C2<R> v[K]) {
    if constexpr (!S::scaled) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            typename S::pair p;
            p.x = (typename S::real)v[c].re;
            p.y = (typename S::real)v[c].im;
            d[(col * K + c) * Vh + i] = p;
        }
    } else {
        float m = 0.0f;
#pragma unroll
        for (int c = 0; c < K; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].re), fabsf((float)v[c].im)));
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const unsigned int lo = S::enc((float)v[c].re * inv);
            const unsigned int hi = S::enc((float)v[c].im * inv);
            d[(col * K + c) * Vh + i] = lo | (hi << 16);
        }
        sc[col * Vh + i] = m;
    }
}

// store_group that also replaces v by the values as stored (16-bit: decoded),
// so a fused epilogue sees exactly what later kernels will load
template <typename S, int K, typename R>
__device__ __forceinline__ void store_group_rt(typename S::pair* __restrict__ d, float* __restrict__ sc,
                                               long Vh, long col, long i, C2<R> v[K]) {
    if constexpr (!S::scaled) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            typename S::pair p;
            p.x = (typename S::real)v[c].re;
            p.y = (typename S::real)v[c].im;
            d[(col * K + c) * Vh + i] = p;
            v[c] = C2<R>{(R)p.x, (R)p.y};
        }
    } else {
        float m = 0.0f;
#pragma unroll
        for (int c = 0; c < K; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].re), fabsf((float)v[c].im)));
        const float inv = m > 0.0f ? 1.0f / m : 0.0f;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const unsigned short lo = S::enc((float)v[c].re * inv);
            const unsigned short hi = S::enc((float)v[c].im * inv);
            d[(col * K + c) * Vh + i] = (unsigned int)lo | ((unsigned int)hi << 16);
            v[c] = C2<R>{(R)(S::dec(lo) * m), (R)(S::dec(hi) * m)};
        }
        sc[col * Vh + i] = m;
    }
}

// LDS element type of fused Gram tiles: FP64 values for FP64 storage, FP32
// otherwise (exact for FP32 and decoded 16-bit data; products are formed in FP64)
template <typename S> struct TileElem { using type = float; };
template <> struct TileElem<F64> { using type = double; };

}  // namespace bcg
