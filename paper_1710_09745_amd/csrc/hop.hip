// Multi-right-hand-side staggered hop (the block Dslash, Sec. 6.2) for gfx950.
//
// Links are stored per output parity as sixteen folded 3x3 matrices per site
// (eta phase, backward sign and Hermitian conjugate applied once at load time),
// so the kernel is a uniform 16-point gather:  out(x) = sum_k W_k(x) in(x + d_k).
// Each matrix is read once per output site and applied to a register tile of
// TR right-hand sides; the workgroup's other waves work on other right-hand-side
// tiles of the same 64 sites, so the same link lines are served from the L1/L2
// caches (cache tiling across waves, register tiling within a lane: the hybrid
// of Sec. 6.2, re-shaped for 64-wide wavefronts).
//
// Layouts: W [NL][9][Vh] pairs; vectors [N][3][Vh] pairs (colour planes per
// right-hand side, sites contiguous so every load of a wave is one coalesced
// 64-site segment).
#include "device_common.h"
#include "internal.h"

namespace bcg {

__device__ __forceinline__ int lex_of(const Geom& g, int y0, int y1, int y2, int y3) {
    return y0 + g.L[0] * (y1 + g.L[1] * (y2 + g.L[2] * y3));
}

// One thread per (output site, folded matrix k).  fat/lng: canonical complex128
// [4][V][3][3] on the device.
template <typename T>
__global__ void __launch_bounds__(256)
k_pack_links(const double2* __restrict__ fat, const double2* __restrict__ lng,
             typename Store<T>::pair* __restrict__ W, Geom g, int parity, int nl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= g.Vh || k >= nl) return;
    int x[4];
    site_coords(g, i, parity, x);
    const int mu = nl == 16 ? (k >> 2) : (k >> 1);
    const int j = nl == 16 ? (k & 3) : (k & 1);
    const int hop = (j & 2) ? 3 : 1;
    const bool bwd = j & 1;
    const double2* U = (j & 2) ? lng : fat;
    const long V = 2L * g.Vh;
    int y[4] = {x[0], x[1], x[2], x[3]};
    if (bwd) {
        int v = y[mu] - hop;
        while (v < 0) v += g.L[mu];
        y[mu] = v;
    }
    const long src = ((long)mu * V + lex_of(g, y[0], y[1], y[2], y[3])) * 9;
    const double s = (double)eta_sign(x, mu) * (bwd ? -1.0 : 1.0);
    using P = typename Store<T>::pair;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            // forward: W_ab = s U_ab;  backward: W_ab = s conj(U_ba)
            const double2 u = bwd ? U[src + 3 * b + a] : U[src + 3 * a + b];
            P w;
            w.x = (T)(s * u.x);
            w.y = (T)(bwd ? -s * u.y : s * u.y);
            W[((long)k * 9 + 3 * a + b) * g.Vh + i] = w;
        }
}

// Epilogues of the hop.
enum { EPI_PLAIN = 0, EPI_MASS = 1, EPI_MASS_DOT = 2 };

// out = D_{p,1-p} in (EPI_PLAIN), or out = m2 * ctr - D_{p,1-p} in (EPI_MASS),
// plus, for EPI_MASS_DOT (one right-hand side), a per-workgroup partial of
// Re <ctr, out> written to dot[blockIdx.x].
//
// Thread layout: blockDim.x = 256 = spb sites x tpb right-hand-side tiles, spb a
// multiple of 64, so each wave covers 64 consecutive sites of one tile.
template <typename T, int TR, int NL, int EPI>
__global__ void __launch_bounds__(256)
k_hop(const typename Store<T>::pair* __restrict__ W, const typename Store<T>::pair* __restrict__ in,
      typename Store<T>::pair* __restrict__ out, const typename Store<T>::pair* __restrict__ ctr,
      double m2d, int N, Geom g, int out_parity, int spb, const int* __restrict__ halt,
      double* __restrict__ dot) {
    using R = typename Store<T>::real;
    using P = typename Store<T>::pair;
    if (halt != nullptr && *halt) return;
    const int lane_site = threadIdx.x % spb;
    const int i = blockIdx.x * spb + lane_site;
    const int tile = blockIdx.y * (256 / spb) + threadIdx.x / spb;
    const int r0 = tile * TR;
    const bool active = (i < g.Vh) && (r0 < N);
    const long Vh = g.Vh;
    double mydot = 0.0;
    if (active) {
        int x[4];
        site_coords(g, i, out_parity, x);
        C2<R> acc[TR][3];
#pragma unroll
        for (int r = 0; r < TR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] = c2<R>(0, 0);
        // not unrolled: one folded matrix (18 reals) live at a time keeps the
        // register tile of TR right-hand sides resident without spilling
#pragma unroll 1
        for (int k = 0; k < NL; ++k) {
            const int nb = neighbour_cb(g, x, hop_mu<NL>(k), hop_d<NL>(k));
            C2<R> w[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e] = ld(W + ((long)k * 9 + e) * Vh + i);
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                if (r0 + r < N) {
                    const P* src = in + (long)(r0 + r) * 3 * Vh + nb;
                    const C2<R> v0 = ld(src), v1 = ld(src + Vh), v2 = ld(src + 2 * Vh);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        cmac(acc[r][a], w[3 * a + 0], v0);
                        cmac(acc[r][a], w[3 * a + 1], v1);
                        cmac(acc[r][a], w[3 * a + 2], v2);
                    }
                }
            }
        }
        const R m2 = (R)m2d;
#pragma unroll
        for (int r = 0; r < TR; ++r) {
            if (r0 + r < N) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const long o = ((long)(r0 + r) * 3 + c) * Vh + i;
                    C2<R> v = acc[r][c];
                    if (EPI != EPI_PLAIN) {
                        const C2<R> z = ld(ctr + o);
                        v.re = m2 * z.re - v.re;
                        v.im = m2 * z.im - v.im;
                        if (EPI == EPI_MASS_DOT)
                            mydot += (double)z.re * (double)v.re + (double)z.im * (double)v.im;
                    }
                    P pv;
                    pv.x = v.re;
                    pv.y = v.im;
                    out[o] = pv;
                }
            }
        }
    }
    if (EPI == EPI_MASS_DOT) {
        __shared__ double red[4];
        for (int off = 32; off > 0; off >>= 1) mydot += __shfl_xor(mydot, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mydot;
        __syncthreads();
        if (threadIdx.x == 0) dot[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
hipError_t pack_links(Prec prec, const void* fat, const void* lng, void* W, const Geom& g,
                      int parity, int nl, hipStream_t s) {
    dim3 grid((g.Vh + 255) / 256, nl);
    if (prec == Prec::FP64)
        hipLaunchKernelGGL(k_pack_links<double>, grid, dim3(256), 0, s, (const double2*)fat,
                           (const double2*)lng, (double2*)W, g, parity, nl);
    else
        hipLaunchKernelGGL(k_pack_links<float>, grid, dim3(256), 0, s, (const double2*)fat,
                           (const double2*)lng, (float2*)W, g, parity, nl);
    return hipGetLastError();
}

HopShape hop_shape(int N) {
    // register tile TR and tiles per workgroup tpb
    HopShape h;
    if (N <= 1) { h.tr = 1; h.tpb = 1; }
    else if (N <= 2) { h.tr = 2; h.tpb = 1; }
    else if (N <= 4) { h.tr = 4; h.tpb = 1; }
    else if (N <= 8) { h.tr = 4; h.tpb = 2; }
    else if (N <= 16) { h.tr = 4; h.tpb = 4; }
    else { h.tr = 8; h.tpb = 4; }
    return h;
}

template <typename T, int TR, int NL>
static void launch_hop_t(const void* W, const void* in, void* out, const void* ctr, double m2,
                         int N, const Geom& g, int out_parity, int epi, int tpb,
                         const int* halt, double* dot, hipStream_t s) {
    using P = typename Store<T>::pair;
    const int spb = 256 / tpb;
    const int ntiles = (N + TR - 1) / TR;
    dim3 grid((g.Vh + spb - 1) / spb, (ntiles + tpb - 1) / tpb);
    if (epi == EPI_PLAIN)
        hipLaunchKernelGGL((k_hop<T, TR, NL, EPI_PLAIN>), grid, dim3(256), 0, s, (const P*)W,
                           (const P*)in, (P*)out, (const P*)ctr, m2, N, g, out_parity, spb, halt, dot);
    else if (epi == EPI_MASS)
        hipLaunchKernelGGL((k_hop<T, TR, NL, EPI_MASS>), grid, dim3(256), 0, s, (const P*)W,
                           (const P*)in, (P*)out, (const P*)ctr, m2, N, g, out_parity, spb, halt, dot);
    else
        hipLaunchKernelGGL((k_hop<T, TR, NL, EPI_MASS_DOT>), grid, dim3(256), 0, s, (const P*)W,
                           (const P*)in, (P*)out, (const P*)ctr, m2, N, g, out_parity, spb, halt, dot);
}

template <typename T, int NL>
static void launch_hop_nl(const void* W, const void* in, void* out, const void* ctr, double m2,
                          int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                          const int* halt, double* dot, hipStream_t s) {
    switch (h.tr) {
        case 1: launch_hop_t<T, 1, NL>(W, in, out, ctr, m2, N, g, out_parity, epi, h.tpb, halt, dot, s); break;
        case 2: launch_hop_t<T, 2, NL>(W, in, out, ctr, m2, N, g, out_parity, epi, h.tpb, halt, dot, s); break;
        case 4: launch_hop_t<T, 4, NL>(W, in, out, ctr, m2, N, g, out_parity, epi, h.tpb, halt, dot, s); break;
        default: launch_hop_t<T, 8, NL>(W, in, out, ctr, m2, N, g, out_parity, epi, h.tpb, halt, dot, s); break;
    }
}

int hop_dot_blocks(const Geom& g) { return (g.Vh + 255) / 256; }

hipError_t launch_hop(Prec prec, int nl, const void* W, const void* in, void* out, const void* ctr,
                      double m2, int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                      const int* halt, double* dot, hipStream_t s) {
    if (epi == EPI_MASS_DOT && (N != 1 || h.tpb != 1 || h.tr != 1)) return hipErrorInvalidValue;
    if (prec == Prec::FP64) {
        if (nl == 16) launch_hop_nl<double, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, s);
        else launch_hop_nl<double, 8>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, s);
    } else if (prec == Prec::FP32) {
        if (nl == 16) launch_hop_nl<float, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, s);
        else launch_hop_nl<float, 8>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bcg
