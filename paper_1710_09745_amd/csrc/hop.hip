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
#include <type_traits>

#include "device_common.h"
#include "gram_tile.h"
#include "internal.h"
#include "storage.h"

namespace bcg {

__device__ __forceinline__ int lex_of(const Geom& g, int y0, int y1, int y2, int y3) {
    return y0 + g.L[0] * (y1 + g.L[1] * (y2 + g.L[2] * y3));
}

// One thread per (output site, folded matrix k): FP64 folded links.  fat/lng:
// canonical complex128 [4][V][3][3] on the device; lower precisions are made
// from these by the group conversion below.
__global__ void __launch_bounds__(256)
k_pack_links(const double2* __restrict__ fat, const double2* __restrict__ lng,
             double2* __restrict__ W, Geom g, int parity, int nl) {
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
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            // forward: W_ab = s U_ab;  backward: W_ab = s conj(U_ba)
            const double2 u = bwd ? U[src + 3 * b + a] : U[src + 3 * a + b];
            W[((long)k * 9 + 3 * a + b) * g.Vh + i] = make_double2(s * u.x, bwd ? -s * u.y : s * u.y);
        }
}

// [cols][K][Vh] groups from FP64 into another storage policy
template <typename SD, int K>
__global__ void __launch_bounds__(256)
k_group_from64(const double2* __restrict__ src, typename SD::pair* __restrict__ d, float* __restrict__ sc,
               long cols, long Vh) {
    const long n = cols * Vh;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long col = t / Vh, i = t - col * Vh;
        C2<double> v[K];
        load_group<F64, K>(src, nullptr, Vh, col, i, v);
        store_group<SD, K, double>(d, sc, Vh, col, i, v);
    }
}

// Workgroups are handed to the eight XCDs round robin (workgroup b on XCD b % 8),
// and each XCD has its own L2.  Site block it (in the order the workgroups are
// issued) is therefore remapped so that XCD x works through one contiguous eighth
// of the lattice: the z and t neighbours a site block reads were then most likely
// fetched into the same L2 by the workgroups just before it.  A bijection of
// [0, nsb): the first 8*(nsb/8) blocks split into eight contiguous chunks, the
// remainder stays in place.
__device__ __forceinline__ int xcd_block(int it, int nsb) {
    const int q8 = nsb >> 3;
    if (it >= (q8 << 3)) return it;
    return (it & 7) * q8 + (it >> 3);
}

// Epilogues of the hop.
enum { EPI_PLAIN = 0, EPI_MASS = 1, EPI_MASS_DOT = 2 };

// out = D_{p,1-p} in (EPI_PLAIN), or out = m2 * ctr - D_{p,1-p} in (EPI_MASS),
// plus, for EPI_MASS_DOT (one right-hand side), a per-workgroup partial of
// Re <ctr, out> written to dot[blockIdx.x].
//
// Thread layout: blockDim.x = 256 = spb sites x tpb lanes groups, spb a multiple
// of 64, so each wave covers 64 consecutive sites.  A workgroup owns its sites
// for all N right-hand sides: wave group t handles the register tiles t, t + tpb,
// ... of TR columns each.  Keeping every tile of a site in one workgroup keeps
// the re-reads of its links inside one CU (and so one XCD's L2).
template <typename S, int TR, int NL, int EPI, bool PF, int NB, bool GR>
__global__ void __launch_bounds__(256)
k_hop(const typename S::pair* __restrict__ W, const float* __restrict__ Ws,
      const typename S::pair* __restrict__ in, const float* __restrict__ ins,
      typename S::pair* __restrict__ out, float* __restrict__ outs,
      const typename S::pair* __restrict__ ctr, const float* __restrict__ ctrs,
      double m2d, int N, Geom g, int out_parity, int spb, const int* __restrict__ halt,
      double* __restrict__ dot, double2* __restrict__ partials) {
    using R = typename S::real;
    using E = typename TileElem<S>::type;
    extern __shared__ unsigned char lds_raw[];
    C2<E>* tile = reinterpret_cast<C2<E>*>(lds_raw);
    if (halt != nullptr && *halt) return;
    const int tpb = 256 / spb;
    const int lane_site = threadIdx.x % spb;
    const long Vh = g.Vh;
    const int nsb = (g.Vh + spb - 1) / spb;
    const int rows = 3 * spb;
    double mydot = 0.0;
    GramAcc<NB> gacc;
    if constexpr (GR) {
        gacc.zero();
        for (int e = threadIdx.x; e < rows * (NB + 1); e += 256) tile[e] = C2<E>{(E)0, (E)0};
    }
    for (int it = blockIdx.x; it < nsb; it += gridDim.x) {
      const int sb = xcd_block(it, nsb);
      const int i = sb * spb + lane_site;
      if constexpr (GR) __syncthreads();
      if (i < g.Vh) {
        int x[4];
        site_coords(g, i, out_parity, x);
        for (int r0 = (threadIdx.x / spb) * TR; r0 < N; r0 += tpb * TR) {
            C2<R> acc[TR][3];
#pragma unroll
            for (int r = 0; r < TR; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[r][c] = c2<R>(0, 0);
            if constexpr (!PF) {
                // one folded matrix (18 reals) live at a time keeps the register
                // tile of TR right-hand sides resident without spilling
#pragma unroll 1
                for (int k = 0; k < NL; ++k) {
                    const int nb = neighbour_cb(g, x, hop_mu<NL>(k), hop_d<NL>(k));
                    C2<R> w[9];
                    load_group<S, 9, true>(W, Ws, Vh, k, i, w);
#pragma unroll
                    for (int r = 0; r < TR; ++r) {
                        if (r0 + r < N) {
                            C2<R> v[3];
                            load_group<S, 3>(in, ins, Vh, r0 + r, nb, v);
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                cmac(acc[r][a], w[3 * a + 0], v[0]);
                                cmac(acc[r][a], w[3 * a + 1], v[1]);
                                cmac(acc[r][a], w[3 * a + 2], v[2]);
                            }
                        }
                    }
                }
            } else {
                // Software-pipelined over the NL folded matrices: the loads of matrix
                // k+1 and of its TR neighbour vectors are issued before the FMAs of
                // matrix k, so each wave keeps two hops' worth of loads in flight.
                C2<R> w[9], v[TR][3];
                {
                    const int nb = neighbour_cb(g, x, hop_mu<NL>(0), hop_d<NL>(0));
                    load_group<S, 9, true>(W, Ws, Vh, 0, i, w);
    #pragma unroll
                    for (int r = 0; r < TR; ++r)
                        if (r0 + r < N) load_group<S, 3>(in, ins, Vh, r0 + r, nb, v[r]);
                }
    #pragma unroll 1
                for (int k = 0; k < NL; ++k) {
                    C2<R> wc[9], vc[TR][3];
    #pragma unroll
                    for (int e = 0; e < 9; ++e) wc[e] = w[e];
    #pragma unroll
                    for (int r = 0; r < TR; ++r)
    #pragma unroll
                        for (int c = 0; c < 3; ++c) vc[r][c] = v[r][c];
                    if (k + 1 < NL) {
                        const int nb = neighbour_cb(g, x, hop_mu<NL>(k + 1), hop_d<NL>(k + 1));
                        load_group<S, 9, true>(W, Ws, Vh, k + 1, i, w);
    #pragma unroll
                        for (int r = 0; r < TR; ++r)
                            if (r0 + r < N) load_group<S, 3>(in, ins, Vh, r0 + r, nb, v[r]);
                    }
    #pragma unroll
                    for (int r = 0; r < TR; ++r) {
                        if (r0 + r < N) {
    #pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                cmac(acc[r][a], wc[3 * a + 0], vc[r][0]);
                                cmac(acc[r][a], wc[3 * a + 1], vc[r][1]);
                                cmac(acc[r][a], wc[3 * a + 2], vc[r][2]);
                            }
                        }
                    }
                }
            }
            const R m2 = (R)m2d;
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                if (r0 + r < N) {
                    if (EPI != EPI_PLAIN) {
                        C2<R> z[3];
                        load_group<S, 3>(ctr, ctrs, Vh, r0 + r, i, z);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            acc[r][c].re = m2 * z[c].re - acc[r][c].re;
                            acc[r][c].im = m2 * z[c].im - acc[r][c].im;
                            if (EPI == EPI_MASS_DOT)
                                mydot += (double)z[c].re * (double)acc[r][c].re +
                                         (double)z[c].im * (double)acc[r][c].im;
                        }
                    }
                    store_group_rt<S, 3, R>(out, outs, Vh, r0 + r, i, acc[r]);
                    if constexpr (GR) {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            tile[(c * spb + lane_site) * (NB + 1) + r0 + r] = C2<E>{(E)acc[r][c].re, (E)acc[r][c].im};
                    }
                }
            }
        }
      } else if constexpr (GR) {
        for (int r0 = (threadIdx.x / spb) * TR; r0 < N; r0 += tpb * TR)
            for (int r = 0; r < TR && r0 + r < N; ++r)
                for (int c = 0; c < 3; ++c) tile[(c * spb + lane_site) * (NB + 1) + r0 + r] = C2<E>{(E)0, (E)0};
      }
      if constexpr (GR) {
        __syncthreads();
        gram_tile_acc<NB, E>(tile, tile, rows, gacc);
      }
    }
    if constexpr (GR) gram_finish<NB>(gacc, reinterpret_cast<C2<double>*>(lds_raw), partials + (long)blockIdx.x * NB * NB);
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
hipError_t pack_links(const void* fat, const void* lng, void* W, const Geom& g, int parity, int nl,
                      hipStream_t s) {
    dim3 grid((g.Vh + 255) / 256, nl);
    hipLaunchKernelGGL(k_pack_links, grid, dim3(256), 0, s, (const double2*)fat, (const double2*)lng,
                       (double2*)W, g, parity, nl);
    return hipGetLastError();
}

static unsigned grid_for(long n) {
    const long g = (n + 255) / 256;
    return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

hipError_t links_from64(Prec pd, const void* W64, void* Wd, int nl, long Vh, hipStream_t s) {
    const long cols = nl;
    float* sc = (float*)((char*)Wd + (size_t)pd_bytes(pd) * cols * 9 * Vh);
    const dim3 grid(grid_for(cols * Vh));
    switch (pd) {
        case Prec::FP32: hipLaunchKernelGGL((k_group_from64<F32, 9>), grid, dim3(256), 0, s, (const double2*)W64, (float2*)Wd, sc, cols, Vh); break;
        case Prec::FP16: hipLaunchKernelGGL((k_group_from64<H16, 9>), grid, dim3(256), 0, s, (const double2*)W64, (unsigned int*)Wd, sc, cols, Vh); break;
        case Prec::BF16: hipLaunchKernelGGL((k_group_from64<B16, 9>), grid, dim3(256), 0, s, (const double2*)W64, (unsigned int*)Wd, sc, cols, Vh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

HopShape hop_shape(int N, int tr, int tpb, int pf) {
    // default register tile TR and lane groups per workgroup tpb by N; nonzero
    // arguments override them (tuning), pf selects the software-pipelined loop
    HopShape h;
    if (N <= 1) { h.tr = 1; h.tpb = 1; }
    else if (N <= 2) { h.tr = 2; h.tpb = 1; }
    else if (N <= 4) { h.tr = 4; h.tpb = 1; }
    else if (N <= 8) { h.tr = 4; h.tpb = 2; }
    else if (N <= 16) { h.tr = 4; h.tpb = 4; }
    else { h.tr = 8; h.tpb = 4; }
    h.pf = pf > 0 ? 1 : 0;
    if (N > 1 && (tr == 1 || tr == 2 || tr == 4 || tr == 8)) h.tr = tr;
    if (N > 1 && (tpb == 1 || tpb == 2 || tpb == 4)) h.tpb = tpb;
    return h;
}

// LDS bytes of the fused T^H T epilogue for this shape, or 0 if over the 64 KB budget
size_t hop_tile_bytes(Prec prec, int N, const HopShape& h) {
    const int spb = 256 / h.tpb;
    const size_t e = (prec == Prec::FP64) ? 16 : 8;
    const size_t b = (size_t)3 * spb * (pad_n(N) + 1) * e;
    return b <= 65536 ? b : 0;
}

int hop_grid(const Geom& g, const HopShape& h, bool fused) {
    const int spb = 256 / h.tpb;
    const int nsb = (g.Vh + spb - 1) / spb;
    return fused ? (nsb < GRAM_BLOCKS ? nsb : GRAM_BLOCKS) : nsb;
}

template <typename S, int TR, int NL, bool PF, int NB, bool GR>
static void launch_hop_g(const void* W, const void* in, void* out, const void* ctr, double m2, int N,
                         const Geom& g, int out_parity, int epi, const HopShape& h, const int* halt,
                         double* dot, double2* partials, hipStream_t s) {
    using P = typename S::pair;
    const long Vh = g.Vh;
    auto scale = [&](const void* p, long cols, int K) -> float* {
        return S::scaled && p ? (float*)((char*)p + (size_t)S::bytes * cols * K * Vh) : nullptr;
    };
    const int spb = 256 / h.tpb;
    dim3 grid(hop_grid(g, h, GR));
    const size_t lds = GR ? (size_t)3 * spb * (NB + 1) * sizeof(C2<typename TileElem<S>::type>) : 0;
    float* Ws = scale(W, NL, 9);
    float* ins = scale(in, N, 3);
    float* outs = scale(out, N, 3);
    float* ctrs = scale(ctr, N, 3);
#define HOP_GO(E)                                                                                      \
    hipLaunchKernelGGL((k_hop<S, TR, NL, E, PF, NB, GR>), grid, dim3(256), lds, s, (const P*)W, Ws,        \
                       (const P*)in, ins, (P*)out, outs, (const P*)ctr, ctrs, m2, N, g, out_parity, spb, \
                       halt, dot, partials)
    if (epi == EPI_PLAIN) HOP_GO(EPI_PLAIN);
    else if constexpr (!GR) {
        if (epi == EPI_MASS) HOP_GO(EPI_MASS);
        else if constexpr (TR == 1) HOP_GO(EPI_MASS_DOT);
    }
#undef HOP_GO
}

template <typename S, int TR, int NL, bool PF>
static void launch_hop_t(const void* W, const void* in, void* out, const void* ctr, double m2,
                         int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                         const int* halt, double* dot, double2* partials, hipStream_t s) {
#define HG(NBV, GRV) launch_hop_g<S, TR, NL, PF, NBV, GRV>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s)
    if (partials == nullptr) return HG(1, false);
    switch (pad_n(N)) {
        case 1: return HG(1, true);
        case 2: return HG(2, true);
        case 4: return HG(4, true);
        case 8: return HG(8, true);
        case 16: return HG(16, true);
        default:
            if constexpr (!std::is_same<S, F64>::value) return HG(32, true);
    }
#undef HG
}

template <typename S, int NL>
static void launch_hop_nl(const void* W, const void* in, void* out, const void* ctr, double m2,
                          int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                          const int* halt, double* dot, double2* partials, hipStream_t s) {
#define HOP_TR(T)                                                                                          \
    (h.pf ? launch_hop_t<S, T, NL, true>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s) \
          : launch_hop_t<S, T, NL, false>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s))
    switch (h.tr) {
        case 1: HOP_TR(1); break;
        case 2: HOP_TR(2); break;
        case 4: HOP_TR(4); break;
        default: HOP_TR(8); break;
    }
#undef HOP_TR
}

template <typename S>
static void launch_hop_s(int nl, const void* W, const void* in, void* out, const void* ctr, double m2,
                         int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                         const int* halt, double* dot, double2* partials, hipStream_t s) {
    if (nl == 16) launch_hop_nl<S, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s);
    else launch_hop_nl<S, 8>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s);
}

int hop_dot_blocks(const Geom& g) { return (g.Vh + 255) / 256; }

hipError_t launch_hop(Prec prec, int nl, const void* W, const void* in, void* out, const void* ctr,
                      double m2, int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                      const int* halt, double* dot, double2* partials, hipStream_t s) {
    if (epi == EPI_MASS_DOT && (N != 1 || h.tpb != 1 || h.tr != 1)) return hipErrorInvalidValue;
    if (partials != nullptr && (epi != EPI_PLAIN || hop_tile_bytes(prec, N, h) == 0))
        return hipErrorInvalidValue;
    switch (prec) {
        case Prec::FP64: launch_hop_s<F64>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s); break;
        case Prec::FP32: launch_hop_s<F32>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s); break;
        case Prec::FP16: launch_hop_s<H16>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s); break;
        case Prec::BF16: launch_hop_s<B16>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, s); break;
    }
    return hipGetLastError();
}

}  // namespace bcg
