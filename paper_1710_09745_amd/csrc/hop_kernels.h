// Kernels of the multi-right-hand-side staggered hop and their launch templates;
// included by one translation unit per storage precision (hop_<prec>.hip), so the
// many instantiations compile in parallel.  See hop.hip for the design.
#pragma once
#include <type_traits>

#include "device_common.h"
#include "gram_tile.h"
#include "internal.h"
#include "storage.h"

namespace bcg {

enum { EPI_PLAIN = 0, EPI_MASS = 1, EPI_MASS_DOT = 2 };

// Loads of one folded matrix and of the TR neighbour vectors it multiplies.
template <typename S, int TR> struct HopOperands {
    C2<typename S::real> w[9];
    C2<typename S::real> v[TR][3];
};

// Per-XCD task queues of the site-parallel hop.  The site blocks are grouped into
// cells of bpc consecutive blocks (a quarter of a time slice where it divides), and
// cell c belongs to queue c mod 8, so at any moment the eight XCDs work on eight
// neighbouring cells and the workgroups of one XCD on consecutive blocks of one
// cell: the x, y and z neighbours of a cell then stay in that XCD's L2 and the
// t neighbours are the cells the XCDs read a few steps earlier or later.  Queue q
// holds, for each tile group in turn, the blocks of its cells in order.
__device__ __forceinline__ int hop_queue_cells(const HopQueue& q, int qq) {
    return qq < q.ncell ? (q.ncell - 1 - qq) / 8 + 1 : 0;
}
__device__ __forceinline__ int hop_queue_tasks(const HopQueue& q, int qq, int ntg) {
    return hop_queue_cells(q, qq) * q.bpc * ntg;
}
// task (tile group tg, site block sb) as tg * nsb + sb for entry li of queue qq
__device__ __forceinline__ int hop_queue_task(const HopQueue& q, int qq, int li, int ntg) {
    const int per_tg = hop_queue_cells(q, qq) * q.bpc;
    const int tg = li / per_tg;
    const int r = li - tg * per_tg;
    const int k = r / q.bpc;
    const int cell = qq + 8 * k;
    const int sb = cell * q.bpc + (r - k * q.bpc);
    (void)ntg;
    return tg * (q.ncell * q.bpc) + sb;
}

// Issue every load of hop k of direction mu (all independent, so the wave has
// 9 + 3 TR loads in flight before its first FMA).  Returns nothing; the
// neighbour index is formed from the site's coordinate along mu with the
// periodic wrap applied with uniform strides.
template <typename S, int TR, int NL>
__device__ __forceinline__ void hop_fetch(HopOperands<S, TR>& o, int k, int j, int xm, int Lm, int sm, int lex,
                                          unsigned site_vo, unsigned site_so, unsigned plane,
                                          const char* Wb, const float* Wsb, long Vh,
                                          const rsrc_t* vin, const rsrc_t* vins) {
    const int hop = (NL == 16 && (j & 2)) ? 3 : 1;
    const int d = (j & 1) ? -hop : hop;
    int v = xm + d;
    int nbl = lex + d * sm;
    const int wrap = Lm * sm;
    if (v >= Lm) { v -= Lm; nbl -= wrap; }
    if (v >= Lm) nbl -= wrap;
    if (v < 0) { v += Lm; nbl += wrap; }
    if (v < 0) nbl += wrap;
    const unsigned nb = (unsigned)nbl >> 1;
    const rsrc_t wr = make_rsrc(Wb + (size_t)k * 9 * plane);
    const rsrc_t wsr = S::scaled ? make_rsrc(Wsb + (size_t)k * Vh) : wr;
    buf_group<S, 9, AUX_NONE>(wr, wsr, site_vo, site_so, plane, o.w);
#pragma unroll
    for (int r = 0; r < TR; ++r) buf_group<S, 3, AUX_NONE>(vin[r], vins[r], nb * S::bytes, nb * 4u, plane, o.v[r]);
}

template <typename S, int TR>
__device__ __forceinline__ void hop_fma(const HopOperands<S, TR>& o, C2<typename S::real> acc[TR][3]) {
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cmac(acc[r][a], o.w[3 * a + 0], o.v[r][0]);
            cmac(acc[r][a], o.w[3 * a + 1], o.v[r][1]);
            cmac(acc[r][a], o.w[3 * a + 2], o.v[r][2]);
        }
}

// out = D_{p,1-p} in (EPI_PLAIN), or out = m2 * ctr - D_{p,1-p} in (EPI_MASS),
// plus, for EPI_MASS_DOT (one right-hand side), a per-workgroup partial of
// Re <ctr, out> written to dot[blockIdx.x].
//
// Thread layout: blockDim.x = 256 = spb sites x tpb lane groups, spb a multiple
// of 64, so each wave covers 64 consecutive sites and one lane group.  A
// workgroup owns its sites for all N right-hand sides: lane group t handles the
// register tiles t, t + tpb, ... of TR columns each.  Keeping every tile of a
// site in one workgroup keeps the re-reads of its links inside one CU (and so
// one XCD's L2).  A ragged last tile repeats column N - 1 in its spare slots
// (loads stay unconditional so they issue together; only the stores are masked),
// and lanes past the last site work on site Vh - 1 without storing.
// PF: two hops per loop trip, so twice the loads are in flight per wave.
template <typename S, int TR, int NL, int EPI, bool PF, int NB, bool GR>
__global__ void __launch_bounds__(256)
k_hop(const typename S::pair* __restrict__ W, const float* __restrict__ Ws,
      const typename S::pair* __restrict__ in, const float* __restrict__ ins,
      typename S::pair* __restrict__ out, float* __restrict__ outs,
      const typename S::pair* __restrict__ ctr, const float* __restrict__ ctrs,
      double m2d, int N, Geom g, int out_parity, int spb, int ntg, const int* __restrict__ halt,
      double* __restrict__ dot, double2* __restrict__ partials, HopQueue q) {
    using R = typename S::real;
    using E = typename TileElem<S>::type;
    constexpr int NJ = NL / 4;  // hops per direction
    extern __shared__ unsigned char lds_raw[];
    C2<E>* tile = reinterpret_cast<C2<E>*>(lds_raw);
    if (halt != nullptr && *halt) return;
    const int tpb = 256 / spb;
    const int lane_site = threadIdx.x % spb;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / spb);
    const long Vh = g.Vh;
    const unsigned plane = (unsigned)Vh * S::bytes;
    const int nsb = (g.Vh + spb - 1) / spb;
    const int rows = 3 * spb;
    const int st[4] = {1, g.L[0], g.L[0] * g.L[1], g.L[0] * g.L[1] * g.L[2]};
    const char* Wb = reinterpret_cast<const char*>(W);
    double mydot = 0.0;
    GramAcc<NB> gacc;
    if constexpr (GR) {
        gacc.zero();
        for (int e = threadIdx.x; e < rows * (NB + 1); e += 256) tile[e] = C2<E>{(E)0, (E)0};
    }
    const int bps = blocks_per_slice(g, spb);
    const int gcols = tpb * TR;  // columns of one tile group
    // task order: with a queue, the workgroups of each XCD take the cells of their own
    // queue in order (then help drain the others); otherwise a static grid-stride walk
    __shared__ int s_task;
    const int xcd = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u);  // XCC_ID, bits 3:0
    int qi = 0;                                                               // queues visited
    auto next_task = [&](int prev) -> int {
        if (q.ctr == nullptr) return prev < 0 ? (int)blockIdx.x : prev + (int)gridDim.x;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = -1;
            while (qi < 8) {
                const int qq = (xcd + qi) & 7;
                const int n = hop_queue_tasks(q, qq, ntg);
                const int li = atomicAdd(&q.ctr[qq], 1);
                if (li < n) {
                    t = hop_queue_task(q, qq, li, ntg);
                    break;
                }
                ++qi;
            }
            s_task = t;
        }
        __syncthreads();
        return s_task;
    };
    for (int it = next_task(-1); it >= 0 && it < nsb * ntg; it = next_task(it)) {
        int sb, tg;
        if (q.ctr != nullptr) {
            tg = it / nsb;
            sb = it - tg * nsb;
        } else {
            xcd_task_tm(it, nsb, ntg, bps, sb, tg);
        }
        const int cend = (ntg == 1) ? N : min(N, (tg + 1) * gcols);
        const int i0 = sb * spb + lane_site;
        const bool live = i0 < g.Vh;
        const int i = live ? i0 : g.Vh - 1;
        if constexpr (GR) __syncthreads();
        int x[4];
        site_coords(g, i, out_parity, x);
        const int lex = x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
        const unsigned site_vo = (unsigned)i * S::bytes, site_so = (unsigned)i * 4u;
        for (int r0 = tg * gcols + grp * TR; r0 < cend; r0 += gcols) {
            rsrc_t vin[TR], vins[TR];
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                const int col = r0 + r < N ? r0 + r : N - 1;
                vin[r] = make_rsrc(reinterpret_cast<const char*>(in) + (size_t)col * 3 * plane);
                vins[r] = S::scaled ? make_rsrc(ins + (size_t)col * Vh) : vin[r];
            }
            C2<R> acc[TR][3];
#pragma unroll
            for (int r = 0; r < TR; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[r][c] = c2<R>(0, 0);
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                const int xm = x[mu], Lm = g.L[mu], sm = st[mu];
                if constexpr (!PF) {
#pragma unroll 1
                    for (int j = 0; j < NJ; ++j) {
                        HopOperands<S, TR> o;
                        hop_fetch<S, TR, NL>(o, mu * NJ + j, j, xm, Lm, sm, lex, site_vo, site_so, plane, Wb, Ws,
                                             Vh, vin, vins);
                        hop_fma<S, TR>(o, acc);
                    }
                } else {
#pragma unroll 1
                    for (int j = 0; j < NJ; j += 2) {
                        HopOperands<S, TR> o0, o1;
                        hop_fetch<S, TR, NL>(o0, mu * NJ + j, j, xm, Lm, sm, lex, site_vo, site_so, plane, Wb, Ws,
                                             Vh, vin, vins);
                        hop_fetch<S, TR, NL>(o1, mu * NJ + j + 1, j + 1, xm, Lm, sm, lex, site_vo, site_so, plane,
                                             Wb, Ws, Vh, vin, vins);
                        hop_fma<S, TR>(o0, acc);
                        hop_fma<S, TR>(o1, acc);
                    }
                }
            }
            const R m2 = (R)m2d;
#pragma unroll
            for (int r = 0; r < TR; ++r) {
                if (r0 + r < N) {
                    C2<R> z[3];
                    if (EPI != EPI_PLAIN) {
                        load_group<S, 3>(ctr, ctrs, Vh, r0 + r, i, z);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            acc[r][c].re = m2 * z[c].re - acc[r][c].re;
                            acc[r][c].im = m2 * z[c].im - acc[r][c].im;
                        }
                    }
                    if (live) store_group_rt<S, 3, R>(out, outs, Vh, r0 + r, i, acc[r]);
                    // p^H A p of the values as stored (what the CG update reads)
                    if (EPI == EPI_MASS_DOT && live)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            mydot += (double)z[c].re * (double)acc[r][c].re + (double)z[c].im * (double)acc[r][c].im;
                    if constexpr (GR) {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            tile[(c * spb + lane_site) * (NB + 1) + r0 + r] =
                                live ? C2<E>{(E)acc[r][c].re, (E)acc[r][c].im} : C2<E>{(E)0, (E)0};
                    }
                }
            }
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
    if (q.ctr != nullptr && threadIdx.x == 0) {
        // every workgroup has drained all eight queues when it gets here; the last one
        // to arrive resets the counters for the next launch
        __threadfence();
        if (atomicAdd(&q.ctr[8], 1) == (int)gridDim.x - 1) {
            for (int i = 0; i < 9; ++i) atomicExch(&q.ctr[i], 0);
        }
    }
}

// Lane-split hop: lane l of a wave takes site l % SR of a block of SR consecutive
// output sites and the 64 / SR directions mu = (l / SR) * DL ... (l / SR) * DL + DL - 1
// (DL = SR / 16), and applies the NL/4 folded matrices of each of its directions
// (forward and backward, one and three hops) to a register tile of TR right-hand
// sides.  SR = 16: one direction per lane, four per wave; SR = 32: two per lane, so
// each load instruction covers two runs of 32 sites instead of four of 16 (fewer
// cache lines per instruction) for twice the hops per lane.  The direction sums of
// a site meet through a butterfly of cross-lane exchanges (xor SR, ..., xor 32):
// every lane of the site ends with the same bits, so the result does not depend on
// the lane order.  The waves of a workgroup are tpw right-hand-side tiles of the
// same sites (their link loads meet in the CU's L1) and 4 / tpw blocks of SR sites.
// The grid is (site blocks) x (tile groups), walked so that each XCD takes a
// contiguous range of site blocks with all their tile groups one after the other.
// The folded links are addressed with one 32-bit byte offset per lane:
// NL * 9 * Vh * bytes < 4 GiB (checked by the launcher).
// EPI_MASS_DOT (TR = 1): dot[blockIdx.x] = Re <ctr, out> over the workgroup's sites.
template <typename S, int TR, int NL, int EPI, bool PF, int SR>
__global__ void __launch_bounds__(256)
k_hop_ls(const typename S::pair* __restrict__ W, const float* __restrict__ Ws,
         const typename S::pair* __restrict__ in, const float* __restrict__ ins,
         typename S::pair* __restrict__ out, float* __restrict__ outs,
         const typename S::pair* __restrict__ ctr, const float* __restrict__ ctrs,
         double m2d, int N, Geom g, int out_parity, int ntiles, int tpw, const int* __restrict__ halt,
         double* __restrict__ dot) {
    static_assert(SR == 16 || SR == 32, "site runs of 16 or 32");
    using R = typename S::real;
    constexpr int NJ = NL / 4;   // hops per direction
    constexpr int NG = 64 / SR;  // direction groups per wave
    constexpr int DL = 4 / NG;   // directions per lane
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sgn = 4 / tpw;                        // blocks of SR sites per workgroup
    const int nsb = (g.Vh + SR * sgn - 1) / (SR * sgn);
    const int ntg = (ntiles + tpw - 1) / tpw;       // tile groups
    int sb, tg;
    xcd_task_tm(blockIdx.x, nsb, ntg, blocks_per_slice(g, SR * sgn), sb, tg);
    const int tile_w = tg * tpw + w % tpw;
    const bool tile_ok = tile_w < ntiles;
    const int r0 = (tile_ok ? tile_w : ntiles - 1) * TR;
    const int s16 = lane % SR, grp = lane / SR;
    const long Vh = g.Vh;
    const unsigned plane = (unsigned)Vh * S::bytes;
    const int i0 = sb * SR * sgn + (w / tpw) * SR + s16;
    const bool live = i0 < g.Vh;
    const int i = live ? i0 : g.Vh - 1;  // spare lanes work on the last site and store nothing
    int x[4];
    site_coords(g, i, out_parity, x);
    const int lex = x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
    rsrc_t vin[TR], vins[TR];
#pragma unroll
    for (int r = 0; r < TR; ++r) {
        const int col = r0 + r < N ? r0 + r : N - 1;
        vin[r] = make_rsrc(reinterpret_cast<const char*>(in) + (size_t)col * 3 * plane);
        vins[r] = S::scaled ? make_rsrc(ins + (size_t)col * Vh) : vin[r];
    }
    const rsrc_t wr = make_rsrc(W);
    const rsrc_t wsr = S::scaled ? make_rsrc(Ws) : wr;
    C2<R> acc[TR][3];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][c] = c2<R>(0, 0);
#pragma unroll
    for (int dd = 0; dd < DL; ++dd) {
        const int mu = grp * DL + dd;
        const int sm = mu == 0 ? 1 : (mu == 1 ? g.L[0] : (mu == 2 ? g.L[0] * g.L[1] : g.L[0] * g.L[1] * g.L[2]));
        const int xm = mu == 0 ? x[0] : (mu == 1 ? x[1] : (mu == 2 ? x[2] : x[3]));
        const int Lm = mu == 0 ? g.L[0] : (mu == 1 ? g.L[1] : (mu == 2 ? g.L[2] : g.L[3]));
        auto fetch = [&](HopOperands<S, TR>& o, int j) {
            const int hop = (NL == 16 && (j & 2)) ? 3 : 1;
            const int d = (j & 1) ? -hop : hop;
            int v = xm + d;
            int nbl = lex + d * sm;
            const int wrap = Lm * sm;
            if (v >= Lm) { v -= Lm; nbl -= wrap; }
            if (v >= Lm) nbl -= wrap;
            if (v < 0) { v += Lm; nbl += wrap; }
            if (v < 0) nbl += wrap;
            const unsigned nb = (unsigned)nbl >> 1;
            const unsigned k = (unsigned)(mu * NJ + j);
            buf_group<S, 9, AUX_NONE>(wr, wsr, (k * 9u * (unsigned)Vh + (unsigned)i) * S::bytes,
                                    (k * (unsigned)Vh + (unsigned)i) * 4u, plane, o.w);
#pragma unroll
            for (int r = 0; r < TR; ++r)
                buf_group<S, 3, AUX_NONE>(vin[r], vins[r], nb * S::bytes, nb * 4u, plane, o.v[r]);
        };
        if constexpr (!PF) {
#pragma unroll 1
            for (int j = 0; j < NJ; ++j) {
                HopOperands<S, TR> o;
                fetch(o, j);
                hop_fma<S, TR>(o, acc);
            }
        } else {
#pragma unroll 1
            for (int j = 0; j < NJ; j += 2) {
                HopOperands<S, TR> o0, o1;
                fetch(o0, j);
                fetch(o1, j + 1);
                hop_fma<S, TR>(o0, acc);
                hop_fma<S, TR>(o1, acc);
            }
        }
    }
    // sum over the direction groups of the site: xor SR, ..., xor 32
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int off = SR; off < 64; off <<= 1) {
                acc[r][c].re += __shfl_xor(acc[r][c].re, off, 64);
                acc[r][c].im += __shfl_xor(acc[r][c].im, off, 64);
            }
    // lane group grp finishes right-hand sides r = grp, grp + NG, ... of the tile
    const R m2 = (R)m2d;
    double mydot = 0.0;
#pragma unroll
    for (int r = 0; r < TR; ++r) {
        if ((r % NG) == grp && tile_ok && r0 + r < N) {
            C2<R> v[3] = {acc[r][0], acc[r][1], acc[r][2]};
            C2<R> z[3];
            if (EPI != EPI_PLAIN) {
                load_group<S, 3>(ctr, ctrs, Vh, r0 + r, i, z);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[c].re = m2 * z[c].re - v[c].re;
                    v[c].im = m2 * z[c].im - v[c].im;
                }
            }
            if (live) store_group_rt<S, 3, R>(out, outs, Vh, r0 + r, i, v);
            // p^H A p of the values as stored (what the CG update reads)
            if (EPI == EPI_MASS_DOT && live)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    mydot += (double)z[c].re * (double)v[c].re + (double)z[c].im * (double)v[c].im;
        }
    }
    if (EPI == EPI_MASS_DOT) {
        // TR == 1, tpw == 1: four waves of SR sites each; lanes of groups > 0 hold 0
        __shared__ double red[4];
        for (int off = 32; off > 0; off >>= 1) mydot += __shfl_xor(mydot, off, 64);
        if (lane == 0) red[w] = mydot;
        __syncthreads();
        if (threadIdx.x == 0) dot[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

template <typename S, int TR, int NL, bool PF, int NB, bool GR>
static void launch_hop_g(const void* W, const void* in, void* out, const void* ctr, double m2, int N,
                         const Geom& g, int out_parity, int epi, const HopShape& h, const int* halt,
                         double* dot, double2* partials, int* queue, hipStream_t s) {
    using P = typename S::pair;
    const long Vh = g.Vh;
    auto scale = [&](const void* p, long cols, int K) -> float* {
        return S::scaled && p ? (float*)((char*)p + (size_t)S::bytes * cols * K * Vh) : nullptr;
    };
    const int spb = 256 / h.tpb;
    const int ntg = GR ? 1 : (N + h.tpb * TR - 1) / (h.tpb * TR);
    dim3 grid(GR ? hop_grid(g, h, true) : (unsigned)(((g.Vh + spb - 1) / spb) * ntg));
    const size_t lds = GR ? (size_t)3 * spb * (NB + 1) * sizeof(C2<typename TileElem<S>::type>) : 0;
    float* Ws = scale(W, NL, 9);
    float* ins = scale(in, N, 3);
    float* outs = scale(out, N, 3);
    float* ctrs = scale(ctr, N, 3);
    HopQueue q{};
    if (!GR && queue != nullptr && h.queue_wpc > 0) {
        q = hop_queue_layout(g, spb, queue);
        if (q.ctr != nullptr) {
            const unsigned pg = 256u * (unsigned)h.queue_wpc;
            if (pg < grid.x) grid.x = pg;
        }
    }
#define HOP_GO(E)                                                                                      \
    BCG_TIMED_LAUNCH((k_hop<S, TR, NL, E, PF, NB, GR>), grid, dim3(256), lds, s, (const P*)W, Ws,          \
                       (const P*)in, ins, (P*)out, outs, (const P*)ctr, ctrs, m2, N, g, out_parity, spb, \
                       ntg, halt, dot, partials, q)
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
                         const int* halt, double* dot, double2* partials, int* queue, hipStream_t s) {
#define HG(NBV, GRV) launch_hop_g<S, TR, NL, PF, NBV, GRV>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s)
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

template <typename S, int TR, int NL, bool PF, int SR>
static void launch_hop_ls(const void* W, const void* in, void* out, const void* ctr, double m2, int N,
                          const Geom& g, int out_parity, int epi, const int* halt, double* dot, hipStream_t s) {
    using P = typename S::pair;
    const long Vh = g.Vh;
    auto scale = [&](const void* p, long cols, int K) -> float* {
        return S::scaled && p ? (float*)((char*)p + (size_t)S::bytes * cols * K * Vh) : nullptr;
    };
    const int ntiles = (N + TR - 1) / TR;
    const int tpw = ntiles < 4 ? (ntiles < 2 ? 1 : 2) : 4;
    const int sgn = 4 / tpw;
    const long nsb = (Vh + SR * sgn - 1) / (SR * sgn);
    const dim3 grid((unsigned)(nsb * ((ntiles + tpw - 1) / tpw)));
    const float* Ws = scale(W, NL, 9);
    const float* ins = scale(in, N, 3);
    float* outs = scale(out, N, 3);
    const float* ctrs = scale(ctr, N, 3);
#define HOP_LS(E)                                                                                        \
    BCG_TIMED_LAUNCH((k_hop_ls<S, TR, NL, E, PF, SR>), grid, dim3(256), 0, s, (const P*)W, Ws, (const P*)in, \
                       ins, (P*)out, outs, (const P*)ctr, ctrs, m2, N, g, out_parity, ntiles, tpw, halt, dot)
    if (epi == EPI_PLAIN) HOP_LS(EPI_PLAIN);
    else if (epi == EPI_MASS) HOP_LS(EPI_MASS);
    else if constexpr (TR == 1) HOP_LS(EPI_MASS_DOT);
#undef HOP_LS
}

template <typename S, int NL>
static void launch_hop_nl(const void* W, const void* in, void* out, const void* ctr, double m2,
                          int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                          const int* halt, double* dot, double2* partials, int* queue, hipStream_t s) {
    if (h.split) {
#define HOP_DT(T)                                                                                        \
    (h.split == 2 ? (h.pf ? launch_hop_ls<S, T, NL, true, 32>(W, in, out, ctr, m2, N, g, out_parity, epi, halt, dot, s)   \
                          : launch_hop_ls<S, T, NL, false, 32>(W, in, out, ctr, m2, N, g, out_parity, epi, halt, dot, s))  \
                  : (h.pf ? launch_hop_ls<S, T, NL, true, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, halt, dot, s)   \
                          : launch_hop_ls<S, T, NL, false, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, halt, dot, s)))
        switch (h.tr) {
            case 1: HOP_DT(1); break;
            case 2: HOP_DT(2); break;
            case 4: HOP_DT(4); break;
            default: HOP_DT(8); break;
        }
#undef HOP_DT
        return;
    }
#define HOP_TR(T)                                                                                          \
    (h.pf ? launch_hop_t<S, T, NL, true>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s) \
          : launch_hop_t<S, T, NL, false>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s))
    switch (h.tr) {
        case 1: HOP_TR(1); break;
        case 2: HOP_TR(2); break;
        case 4: HOP_TR(4); break;
        default: HOP_TR(8); break;
    }
#undef HOP_TR
}

template <typename S>
void launch_hop_s(int nl, const void* W, const void* in, void* out, const void* ctr, double m2,
                         int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                         const int* halt, double* dot, double2* partials, int* queue, hipStream_t s) {
    if (nl == 16) launch_hop_nl<S, 16>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s);
    else launch_hop_nl<S, 8>(W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s);
}

}  // namespace bcg
