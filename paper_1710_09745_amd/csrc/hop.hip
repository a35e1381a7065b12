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
//
// This file holds the link packing, the launch-shape choice and the dispatch;
// the kernels are in hop_kernels.h, instantiated once per storage precision by
// hop_f64.hip, hop_f32.hip, hop_h16.hip, hop_b16.hip and hop_x16.hip.
#include "device_common.h"
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

// Epilogues of the hop.
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
        case Prec::FX16: hipLaunchKernelGGL((k_group_from64<X16, 9>), grid, dim3(256), 0, s, (const double2*)W64, (unsigned int*)Wd, sc, cols, Vh); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

HopShape hop_shape(Prec p, int N, int tr, int tpb, int pf, int kernel, const Geom& g, bool fused, int sched) {
    HopShape h;
    // default kernel: the site-parallel kernel when its grid fills the chip four
    // times over, the lane-split kernel on smaller lattices (measured on MI355X:
    // 16^4 and 32^3 x 64 at N = 4 ... 64); below 16 bytes per stored complex number
    // the lane-split kernel takes runs of 32 sites, so that a load instruction covers
    // whole cache lines (16^4, N = 16, FP32: 27.0 / 29.4 us against 29.6 / 32.6 us
    // per hop; FP64 even); at N = 1 only on large lattices, where the grid of
    // 128-site workgroups still fills the chip (32^3 x 64 FP32: 310 / 298 us against
    // 337 / 330 us; 16^4: 10.3 / 10.0 against 9.2 / 8.2 us); the CG path's hop with
    // the fused dot takes the same run length
    const bool small_lattice = g.Vh / 128 < 4 * 256;
    if (fused) h.split = 0;
    else if (kernel == 1) h.split = 1;
    else if (kernel == 3) h.split = 2;
    else if (kernel == 2) h.split = 0;
    else if (N == 1) h.split = (p == Prec::FP64 || small_lattice) ? 1 : 2;
    else h.split = small_lattice ? (p == Prec::FP64 ? 1 : 2) : 0;
    if (h.split) {
        h.tpb = 1;
        h.pf = pf > 0 ? 1 : 0;
        h.tr = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
        if (tr == 1 || tr == 2 || tr == 4 || tr == 8) h.tr = tr;
        if (N <= 1) h.tr = 1;
        return h;
    }
    // site-parallel: register tile TR and lane groups tpb by N; a workgroup covers
    // tpb x TR columns and N > 16 takes several sweeps over the lattice, one per
    // group of 16 columns (narrower sweeps re-read the links more often than they
    // save in neighbour re-fetches: measured slower at 32^3 x 64)
    h.pf = 1;
    if (N <= 1) { h.tr = 1; h.tpb = 1; }
    else if (N <= 2) { h.tr = 2; h.tpb = 1; }
    else if (N <= 4) { h.tr = 4; h.tpb = 1; }
    else if (N <= 8) { h.tr = 4; h.tpb = 2; }
    else { h.tr = 8; h.tpb = 2; }
    if (pf == 1) h.pf = 1;
    else if (pf == 2) h.pf = 0;
    if (N > 1 && (tr == 1 || tr == 2 || tr == 4 || tr == 8)) h.tr = tr;
    if (N > 1 && (tpb == 1 || tpb == 2 || tpb == 4)) h.tpb = tpb;
    // per-XCD task queues (not with the fused Gram epilogue, whose per-workgroup
    // partials must not depend on which workgroup did which task)
    h.queue_wpc = 0;
    if (!fused) {
        if (sched == 2) h.queue_wpc = 1;
        else if (sched == 3) h.queue_wpc = 2;
        else if (sched == 4) h.queue_wpc = 4;
        else if (sched == 5) h.queue_wpc = 8;
    }
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

// one translation unit per storage precision instantiates the launch templates
template <typename S>
void launch_hop_s(int nl, const void* W, const void* in, void* out, const void* ctr, double m2, int N,
                  const Geom& g, int out_parity, int epi, const HopShape& h, const int* halt, double* dot,
                  double2* partials, int* queue, hipStream_t s);
extern template void launch_hop_s<F64>(int, const void*, const void*, void*, const void*, double, int, const Geom&,
                                       int, int, const HopShape&, const int*, double*, double2*, int*, hipStream_t);
extern template void launch_hop_s<F32>(int, const void*, const void*, void*, const void*, double, int, const Geom&,
                                       int, int, const HopShape&, const int*, double*, double2*, int*, hipStream_t);
extern template void launch_hop_s<H16>(int, const void*, const void*, void*, const void*, double, int, const Geom&,
                                       int, int, const HopShape&, const int*, double*, double2*, int*, hipStream_t);
extern template void launch_hop_s<B16>(int, const void*, const void*, void*, const void*, double, int, const Geom&,
                                       int, int, const HopShape&, const int*, double*, double2*, int*, hipStream_t);
extern template void launch_hop_s<X16>(int, const void*, const void*, void*, const void*, double, int, const Geom&,
                                       int, int, const HopShape&, const int*, double*, double2*, int*, hipStream_t);

// dot partials of the one-column lane-split hop: at most one per 64 sites (runs of 16)
int hop_dot_blocks(const Geom& g) { return (g.Vh + 63) / 64; }

HopQueue hop_queue_layout(const Geom& g, int spb, int* ctr) {
    HopQueue q{};
    if (ctr == nullptr || !g.slab) return q;
    const int nsb = (g.Vh + spb - 1) / spb;
    const int slice = g.L[0] * g.L[1] * g.L[2] / 2;
    int bpc = 0;
    if (slice % spb == 0) {
        const int bps = slice / spb;
        for (int Q : {4, 2, 1})
            if (bps % Q == 0) {
                bpc = bps / Q;
                break;
            }
    }
    if (bpc == 0 || nsb % bpc != 0) bpc = 1;
    q.ctr = ctr;
    q.bpc = bpc;
    q.ncell = nsb / bpc;
    return q;
}

hipError_t launch_hop(Prec prec, int nl, const void* W, const void* in, void* out, const void* ctr,
                      double m2, int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                      const int* halt, double* dot, double2* partials, int* queue, hipStream_t s) {
    if (epi == EPI_MASS_DOT_ && (N != 1 || h.tr != 1 || !h.split)) return hipErrorInvalidValue;
    if (h.split && (double)nl * 9.0 * (double)g.Vh * pd_bytes(prec) >= 4294967296.0) {
        // links beyond 32-bit lane offsets: the site-parallel kernel re-bases per matrix
        if (epi == EPI_MASS_DOT_) return hipErrorInvalidValue;
        HopShape h2 = hop_shape(prec, N, 0, 0, 0, 2, g, false);
        return launch_hop(prec, nl, W, in, out, ctr, m2, N, g, out_parity, epi, h2, halt, dot, partials, queue, s);
    }
    if (partials != nullptr && (epi != EPI_PLAIN_ || h.split || hop_tile_bytes(prec, N, h) == 0))
        return hipErrorInvalidValue;
    switch (prec) {
        case Prec::FP64: launch_hop_s<F64>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s); break;
        case Prec::FP32: launch_hop_s<F32>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s); break;
        case Prec::FP16: launch_hop_s<H16>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s); break;
        case Prec::BF16: launch_hop_s<B16>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s); break;
        case Prec::FX16: launch_hop_s<X16>(nl, W, in, out, ctr, m2, N, g, out_parity, epi, h, halt, dot, partials, queue, s); break;
    }
    return hipGetLastError();
}

}  // namespace bcg
