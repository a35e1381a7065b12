// Device-side helpers shared by the gfx950 kernels: storage types, complex
// arithmetic on (re, im) register pairs, lattice geometry of the even-odd
// checkerboard, and the ordering of the sixteen folded hop matrices.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcg {

// ---------------------------------------------------------------------------------------------
// Storage precisions.  Block vectors and links are stored as interleaved complex
// pairs in the storage type; arithmetic runs in Real (FP64 for FP64 storage,
// FP32 otherwise).
// ---------------------------------------------------------------------------------------------
template <typename T> struct Store;
template <> struct Store<double> {
    using pair = double2;
    using real = double;
};
template <> struct Store<float> {
    using pair = float2;
    using real = float;
};

template <typename R> struct C2 {
    R re, im;
};

template <typename R> __device__ __forceinline__ C2<R> c2(R a, R b) { return C2<R>{a, b}; }

template <typename P> __device__ __forceinline__ auto ld(const P* p) -> C2<decltype(p->x)> {
    P v = *p;
    return C2<decltype(p->x)>{v.x, v.y};
}

// acc += a * b
template <typename R> __device__ __forceinline__ void cmac(C2<R>& acc, C2<R> a, C2<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R> __device__ __forceinline__ void cmac_conj(C2<R>& acc, C2<R> a, C2<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

// ---------------------------------------------------------------------------------------------
// Lattice geometry.  lex = x0 + L0*(x1 + L1*(x2 + L2*x3)); parity = (x0+x1+x2+x3) & 1;
// checkerboard index cb = lex >> 1.  All extents are even.
// ---------------------------------------------------------------------------------------------
struct Geom {
    int L[4];
    int Vh;
    int slab;  // 1: XCD slab order of site blocks (xcd_task), 0: identity order
};

// coordinates of the site with checkerboard index cb on parity p
__device__ __forceinline__ void site_coords(const Geom& g, int cb, int p, int x[4]) {
    const int l = 2 * cb;
    int r = l / g.L[0];
    x[0] = l - r * g.L[0];
    int r2 = r / g.L[1];
    x[1] = r - r2 * g.L[1];
    x[3] = r2 / g.L[2];
    x[2] = r2 - x[3] * g.L[2];
    x[0] += ((x[0] + x[1] + x[2] + x[3]) & 1) ^ p;
}

// checkerboard index of x + d*mu (|d| <= 3), periodic
__device__ __forceinline__ int neighbour_cb(const Geom& g, const int x[4], int mu, int d) {
    int y0 = x[0], y1 = x[1], y2 = x[2], y3 = x[3];
    int v = x[mu] + d;
    const int L = g.L[mu];
    if (v >= L) v -= L;
    if (v >= L) v -= L;
    if (v < 0) v += L;
    if (v < 0) v += L;
    if (mu == 0) y0 = v;
    else if (mu == 1) y1 = v;
    else if (mu == 2) y2 = v;
    else y3 = v;
    return (y0 + g.L[0] * (y1 + g.L[1] * (y2 + g.L[2] * y3))) >> 1;
}

// Site-block order for XCD locality.  Workgroups are handed to the eight XCDs
// round robin (workgroup b on XCD b % 8), and each XCD has its own L2.  With bps
// site blocks per time slice (bps % 8 == 0 and nsb a multiple of bps), XCD x takes
// the x-th eighth of every time slice and all XCDs sweep the slices together: the
// slices a stencil reaches (t +- 3) are then shared in the Infinity Cache, and every
// kernel that uses this order puts a site on the same XCD, so a block vector written
// by one kernel is re-read from that XCD's L2 by the next.  Tasks are (site block,
// tile group) pairs with the ntg tile groups of a block consecutive on its XCD.
// Otherwise the identity order.  A bijection of [0, nsb * ntg).
__device__ __forceinline__ void xcd_task(int b, int nsb, int ntg, int bps, int& sb, int& tg) {
    if (bps > 0 && (bps & 7) == 0 && nsb % bps == 0) {
        const int x = b & 7, q = b >> 3;
        const int per_t = (bps >> 3) * ntg;
        const int t = q / per_t, r = q - t * per_t;
        const int k = r / ntg;
        tg = r - k * ntg;
        sb = t * bps + x * (bps >> 3) + k;
        return;
    }
    sb = b / ntg;
    tg = b - sb * ntg;
}

// Column-tile-major order: every site block of tile group 0, then of tile group 1,
// ... (one sweep over the lattice per group of columns, each sweep in the slab
// order above), so the stencil window of one sweep is a group's columns only.
__device__ __forceinline__ void xcd_task_tm(int b, int nsb, int ntg, int bps, int& sb, int& tg) {
    tg = b / nsb;
    int unused;
    xcd_task(b - tg * nsb, nsb, 1, bps, sb, unused);
    (void)ntg;
}

// site blocks of spb sites per time slice, or 0 when a slice is not a whole number of blocks
__host__ __device__ inline int blocks_per_slice(const Geom& g, int spb) {
    if (!g.slab) return 0;
    const int slice = g.L[0] * g.L[1] * g.L[2] / 2;
    return (slice % spb == 0) ? slice / spb : 0;
}

// staggered phase eta_mu(x)
__device__ __forceinline__ int eta_sign(const int x[4], int mu) {
    int s = 0;
    if (mu > 0) s += x[0];
    if (mu > 1) s += x[1];
    if (mu > 2) s += x[2];
    return (s & 1) ? -1 : 1;
}

// The NL folded matrices of an output site, k = 0 .. NL-1.  Improved (NL = 16):
// k = 4 mu + j with j = 0 fat forward (+1), 1 fat backward (-1), 2 long forward
// (+3), 3 long backward (-3).  Naive (NL = 8): k = 2 mu + j, j = 0 forward,
// 1 backward.  W_k(x) already carries eta_mu(x), the sign of the backward hop
// and the Hermitian conjugate, so (D psi)(x) = sum_k W_k(x) psi(x + d_k).
template <int NL> __device__ __forceinline__ int hop_mu(int k) { return NL == 16 ? (k >> 2) : (k >> 1); }
template <int NL> __device__ __forceinline__ int hop_d(int k) {
    const int j = NL == 16 ? (k & 3) : (k & 1);
    return ((j & 2) ? 3 : 1) * ((j & 1) ? -1 : 1);
}

// Device state of a running solve.  Written by the single-workgroup N x N
// kernels, read by every iteration kernel.
struct SolveState {
    int halt;          // nonzero: skip the remaining iteration kernels
    int reason;        // HALT_* below
    int pb_mode;       // what pass B does this iteration: PB_FULL, PB_X_ONLY, PB_SKIP
    int iters;         // active iterations so far
    double max_relres; // max_i relative iterated residual at the last active iteration
    double rho_ru;     // max relative residual at the last reliable update
    double tol;
    double ru_delta;
    double best_relres; // smallest max_relres since the last reliable update (or the start)
    int best_it;       // iteration at which best_relres was reached
    int ru_window;     // > 0: reliable update after this many iterations without a new best_relres
    double relres[64];
    double bnorm[64];
};
enum { HALT_NONE = 0, HALT_CONVERGED = 1, HALT_RU = 2, HALT_BREAKDOWN_G = 3, HALT_BREAKDOWN_H = 4, HALT_DONE = 5 };
enum { PB_FULL = 0, PB_X_ONLY = 1, PB_SKIP = 2 };

}  // namespace bcg
