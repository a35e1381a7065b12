// Register-blocked Gram accumulation over a tile of rows staged in LDS, shared
// by the stand-alone Gram kernel and the kernels that fuse a Gram product into
// their epilogue (reduction multi-BLAS, Sec. 6.4).
//
// A tile holds R rows of NB columns (row stride LD = NB + 1 complex numbers to
// spread LDS banks).  256 threads split the NB x NB result into register blocks
// of RB x RB and the rows into G = 256 / (NB/RB)^2 row groups; each thread
// accumulates conj(A[row, i]) B[row, j] in FP64 for its block over its rows.
// gram_finish sums the row groups in a fixed order (shuffles within a wave, then
// the four waves in turn through LDS) and writes the workgroup's NB x NB partial.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace bcg {

template <int NB> struct GramBlk;
template <> struct GramBlk<1> { static constexpr int RB = 1; };
template <> struct GramBlk<2> { static constexpr int RB = 1; };
template <> struct GramBlk<4> { static constexpr int RB = 1; };
template <> struct GramBlk<8> { static constexpr int RB = 2; };
template <> struct GramBlk<16> { static constexpr int RB = 4; };
template <> struct GramBlk<32> { static constexpr int RB = 4; };
template <> struct GramBlk<64> { static constexpr int RB = 4; };

template <int NB> struct GramGeo {
    static constexpr int RB = GramBlk<NB>::RB;
    static constexpr int NBB = NB / RB;
    static constexpr int NBLK = NBB * NBB;
    static constexpr int G = 256 / NBLK;
    static constexpr int LD = NB + 1;
};

template <int NB> struct GramAcc {
    C2<double> a[GramBlk<NB>::RB][GramBlk<NB>::RB];
    __device__ void zero() {
#pragma unroll
        for (int m = 0; m < GramBlk<NB>::RB; ++m)
#pragma unroll
            for (int n = 0; n < GramBlk<NB>::RB; ++n) a[m][n] = C2<double>{0.0, 0.0};
    }
};

// acc += sum over rows r of this thread's group: conj(A[r, i]) B[r, j] for its block
template <int NB, typename E>
__device__ __forceinline__ void gram_tile_acc(const C2<E>* __restrict__ As, const C2<E>* __restrict__ Bs,
                                              int R, GramAcc<NB>& acc) {
    using Geo = GramGeo<NB>;
    constexpr int RB = Geo::RB;
    const int t = threadIdx.x;
    const int blk = t % Geo::NBLK, grp = t / Geo::NBLK;
    const int bi = blk / Geo::NBB, bj = blk % Geo::NBB;
    for (int r = grp; r < R; r += Geo::G) {
        C2<double> a[RB], b[RB];
#pragma unroll
        for (int m = 0; m < RB; ++m) {
            const C2<E> x = As[r * Geo::LD + bi * RB + m];
            const C2<E> y = Bs[r * Geo::LD + bj * RB + m];
            a[m] = C2<double>{(double)x.re, (double)x.im};
            b[m] = C2<double>{(double)y.re, (double)y.im};
        }
#pragma unroll
        for (int m = 0; m < RB; ++m)
#pragma unroll
            for (int n = 0; n < RB; ++n) cmac_conj(acc.a[m][n], a[m], b[n]);
    }
}

// Sum the row groups of the workgroup in a fixed order and write its NB x NB
// partial to out[i*NB + j].  red: LDS scratch of NB*NB C2<double> (unused when
// G == 1).  Must be called by all 256 threads; begins with a barrier.
template <int NB>
__device__ void gram_finish(GramAcc<NB>& acc, C2<double>* red, double2* __restrict__ out) {
    using Geo = GramGeo<NB>;
    constexpr int RB = Geo::RB;
    const int t = threadIdx.x;
    const int blk = t % Geo::NBLK;
    const int bi = blk / Geo::NBB, bj = blk % Geo::NBB;
    if (Geo::G == 1) {
#pragma unroll
        for (int m = 0; m < RB; ++m)
#pragma unroll
            for (int n = 0; n < RB; ++n)
                out[(bi * RB + m) * NB + bj * RB + n] = make_double2(acc.a[m][n].re, acc.a[m][n].im);
        return;
    }
    if (Geo::NBLK < 64) {
#pragma unroll
        for (int off = Geo::NBLK; off < 64; off <<= 1)
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int n = 0; n < RB; ++n) {
                    acc.a[m][n].re += __shfl_xor(acc.a[m][n].re, off, 64);
                    acc.a[m][n].im += __shfl_xor(acc.a[m][n].im, off, 64);
                }
    }
    __syncthreads();
    const int wave = t >> 6, lane = t & 63;
    const bool holder = (Geo::NBLK >= 64) || (lane < Geo::NBLK);
    for (int w = 0; w < 4; ++w) {
        if (wave == w && holder) {
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int n = 0; n < RB; ++n) {
                    const int idx = (bi * RB + m) * NB + bj * RB + n;
                    if (w == 0) red[idx] = acc.a[m][n];
                    else {
                        red[idx].re += acc.a[m][n].re;
                        red[idx].im += acc.a[m][n].im;
                    }
                }
        }
        __syncthreads();
    }
    for (int e = t; e < NB * NB; e += 256) out[e] = make_double2(red[e].re, red[e].im);
}

}  // namespace bcg
