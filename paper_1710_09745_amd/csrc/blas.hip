// Block BLAS for blockCGrQ on gfx950: reduction multi-BLAS (Gram products,
// Sec. 6.4), streaming multi-BLAS (block caxpy with a small N x N matrix,
// Sec. 6.3), layout conversion, and the vector kernels of the single
// right-hand-side CG baseline.
//
// Block vectors are [N][3][Vh] complex pairs (colour planes per column).  The
// streaming kernels map the 64 lanes of a wave onto 64 consecutive sites and a
// wave-uniform group of CPT output columns, so every vector load is one
// coalesced 64-site segment and every coefficient of the small matrix is a
// wave-uniform (scalar-cache) load; the other column groups of the same sites
// run in the workgroup's other waves and re-read the same lines from L1/L2, so
// HBM traffic stays linear in N (Sec. 6.3).  The Gram kernels stage a tile of
// rows of both block vectors in LDS and accumulate register blocks of the N x N
// result in FP64; partial results per workgroup are summed in a fixed order by
// a second kernel, so every reduction is deterministic.
#include <cstdlib>
#include <type_traits>

#include "device_common.h"
#include "gram_tile.h"
#include "internal.h"
#include "storage.h"

namespace bcg {

template <typename T> using PairT = typename Store<T>::pair;

// scale array of a [cols][K][Vh] block allocation in policy S (nullptr if unscaled)
template <typename S> static inline float* scale_of(const void* p, long cols, int K, long Vh) {
    if (!S::scaled || p == nullptr) return nullptr;
    return (float*)((char*)p + (size_t)S::bytes * cols * K * Vh);
}

template <typename P> __device__ __forceinline__ C2<double> ldd(const P* p) {
    const P v = *p;
    return C2<double>{(double)v.x, (double)v.y};
}
template <typename P, typename R> __device__ __forceinline__ void st(P* p, C2<R> v) {
    P w;
    w.x = v.re;
    w.y = v.im;
    *p = w;
}
__device__ __forceinline__ C2<double> dld(const double2* p) {
    const double2 v = *p;
    return C2<double>{v.x, v.y};
}

// ---------------------------------------------------------------------------------------------
// Gram:  partials[b][i*NB + j] = sum_{rows of workgroup b} conj(A[row, i]) B[row, j]
// ---------------------------------------------------------------------------------------------
template <int NB> struct GramCfg;
template <> struct GramCfg<1> { static constexpr int S = 64, RB = 1; };
template <> struct GramCfg<2> { static constexpr int S = 64, RB = 1; };
template <> struct GramCfg<4> { static constexpr int S = 64, RB = 1; };
template <> struct GramCfg<8> { static constexpr int S = 64, RB = 2; };
template <> struct GramCfg<16> { static constexpr int S = 32, RB = 4; };
template <> struct GramCfg<32> { static constexpr int S = 16, RB = 4; };
template <> struct GramCfg<64> { static constexpr int S = 8, RB = 4; };

template <typename S, int NB>
__global__ void __launch_bounds__(256)
k_gram(const typename S::pair* __restrict__ A, const float* __restrict__ As_,
       const typename S::pair* __restrict__ B, const float* __restrict__ Bs_, int N, int Vh,
       double2* __restrict__ partials, const int* __restrict__ halt) {
    if (halt != nullptr && *halt) return;
    constexpr int SITES = GramCfg<NB>::S;
    constexpr int R = 3 * SITES, LD = NB + 1;
    constexpr int EPT = (R * NB + 255) / 256;   // tile elements per thread
    __shared__ C2<double> As[R * LD];
    __shared__ C2<double> Bs[R * LD];
    const bool same = (A == B);
    const int t = threadIdx.x;
    GramAcc<NB> acc;
    acc.zero();
    for (int e = t; e < R * LD; e += 256) {
        As[e] = C2<double>{0.0, 0.0};
        Bs[e] = C2<double>{0.0, 0.0};
    }
    // the next tile is loaded into registers while the current one is reduced
    C2<double> ra[EPT], rb[EPT];
    auto fetch = [&](int tile) {
        const int site0 = tile * SITES;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = t + 256 * k;
            const int sidx = e % SITES, c = (e / SITES) % 3, j = e / R;
            const int site = site0 + sidx;
            ra[k] = C2<double>{0.0, 0.0};
            rb[k] = C2<double>{0.0, 0.0};
            if (j < N && site < Vh) {
                ra[k] = load_one_d<S, 3>(A, As_, Vh, j, c, site);
                if (!same) rb[k] = load_one_d<S, 3>(B, Bs_, Vh, j, c, site);
            }
        }
    };
    const int ntiles = (Vh + SITES - 1) / SITES;
    if (blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = t + 256 * k;
            const int sidx = e % SITES, c = (e / SITES) % 3, j = e / R;
            if (j < N) {
                As[(c * SITES + sidx) * LD + j] = ra[k];
                if (!same) Bs[(c * SITES + sidx) * LD + j] = rb[k];
            }
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) fetch(tile + gridDim.x);
        gram_tile_acc<NB, double>(As, same ? As : Bs, R, acc);
    }
    gram_finish<NB>(acc, As, partials + (long)blockIdx.x * NB * NB);
}

// ---------------------------------------------------------------------------------------------
// Gram on the matrix cores (NB = 16, 32, 64).  Each wave takes chunks of ROWS
// consecutive rows (sites of one colour), stages them in LDS (loaded site-
// coalesced, exact in the tile's element type), and feeds 16 x 4 slices to
// v_mfma_f64_16x16x4f64: with X = Xr + i Xi and 16-column tiles a, b,
//   Re G_ab = Xr_a^T Yr_b + Xi_a^T Yi_b,   Im G_ab = Xr_a^T Yi_b - Xi_a^T Yr_b.
// Only tiles a <= b are formed (the Gram is Hermitian; the lower tiles are
// written as the conjugate transpose).  For A == B the diagonal tile needs three
// products: Re G_aa as above and Im G_aa = M - M^T with M = Xr_a^T Xi_a.
// Operand layout of the 16x16x4 instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element r of lane l is D[4 r + l / 16][l % 16].
// The four waves' accumulators are summed in a fixed order in LDS at the end.
// ---------------------------------------------------------------------------------------------
typedef double dvec4 __attribute__((ext_vector_type(4)));

// sites i and i + 1 (i even) of plane (col, c) of a 16-bit [N][3][Vh] field with its
// per-(column, site) scales, decoded to float: one 8-byte load each for the packed
// pairs and the two scales (the same values load_one_d gives)
template <typename S>
__device__ __forceinline__ void load_two(const typename S::pair* __restrict__ d, const float* __restrict__ sc,
                                         long Vh, long col, int c, long i, C2<float>& v0, C2<float>& v1) {
    const uint2 u = *reinterpret_cast<const uint2*>(d + (col * 3 + c) * Vh + i);
    const float2 s = *reinterpret_cast<const float2*>(sc + col * Vh + i);
    v0 = C2<float>{S::dec((unsigned short)(u.x & 0xffffu)) * s.x, S::dec((unsigned short)(u.x >> 16)) * s.x};
    v1 = C2<float>{S::dec((unsigned short)(u.y & 0xffffu)) * s.y, S::dec((unsigned short)(u.y >> 16)) * s.y};
}

template <typename S, int NB, bool SAME> struct MfmaGram {
    using E = typename TileElem<S>::type;
    static constexpr int NT = NB / 16;
    static constexpr int NUP = NT * (NT + 1) / 2;
    // rows per wave chunk: 16, or 8 or 4 when the per-wave tiles would exceed 64 KB per
    // workgroup; 16-bit storage takes 64 or 32 rows when they fit, so that the lanes of a
    // column group (two sites each) cover 256 or 128 contiguous bytes per load
    static constexpr int TB = 4 * (NB + 1) * (int)sizeof(C2<E>) * (SAME ? 1 : 2);  // bytes per row
    static constexpr int ROWS16 = (16 * TB <= 65536) ? 16 : ((8 * TB <= 65536) ? 8 : 4);
    static constexpr int ROWS = !S::scaled ? ROWS16 : ((64 * TB <= 65536) ? 64 : ((32 * TB <= 65536) ? 32 : ROWS16));
    static constexpr int LD = NB + 1;
    static constexpr size_t tile_bytes = (size_t)4 * ROWS * LD * sizeof(C2<E>) * (SAME ? 1 : 2);
};

template <typename S, int NB, bool SAME>
__global__ void __launch_bounds__(256)
k_gram_mfma(const typename S::pair* __restrict__ A, const float* __restrict__ As_,
            const typename S::pair* __restrict__ B, const float* __restrict__ Bs_, int N, int Vh,
            double2* __restrict__ partials, const int* __restrict__ halt) {
    using G = MfmaGram<S, NB, SAME>;
    using E = typename G::E;
    // 16-bit storage: a lane fetches two consecutive sites per column with one 8-byte
    // load of the packed pairs and one of the scales (the 4-byte loads of one site at a
    // time made this Gram load-issue bound at twice the FP32 time for the same bytes)
    constexpr int SPL = S::scaled ? 2 : 1;  // sites per lane in a fetch
    constexpr int NT = G::NT, ROWS = G::ROWS, LD = G::LD, QG = 64 * SPL / ROWS;
    extern __shared__ unsigned char lds_raw[];
    C2<E>* ta = reinterpret_cast<C2<E>*>(lds_raw);
    C2<E>* tb = SAME ? ta : ta + 4 * ROWS * LD;
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    C2<E>* wa = ta + w * ROWS * LD;
    C2<E>* wb = tb + w * ROWS * LD;
    // accumulators per upper tile: Re G and Im G; for A == B the diagonal tiles keep
    // M = Xr^T Xi in the second one (Im G = M - M^T at the end)
    dvec4 acc_re[G::NUP], acc_im[G::NUP];
#pragma unroll
    for (int t = 0; t < G::NUP; ++t) {
        acc_re[t] = dvec4{0.0, 0.0, 0.0, 0.0};
        acc_im[t] = dvec4{0.0, 0.0, 0.0, 0.0};
    }
    const int nchunks = ((Vh + ROWS - 1) / ROWS) * 3;
    const int ls = lane % (ROWS / SPL), lq = lane / (ROWS / SPL);
    // the next chunk is loaded into registers while the current one is multiplied
    C2<E> ra[SPL * NB / QG], rb[SAME ? 1 : SPL * NB / QG];
    auto fetch = [&](int ch) {
        const int c = ch % 3, site = (ch / 3) * ROWS + SPL * ls;
#pragma unroll
        for (int jj = 0; jj < NB / QG; ++jj) {
            const int j = jj * QG + lq;
            if constexpr (SPL == 1) {
                const bool ok = site < Vh && j < N;
                C2<double> v{0.0, 0.0};
                if (ok) v = load_one_d<S, 3>(A, As_, Vh, j, c, site);
                ra[jj] = C2<E>{(E)v.re, (E)v.im};
                if constexpr (!SAME) {
                    C2<double> u{0.0, 0.0};
                    if (ok) u = load_one_d<S, 3>(B, Bs_, Vh, j, c, site);
                    rb[jj] = C2<E>{(E)u.re, (E)u.im};
                }
            } else {
                C2<E> v0{0.0f, 0.0f}, v1{0.0f, 0.0f}, u0{0.0f, 0.0f}, u1{0.0f, 0.0f};
                if (j < N && site + 1 < Vh) {  // site is even and Vh a multiple of 8: aligned
                    load_two<S>(A, As_, Vh, j, c, site, v0, v1);
                    if constexpr (!SAME) load_two<S>(B, Bs_, Vh, j, c, site, u0, u1);
                } else if (j < N && site < Vh) {
                    const C2<double> a = load_one_d<S, 3>(A, As_, Vh, j, c, site);
                    v0 = C2<E>{(E)a.re, (E)a.im};
                    if constexpr (!SAME) {
                        const C2<double> b = load_one_d<S, 3>(B, Bs_, Vh, j, c, site);
                        u0 = C2<E>{(E)b.re, (E)b.im};
                    }
                }
                ra[2 * jj] = v0;
                ra[2 * jj + 1] = v1;
                if constexpr (!SAME) {
                    rb[2 * jj] = u0;
                    rb[2 * jj + 1] = u1;
                }
            }
        }
    };
    const int stride = gridDim.x * 4;
    int ch = blockIdx.x * 4 + w;
    if (ch < nchunks) fetch(ch);
    for (; ch < nchunks; ch += stride) {
        // stage ROWS x NB: lane (ls, lq) holds columns lq, lq + QG, ...
#pragma unroll
        for (int jj = 0; jj < NB / QG; ++jj)
#pragma unroll
            for (int q = 0; q < SPL; ++q) {
                wa[(SPL * ls + q) * LD + jj * QG + lq] = ra[SPL * jj + q];
                if constexpr (!SAME) wb[(SPL * ls + q) * LD + jj * QG + lq] = rb[SPL * jj + q];
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ch + stride < nchunks) fetch(ch + stride);
#pragma unroll
        for (int kk = 0; kk < ROWS / 4; ++kk) {
            const int row = 4 * kk + (lane >> 4), col = lane & 15;
            double ar[NT], ai[NT], br[NT], bi[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const C2<E> a = wa[row * LD + 16 * t + col];
                ar[t] = (double)a.re;
                ai[t] = (double)a.im;
                if (!SAME) {
                    const C2<E> b = wb[row * LD + 16 * t + col];
                    br[t] = (double)b.re;
                    bi[t] = (double)b.im;
                } else {
                    br[t] = ar[t];
                    bi[t] = ai[t];
                }
            }
            int u = 0;
#pragma unroll
            for (int ta_ = 0; ta_ < NT; ++ta_)
#pragma unroll
                for (int tb_ = ta_; tb_ < NT; ++tb_, ++u) {
                    acc_re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ta_], br[tb_], acc_re[u], 0, 0, 0);
                    acc_re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[ta_], bi[tb_], acc_re[u], 0, 0, 0);
                    acc_im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[ta_], bi[tb_], acc_im[u], 0, 0, 0);
                    if (!(SAME && ta_ == tb_))
                        acc_im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[ta_], br[tb_], acc_im[u], 0, 0, 0);
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // fixed-order sum of the four waves, one upper tile at a time
    __syncthreads();
    double* red = reinterpret_cast<double*>(lds_raw);  // [4 waves][2][256]
    double2* out = partials + (long)blockIdx.x * NB * NB;
    int u = 0;
#pragma unroll
    for (int ta_ = 0; ta_ < NT; ++ta_)
#pragma unroll
        for (int tb_ = ta_; tb_ < NT; ++tb_, ++u) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = (4 * r + (lane >> 4)) * 16 + (lane & 15);
                red[(w * 2 + 0) * 256 + e] = acc_re[u][r];
                red[(w * 2 + 1) * 256 + e] = acc_im[u][r];
            }
            __syncthreads();
            {
                const int e = threadIdx.x, i = e >> 4, j = e & 15;
                const int et = j * 16 + i;  // transposed entry
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    re += red[(v * 2 + 0) * 256 + e];
                    if (SAME && ta_ == tb_) im += red[(v * 2 + 1) * 256 + e] - red[(v * 2 + 1) * 256 + et];
                    else im += red[(v * 2 + 1) * 256 + e];
                }
                const int gi = 16 * ta_ + i, gj = 16 * tb_ + j;
                out[gi * NB + gj] = make_double2(re, im);
                if (ta_ != tb_) out[gj * NB + gi] = make_double2(re, -im);
            }
            __syncthreads();
        }
}

template <typename S, int NB>
static void gram_mfma_go(const void* A, const void* B, int N, int Vh, double2* partials, const int* halt,
                         hipStream_t s, int grid) {
    using P = typename S::pair;
    const float* as = scale_of<S>(A, N, 3, Vh);
    const float* bs = scale_of<S>(B, N, 3, Vh);
    if (A == B) {
        using G = MfmaGram<S, NB, true>;
        const size_t lds = G::tile_bytes > 4 * 2 * 256 * 8 ? G::tile_bytes : 4 * 2 * 256 * 8;
        hipLaunchKernelGGL((k_gram_mfma<S, NB, true>), dim3(grid), dim3(256), lds, s, (const P*)A, as, (const P*)B,
                           bs, N, Vh, partials, halt);
    } else {
        using G = MfmaGram<S, NB, false>;
        const size_t lds = G::tile_bytes > 4 * 2 * 256 * 8 ? G::tile_bytes : 4 * 2 * 256 * 8;
        hipLaunchKernelGGL((k_gram_mfma<S, NB, false>), dim3(grid), dim3(256), lds, s, (const P*)A, as,
                           (const P*)B, bs, N, Vh, partials, halt);
    }
}

// workgroups of the matrix-core Gram: one wave per 16-row chunk at most (the
// kernel strides over chunks, so the grid does not depend on its chunk size)
static int gram_mfma_grid(int Vh) {
    const int waves = (((Vh + 15) / 16) * 3 + 3) / 4;
    return waves < GRAM_BLOCKS ? waves : GRAM_BLOCKS;
}

template <typename S>
static void gram_t(const void* A, const void* B, int N, int Vh, double2* partials, const int* halt,
                   hipStream_t s, int nb, bool mfma) {
    using P = typename S::pair;
    if (mfma && nb >= 16) {
        const int grid = gram_mfma_grid(Vh);
        if (nb == 16) gram_mfma_go<S, 16>(A, B, N, Vh, partials, halt, s, grid);
        else if (nb == 32) gram_mfma_go<S, 32>(A, B, N, Vh, partials, halt, s, grid);
        else gram_mfma_go<S, 64>(A, B, N, Vh, partials, halt, s, grid);
        return;
    }
    float* as = scale_of<S>(A, N, 3, Vh);
    float* bs = scale_of<S>(B, N, 3, Vh);
    auto go = [&](auto kern, int sites) {
        const int ntiles = (Vh + sites - 1) / sites;
        const int grid = ntiles < GRAM_BLOCKS ? ntiles : GRAM_BLOCKS;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, (const P*)A, as, (const P*)B, bs, N, Vh,
                           partials, halt);
    };
    switch (nb) {
        case 1: go(k_gram<S, 1>, GramCfg<1>::S); break;
        case 2: go(k_gram<S, 2>, GramCfg<2>::S); break;
        case 4: go(k_gram<S, 4>, GramCfg<4>::S); break;
        case 8: go(k_gram<S, 8>, GramCfg<8>::S); break;
        case 16: go(k_gram<S, 16>, GramCfg<16>::S); break;
        case 32: go(k_gram<S, 32>, GramCfg<32>::S); break;
        default: go(k_gram<S, 64>, GramCfg<64>::S); break;
    }
}

static int gram_sites(int nb) {
    switch (nb) {
        case 16: return GramCfg<16>::S;
        case 32: return GramCfg<32>::S;
        case 64: return GramCfg<64>::S;
        default: return 64;
    }
}

static int gram_nparts(int Vh, int nb, bool mfma) {
    if (mfma && nb >= 16) return gram_mfma_grid(Vh);
    const int S = gram_sites(nb);
    const int ntiles = (Vh + S - 1) / S;
    return ntiles < GRAM_BLOCKS ? ntiles : GRAM_BLOCKS;
}

hipError_t launch_gram(Prec prec, const void* A, const void* B, int N, int Vh, double2* partials,
                       const int* halt, bool mfma, hipStream_t s) {
    const int nb = pad_n(N);
    switch (prec) {
        case Prec::FP64: gram_t<F64>(A, B, N, Vh, partials, halt, s, nb, mfma); break;
        case Prec::FP32: gram_t<F32>(A, B, N, Vh, partials, halt, s, nb, mfma); break;
        case Prec::FP16: gram_t<H16>(A, B, N, Vh, partials, halt, s, nb, mfma); break;
        case Prec::BF16: gram_t<B16>(A, B, N, Vh, partials, halt, s, nb, mfma); break;
        case Prec::FX16: gram_t<X16>(A, B, N, Vh, partials, halt, s, nb, mfma); break;
    }
    return hipGetLastError();
}

int gram_parts(int N, int Vh, bool mfma) { return gram_nparts(Vh, pad_n(N), mfma); }

// out[i*64 + j] = sum_b pa[b][e] + alpha * sum_b pb[b][e], e = i*NB + j, in a fixed
// order: 256 / LPE entries per workgroup, LPE lanes per entry each summing every
// LPE-th partial (16 independent loads in flight per lane), then the LPE lane totals.
template <int LPE>
__device__ __forceinline__ void partial_sum(const double2* __restrict__ part, int P, int NN, int e,
                                            int lane, double& sr, double& si) {
    for (int p0 = lane; p0 < P; p0 += LPE * 16) {
        double2 v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int p = p0 + LPE * u;
            v[u] = p < P ? part[(long)p * NN + e] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            sr += v[u].x;
            si += v[u].y;
        }
    }
}

template <int LPE>
__global__ void __launch_bounds__(256)
k_gram_reduce(const double2* __restrict__ pa, int na, const double2* __restrict__ pb, int nb,
              double alpha, int NB, int N, double2* __restrict__ out, const int* __restrict__ halt) {
    constexpr int EPW = 256 / LPE;  // entries per workgroup
    if (halt != nullptr && *halt) return;
    __shared__ double2 red[2][EPW][LPE + 1];
    const int ent = threadIdx.x / LPE, lane = threadIdx.x % LPE;
    const int e = blockIdx.x * EPW + ent;
    const int NN = NB * NB;
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    if (e < NN) {
        partial_sum<LPE>(pa, na, NN, e, lane, ar, ai);
        if (pb != nullptr) partial_sum<LPE>(pb, nb, NN, e, lane, br, bi);
    }
    red[0][ent][lane] = make_double2(ar, ai);
    red[1][ent][lane] = make_double2(br, bi);
    __syncthreads();
    if (lane == 0 && e < NN) {
        double tr = 0.0, ti = 0.0, ur = 0.0, ui = 0.0;
        for (int g = 0; g < LPE; ++g) {
            tr += red[0][ent][g].x;
            ti += red[0][ent][g].y;
            ur += red[1][ent][g].x;
            ui += red[1][ent][g].y;
        }
        const int i = e / NB, j = e % NB;
        if (i < N && j < N) out[i * MAXN + j] = make_double2(tr + alpha * ur, ti + alpha * ui);
    }
}

constexpr int REDUCE_LPE = 32;

hipError_t launch_gram_reduce(const double2* pa, int na, const double2* pb, int nb, double alpha, int N,
                              double2* out, const int* halt, hipStream_t s) {
    const int NBv = pad_n(N);
    constexpr int EPW = 256 / REDUCE_LPE;
    const int grid = (NBv * NBv + EPW - 1) / EPW;
    hipLaunchKernelGGL(k_gram_reduce<REDUCE_LPE>, dim3(grid), dim3(256), 0, s, pa, na, pb, nb, alpha, NBv, N, out,
                       halt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Fused Gram epilogues.  A workgroup owns 64 consecutive sites (one per lane) and
// all N columns; with GR the kernel is persistent over such site tiles, stages
// the block it produces (3 colours x 64 sites = 192 rows, NB columns) in LDS and
// accumulates its Gram there (gram_tile.h), writing one NB x NB partial per
// workgroup.  Without GR it is one tile per workgroup and no LDS.
// ---------------------------------------------------------------------------------------------
template <typename S, int NB> struct FusedTile {
    using E = typename TileElem<S>::type;
    static constexpr int ROWS = 192;
    static constexpr size_t bytes = (size_t)ROWS * (NB + 1) * sizeof(C2<E>);
};

// LDS bytes a fused epilogue of precision prec and block size N would need, or 0
// when it does not fit the 64 KB LDS budget the fused epilogues keep per workgroup.
size_t fused_tile_bytes(Prec prec, int N) {
    const int nb = pad_n(N);
    const size_t e = (prec == Prec::FP64) ? 16 : 8;
    const size_t b = (size_t)192 * (nb + 1) * e;
    return b <= 65536 ? b : 0;
}

int fused_grid(int Vh) {
    const int nsb = (Vh + 63) / 64;
    return nsb < GRAM_BLOCKS ? nsb : GRAM_BLOCKS;
}

template <typename E, typename R>
__device__ __forceinline__ void tile_put(C2<E>* tile, int NBp1, int lane, int j, const C2<R> v[3], bool valid) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
        tile[(c * 64 + lane) * NBp1 + j] = valid ? C2<E>{(E)v[c].re, (E)v[c].im} : C2<E>{(E)0, (E)0};
}

// ---------------------------------------------------------------------------------------------
// Pass A:  Q <- Q - AP beta   (Alg. 1: Q S = Q - A P beta, before its QR);
// with GR also the partials of H = Qt^H Qt (Alg. 2 on Qt).
// ---------------------------------------------------------------------------------------------
template <typename S, int CPT, int NB, bool GR, int LB = std::is_same<S, F64>::value ? 2 : 4>
__global__ void __launch_bounds__(256)
k_pass_a(typename S::pair* __restrict__ Q, float* __restrict__ Qs, const typename S::pair* __restrict__ AP,
         const float* __restrict__ APs, const double2* __restrict__ beta, int N, int Vh,
         const int* __restrict__ halt, double2* __restrict__ partials, int bps) {
    using R = typename S::real;
    using E = typename TileElem<S>::type;
    extern __shared__ unsigned char lds_raw[];
    C2<E>* tile = reinterpret_cast<C2<E>*>(lds_raw);
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar coefficient loads
    const int nsb = (Vh + 63) / 64;
    GramAcc<NB> acc;
    if constexpr (GR) {
        acc.zero();
        for (int e = threadIdx.x; e < FusedTile<S, NB>::ROWS * (NB + 1); e += 256)
            tile[e] = C2<E>{(E)0, (E)0};
    }
    for (int it = blockIdx.x; it < nsb; it += gridDim.x) {
        int sb, tg_unused;
        xcd_task(it, nsb, 1, bps, sb, tg_unused);
        const int i0 = sb * 64 + lane;
        const bool valid = i0 < Vh;
        const int i = valid ? i0 : Vh - 1;  // spare lanes compute on the last site, store nothing
        if constexpr (GR) __syncthreads();
        for (int j0 = wave * CPT; j0 < N; j0 += 4 * CPT) {
            C2<R> acc2[CPT][3];
#pragma unroll
            for (int m = 0; m < CPT; ++m)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc2[m][c] = C2<R>{0, 0};
            // LB columns of AP per trip, loaded together (a ragged trip repeats column N - 1)
            for (int l0 = 0; l0 < N; l0 += LB) {
                C2<R> a[LB][3];
#pragma unroll
                for (int u = 0; u < LB; ++u) load_group<S, 3>(AP, APs, Vh, l0 + u < N ? l0 + u : N - 1, i, a[u]);
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    if (l0 + u < N) {
#pragma unroll
                        for (int m = 0; m < CPT; ++m) {
                            if (j0 + m < N) {
                                const double2 bd = beta[(l0 + u) * MAXN + j0 + m];
                                const C2<R> b{(R)bd.x, (R)bd.y};
#pragma unroll
                                for (int c = 0; c < 3; ++c) cmac(acc2[m][c], a[u][c], b);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N) {
                    C2<R> q[3];
                    load_group<S, 3>(Q, Qs, Vh, j0 + m, i, q);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        q[c].re -= acc2[m][c].re;
                        q[c].im -= acc2[m][c].im;
                    }
                    if (valid) store_group_rt<S, 3, R>(Q, Qs, Vh, j0 + m, i, q);
                    if constexpr (GR) tile_put<E, R>(tile, NB + 1, lane, j0 + m, q, valid);
                }
            }
        }
        if constexpr (GR) {
            __syncthreads();
            gram_tile_acc<NB, E>(tile, tile, FusedTile<S, NB>::ROWS, acc);
        }
    }
    if constexpr (GR) gram_finish<NB>(acc, reinterpret_cast<C2<double>*>(lds_raw), partials + (long)blockIdx.x * NB * NB);
}

// columns per thread of the streaming passes (cpt_req 1, 2 or 4 overrides the default 4)
static int pass_cpt(int N, int cpt_req) {
    const int c = (cpt_req == 1 || cpt_req == 2 || cpt_req == 4) ? cpt_req : 4;
    return N < c ? (N == 1 ? 1 : (N == 2 ? 2 : c)) : c;
}

// Pass A on the vector ALUs with beta staged in LDS (blocks of 16 columns, as
// k_pass_b_st), persistent over site blocks.  Pass A reads one coefficient matrix,
// and its scalar-load version measured faster (32^3 x 64, N = 16 ... 64), so this
// one is used only on request.
template <typename S, int LB = std::is_same<S, F64>::value ? 2 : 4>
__global__ void __launch_bounds__(256)
k_pass_a_st(typename S::pair* __restrict__ Q, float* __restrict__ Qs, const typename S::pair* __restrict__ AP,
            const float* __restrict__ APs, const double2* __restrict__ beta, int N, int Vh,
            const int* __restrict__ halt, int bps) {
    using R = typename S::real;
    constexpr int CPT = 4;
    extern __shared__ double2 cfs[];  // [N][16]
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nsb = (Vh + 63) / 64;
    for (int jb = 0; jb < N; jb += 16) {
        __syncthreads();
        for (int e = threadIdx.x; e < N * 16; e += 256) {
            const int l = e >> 4, j = jb + (e & 15);
            cfs[e] = j < N ? beta[l * MAXN + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int j0 = jb + wave * CPT;
        if (j0 >= N) continue;
        const int jl = wave * CPT;
        for (int it = blockIdx.x; it < nsb; it += gridDim.x) {
            int sb, tg_unused;
            xcd_task(it, nsb, 1, bps, sb, tg_unused);
            const int i0 = sb * 64 + lane;
            const bool valid = i0 < Vh;
            const int i = valid ? i0 : Vh - 1;
            C2<R> acc2[CPT][3];
#pragma unroll
            for (int m = 0; m < CPT; ++m)
#pragma unroll
                for (int c = 0; c < 3; ++c) acc2[m][c] = C2<R>{0, 0};
            for (int l0 = 0; l0 < N; l0 += LB) {
                C2<R> a[LB][3];
#pragma unroll
                for (int u = 0; u < LB; ++u) load_group<S, 3>(AP, APs, Vh, l0 + u < N ? l0 + u : N - 1, i, a[u]);
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    if (l0 + u < N) {
#pragma unroll
                        for (int m = 0; m < CPT; ++m) {
                            const double2 bd = cfs[(l0 + u) * 16 + jl + m];
                            const C2<R> b{(R)bd.x, (R)bd.y};
#pragma unroll
                            for (int c = 0; c < 3; ++c) cmac(acc2[m][c], a[u][c], b);
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N && valid) {
                    C2<R> q[3];
                    load_group<S, 3>(Q, Qs, Vh, j0 + m, i, q);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        q[c].re -= acc2[m][c].re;
                        q[c].im -= acc2[m][c].im;
                    }
                    store_group<S, 3, R>(Q, Qs, Vh, j0 + m, i, q);
                }
            }
        }
    }
}

template <typename S, int CPT, int NB, bool GR>
static void pass_a_go(void* Q, const void* AP, const double2* beta, int N, int Vh, const int* halt,
                      double2* partials, int bps, bool staged, hipStream_t s) {
    using P = typename S::pair;
    if constexpr (!GR) {
        if (CPT == 4 && staged) {
            const int nsb = (Vh + 63) / 64;
            const int grid = nsb < 2048 ? nsb : 2048;
            hipLaunchKernelGGL((k_pass_a_st<S>), dim3(grid), dim3(256), (size_t)N * 16 * sizeof(double2), s, (P*)Q,
                               scale_of<S>(Q, N, 3, Vh), (const P*)AP, scale_of<S>(AP, N, 3, Vh), beta, N, Vh, halt,
                               bps);
            return;
        }
    }
    const int grid = GR ? fused_grid(Vh) : (Vh + 63) / 64;
    const size_t lds = GR ? FusedTile<S, NB>::bytes : 0;
    hipLaunchKernelGGL((k_pass_a<S, CPT, NB, GR>), dim3(grid), dim3(256), lds, s, (P*)Q, scale_of<S>(Q, N, 3, Vh),
                       (const P*)AP, scale_of<S>(AP, N, 3, Vh), beta, N, Vh, halt, partials, bps);
}

template <typename S, int CPT>
static void pass_a_nb(void* Q, const void* AP, const double2* beta, int N, int Vh, const int* halt,
                      double2* partials, int bps, bool staged, hipStream_t s) {
    if (partials == nullptr) return pass_a_go<S, CPT, 1, false>(Q, AP, beta, N, Vh, halt, nullptr, bps, staged, s);
    switch (pad_n(N)) {
        case 1: return pass_a_go<S, CPT, 1, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
        case 2: return pass_a_go<S, CPT, 2, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
        case 4: return pass_a_go<S, CPT, 4, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
        case 8: return pass_a_go<S, CPT, 8, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
        case 16: return pass_a_go<S, CPT, 16, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
        default:
            if constexpr (!std::is_same<S, F64>::value) return pass_a_go<S, CPT, 32, true>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
    }
}

template <typename S>
static void pass_a_t(void* Q, const void* AP, const double2* beta, int N, int Vh, const int* halt,
                     double2* partials, int cpt_req, int bps, bool staged, hipStream_t s) {
    const int cpt = pass_cpt(N, cpt_req);
    if (cpt == 1) pass_a_nb<S, 1>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
    else if (cpt == 2) pass_a_nb<S, 2>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
    else pass_a_nb<S, 4>(Q, AP, beta, N, Vh, halt, partials, bps, staged, s);
}

// Pass A on the matrix cores (FP32 / FP64 storage, 16 < N <= 32), the same
// transposed-tile scheme as pass B: Qt^T[j][r] = Q^T[j][r] - sum_l beta^T[j][l] AP^T[l][r]
// with beta (Hermitian, staged in LDS) as the A operand and 16 rows of AP as the
// B operand, FP64 products.
template <typename S, int NT>
__global__ void __launch_bounds__(256)
k_pass_a_mfma(typename S::pair* __restrict__ Q, const typename S::pair* __restrict__ AP,
              const double2* __restrict__ beta, int N, int Vh, const int* __restrict__ halt) {
    using PR = typename S::pair;
    using R = typename S::real;
    constexpr int NQ = 4 * NT;
    constexpr int NP = 16 * NT;
    extern __shared__ double2 cf[];  // [NP][NP] beta, zero outside N x N
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, k4 = lane >> 4;
    for (int e = threadIdx.x; e < NP * NP; e += 256) {
        const int l = e / NP, j = e % NP;
        cf[e] = (l < N && j < N) ? beta[l * MAXN + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long ngroups = (nrb + 3) / 4;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const long rb0 = g * 4 + w;
        const bool rb_ok = rb0 < nrb;
        const long rb = rb_ok ? rb0 : nrb - 1;
        const int c = (int)(rb % 3);
        const int site = (int)(rb / 3) * 16 + r16;
        const bool live = rb_ok && site < Vh;
        const int si = site < Vh ? site : Vh - 1;
        R ar[NQ], ai[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int l = 4 * q + k4;
            const bool ok = l < N;
            const PR a = AP[((long)(ok ? l : N - 1) * 3 + c) * Vh + si];
            ar[q] = ok ? a.x : (R)0;
            ai[q] = ok ? a.y : (R)0;
        }
#pragma unroll 1
        for (int jt = 0; jt < NT; ++jt) {
            const int jo = jt * 16 + r16;
            dvec4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int l = 4 * q + k4;
                const double2 m = cf[l * NP + jo];
                const double dr = (double)ar[q], di = (double)ai[q];
                yr = __builtin_amdgcn_mfma_f64_16x16x4f64(m.x, dr, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f64_16x16x4f64(m.x, di, yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f64_16x16x4f64(-m.y, di, yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f64_16x16x4f64(m.y, dr, yi, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int j = jt * 16 + 4 * m + k4;
                if (!live || j >= N) continue;
                const long o = ((long)j * 3 + c) * Vh + site;
                PR qv = Q[o];
                qv.x = (R)((double)qv.x - yr[m]);
                qv.y = (R)((double)qv.y - yi[m]);
                Q[o] = qv;
            }
        }
    }
}

// Pass A on the matrix cores for FP32 storage and 32 < N <= 64: the layout of
// k_pass_a_mfma with beta staged in FP32 (32 KB) and the products on
// v_mfma_f32_16x16x4f32 (FP32 storage, FP32 arithmetic, as the vector kernel).
#define F32_ACC_ROW(m, l) (4 * ((l) >> 4) + (m))
__global__ void __launch_bounds__(256)
k_pass_a_mfma32(float2* __restrict__ Q, const float2* __restrict__ AP, const double2* __restrict__ beta, int N,
                int Vh, const int* __restrict__ halt) {
    constexpr int NT = 4, NQ = 16, NP = 64;
    typedef float fvec4 __attribute__((ext_vector_type(4)));
    extern __shared__ float2 cb[];  // [NP][NP] beta in FP32, zero outside N x N
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, k4 = lane >> 4;
    for (int e = threadIdx.x; e < NP * NP; e += 256) {
        const int l = e / NP, j = e % NP;
        const double2 b = (l < N && j < N) ? beta[l * MAXN + j] : make_double2(0.0, 0.0);
        cb[e] = make_float2((float)b.x, (float)b.y);
    }
    __syncthreads();
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long ngroups = (nrb + 3) / 4;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const long rb0 = g * 4 + w;
        const bool rb_ok = rb0 < nrb;
        const long rb = rb_ok ? rb0 : nrb - 1;
        const int c = (int)(rb % 3);
        const int site = (int)(rb / 3) * 16 + r16;
        const bool live = rb_ok && site < Vh;
        const int si = site < Vh ? site : Vh - 1;
        float ar[NQ], ai[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int l = 4 * q + k4;
            const bool ok = l < N;
            const float2 a = AP[((long)(ok ? l : N - 1) * 3 + c) * Vh + si];
            ar[q] = ok ? a.x : 0.0f;
            ai[q] = ok ? a.y : 0.0f;
        }
#pragma unroll 1
        for (int jt = 0; jt < NT; ++jt) {
            if (jt * 16 >= N) break;
            const int jo = jt * 16 + r16;
            fvec4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int l = 4 * q + k4;
                const float2 m = cb[l * NP + jo];
                yr = __builtin_amdgcn_mfma_f32_16x16x4f32(m.x, ar[q], yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x4f32(m.x, ai[q], yi, 0, 0, 0);
                yr = __builtin_amdgcn_mfma_f32_16x16x4f32(-m.y, ai[q], yr, 0, 0, 0);
                yi = __builtin_amdgcn_mfma_f32_16x16x4f32(m.y, ar[q], yi, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int j = jt * 16 + F32_ACC_ROW(m, lane);
                if (!live || j >= N) continue;
                const long o = ((long)j * 3 + c) * Vh + site;
                float2 qv = Q[o];
                qv.x -= yr[m];
                qv.y -= yi[m];
                Q[o] = qv;
            }
        }
    }
}
#undef F32_ACC_ROW

hipError_t launch_pass_a(Prec prec, void* Q, const void* AP, const double2* beta, int N, int Vh,
                         const int* halt, double2* partials, int cpt, int bps, int kernel, hipStream_t s) {
    if (partials != nullptr && fused_tile_bytes(prec, N) == 0) return hipErrorInvalidValue;
    if ((kernel == 0 || kernel == 1) && partials == nullptr && N > 16 && N <= 32 &&
        (prec == Prec::FP64 || prec == Prec::FP32)) {
        const long groups = ((long)((Vh + 15) / 16) * 3 + 3) / 4;
        const dim3 grid((unsigned)(groups < 2048 ? groups : 2048));
        const size_t lds = (size_t)32 * 32 * sizeof(double2);
        if (prec == Prec::FP64)
            hipLaunchKernelGGL((k_pass_a_mfma<F64, 2>), grid, dim3(256), lds, s, (double2*)Q, (const double2*)AP,
                               beta, N, Vh, halt);
        else
            hipLaunchKernelGGL((k_pass_a_mfma<F32, 2>), grid, dim3(256), lds, s, (float2*)Q, (const float2*)AP,
                               beta, N, Vh, halt);
        return hipGetLastError();
    }
    if ((kernel == 0 || kernel == 1) && partials == nullptr && N > 32 && N <= 64 && prec == Prec::FP32) {
        const long groups = ((long)((Vh + 15) / 16) * 3 + 3) / 4;
        const dim3 grid((unsigned)(groups < 2048 ? groups : 2048));
        hipLaunchKernelGGL(k_pass_a_mfma32, grid, dim3(256), (size_t)64 * 64 * sizeof(float2), s, (float2*)Q,
                           (const float2*)AP, beta, N, Vh, halt);
        return hipGetLastError();
    }
    if ((kernel == 0 || kernel == 1) && partials == nullptr && N > 32 && N <= 64 && prec == Prec::FP64) {
        // four column tiles, beta in FP64 (64 KB of LDS: two workgroups per CU); at N = 64
        // 1.41x (16^4) and 1.69x (32^3 x 64) faster than the vector kernel
        // (FP64 pass B stays on the vector kernel for N > 32: a matrix-core version with
        // packed triangular S^{-1} and S^H measured slower at four waves per CU)
        const long groups = ((long)((Vh + 15) / 16) * 3 + 3) / 4;
        const dim3 grid((unsigned)(groups < 2048 ? groups : 2048));
        hipLaunchKernelGGL((k_pass_a_mfma<F64, 4>), grid, dim3(256), (size_t)64 * 64 * sizeof(double2), s,
                           (double2*)Q, (const double2*)AP, beta, N, Vh, halt);
        return hipGetLastError();
    }
    switch (prec) {
        case Prec::FP64: pass_a_t<F64>(Q, AP, beta, N, Vh, halt, partials, cpt, bps, kernel == 2, s); break;
        case Prec::FP32: pass_a_t<F32>(Q, AP, beta, N, Vh, halt, partials, cpt, bps, kernel == 2, s); break;
        case Prec::FP16: pass_a_t<H16>(Q, AP, beta, N, Vh, halt, partials, cpt, bps, kernel == 2, s); break;
        case Prec::BF16: pass_a_t<B16>(Q, AP, beta, N, Vh, halt, partials, cpt, bps, kernel == 2, s); break;
        case Prec::FX16: pass_a_t<X16>(Q, AP, beta, N, Vh, halt, partials, cpt, bps, kernel == 2, s); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Pass B (Alg. 1, with the X update of the same iteration deferred to here, Sec. 6.2):
//   X  += P (beta C)                      (old P; formed and added in FP64)
//   Qn  = Qt S^{-1}                       (S^{-1} upper triangular: l <= j only)
//   Pn  = Qn + P S^H                      (S^H lower triangular: l >= j only)
// Qn, Pn are written to other buffers than Qt, P (ping-pong), so there is no
// in-place hazard between the waves that read all columns and those that write.
// With GR also the partials of Pn^H Pn (the P^H P term of the next iteration's
// G = 4 m^2 P^H P + T^H T).
// ---------------------------------------------------------------------------------------------
template <typename S, int CPT, int NB, bool GR, int LB = std::is_same<S, F64>::value ? 2 : 4>
__global__ void __launch_bounds__(256)
k_pass_b(double2* __restrict__ X, const typename S::pair* __restrict__ Qt, const float* __restrict__ Qts,
         const typename S::pair* __restrict__ P, const float* __restrict__ Ps,
         typename S::pair* __restrict__ Qn, float* __restrict__ Qns, typename S::pair* __restrict__ Pn,
         float* __restrict__ Pns, const double2* __restrict__ betaC, const double2* __restrict__ Sinv,
         const double2* __restrict__ SH, int N, int Vh, const SolveState* __restrict__ stt,
         double2* __restrict__ partials, int bps) {
    using R = typename S::real;
    using E = typename TileElem<S>::type;
    extern __shared__ unsigned char lds_raw[];
    C2<E>* tile = reinterpret_cast<C2<E>*>(lds_raw);
    const int mode = stt->pb_mode;
    if (mode == PB_SKIP) return;
    const bool full = (mode == PB_FULL);
    const bool gram = GR && full;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar coefficient loads
    const int nsb = (Vh + 63) / 64;
    GramAcc<NB> acc;
    if constexpr (GR) {
        acc.zero();
        for (int e = threadIdx.x; e < FusedTile<S, NB>::ROWS * (NB + 1); e += 256)
            tile[e] = C2<E>{(E)0, (E)0};
    }
    for (int it = blockIdx.x; it < nsb; it += gridDim.x) {
        int sb, tg_unused;
        xcd_task(it, nsb, 1, bps, sb, tg_unused);
        const int i0 = sb * 64 + lane;
        const bool valid = i0 < Vh;
        const int i = valid ? i0 : Vh - 1;  // spare lanes compute on the last site, store nothing
        if (gram) __syncthreads();
        for (int j0 = wave * CPT; j0 < N; j0 += 4 * CPT) {
            C2<double> xa[CPT][3];
            C2<R> qa[CPT][3], pa[CPT][3];
#pragma unroll
            for (int m = 0; m < CPT; ++m)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xa[m][c] = C2<double>{0.0, 0.0};
                    qa[m][c] = C2<R>{0, 0};
                    pa[m][c] = C2<R>{0, 0};
                }
            // LB columns of P (and of Qt while S^{-1} has entries for this tile) per
            // trip, loaded together; a ragged trip repeats column N - 1
            for (int l0 = 0; l0 < N; l0 += LB) {
                const bool needq = full && l0 < j0 + CPT;
                C2<R> p[LB][3], q[LB][3];
#pragma unroll
                for (int u = 0; u < LB; ++u) load_group<S, 3>(P, Ps, Vh, l0 + u < N ? l0 + u : N - 1, i, p[u]);
                if (needq) {
#pragma unroll
                    for (int u = 0; u < LB; ++u) load_group<S, 3>(Qt, Qts, Vh, l0 + u < N ? l0 + u : N - 1, i, q[u]);
                }
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int l = l0 + u;
                    if (l >= N) break;
#pragma unroll
                    for (int m = 0; m < CPT; ++m) {
                        if (j0 + m < N) {
                            const double2 bc = betaC[l * MAXN + j0 + m];
#pragma unroll
                            for (int c = 0; c < 3; ++c)
                                cmac(xa[m][c], C2<double>{(double)p[u][c].re, (double)p[u][c].im}, C2<double>{bc.x, bc.y});
                        }
                    }
                    if (full) {
#pragma unroll
                        for (int m = 0; m < CPT; ++m) {
                            if (j0 + m < N && l >= j0 + m) {
                                const double2 sh = SH[l * MAXN + j0 + m];
                                const C2<R> b{(R)sh.x, (R)sh.y};
#pragma unroll
                                for (int c = 0; c < 3; ++c) cmac(pa[m][c], p[u][c], b);
                            }
                        }
                        if (needq) {
#pragma unroll
                            for (int m = 0; m < CPT; ++m) {
                                if (j0 + m < N && l <= j0 + m) {
                                    const double2 si = Sinv[l * MAXN + j0 + m];
                                    const C2<R> b{(R)si.x, (R)si.y};
#pragma unroll
                                    for (int c = 0; c < 3; ++c) cmac(qa[m][c], q[u][c], b);
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N) {
                    if (valid) {
                        double2 xv[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) xv[c] = X[((long)(j0 + m) * 3 + c) * Vh + i];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            xv[c].x += xa[m][c].re;
                            xv[c].y += xa[m][c].im;
                            X[((long)(j0 + m) * 3 + c) * Vh + i] = xv[c];
                        }
                    }
                    if (full) {
                        if (valid) {
                            store_group<S, 3, R>(Qn, Qns, Vh, j0 + m, i, qa[m]);
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                pa[m][c].re += qa[m][c].re;
                                pa[m][c].im += qa[m][c].im;
                            }
                            store_group_rt<S, 3, R>(Pn, Pns, Vh, j0 + m, i, pa[m]);
                        }
                        if constexpr (GR) tile_put<E, R>(tile, NB + 1, lane, j0 + m, pa[m], valid);
                    }
                }
            }
        }
        if (gram) {
            __syncthreads();
            gram_tile_acc<NB, E>(tile, tile, FusedTile<S, NB>::ROWS, acc);
        }
    }
    if (gram) gram_finish<NB>(acc, reinterpret_cast<C2<double>*>(lds_raw), partials + (long)blockIdx.x * NB * NB);
}

// Pass B on the vector ALUs with the coefficients in LDS.  The coefficient reads
// of the kernel above are wave-uniform scalar loads, and a 64 x 64 FP64 matrix
// does not stay in the scalar cache, so every column step waited on L2.  Here the
// workgroup stages a block of 16 columns of beta C, S^{-1} and S^H ([3][N][16], at
// most 48 KB) in LDS and then sweeps its share of the site blocks for those
// columns (wave w takes columns 4w .. 4w+3 of the block); the coefficient reads are
// LDS broadcasts.  Persistent grid: block jb is staged once per workgroup.
template <typename S, int LB = std::is_same<S, F64>::value ? 2 : 4>
__global__ void __launch_bounds__(256)
k_pass_b_st(double2* __restrict__ X, const typename S::pair* __restrict__ Qt, const float* __restrict__ Qts,
            const typename S::pair* __restrict__ P, const float* __restrict__ Ps,
            typename S::pair* __restrict__ Qn, float* __restrict__ Qns, typename S::pair* __restrict__ Pn,
            float* __restrict__ Pns, const double2* __restrict__ betaC, const double2* __restrict__ Sinv,
            const double2* __restrict__ SH, int N, int Vh, const SolveState* __restrict__ stt, int bps) {
    using R = typename S::real;
    constexpr int CPT = 4;
    extern __shared__ double2 cfs[];  // [3][N][16]
    const int mode = stt->pb_mode;
    if (mode == PB_SKIP) return;
    const bool full = (mode == PB_FULL);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nsb = (Vh + 63) / 64;
    for (int jb = 0; jb < N; jb += 16) {
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * N * 16; e += 256) {
            const int mat = e / (N * 16), rem = e - mat * N * 16;
            const int l = rem >> 4, j = jb + (rem & 15);
            const double2* M = mat == 0 ? betaC : (mat == 1 ? Sinv : SH);
            cfs[e] = j < N ? M[l * MAXN + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int j0 = jb + wave * CPT;
        if (j0 >= N) continue;
        const int jl = wave * CPT;  // column of the staged block
        const double2* cb = cfs;
        const double2* ci = cfs + N * 16;
        const double2* ch = cfs + 2 * N * 16;
        for (int it = blockIdx.x; it < nsb; it += gridDim.x) {
            int sb, tg_unused;
            xcd_task(it, nsb, 1, bps, sb, tg_unused);
            const int i0 = sb * 64 + lane;
            const bool valid = i0 < Vh;
            const int i = valid ? i0 : Vh - 1;
            C2<double> xa[CPT][3];
            C2<R> qa[CPT][3], pa[CPT][3];
#pragma unroll
            for (int m = 0; m < CPT; ++m)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xa[m][c] = C2<double>{0.0, 0.0};
                    qa[m][c] = C2<R>{0, 0};
                    pa[m][c] = C2<R>{0, 0};
                }
            for (int l0 = 0; l0 < N; l0 += LB) {
                const bool needq = full && l0 < j0 + CPT;
                C2<R> p[LB][3], q[LB][3];
#pragma unroll
                for (int u = 0; u < LB; ++u) load_group<S, 3>(P, Ps, Vh, l0 + u < N ? l0 + u : N - 1, i, p[u]);
                if (needq) {
#pragma unroll
                    for (int u = 0; u < LB; ++u) load_group<S, 3>(Qt, Qts, Vh, l0 + u < N ? l0 + u : N - 1, i, q[u]);
                }
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int l = l0 + u;
                    if (l >= N) break;
#pragma unroll
                    for (int m = 0; m < CPT; ++m) {
                        const double2 bc = cb[l * 16 + jl + m];
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            cmac(xa[m][c], C2<double>{(double)p[u][c].re, (double)p[u][c].im}, C2<double>{bc.x, bc.y});
                    }
                    if (full) {
#pragma unroll
                        for (int m = 0; m < CPT; ++m) {
                            if (l >= j0 + m) {
                                const double2 sh = ch[l * 16 + jl + m];
                                const C2<R> b{(R)sh.x, (R)sh.y};
#pragma unroll
                                for (int c = 0; c < 3; ++c) cmac(pa[m][c], p[u][c], b);
                            }
                        }
                        if (needq) {
#pragma unroll
                            for (int m = 0; m < CPT; ++m) {
                                if (l <= j0 + m) {
                                    const double2 si = ci[l * 16 + jl + m];
                                    const C2<R> b{(R)si.x, (R)si.y};
#pragma unroll
                                    for (int c = 0; c < 3; ++c) cmac(qa[m][c], q[u][c], b);
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N && valid) {
                    double2 xv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) xv[c] = X[((long)(j0 + m) * 3 + c) * Vh + i];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        xv[c].x += xa[m][c].re;
                        xv[c].y += xa[m][c].im;
                        X[((long)(j0 + m) * 3 + c) * Vh + i] = xv[c];
                    }
                    if (full) {
                        store_group<S, 3, R>(Qn, Qns, Vh, j0 + m, i, qa[m]);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            pa[m][c].re += qa[m][c].re;
                            pa[m][c].im += qa[m][c].im;
                        }
                        store_group<S, 3, R>(Pn, Pns, Vh, j0 + m, i, pa[m]);
                    }
                }
            }
        }
    }
}

template <typename S, int CPT, int NB, bool GR>
static void pass_b_go(double2* X, const void* Qt, const void* P, void* Qn, void* Pn, const double2* betaC,
                      const double2* Sinv, const double2* SH, int N, int Vh, const SolveState* st,
                      double2* partials, int bps, bool staged, hipStream_t s) {
    using PP = typename S::pair;
    if constexpr (!GR) {
        if (CPT == 4 && staged) {
            const int nsb = (Vh + 63) / 64;
            const int grid = nsb < 2048 ? nsb : 2048;
            hipLaunchKernelGGL((k_pass_b_st<S>), dim3(grid), dim3(256), (size_t)3 * N * 16 * sizeof(double2), s, X,
                               (const PP*)Qt, scale_of<S>(Qt, N, 3, Vh), (const PP*)P, scale_of<S>(P, N, 3, Vh),
                               (PP*)Qn, scale_of<S>(Qn, N, 3, Vh), (PP*)Pn, scale_of<S>(Pn, N, 3, Vh), betaC, Sinv,
                               SH, N, Vh, st, bps);
            return;
        }
    }
    const int grid = GR ? fused_grid(Vh) : (Vh + 63) / 64;
    const size_t lds = GR ? FusedTile<S, NB>::bytes : 0;
    hipLaunchKernelGGL((k_pass_b<S, CPT, NB, GR>), dim3(grid), dim3(256), lds, s, X, (const PP*)Qt,
                       scale_of<S>(Qt, N, 3, Vh), (const PP*)P, scale_of<S>(P, N, 3, Vh), (PP*)Qn,
                       scale_of<S>(Qn, N, 3, Vh), (PP*)Pn, scale_of<S>(Pn, N, 3, Vh), betaC, Sinv, SH, N, Vh,
                       st, partials, bps);
}

template <typename S, int CPT>
static void pass_b_nb(double2* X, const void* Qt, const void* P, void* Qn, void* Pn, const double2* betaC,
                      const double2* Sinv, const double2* SH, int N, int Vh, const SolveState* st,
                      double2* partials, int bps, bool staged, hipStream_t s) {
#define PBG(NBV, GRV) pass_b_go<S, CPT, NBV, GRV>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, st, partials, bps, staged, s)
    if (partials == nullptr) return PBG(1, false);
    switch (pad_n(N)) {
        case 1: return PBG(1, true);
        case 2: return PBG(2, true);
        case 4: return PBG(4, true);
        case 8: return PBG(8, true);
        case 16: return PBG(16, true);
        default:
            if constexpr (!std::is_same<S, F64>::value) return PBG(32, true);
    }
#undef PBG
}

template <typename S>
static void pass_b_t(double2* X, const void* Qt, const void* P, void* Qn, void* Pn, const double2* betaC,
                     const double2* Sinv, const double2* SH, int N, int Vh, const SolveState* st,
                     double2* partials, int cpt_req, int bps, bool staged, hipStream_t s) {
    const int cpt = pass_cpt(N, cpt_req);
    if (cpt == 1) pass_b_nb<S, 1>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, st, partials, bps, staged, s);
    else if (cpt == 2) pass_b_nb<S, 2>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, st, partials, bps, staged, s);
    else pass_b_nb<S, 4>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, st, partials, bps, staged, s);
}

// ---------------------------------------------------------------------------------------------
// Pass B on the matrix cores (FP32 and FP64 storage, N > 16).  Transposed, every
// output column tile is a small GEMM  Y^T[j][r] = sum_l M^T[j][l] D^T[l][r]  with a
// coefficient matrix M (beta C, S^{-1} or S^H) as the 16 x 4 A operand and the data
// (P or Qt over a block of 16 rows: 16 consecutive sites of one colour) as the
// 4 x 16 B operand, in FP64 (v_mfma_f64_16x16x4f64; a complex product is four real
// ones).  A wave owns one row block: it loads all N columns of P and Qt for its rows
// once (each load: 4 columns x 16 consecutive sites) into registers and then walks
// the NT output column tiles.  Accumulator element m of lane l is column 4m + l/16
// of the tile at row l % 16, so each store also covers 4 columns x 16 sites.  S^{-1}
// is upper and S^H lower triangular: K-steps wholly outside a triangle are skipped.
// Coefficients beyond N x N are treated as zero (their storage is never written).
// ---------------------------------------------------------------------------------------------
template <typename S, int NT>
__global__ void __launch_bounds__(256)
k_pass_b_mfma(double2* __restrict__ X, const typename S::pair* __restrict__ Qt,
              const typename S::pair* __restrict__ P, typename S::pair* __restrict__ Qn,
              typename S::pair* __restrict__ Pn, const double2* __restrict__ betaC,
              const double2* __restrict__ Sinv, const double2* __restrict__ SH, int N, int Vh,
              const SolveState* __restrict__ stt) {
    using PR = typename S::pair;
    using R = typename S::real;
    constexpr int NQ = 4 * NT;      // K-steps of four columns
    constexpr int NP = 16 * NT;     // N padded to whole tiles
    extern __shared__ double2 cf[];  // [3][NP][NP] coefficient matrices, zero outside N x N
    const int mode = stt->pb_mode;
    if (mode == PB_SKIP) return;
    const bool full = (mode == PB_FULL);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, k4 = lane >> 4;
    for (int e = threadIdx.x; e < 3 * NP * NP; e += 256) {
        const int mat = e / (NP * NP), rem = e - mat * NP * NP;
        const int l = rem / NP, j = rem % NP;
        const double2* M = mat == 0 ? betaC : (mat == 1 ? Sinv : SH);
        cf[e] = (l < N && j < N) ? M[l * MAXN + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long ngroups = (nrb + 3) / 4;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const long rb0 = g * 4 + w;
        const bool rb_ok = rb0 < nrb;
        const long rb = rb_ok ? rb0 : nrb - 1;
        const int c = (int)(rb % 3);
        const int site = (int)(rb / 3) * 16 + r16;
        const bool live = rb_ok && site < Vh;
        const int si = site < Vh ? site : Vh - 1;
        // lane (r16, k4) holds column 4q + k4 of row (site, c) for every K-step q
        R pr[NQ], pi[NQ], qr[NQ], qi[NQ];  // storage precision; exact in FP64 at use
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int l = 4 * q + k4;
            const bool ok = l < N;
            const int lc = ok ? l : N - 1;
            const PR a = P[((long)lc * 3 + c) * Vh + si];
            const PR b = Qt[((long)lc * 3 + c) * Vh + si];
            pr[q] = ok ? a.x : (R)0;
            pi[q] = ok ? a.y : (R)0;
            qr[q] = ok ? b.x : (R)0;
            qi[q] = ok ? b.y : (R)0;
        }
#pragma unroll 1
        for (int jt = 0; jt < NT; ++jt) {
            const int jo = jt * 16 + r16;  // coefficient column of this lane (A-operand row)
            dvec4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
            dvec4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};  // Qt S^{-1}
            dvec4 br = {0, 0, 0, 0}, bi = {0, 0, 0, 0};  // P S^H
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int l = 4 * q + k4;
                const double dpr = (double)pr[q], dpi = (double)pi[q];
                const double dqr = (double)qr[q], dqi = (double)qi[q];
                const double2 m1 = cf[(0 * NP + l) * NP + jo];
                const bool uq = full && q <= 4 * jt + 3;
                const bool up = full && q >= 4 * jt;
                const double2 m2 = uq ? cf[(1 * NP + l) * NP + jo] : make_double2(0.0, 0.0);
                const double2 m3 = up ? cf[(2 * NP + l) * NP + jo] : make_double2(0.0, 0.0);
                // independent accumulators interleaved between the two halves of each product
                xr = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.x, dpr, xr, 0, 0, 0);
                xi = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.x, dpi, xi, 0, 0, 0);
                if (uq) {
                    ar = __builtin_amdgcn_mfma_f64_16x16x4f64(m2.x, dqr, ar, 0, 0, 0);
                    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(m2.x, dqi, ai, 0, 0, 0);
                }
                if (up) {
                    br = __builtin_amdgcn_mfma_f64_16x16x4f64(m3.x, dpr, br, 0, 0, 0);
                    bi = __builtin_amdgcn_mfma_f64_16x16x4f64(m3.x, dpi, bi, 0, 0, 0);
                }
                xr = __builtin_amdgcn_mfma_f64_16x16x4f64(-m1.y, dpi, xr, 0, 0, 0);
                xi = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.y, dpr, xi, 0, 0, 0);
                if (uq) {
                    ar = __builtin_amdgcn_mfma_f64_16x16x4f64(-m2.y, dqi, ar, 0, 0, 0);
                    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(m2.y, dqr, ai, 0, 0, 0);
                }
                if (up) {
                    br = __builtin_amdgcn_mfma_f64_16x16x4f64(-m3.y, dpi, br, 0, 0, 0);
                    bi = __builtin_amdgcn_mfma_f64_16x16x4f64(m3.y, dpr, bi, 0, 0, 0);
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int j = jt * 16 + 4 * m + k4;
                if (!live || j >= N) continue;
                const long o = ((long)j * 3 + c) * Vh + site;
                double2 xv = X[o];
                xv.x += xr[m];
                xv.y += xi[m];
                X[o] = xv;
                if (full) {
                    PR qv, pv;
                    qv.x = (R)ar[m];
                    qv.y = (R)ai[m];
                    // P = Q + P S^H with Q as stored
                    pv.x = (R)((double)qv.x + br[m]);
                    pv.y = (R)((double)qv.y + bi[m]);
                    Qn[o] = qv;
                    Pn[o] = pv;
                }
            }
        }
    }
}

// Pass B on the matrix cores for FP32 storage and 32 < N <= 64 (NT = 4 column tiles).
// The layout of k_pass_b_mfma, but the three 64 x 64 coefficient matrices do not fit
// LDS in FP64 (192 KB), so beta C stays FP64 (64 KB, the X increment in FP64 as in
// the vector kernels) while S^{-1} and S^H are staged in FP32 (32 KB each) and the
// Q and P products run on v_mfma_f32_16x16x4f32 (FP32 storage and FP32 arithmetic,
// as the vector kernels).  128 KB of LDS: one workgroup of NW waves per CU, persistent.
// Accumulator element m of lane l of the FP32 instruction holds row
// F32_ACC_ROW(m, l) of its 16 x 16 tile (checked on the device by an in-bounds probe).
#define F32_ACC_ROW(m, l) (4 * ((l) >> 4) + (m))
template <int NW>
__global__ void __launch_bounds__(64 * NW)
k_pass_b_mfma32(double2* __restrict__ X, const float2* __restrict__ Qt, const float2* __restrict__ P,
                float2* __restrict__ Qn, float2* __restrict__ Pn, const double2* __restrict__ betaC,
                const double2* __restrict__ Sinv, const double2* __restrict__ SH, int N, int Vh,
                const SolveState* __restrict__ stt) {
    constexpr int NT = 4, NQ = 16, NP = 64;
    typedef float fvec4 __attribute__((ext_vector_type(4)));
    extern __shared__ double2 cf64[];                                  // [NP][NP] beta C
    float2* cf32 = reinterpret_cast<float2*>(cf64 + NP * NP);          // [2][NP][NP] S^{-1}, S^H
    const int mode = stt->pb_mode;
    if (mode == PB_SKIP) return;
    const bool full = (mode == PB_FULL);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, k4 = lane >> 4;
    for (int e = threadIdx.x; e < NP * NP; e += 64 * NW) {
        const int l = e / NP, j = e % NP;
        const bool in = l < N && j < N;
        cf64[e] = in ? betaC[l * MAXN + j] : make_double2(0.0, 0.0);
        const double2 a = in ? Sinv[l * MAXN + j] : make_double2(0.0, 0.0);
        const double2 b = in ? SH[l * MAXN + j] : make_double2(0.0, 0.0);
        cf32[e] = make_float2((float)a.x, (float)a.y);
        cf32[NP * NP + e] = make_float2((float)b.x, (float)b.y);
    }
    __syncthreads();
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long ngroups = (nrb + NW - 1) / NW;
    for (long g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const long rb0 = g * NW + w;
        const bool rb_ok = rb0 < nrb;
        const long rb = rb_ok ? rb0 : nrb - 1;
        const int c = (int)(rb % 3);
        const int site = (int)(rb / 3) * 16 + r16;
        const bool live = rb_ok && site < Vh;
        const int si = site < Vh ? site : Vh - 1;
        float pr[NQ], pi[NQ], qr[NQ], qi[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int l = 4 * q + k4;
            const bool ok = l < N;
            const int lc = ok ? l : N - 1;
            const float2 a = P[((long)lc * 3 + c) * Vh + si];
            const float2 b = Qt[((long)lc * 3 + c) * Vh + si];
            pr[q] = ok ? a.x : 0.0f;
            pi[q] = ok ? a.y : 0.0f;
            qr[q] = ok ? b.x : 0.0f;
            qi[q] = ok ? b.y : 0.0f;
        }
#pragma unroll 1
        for (int jt = 0; jt < NT; ++jt) {
            if (jt * 16 >= N) break;
            const int jo = jt * 16 + r16;  // coefficient column of this lane (A-operand row)
            dvec4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
            fvec4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};  // Qt S^{-1}
            fvec4 br = {0, 0, 0, 0}, bi = {0, 0, 0, 0};  // P S^H
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int l = 4 * q + k4;
                const double2 m1 = cf64[l * NP + jo];
                const bool uq = full && q <= 4 * jt + 3;
                const bool up = full && q >= 4 * jt;
                const double dpr = (double)pr[q], dpi = (double)pi[q];
                xr = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.x, dpr, xr, 0, 0, 0);
                xi = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.x, dpi, xi, 0, 0, 0);
                if (uq) {
                    const float2 m2 = cf32[l * NP + jo];
                    ar = __builtin_amdgcn_mfma_f32_16x16x4f32(m2.x, qr[q], ar, 0, 0, 0);
                    ai = __builtin_amdgcn_mfma_f32_16x16x4f32(m2.x, qi[q], ai, 0, 0, 0);
                    ar = __builtin_amdgcn_mfma_f32_16x16x4f32(-m2.y, qi[q], ar, 0, 0, 0);
                    ai = __builtin_amdgcn_mfma_f32_16x16x4f32(m2.y, qr[q], ai, 0, 0, 0);
                }
                if (up) {
                    const float2 m3 = cf32[NP * NP + l * NP + jo];
                    br = __builtin_amdgcn_mfma_f32_16x16x4f32(m3.x, pr[q], br, 0, 0, 0);
                    bi = __builtin_amdgcn_mfma_f32_16x16x4f32(m3.x, pi[q], bi, 0, 0, 0);
                    br = __builtin_amdgcn_mfma_f32_16x16x4f32(-m3.y, pi[q], br, 0, 0, 0);
                    bi = __builtin_amdgcn_mfma_f32_16x16x4f32(m3.y, pr[q], bi, 0, 0, 0);
                }
                xr = __builtin_amdgcn_mfma_f64_16x16x4f64(-m1.y, dpi, xr, 0, 0, 0);
                xi = __builtin_amdgcn_mfma_f64_16x16x4f64(m1.y, dpr, xi, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                // FP64 accumulator m of lane l: output column 4m + l/16 of the tile
                const int j = jt * 16 + 4 * m + k4;
                if (live && j < N) {
                    const long o = ((long)j * 3 + c) * Vh + site;
                    double2 xv = X[o];
                    xv.x += xr[m];
                    xv.y += xi[m];
                    X[o] = xv;
                }
            }
            if (full) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int j = jt * 16 + F32_ACC_ROW(m, lane);
                    if (live && j < N) {
                        const long o = ((long)j * 3 + c) * Vh + site;
                        const float2 qv = make_float2(ar[m], ai[m]);
                        Qn[o] = qv;
                        Pn[o] = make_float2(qv.x + br[m], qv.y + bi[m]);   // P = Q + P S^H
                    }
                }
            }
        }
    }
}
#undef F32_ACC_ROW

// eight waves share the one workgroup per CU that the 128 KB of LDS allows (two per
// SIMD, 254 VGPRs each): 1.49x faster than four waves at N = 64 on 32^3 x 64
constexpr int PASS_B32_NW = 8;
constexpr size_t PASS_B32_LDS = (size_t)64 * 64 * sizeof(double2) + (size_t)2 * 64 * 64 * sizeof(float2);

static bool pass_b_mfma32_ok(Prec prec, int N, bool fused) {
    return !fused && N > 32 && N <= 64 && prec == Prec::FP32;
}

static void pass_b_mfma32_go(double2* X, const void* Qt, const void* P, void* Qn, void* Pn, const double2* betaC,
                             const double2* Sinv, const double2* SH, int N, int Vh, const SolveState* st,
                             hipStream_t s) {
    constexpr int NW = PASS_B32_NW;
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long groups = (nrb + NW - 1) / NW;
    const dim3 grid((unsigned)(groups < 256 ? groups : 256));
    hipLaunchKernelGGL(k_pass_b_mfma32<PASS_B32_NW>, grid, dim3(64 * NW), PASS_B32_LDS, s, X, (const float2*)Qt,
                       (const float2*)P, (float2*)Qn, (float2*)Pn, betaC, Sinv, SH, N, Vh, st);
}

hipError_t blas_setup() {
    return hipFuncSetAttribute((const void*)k_pass_b_mfma32<PASS_B32_NW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)PASS_B32_LDS);
}

// matrix-core pass B applies (FP32 / FP64 storage, no fused Gram, 16 < N <= 32:
// all three coefficient matrices fit in LDS; measured 1.4x faster than the vector
// kernel at N = 32 on 32^3 x 64, while at N = 64 the per-tile staging makes it slower)
// (the 16-bit formats stay on the vector kernel: a group's scale spans three
// colours, and a three-wave matrix-core variant measured no faster at N = 32)
static bool pass_b_mfma_ok(Prec prec, int N, bool fused) {
    return !fused && N > 16 && N <= 32 && (prec == Prec::FP64 || prec == Prec::FP32);
}

template <typename S>
static void pass_b_mfma_t(double2* X, const void* Qt, const void* P, void* Qn, void* Pn, const double2* betaC,
                          const double2* Sinv, const double2* SH, int N, int Vh, const SolveState* st,
                          hipStream_t s) {
    using PP = typename S::pair;
    const long nrb = (long)((Vh + 15) / 16) * 3;
    const long groups = (nrb + 3) / 4;
    // persistent over groups of four row blocks: the staged coefficients are reused
    const dim3 grid((unsigned)(groups < 2048 ? groups : 2048));
#define PBM(T)                                                                                          \
    hipLaunchKernelGGL((k_pass_b_mfma<S, T>), grid, dim3(256),                                          \
                       (size_t)3 * (16 * T) * (16 * T) * sizeof(double2), s, X,                        \
                       (const PP*)Qt, (const PP*)P, (PP*)Qn, (PP*)Pn, betaC, Sinv, SH, N, Vh, st)
    PBM(2);
#undef PBM
}

hipError_t launch_pass_b(Prec prec, double2* X, const void* Qt, const void* P, void* Qn, void* Pn,
                         const double2* betaC, const double2* Sinv, const double2* SH, int N,
                         int Vh, const SolveState* state, double2* partials, int cpt, int bps, int kernel,
                         hipStream_t s) {
    if (partials != nullptr && fused_tile_bytes(prec, N) == 0) return hipErrorInvalidValue;
    const bool staged = kernel != 3;
    if ((kernel == 0 || kernel == 1) && pass_b_mfma_ok(prec, N, partials != nullptr)) {
        if (prec == Prec::FP64) pass_b_mfma_t<F64>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, s);
        else pass_b_mfma_t<F32>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, s);
        return hipGetLastError();
    }
    if ((kernel == 0 || kernel == 1) && pass_b_mfma32_ok(prec, N, partials != nullptr)) {
        pass_b_mfma32_go(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, s);
        return hipGetLastError();
    }

    switch (prec) {
        case Prec::FP64: pass_b_t<F64>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, partials, cpt, bps, staged, s); break;
        case Prec::FP32: pass_b_t<F32>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, partials, cpt, bps, staged, s); break;
        case Prec::FP16: pass_b_t<H16>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, partials, cpt, bps, staged, s); break;
        case Prec::BF16: pass_b_t<B16>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, partials, cpt, bps, staged, s); break;
        case Prec::FX16: pass_b_t<X16>(X, Qt, P, Qn, Pn, betaC, Sinv, SH, N, Vh, state, partials, cpt, bps, staged, s); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Y <- Z + X M   (block caxpy, Eq. 3), all buffers distinct; Z may be NULL.
// ---------------------------------------------------------------------------------------------
template <typename SX, typename SY, int CPT>
__global__ void __launch_bounds__(256)
k_bmul(const typename SX::pair* __restrict__ X, const float* __restrict__ Xs,
       const typename SY::pair* __restrict__ Z, const float* __restrict__ Zs,
       typename SY::pair* __restrict__ Y, float* __restrict__ Ys, const double2* __restrict__ M, int N,
       int Nout, int Vh, const int* __restrict__ skip) {
    if (skip != nullptr && *skip) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar coefficient loads
    const int i = blockIdx.x * 64 + lane;
    if (i >= Vh) return;
    for (int j0 = wave * CPT; j0 < Nout; j0 += 4 * CPT) {
        C2<double> acc[CPT][3];
#pragma unroll
        for (int m = 0; m < CPT; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[m][c] = C2<double>{0.0, 0.0};
#pragma unroll 4
        for (int l = 0; l < N; ++l) {
            C2<typename SX::real> a[3];
            load_group<SX, 3>(X, Xs, Vh, l, i, a);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < Nout) {
                    const C2<double> b = dld(M + l * MAXN + j0 + m);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        cmac(acc[m][c], C2<double>{(double)a[c].re, (double)a[c].im}, b);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (j0 + m < Nout) {
                if (Z != nullptr) {
                    C2<typename SY::real> z[3];
                    load_group<SY, 3>(Z, Zs, Vh, j0 + m, i, z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        acc[m][c].re += (double)z[c].re;
                        acc[m][c].im += (double)z[c].im;
                    }
                }
                store_group<SY, 3, double>(Y, Ys, Vh, j0 + m, i, acc[m]);
            }
        }
    }
}

// Each wave re-reads the N input columns of its sites once per group of CPT output
// columns, so 32 or more outputs take groups of 8 (every wave one group at 32):
// half the re-reads of groups of 4, with the same summation order per output.
template <typename SX, typename SY>
static void bmul_t(const void* X, const void* Z, void* Y, const double2* M, int N, int Nout, int Vh,
                   const int* skip, hipStream_t s) {
    dim3 grid((Vh + 63) / 64);
#define BMUL_GO(CPTV)                                                                                           \
    hipLaunchKernelGGL((k_bmul<SX, SY, CPTV>), grid, dim3(256), 0, s, (const typename SX::pair*)X,           \
                       scale_of<SX>(X, N, 3, Vh), (const typename SY::pair*)Z, scale_of<SY>(Z, Nout, 3, Vh), \
                       (typename SY::pair*)Y, scale_of<SY>(Y, Nout, 3, Vh), M, N, Nout, Vh, skip)
    if (Nout >= 32) BMUL_GO(8);
    else BMUL_GO(4);
#undef BMUL_GO
}

template <typename SX>
static hipError_t bmul_y(Prec py, const void* X, const void* Z, void* Y, const double2* M, int N, int Vh,
                         const int* skip, hipStream_t s) {
    switch (py) {
        case Prec::FP64: bmul_t<SX, F64>(X, Z, Y, M, N, N, Vh, skip, s); break;
        case Prec::FP32: bmul_t<SX, F32>(X, Z, Y, M, N, N, Vh, skip, s); break;
        case Prec::FP16: bmul_t<SX, H16>(X, Z, Y, M, N, N, Vh, skip, s); break;
        case Prec::BF16: bmul_t<SX, B16>(X, Z, Y, M, N, N, Vh, skip, s); break;
        case Prec::FX16: bmul_t<SX, X16>(X, Z, Y, M, N, N, Vh, skip, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_bmul_rect(Prec px, const void* X, const double2* Z, double2* Y, const double2* M, int Nin,
                            int Nout, int Vh, const int* skip, hipStream_t s) {
    switch (px) {
        case Prec::FP64: bmul_t<F64, F64>(X, Z, Y, M, Nin, Nout, Vh, skip, s); break;
        case Prec::FP32: bmul_t<F32, F64>(X, Z, Y, M, Nin, Nout, Vh, skip, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bmul(Prec px, const void* X, Prec py, const void* Z, void* Y, const double2* M,
                       int N, int Vh, const int* skip, hipStream_t s) {
    switch (px) {
        case Prec::FP64: return bmul_y<F64>(py, X, Z, Y, M, N, Vh, skip, s);
        case Prec::FP32: return bmul_y<F32>(py, X, Z, Y, M, N, Vh, skip, s);
        case Prec::FP16: return bmul_y<H16>(py, X, Z, Y, M, N, Vh, skip, s);
        case Prec::BF16: return bmul_y<B16>(py, X, Z, Y, M, N, Vh, skip, s);
        case Prec::FX16: return bmul_y<X16>(py, X, Z, Y, M, N, Vh, skip, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// Layout conversion and small vector kernels
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_canon_to_int(const double2* __restrict__ src, double2* __restrict__ dst, int N, long Vh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * Vh) return;
    const long n = t / Vh, i = t - n * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[(n * 3 + c) * Vh + i] = src[t * 3 + c];
}

__global__ void __launch_bounds__(256)
k_int_to_canon(const double2* __restrict__ src, double2* __restrict__ dst, int N, long Vh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * Vh) return;
    const long n = t / Vh, i = t - n * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[t * 3 + c] = src[(n * 3 + c) * Vh + i];
}

hipError_t launch_canon_to_int(const double2* src, double2* dst, int N, int Vh, hipStream_t s) {
    const long n = (long)N * Vh;
    hipLaunchKernelGGL(k_canon_to_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, N, (long)Vh);
    return hipGetLastError();
}

hipError_t launch_int_to_canon(const double2* src, double2* dst, int N, int Vh, hipStream_t s) {
    const long n = (long)N * Vh;
    hipLaunchKernelGGL(k_int_to_canon, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, N, (long)Vh);
    return hipGetLastError();
}

static unsigned stream_grid(long n) {
    long g = (n + 255) / 256;
    return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

__global__ void __launch_bounds__(256) k_fold_x(double2* __restrict__ Y, double2* __restrict__ X, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const double2 x = X[t];
        double2 y = Y[t];
        y.x += x.x;
        y.y += x.y;
        Y[t] = y;
        X[t] = make_double2(0.0, 0.0);
    }
}
hipError_t launch_fold_x(double2* Y, double2* X, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_x, dim3(stream_grid(n)), dim3(256), 0, s, Y, X, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_residual(const double2* __restrict__ B, double2* __restrict__ R, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const double2 b = B[t];
        const double2 a = R[t];
        R[t] = make_double2(b.x - a.x, b.y - a.y);
    }
}
hipError_t launch_residual(const double2* B, double2* R, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(stream_grid(n)), dim3(256), 0, s, B, R, n);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_zero(uint4* __restrict__ p, long n16) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n16; t += (long)gridDim.x * blockDim.x)
        p[t] = make_uint4(0, 0, 0, 0);
}
hipError_t launch_zero(void* p, long bytes, hipStream_t s) {
    if (bytes % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero, dim3(stream_grid(bytes / 16)), dim3(256), 0, s, (uint4*)p, bytes / 16);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ a, uint4* __restrict__ b, long n16) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n16; t += (long)gridDim.x * blockDim.x)
        b[t] = a[t];
}
hipError_t launch_copy(const void* src, void* dst, long bytes, hipStream_t s) {
    if (bytes % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3(stream_grid(bytes / 16)), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, bytes / 16);
    return hipGetLastError();
}

// One step of the Chebyshev basis of the s-step solver:
// Vn = a (AV - c V) - Vm  (Vm may be NULL = 0), n complex entries of FP64 or FP32
// storage, formed in FP64 and rounded once on the store
template <typename P>
__global__ void __launch_bounds__(256) k_cheb_step(P* __restrict__ Vn, const P* __restrict__ AV,
                                                   const P* __restrict__ V, const P* __restrict__ Vm,
                                                   double a, double c, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const P av = AV[t], v = V[t];
        double rx = a * ((double)av.x - c * (double)v.x), ry = a * ((double)av.y - c * (double)v.y);
        if (Vm != nullptr) {
            const P m = Vm[t];
            rx -= (double)m.x;
            ry -= (double)m.y;
        }
        P r;
        r.x = rx;
        r.y = ry;
        Vn[t] = r;
    }
}
hipError_t launch_cheb_step(Prec p, void* Vn, const void* AV, const void* V, const void* Vm, double a, double c,
                            long n, hipStream_t s) {
    if (p == Prec::FP64)
        hipLaunchKernelGGL(k_cheb_step<double2>, dim3(stream_grid(n)), dim3(256), 0, s, (double2*)Vn,
                           (const double2*)AV, (const double2*)V, (const double2*)Vm, a, c, n);
    else if (p == Prec::FP32)
        hipLaunchKernelGGL(k_cheb_step<float2>, dim3(stream_grid(n)), dim3(256), 0, s, (float2*)Vn,
                           (const float2*)AV, (const float2*)V, (const float2*)Vm, a, c, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// v = w / *nrm (FP64 pairs, n entries; *nrm > 0 read on the device)
__global__ void __launch_bounds__(256) k_scale_inv(double2* __restrict__ v, const double2* __restrict__ w,
                                                   const double* __restrict__ nrm, long n) {
    const double r = 1.0 / *nrm;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const double2 x = w[t];
        v[t] = make_double2(x.x * r, x.y * r);
    }
}
hipError_t launch_scale_inv(double2* v, const double2* w, const double* nrm, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv, dim3(stream_grid(n)), dim3(256), 0, s, v, w, nrm, n);
    return hipGetLastError();
}

// per-column sum of |V|^2 over each workgroup's sites: partials[b*N + j]
__global__ void __launch_bounds__(256)
k_colnorm2(const double2* __restrict__ V, int N, int Vh, double* __restrict__ partials) {
    __shared__ double red[4];
    for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < Vh; i += (long)gridDim.x * 256)
            for (int c = 0; c < 3; ++c) {
                const double2 v = V[((long)j * 3 + c) * Vh + i];
                s += v.x * v.x + v.y * v.y;
            }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partials[(long)blockIdx.x * N + j] = red[0] + red[1] + red[2] + red[3];
    }
}
static int norm_blocks(int Vh) {
    const int g = (Vh + 255) / 256;
    return g < NORM_BLOCKS ? g : NORM_BLOCKS;
}
hipError_t launch_colnorm2(const double2* V, int N, int Vh, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_colnorm2, dim3(norm_blocks(Vh)), dim3(256), 0, s, V, N, Vh, partials);
    return hipGetLastError();
}

// out[j] = sum_b partials[b*N + j] (its square root if take_sqrt): one wave per
// column, lanes strided over the partials, then a fixed butterfly (deterministic)
__global__ void __launch_bounds__(1024)
k_colnorm_reduce(const double* __restrict__ partials, int N, int P, double* __restrict__ out, int take_sqrt) {
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int j = wave; j < N; j += nw) {
        double s = 0.0;
        for (int b = lane; b < P; b += 64) s += partials[(long)b * N + j];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) out[j] = take_sqrt ? sqrt(s) : s;
    }
}
hipError_t launch_colnorm_reduce(const double* partials, int N, int Vh, double* out, int take_sqrt,
                                 hipStream_t s) {
    const int waves = N < 16 ? N : 16;
    hipLaunchKernelGGL(k_colnorm_reduce, dim3(1), dim3(64 * waves), 0, s, partials, N, norm_blocks(Vh), out,
                       take_sqrt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// CG baseline (Hestenes-Stiefel), one right-hand side, FP64
// ---------------------------------------------------------------------------------------------
__device__ double block_sum_1024(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// rr = ||r||^2 from the norm partials (r = b, p = b, x = 0 are set by copies
// beforehand).  restart = 0: a new solve, ||b|| = ||r||; restart = 1: r = b - A x
// after a true-residual check, ||b|| and the iteration count are kept.
__global__ void __launch_bounds__(1024)
k_cg_init(const double* __restrict__ partials, int P, CgState* st, double tol, int restart) {
    __shared__ double red[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < P; b += blockDim.x) v += partials[b];
    const double s = block_sum_1024(v, red);
    if (threadIdx.x == 0) {
        st->rr = s;
        if (!restart) {
            st->bnorm = sqrt(s);
            st->iters = 0;
        }
        st->tol = tol;
        st->relres = sqrt(s) / st->bnorm;
        st->rr_prev = s;
        st->ru_delta = 0.0;
        st->rho_ru = st->relres;
        st->halt = (s > 0.0) ? 0 : 1;
        st->reason = (s > 0.0) ? HALT_NONE : HALT_CONVERGED;
    }
}
hipError_t launch_cg_init(const double* partials, int Vh, CgState* st, double tol, int restart,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1024), 0, s, partials, norm_blocks(Vh), st, tol, restart);
    return hipGetLastError();
}

__global__ void __launch_bounds__(1024) k_cg_alpha(const double* __restrict__ dot, int P, CgState* st) {
    if (st->halt) return;
    __shared__ double red[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < P; b += blockDim.x) v += dot[b];
    const double pap = block_sum_1024(v, red);
    if (threadIdx.x == 0) {
        if (!(pap > 0.0)) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_G;
        } else {
            st->alpha = st->rr / pap;
        }
    }
}
hipError_t launch_cg_alpha(const double* dot_partials, int nparts, CgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, dot_partials, nparts, st);
    return hipGetLastError();
}

// x += alpha p; r -= alpha Ap; partial ||r||^2
__global__ void __launch_bounds__(256)
k_cg_update1(double2* __restrict__ x, double2* __restrict__ r, const double2* __restrict__ p,
             const double2* __restrict__ Ap, long n, double* __restrict__ partials, const CgState* __restrict__ st) {
    if (st->halt) return;
    const double a = st->alpha;
    double s = 0.0;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
        const double2 pv = p[t], av = Ap[t];
        double2 xv = x[t], rv = r[t];
        xv.x = fma(a, pv.x, xv.x);
        xv.y = fma(a, pv.y, xv.y);
        rv.x = fma(-a, av.x, rv.x);
        rv.y = fma(-a, av.y, rv.y);
        x[t] = xv;
        r[t] = rv;
        s += rv.x * rv.x + rv.y * rv.y;
    }
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
static int cg_parts(long n) {
    const long g = (n + 255) / 256;
    return (int)(g < NORM_BLOCKS ? g : NORM_BLOCKS);
}
hipError_t launch_cg_update1(double2* x, double2* r, const double2* p, const double2* Ap, long n,
                             double* partials, CgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update1, dim3(cg_parts(n)), dim3(256), 0, s, x, r, p, Ap, n, partials, st);
    return hipGetLastError();
}

__global__ void __launch_bounds__(1024) k_cg_beta(const double* __restrict__ partials, int P, CgState* st) {
    if (st->halt) return;
    __shared__ double red[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < P; b += blockDim.x) v += partials[b];
    const double rr = block_sum_1024(v, red);
    if (threadIdx.x == 0) {
        st->iters += 1;
        st->relres = sqrt(rr) / st->bnorm;
        st->beta = rr / st->rr;
        st->rr_prev = st->rr;
        st->rr = rr;
        if (st->relres <= st->tol) {
            st->halt = 1;
            st->reason = HALT_CONVERGED;
        } else if (st->ru_delta > 0.0 && st->relres <= st->ru_delta * st->rho_ru) {
            st->halt = 1;
            st->reason = HALT_RU;
        }
    }
}
hipError_t launch_cg_beta(const double* partials, long n, CgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, s, partials, cg_parts(n), st);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_cg_update2(double2* __restrict__ p, const double2* __restrict__ r, long n, const CgState* __restrict__ st) {
    if (st->halt) return;
    const double b = st->beta;
    for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
        const double2 rv = r[t];
        double2 pv = p[t];
        pv.x = fma(b, pv.x, rv.x);
        pv.y = fma(b, pv.y, rv.y);
        p[t] = pv;
    }
}
hipError_t launch_cg_update2(double2* p, const double2* r, long n, CgState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update2, dim3(stream_grid(n)), dim3(256), 0, s, p, r, n, st);
    return hipGetLastError();
}

// x += alpha p (x FP64); r -= alpha Ap (stored in S); partial ||r||^2 of r as stored.
// One thread per site: the three colour components share a scale in the 16-bit formats.
template <typename S>
__global__ void __launch_bounds__(256)
k_cg_update1_s(double2* __restrict__ x, typename S::pair* __restrict__ r, float* __restrict__ rs,
               const typename S::pair* __restrict__ p, const float* __restrict__ ps,
               const typename S::pair* __restrict__ Ap, const float* __restrict__ Aps, int Vh,
               double* __restrict__ partials, const CgState* __restrict__ st) {
    if (st->halt) return;
    using R = typename S::real;
    const double a = st->alpha;
    double sum = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < Vh; i += gridDim.x * 256) {
        C2<R> pv[3], av[3], rv[3];
        load_group<S, 3>(p, ps, Vh, 0, i, pv);
        load_group<S, 3>(Ap, Aps, Vh, 0, i, av);
        load_group<S, 3>(r, rs, Vh, 0, i, rv);
        C2<double> rn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 xv = x[(long)c * Vh + i];
            xv.x = fma(a, (double)pv[c].re, xv.x);
            xv.y = fma(a, (double)pv[c].im, xv.y);
            x[(long)c * Vh + i] = xv;
            rn[c] = C2<double>{fma(-a, (double)av[c].re, (double)rv[c].re), fma(-a, (double)av[c].im, (double)rv[c].im)};
        }
        store_group_rt<S, 3, double>(r, rs, Vh, 0, i, rn);
#pragma unroll
        for (int c = 0; c < 3; ++c) sum += rn[c].re * rn[c].re + rn[c].im * rn[c].im;
    }
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// p = r + beta p in storage S
template <typename S>
__global__ void __launch_bounds__(256)
k_cg_update2_s(typename S::pair* __restrict__ p, float* __restrict__ ps, const typename S::pair* __restrict__ r,
               const float* __restrict__ rs, int Vh, const CgState* __restrict__ st) {
    if (st->halt) return;
    using R = typename S::real;
    const double b = st->beta;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < Vh; i += gridDim.x * 256) {
        C2<R> pv[3], rv[3];
        load_group<S, 3>(p, ps, Vh, 0, i, pv);
        load_group<S, 3>(r, rs, Vh, 0, i, rv);
        C2<double> pn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            pn[c] = C2<double>{fma(b, (double)pv[c].re, (double)rv[c].re), fma(b, (double)pv[c].im, (double)rv[c].im)};
        store_group<S, 3, double>(p, ps, Vh, 0, i, pn);
    }
}

template <typename S>
static void cg_update1_t(double2* x, void* r, const void* p, const void* Ap, int Vh, double* partials,
                         CgState* st, hipStream_t s) {
    using P = typename S::pair;
    hipLaunchKernelGGL(k_cg_update1_s<S>, dim3(cg_parts(Vh)), dim3(256), 0, s, x, (P*)r, scale_of<S>(r, 1, 3, Vh),
                       (const P*)p, scale_of<S>(p, 1, 3, Vh), (const P*)Ap, scale_of<S>(Ap, 1, 3, Vh), Vh,
                       partials, st);
}
template <typename S>
static void cg_update2_t(void* p, const void* r, int Vh, CgState* st, hipStream_t s) {
    using P = typename S::pair;
    hipLaunchKernelGGL(k_cg_update2_s<S>, dim3(stream_grid(Vh)), dim3(256), 0, s, (P*)p, scale_of<S>(p, 1, 3, Vh),
                       (const P*)r, scale_of<S>(r, 1, 3, Vh), Vh, st);
}
hipError_t launch_cg_update1_s(Prec prec, double2* x, void* r, const void* p, const void* Ap, int Vh,
                               double* partials, CgState* st, hipStream_t s) {
    switch (prec) {
        case Prec::FP64: cg_update1_t<F64>(x, r, p, Ap, Vh, partials, st, s); break;
        case Prec::FP32: cg_update1_t<F32>(x, r, p, Ap, Vh, partials, st, s); break;
        case Prec::FP16: cg_update1_t<H16>(x, r, p, Ap, Vh, partials, st, s); break;
        case Prec::BF16: cg_update1_t<B16>(x, r, p, Ap, Vh, partials, st, s); break;
        case Prec::FX16: cg_update1_t<X16>(x, r, p, Ap, Vh, partials, st, s); break;
    }
    return hipGetLastError();
}
hipError_t launch_cg_update2_s(Prec prec, void* p, const void* r, int Vh, CgState* st, hipStream_t s) {
    switch (prec) {
        case Prec::FP64: cg_update2_t<F64>(p, r, Vh, st, s); break;
        case Prec::FP32: cg_update2_t<F32>(p, r, Vh, st, s); break;
        case Prec::FP16: cg_update2_t<H16>(p, r, Vh, st, s); break;
        case Prec::BF16: cg_update2_t<B16>(p, r, Vh, st, s); break;
        case Prec::FX16: cg_update2_t<X16>(p, r, Vh, st, s); break;
    }
    return hipGetLastError();
}

__global__ void __launch_bounds__(1024)
k_cg_ru(const double* __restrict__ partials, int P, CgState* st, int conv_check) {
    __shared__ double red[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < P; b += blockDim.x) v += partials[b];
    const double rr = block_sum_1024(v, red);
    if (threadIdx.x == 0) {
        st->relres = sqrt(rr) / st->bnorm;
        st->rho_ru = st->relres;
        st->beta = rr / st->rr_prev;
        st->rr = rr;
        if (conv_check && st->relres <= st->tol) {
            st->reason = HALT_DONE;
        } else {
            st->halt = 0;
            st->reason = HALT_NONE;
        }
    }
}
hipError_t launch_cg_ru(const double* partials, int Vh, CgState* st, int conv_check, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_ru, dim3(1), dim3(1024), 0, s, partials, norm_blocks(Vh), st, conv_check);
    return hipGetLastError();
}

__global__ void k_cg_set_ru(CgState* st, double ru_delta) {
    if (threadIdx.x == 0) st->ru_delta = ru_delta;
}
hipError_t launch_cg_set_ru(CgState* st, double ru_delta, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_set_ru, dim3(1), dim3(64), 0, s, st, ru_delta);
    return hipGetLastError();
}

}  // namespace bcg
