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
#include "device_common.h"
#include "internal.h"

namespace bcg {

template <typename T> using PairT = typename Store<T>::pair;

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

template <typename T, int NB>
__global__ void __launch_bounds__(256)
k_gram(const PairT<T>* __restrict__ A, const PairT<T>* __restrict__ B, int N, int Vh,
       double2* __restrict__ partials, const int* __restrict__ halt) {
    if (halt != nullptr && *halt) return;
    constexpr int S = GramCfg<NB>::S, RB = GramCfg<NB>::RB;
    constexpr int R = 3 * S, LD = NB + 1;
    constexpr int NBB = NB / RB, NBLK = NBB * NBB, G = 256 / NBLK;
    __shared__ C2<double> As[R * LD];
    __shared__ C2<double> Bs[R * LD];
    const bool same = (A == B);
    const int t = threadIdx.x;
    const int blk = t % NBLK, grp = t / NBLK;
    const int bi = blk / NBB, bj = blk % NBB;
    C2<double> acc[RB][RB];
#pragma unroll
    for (int m = 0; m < RB; ++m)
#pragma unroll
        for (int n = 0; n < RB; ++n) acc[m][n] = C2<double>{0.0, 0.0};
    for (int e = t; e < R * LD; e += 256) {
        As[e] = C2<double>{0.0, 0.0};
        Bs[e] = C2<double>{0.0, 0.0};
    }
    const int ntiles = (Vh + S - 1) / S;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();
        const int site0 = tile * S;
        for (int e = t; e < R * N; e += 256) {
            const int s = e % S;
            const int rest = e / S;
            const int c = rest % 3;
            const int j = rest / 3;
            const int site = site0 + s;
            C2<double> a{0.0, 0.0}, b{0.0, 0.0};
            if (site < Vh) {
                const long o = ((long)j * 3 + c) * Vh + site;
                a = ldd(A + o);
                if (!same) b = ldd(B + o);
            }
            As[(c * S + s) * LD + j] = a;
            if (!same) Bs[(c * S + s) * LD + j] = b;
        }
        __syncthreads();
        const C2<double>* Bp = same ? As : Bs;
        for (int r = grp; r < R; r += G) {
            C2<double> a[RB], b[RB];
#pragma unroll
            for (int m = 0; m < RB; ++m) {
                a[m] = As[r * LD + bi * RB + m];
                b[m] = Bp[r * LD + bj * RB + m];
            }
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int n = 0; n < RB; ++n) cmac_conj(acc[m][n], a[m], b[n]);
        }
    }
    double2* out = partials + (long)blockIdx.x * NB * NB;
    if (G == 1) {
#pragma unroll
        for (int m = 0; m < RB; ++m)
#pragma unroll
            for (int n = 0; n < RB; ++n)
                out[(bi * RB + m) * NB + bj * RB + n] = make_double2(acc[m][n].re, acc[m][n].im);
        return;
    }
    // lanes of one wave that share a register block: reduce them with shuffles
    if (NBLK < 64) {
#pragma unroll
        for (int off = NBLK; off < 64; off <<= 1)
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int n = 0; n < RB; ++n) {
                    acc[m][n].re += __shfl_xor(acc[m][n].re, off, 64);
                    acc[m][n].im += __shfl_xor(acc[m][n].im, off, 64);
                }
    }
    // then the four waves, in order, through LDS
    __syncthreads();
    C2<double>* red = As;
    const int wave = t >> 6, lane = t & 63;
    const bool holder = (NBLK >= 64) || (lane < NBLK);
    for (int w = 0; w < 4; ++w) {
        if (wave == w && holder) {
#pragma unroll
            for (int m = 0; m < RB; ++m)
#pragma unroll
                for (int n = 0; n < RB; ++n) {
                    const int idx = (bi * RB + m) * NB + bj * RB + n;
                    if (w == 0) red[idx] = acc[m][n];
                    else {
                        red[idx].re += acc[m][n].re;
                        red[idx].im += acc[m][n].im;
                    }
                }
        }
        __syncthreads();
    }
    for (int e = t; e < NB * NB; e += 256) out[e] = make_double2(red[e].re, red[e].im);
}

template <typename T>
static void gram_t(const void* A, const void* B, int N, int Vh, double2* partials, const int* halt,
                   hipStream_t s, int nb) {
    auto go = [&](auto kern, int S) {
        const int ntiles = (Vh + S - 1) / S;
        const int grid = ntiles < GRAM_BLOCKS ? ntiles : GRAM_BLOCKS;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, (const PairT<T>*)A, (const PairT<T>*)B,
                           N, Vh, partials, halt);
    };
    switch (nb) {
        case 1: go(k_gram<T, 1>, GramCfg<1>::S); break;
        case 2: go(k_gram<T, 2>, GramCfg<2>::S); break;
        case 4: go(k_gram<T, 4>, GramCfg<4>::S); break;
        case 8: go(k_gram<T, 8>, GramCfg<8>::S); break;
        case 16: go(k_gram<T, 16>, GramCfg<16>::S); break;
        case 32: go(k_gram<T, 32>, GramCfg<32>::S); break;
        default: go(k_gram<T, 64>, GramCfg<64>::S); break;
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

static int gram_nparts(int Vh, int nb) {
    const int S = gram_sites(nb);
    const int ntiles = (Vh + S - 1) / S;
    return ntiles < GRAM_BLOCKS ? ntiles : GRAM_BLOCKS;
}

hipError_t launch_gram(Prec prec, const void* A, const void* B, int N, int Vh, double2* partials,
                       const int* halt, hipStream_t s) {
    const int nb = pad_n(N);
    if (prec == Prec::FP64) gram_t<double>(A, B, N, Vh, partials, halt, s, nb);
    else if (prec == Prec::FP32) gram_t<float>(A, B, N, Vh, partials, halt, s, nb);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// out[i*64 + j] = sum_b partials[b][i*NB + j], b = 0, 1, ... in order
__global__ void __launch_bounds__(1024)
k_gram_reduce(const double2* __restrict__ partials, int NB, int N, int P, double2* __restrict__ out,
              const int* __restrict__ halt) {
    if (halt != nullptr && *halt) return;
    __shared__ double2 red[16][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int NN = NB * NB;
    double sr = 0.0, si = 0.0;
    if (e < NN)
        for (int p = grp; p < P; p += 16) {
            const double2 v = partials[(long)p * NN + e];
            sr += v.x;
            si += v.y;
        }
    red[grp][lane] = make_double2(sr, si);
    __syncthreads();
    if (grp == 0 && e < NN) {
        double tr = 0.0, ti = 0.0;
        for (int g = 0; g < 16; ++g) {
            tr += red[g][lane].x;
            ti += red[g][lane].y;
        }
        const int i = e / NB, j = e % NB;
        if (i < N && j < N) out[i * MAXN + j] = make_double2(tr, ti);
    }
}

hipError_t launch_gram_reduce(const double2* partials, int N, int Vh, double2* out,
                              const int* halt, hipStream_t s) {
    const int nb = pad_n(N);
    const int grid = (nb * nb + 63) / 64;
    hipLaunchKernelGGL(k_gram_reduce, dim3(grid), dim3(1024), 0, s, partials, nb, N,
                       gram_nparts(Vh, nb), out, halt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Pass A:  Q <- Q - AP beta   (Alg. 1: Q S = Q - A P beta, before its QR)
// ---------------------------------------------------------------------------------------------
template <typename T, int CPT>
__global__ void __launch_bounds__(256)
k_pass_a(PairT<T>* __restrict__ Q, const PairT<T>* __restrict__ AP, const double2* __restrict__ beta,
         int N, int Vh, const int* __restrict__ halt) {
    using R = typename Store<T>::real;
    if (halt != nullptr && *halt) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    if (i >= Vh) return;
    for (int j0 = wave * CPT; j0 < N; j0 += 4 * CPT) {
        C2<R> acc[CPT][3];
#pragma unroll
        for (int m = 0; m < CPT; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[m][c] = C2<R>{0, 0};
        for (int l = 0; l < N; ++l) {
            C2<R> a[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] = ld(AP + ((long)l * 3 + c) * Vh + i);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N) {
                    const double2 bd = beta[l * MAXN + j0 + m];
                    const C2<R> b{(R)bd.x, (R)bd.y};
#pragma unroll
                    for (int c = 0; c < 3; ++c) cmac(acc[m][c], a[c], b);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (j0 + m < N) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    PairT<T>* q = Q + ((long)(j0 + m) * 3 + c) * Vh + i;
                    C2<R> v = ld(q);
                    v.re -= acc[m][c].re;
                    v.im -= acc[m][c].im;
                    st(q, v);
                }
            }
        }
    }
}

hipError_t launch_pass_a(Prec prec, void* Q, const void* AP, const double2* beta, int N, int Vh,
                         const int* halt, hipStream_t s) {
    dim3 grid((Vh + 63) / 64);
    if (prec == Prec::FP64) {
        if (N == 1) hipLaunchKernelGGL((k_pass_a<double, 1>), grid, dim3(256), 0, s, (double2*)Q, (const double2*)AP, beta, N, Vh, halt);
        else if (N == 2) hipLaunchKernelGGL((k_pass_a<double, 2>), grid, dim3(256), 0, s, (double2*)Q, (const double2*)AP, beta, N, Vh, halt);
        else hipLaunchKernelGGL((k_pass_a<double, 4>), grid, dim3(256), 0, s, (double2*)Q, (const double2*)AP, beta, N, Vh, halt);
    } else if (prec == Prec::FP32) {
        if (N == 1) hipLaunchKernelGGL((k_pass_a<float, 1>), grid, dim3(256), 0, s, (float2*)Q, (const float2*)AP, beta, N, Vh, halt);
        else if (N == 2) hipLaunchKernelGGL((k_pass_a<float, 2>), grid, dim3(256), 0, s, (float2*)Q, (const float2*)AP, beta, N, Vh, halt);
        else hipLaunchKernelGGL((k_pass_a<float, 4>), grid, dim3(256), 0, s, (float2*)Q, (const float2*)AP, beta, N, Vh, halt);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Pass B (Alg. 1, with the X update of the same iteration deferred to here, Sec. 6.2):
//   X  += P (beta C)                      (old P)
//   Qn  = Qt S^{-1}                       (S^{-1} upper triangular: l <= j only)
//   Pn  = Qn + P S^H                      (S^H lower triangular: l >= j only)
// Qn, Pn are written to other buffers than Qt, P (ping-pong), so there is no
// in-place hazard between the waves that read all columns and those that write.
// ---------------------------------------------------------------------------------------------
template <typename T, int CPT>
__global__ void __launch_bounds__(256)
k_pass_b(double2* __restrict__ X, const PairT<T>* __restrict__ Qt, const PairT<T>* __restrict__ P,
         PairT<T>* __restrict__ Qn, PairT<T>* __restrict__ Pn, const double2* __restrict__ betaC,
         const double2* __restrict__ Sinv, const double2* __restrict__ SH, int N, int Vh,
         const SolveState* __restrict__ stt) {
    using R = typename Store<T>::real;
    const int mode = stt->pb_mode;
    if (mode == PB_SKIP) return;
    const bool full = (mode == PB_FULL);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    if (i >= Vh) return;
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
        for (int l = 0; l < N; ++l) {
            C2<R> p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) p[c] = ld(P + ((long)l * 3 + c) * Vh + i);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N) {
                    const double2 bc = betaC[l * MAXN + j0 + m];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        cmac(xa[m][c], C2<double>{(double)p[c].re, (double)p[c].im}, C2<double>{bc.x, bc.y});
                }
            }
            if (full) {
                if (l >= j0) {
#pragma unroll
                    for (int m = 0; m < CPT; ++m) {
                        if (j0 + m < N && l >= j0 + m) {
                            const double2 sh = SH[l * MAXN + j0 + m];
                            const C2<R> b{(R)sh.x, (R)sh.y};
#pragma unroll
                            for (int c = 0; c < 3; ++c) cmac(pa[m][c], p[c], b);
                        }
                    }
                }
                if (l < j0 + CPT) {
                    C2<R> q[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[c] = ld(Qt + ((long)l * 3 + c) * Vh + i);
#pragma unroll
                    for (int m = 0; m < CPT; ++m) {
                        if (j0 + m < N && l <= j0 + m) {
                            const double2 si = Sinv[l * MAXN + j0 + m];
                            const C2<R> b{(R)si.x, (R)si.y};
#pragma unroll
                            for (int c = 0; c < 3; ++c) cmac(qa[m][c], q[c], b);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (j0 + m < N) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const long o = ((long)(j0 + m) * 3 + c) * Vh + i;
                    double2 xv = X[o];
                    xv.x += xa[m][c].re;
                    xv.y += xa[m][c].im;
                    X[o] = xv;
                    if (full) {
                        st(Qn + o, qa[m][c]);
                        C2<R> pv{qa[m][c].re + pa[m][c].re, qa[m][c].im + pa[m][c].im};
                        st(Pn + o, pv);
                    }
                }
            }
        }
    }
}

hipError_t launch_pass_b(Prec prec, double2* X, const void* Qt, const void* P, void* Qn, void* Pn,
                         const double2* betaC, const double2* Sinv, const double2* SH, int N,
                         int Vh, const SolveState* state, hipStream_t s) {
    dim3 grid((Vh + 63) / 64);
#define PB_LAUNCH(TT, CC)                                                                             \
    hipLaunchKernelGGL((k_pass_b<TT, CC>), grid, dim3(256), 0, s, X, (const PairT<TT>*)Qt,           \
                       (const PairT<TT>*)P, (PairT<TT>*)Qn, (PairT<TT>*)Pn, betaC, Sinv, SH, N, Vh, \
                       state)
    if (prec == Prec::FP64) {
        if (N == 1) PB_LAUNCH(double, 1);
        else if (N == 2) PB_LAUNCH(double, 2);
        else PB_LAUNCH(double, 4);
    } else if (prec == Prec::FP32) {
        if (N == 1) PB_LAUNCH(float, 1);
        else if (N == 2) PB_LAUNCH(float, 2);
        else PB_LAUNCH(float, 4);
    } else {
        return hipErrorInvalidValue;
    }
#undef PB_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Y <- Z + X M   (block caxpy, Eq. 3), all buffers distinct; Z may be NULL.
// ---------------------------------------------------------------------------------------------
template <typename TX, typename TY, int CPT>
__global__ void __launch_bounds__(256)
k_bmul(const PairT<TX>* __restrict__ X, const PairT<TY>* __restrict__ Z, PairT<TY>* __restrict__ Y,
       const double2* __restrict__ M, int N, int Vh, const int* __restrict__ skip) {
    if (skip != nullptr && *skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    if (i >= Vh) return;
    for (int j0 = wave * CPT; j0 < N; j0 += 4 * CPT) {
        C2<double> acc[CPT][3];
#pragma unroll
        for (int m = 0; m < CPT; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[m][c] = C2<double>{0.0, 0.0};
        for (int l = 0; l < N; ++l) {
            C2<double> a[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] = ldd(X + ((long)l * 3 + c) * Vh + i);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (j0 + m < N) {
                    const C2<double> b = dld(M + l * MAXN + j0 + m);
#pragma unroll
                    for (int c = 0; c < 3; ++c) cmac(acc[m][c], a[c], b);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            if (j0 + m < N) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const long o = ((long)(j0 + m) * 3 + c) * Vh + i;
                    C2<double> v = acc[m][c];
                    if (Z != nullptr) {
                        const C2<double> z = ldd(Z + o);
                        v.re += z.re;
                        v.im += z.im;
                    }
                    st(Y + o, v);
                }
            }
        }
    }
}

hipError_t launch_bmul(Prec px, const void* X, Prec py, const void* Z, void* Y, const double2* M,
                       int N, int Vh, const int* skip, hipStream_t s) {
    dim3 grid((Vh + 63) / 64);
#define BM_LAUNCH(TX, TY)                                                                          \
    hipLaunchKernelGGL((k_bmul<TX, TY, 4>), grid, dim3(256), 0, s, (const PairT<TX>*)X,           \
                       (const PairT<TY>*)Z, (PairT<TY>*)Y, M, N, Vh, skip)
    if (px == Prec::FP64 && py == Prec::FP64) BM_LAUNCH(double, double);
    else if (px == Prec::FP64 && py == Prec::FP32) BM_LAUNCH(double, float);
    else if (px == Prec::FP32 && py == Prec::FP32) BM_LAUNCH(float, float);
    else if (px == Prec::FP32 && py == Prec::FP64) BM_LAUNCH(float, double);
    else return hipErrorInvalidValue;
#undef BM_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Layout conversion and small vector kernels
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_canon_to_int(const double2* __restrict__ src, PairT<T>* __restrict__ dst, int N, long Vh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * Vh) return;
    const long n = t / Vh, i = t - n * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double2 v = src[t * 3 + c];
        PairT<T> w;
        w.x = (T)v.x;
        w.y = (T)v.y;
        dst[(n * 3 + c) * Vh + i] = w;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_int_to_canon(const PairT<T>* __restrict__ src, double2* __restrict__ dst, int N, long Vh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * Vh) return;
    const long n = t / Vh, i = t - n * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const PairT<T> v = src[(n * 3 + c) * Vh + i];
        dst[t * 3 + c] = make_double2((double)v.x, (double)v.y);
    }
}

hipError_t launch_canon_to_int(const double2* src, Prec pd, void* dst, int N, int Vh, hipStream_t s) {
    const long n = (long)N * Vh;
    dim3 grid((unsigned)((n + 255) / 256));
    if (pd == Prec::FP64) hipLaunchKernelGGL(k_canon_to_int<double>, grid, dim3(256), 0, s, src, (double2*)dst, N, (long)Vh);
    else if (pd == Prec::FP32) hipLaunchKernelGGL(k_canon_to_int<float>, grid, dim3(256), 0, s, src, (float2*)dst, N, (long)Vh);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_int_to_canon(Prec ps, const void* src, double2* dst, int N, int Vh, hipStream_t s) {
    const long n = (long)N * Vh;
    dim3 grid((unsigned)((n + 255) / 256));
    if (ps == Prec::FP64) hipLaunchKernelGGL(k_int_to_canon<double>, grid, dim3(256), 0, s, (const double2*)src, dst, N, (long)Vh);
    else if (ps == Prec::FP32) hipLaunchKernelGGL(k_int_to_canon<float>, grid, dim3(256), 0, s, (const float2*)src, dst, N, (long)Vh);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(256)
k_convert(const PairT<TS>* __restrict__ src, PairT<TD>* __restrict__ dst, long n) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const PairT<TS> v = src[t];
        PairT<TD> w;
        w.x = (TD)v.x;
        w.y = (TD)v.y;
        dst[t] = w;
    }
}

static unsigned stream_grid(long n) {
    long g = (n + 255) / 256;
    return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

hipError_t launch_convert(Prec ps, const void* src, Prec pd, void* dst, long n, hipStream_t s) {
    const dim3 grid(stream_grid(n));
    if (ps == Prec::FP64 && pd == Prec::FP32) hipLaunchKernelGGL((k_convert<double, float>), grid, dim3(256), 0, s, (const double2*)src, (float2*)dst, n);
    else if (ps == Prec::FP32 && pd == Prec::FP64) hipLaunchKernelGGL((k_convert<float, double>), grid, dim3(256), 0, s, (const float2*)src, (double2*)dst, n);
    else if (ps == Prec::FP64 && pd == Prec::FP64) hipLaunchKernelGGL((k_convert<double, double>), grid, dim3(256), 0, s, (const double2*)src, (double2*)dst, n);
    else if (ps == Prec::FP32 && pd == Prec::FP32) hipLaunchKernelGGL((k_convert<float, float>), grid, dim3(256), 0, s, (const float2*)src, (float2*)dst, n);
    else return hipErrorInvalidValue;
    return hipGetLastError();
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

__global__ void k_colnorm_reduce(const double* __restrict__ partials, int N, int P, double* __restrict__ out, int take_sqrt) {
    const int j = threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int b = 0; b < P; ++b) s += partials[(long)b * N + j];
    out[j] = take_sqrt ? sqrt(s) : s;
}
hipError_t launch_colnorm_reduce(const double* partials, int N, int Vh, double* out, int take_sqrt,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_colnorm_reduce, dim3(1), dim3(64), 0, s, partials, N, norm_blocks(Vh), out,
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
        st->rr = rr;
        if (st->relres <= st->tol) {
            st->halt = 1;
            st->reason = HALT_CONVERGED;
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

}  // namespace bcg
