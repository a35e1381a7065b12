// The small dense N x N steps of blockCGrQ (N <= 64), in FP64, each as one
// workgroup on the device so that the solver loop never waits on the host
// (the paper does these on the host with Eigen, Sec. 6).
//
//   small_init : thin QR of the initial residual (Alg. 2): R^H R = C^H C, C^{-1}
//   small1     : beta = (P^H A P)^{-1} and beta C (Alg. 1)
//   small2     : iterated residual norms sqrt((C^H H C)_ii) / ||b_i|| with
//                H = Qt^H Qt (the residual-norm identity of Sec. 6, tested before
//                the factorisation), stopping and reliable-update tests,
//                H = S^H S, S^{-1}, S^H and C <- S C (Alg. 1 and 2)
//   small_ru   : reliable update (Alg. 3): true residual norms, R = C^ ^H C^,
//                S = C^ C_k^{-1} with C_k the C before this iteration's update
//
// Matrices in global memory are [64][64] complex (row i, column j at i*64 + j).
// The working copies live in LDS (two N x N complex matrices, dynamic).
#include "device_common.h"
#include "internal.h"

namespace bcg {

using Z2 = C2<double>;

__device__ __forceinline__ Z2 zmul(Z2 a, Z2 b) { return Z2{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Z2 zconj(Z2 a) { return Z2{a.re, -a.im}; }
__device__ __forceinline__ Z2 gld(const double2* p) {
    const double2 v = *p;
    return Z2{v.x, v.y};
}
__device__ __forceinline__ void gst(double2* p, Z2 v) { *p = make_double2(v.re, v.im); }

// A <- (M + M^H)/2 for the leading N x N block of a global [64][64] matrix
__device__ void load_herm(Z2* A, const double2* M, int N) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        const Z2 a = gld(M + i * MAXN + j), b = gld(M + j * MAXN + i);
        A[e] = Z2{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
    }
    __syncthreads();
}

// In-place lower Cholesky A = L L^H (L with positive real diagonal, strict upper
// triangle zeroed).  A pivot that is not positive or not finite is a breakdown:
// returns false on every thread.
__device__ bool chol_lower(Z2* A, int N, int* flag) {
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (threadIdx.x == 0) {
            const double d = A[k * N + k].re;
            if (!(d > 0.0) || !isfinite(d)) *flag = 1;
            else A[k * N + k] = Z2{sqrt(d), 0.0};
        }
        __syncthreads();
        if (*flag) return false;
        const double piv = A[k * N + k].re;
        for (int i = k + 1 + threadIdx.x; i < N; i += blockDim.x) {
            const Z2 v = A[i * N + k];
            A[i * N + k] = Z2{v.re / piv, v.im / piv};
        }
        __syncthreads();
        const int m = N - k - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) {
                const Z2 lik = A[i * N + k], ljk = A[j * N + k];
                const Z2 p = zmul(lik, zconj(ljk));
                A[i * N + j].re -= p.re;
                A[i * N + j].im -= p.im;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        if (j > i) A[e] = Z2{0.0, 0.0};
    }
    __syncthreads();
    return true;
}

// Relative pivot test: d_k / H_kk below 1e-14 means column k is numerically in
// the span of the columns before it.  diag: the original diagonal (length N).
__device__ bool chol_lower_checked(Z2* A, int N, int* flag, double* diag) {
    for (int k = threadIdx.x; k < N; k += blockDim.x) diag[k] = A[k * N + k].re;
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        if (threadIdx.x == 0) {
            const double d = A[k * N + k].re;
            if (!(d > 1e-14 * diag[k]) || !isfinite(d)) *flag = 1;
            else A[k * N + k] = Z2{sqrt(d), 0.0};
        }
        __syncthreads();
        if (*flag) return false;
        const double piv = A[k * N + k].re;
        for (int i = k + 1 + threadIdx.x; i < N; i += blockDim.x) {
            const Z2 v = A[i * N + k];
            A[i * N + k] = Z2{v.re / piv, v.im / piv};
        }
        __syncthreads();
        const int m = N - k - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) {
                const Z2 p = zmul(A[i * N + k], zconj(A[j * N + k]));
                A[i * N + j].re -= p.re;
                A[i * N + j].im -= p.im;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        if (j > i) A[e] = Z2{0.0, 0.0};
    }
    __syncthreads();
    return true;
}

// Z = L^{-1} for lower-triangular L with real positive diagonal (column-oriented
// elimination on the identity).
__device__ void tri_inv_lower(const Z2* L, Z2* Zm, int N) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        Zm[e] = Z2{i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const double inv = 1.0 / L[k * N + k].re;
        for (int j = threadIdx.x; j <= k; j += blockDim.x) {
            const Z2 v = Zm[k * N + j];
            Zm[k * N + j] = Z2{v.re * inv, v.im * inv};
        }
        __syncthreads();
        const int w = k + 1, m = N - k - 1;
        for (int e = threadIdx.x; e < m * w; e += blockDim.x) {
            const int i = k + 1 + e / w, j = e % w;
            const Z2 p = zmul(L[i * N + k], Zm[k * N + j]);
            Zm[i * N + j].re -= p.re;
            Zm[i * N + j].im -= p.im;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_state_init(SolveState* st, double tol, double ru_delta, const double* bnorm, int N) {
    const int t = threadIdx.x;
    if (t < MAXN) {
        st->bnorm[t] = t < N ? bnorm[t] : 0.0;
        st->relres[t] = 0.0;
    }
    if (t == 0) {
        st->halt = 0;
        st->reason = HALT_NONE;
        st->pb_mode = PB_FULL;
        st->iters = 0;
        st->max_relres = 1.0;
        st->rho_ru = 1.0;
        st->tol = tol;
        st->ru_delta = ru_delta;
    }
}

__global__ void k_identity(double2* M, int N) {
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) {
        const int i = e / MAXN, j = e % MAXN;
        M[e] = make_double2((i == j && i < N) ? 1.0 : 0.0, 0.0);
    }
}

// initial QR: H = R^H R = C^H C
__global__ void __launch_bounds__(1024)
k_small_init(const double2* __restrict__ H, double2* __restrict__ C, double2* __restrict__ Cinv,
             SolveState* st, int N) {
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* Zm = sm + N * N;
    __shared__ int flag;
    __shared__ double diag[MAXN];
    __shared__ double rel[MAXN];
    load_herm(A, H, N);
    if (!chol_lower_checked(A, N, &flag, diag)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            st->pb_mode = PB_SKIP;
        }
        return;
    }
    tri_inv_lower(A, Zm, N);
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) {
        const int i = e / MAXN, j = e % MAXN;
        Z2 c{0.0, 0.0}, ci{0.0, 0.0};
        if (i < N && j < N && j >= i) {
            c = zconj(A[j * N + i]);     // C = L^H
            ci = zconj(Zm[j * N + i]);   // C^{-1} = (L^{-1})^H
        }
        gst(C + e, c);
        gst(Cinv + e, ci);
    }
    // relative residual of column i = ||C[:, i]|| / ||b_i||  (R = Q C)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s = 0.0;
        for (int m = 0; m <= i; ++m) {  // C[m][i] = conj(L[i][m]), nonzero for m <= i
            const Z2 v = A[i * N + m];
            s += v.re * v.re + v.im * v.im;
        }
        rel[i] = sqrt(s) / st->bnorm[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int i = 0; i < N; ++i) {
            st->relres[i] = rel[i];
            mx = fmax(mx, rel[i]);
        }
        st->max_relres = mx;
        st->rho_ru = mx;
        st->halt = 0;
        st->reason = HALT_NONE;
        st->pb_mode = PB_FULL;
    }
}

// beta = G^{-1} = L^{-H} L^{-1},  betaC = beta C
__global__ void __launch_bounds__(1024)
k_small1(const double2* __restrict__ G, const double2* __restrict__ C, double2* __restrict__ beta,
         double2* __restrict__ betaC, SolveState* st, int N) {
    if (st->halt) return;
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* Zm = sm + N * N;
    __shared__ int flag;
    load_herm(A, G, N);
    if (!chol_lower(A, N, &flag)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_G;
        }
        return;
    }
    tri_inv_lower(A, Zm, N);
    // beta[i][j] = sum_m conj(Z[m][i]) Z[m][j], m >= max(i, j)
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        Z2 s{0.0, 0.0};
        for (int m = (i > j ? i : j); m < N; ++m) {
            const Z2 p = zmul(zconj(Zm[m * N + i]), Zm[m * N + j]);
            s.re += p.re;
            s.im += p.im;
        }
        A[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        gst(beta + i * MAXN + j, A[e]);
        Z2 s{0.0, 0.0};
        for (int m = 0; m <= j; ++m) {   // C upper triangular
            const Z2 p = zmul(A[i * N + m], gld(C + m * MAXN + j));
            s.re += p.re;
            s.im += p.im;
        }
        gst(betaC + i * MAXN + j, s);
    }
}

__global__ void __launch_bounds__(1024)
k_small2(const double2* __restrict__ H, double2* __restrict__ C, double2* __restrict__ Sinv,
         double2* __restrict__ SH, SolveState* st, int N) {
    if (st->halt) {
        if (threadIdx.x == 0) st->pb_mode = PB_SKIP;
        return;
    }
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* W = sm + N * N;
    __shared__ int flag;
    __shared__ double rel[MAXN];
    __shared__ int decision;
    load_herm(A, H, N);
    // W = H C
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        Z2 s{0.0, 0.0};
        for (int m = 0; m <= j; ++m) {
            const Z2 p = zmul(A[i * N + m], gld(C + m * MAXN + j));
            s.re += p.re;
            s.im += p.im;
        }
        W[e] = s;
    }
    __syncthreads();
    // ||r_i||^2 = (C^H H C)_ii = sum_m conj(C[m][i]) W[m][i]
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s = 0.0;
        for (int m = 0; m <= i; ++m) {
            const Z2 c = gld(C + m * MAXN + i), w = W[m * N + i];
            s += c.re * w.re + c.im * w.im;
        }
        rel[i] = sqrt(fmax(s, 0.0)) / st->bnorm[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int i = 0; i < N; ++i) {
            st->relres[i] = rel[i];
            mx = fmax(mx, rel[i]);
        }
        st->max_relres = mx;
        st->iters += 1;
        const bool conv = mx <= st->tol;
        const bool ru = st->ru_delta > 0.0 && mx <= st->ru_delta * st->rho_ru;
        decision = conv ? HALT_CONVERGED : (ru ? HALT_RU : HALT_NONE);
        if (decision != HALT_NONE) {
            st->halt = 1;
            st->reason = decision;
            st->pb_mode = PB_X_ONLY;
        }
    }
    __syncthreads();
    if (decision != HALT_NONE) return;
    if (!chol_lower(A, N, &flag)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            st->pb_mode = PB_X_ONLY;
        }
        return;
    }
    tri_inv_lower(A, W, N);
    // S = L^H; S^H = L; S^{-1} = (L^{-1})^H
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) {
        const int i = e / MAXN, j = e % MAXN;
        Z2 sh{0.0, 0.0}, si{0.0, 0.0};
        if (i < N && j < N) {
            if (j <= i) sh = A[i * N + j];
            if (j >= i) si = zconj(W[j * N + i]);
        }
        gst(SH + e, sh);
        gst(Sinv + e, si);
    }
    __syncthreads();
    // C <- S C, S upper: (S C)[i][j] = sum_{m=i..j} conj(L[m][i]) C[m][j]
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        Z2 s{0.0, 0.0};
        for (int m = i; m <= j; ++m) {
            const Z2 p = zmul(zconj(A[m * N + i]), gld(C + m * MAXN + j));
            s.re += p.re;
            s.im += p.im;
        }
        W[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) gst(C + (e / N) * MAXN + e % N, W[e]);
    if (threadIdx.x == 0) st->pb_mode = PB_FULL;
}

// Reliable update from H = R^H R of the true residual R = B - A Y.
__global__ void __launch_bounds__(1024)
k_small_ru(const double2* __restrict__ H, double2* __restrict__ C, double2* __restrict__ Chinv,
           double2* __restrict__ SH, SolveState* st, double* __restrict__ true_relres,
           int* __restrict__ ru_skip, int conv_check, int N) {
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* W = sm + N * N;
    __shared__ int flag;
    __shared__ double diag[MAXN];
    __shared__ double rel[MAXN];
    __shared__ int done;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        rel[i] = sqrt(fmax(H[i * MAXN + i].x, 0.0)) / st->bnorm[i];
        true_relres[i] = rel[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int i = 0; i < N; ++i) mx = fmax(mx, rel[i]);
        done = (conv_check && mx <= st->tol) ? 1 : 0;
        if (done) {
            st->reason = HALT_DONE;
            *ru_skip = 1;
        }
        st->rho_ru = mx;
        st->max_relres = mx;
    }
    __syncthreads();
    if (done) return;
    load_herm(A, H, N);
    if (!chol_lower_checked(A, N, &flag, diag)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            *ru_skip = 1;
        }
        return;
    }
    tri_inv_lower(A, W, N);
    // C^ = L^H -> temporarily in SH; C^{-1} = (L^{-1})^H -> Chinv
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) {
        const int i = e / MAXN, j = e % MAXN;
        Z2 c{0.0, 0.0}, ci{0.0, 0.0};
        if (i < N && j < N && j >= i) {
            c = zconj(A[j * N + i]);
            ci = zconj(W[j * N + i]);
        }
        gst(SH + e, c);
        gst(Chinv + e, ci);
    }
    __syncthreads();
    // A <- C_k^H (lower), W <- (C_k^H)^{-1} = (C_k^{-1})^H
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        A[e] = (j <= i) ? zconj(gld(C + j * MAXN + i)) : Z2{0.0, 0.0};
    }
    __syncthreads();
    tri_inv_lower(A, W, N);
    // S^ = C^ C_k^{-1} (upper), C_k^{-1}[m][j] = conj(W[j][m])
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        Z2 s{0.0, 0.0};
        for (int m = i; m <= j; ++m) {
            const Z2 p = zmul(gld(SH + i * MAXN + m), zconj(W[j * N + m]));
            s.re += p.re;
            s.im += p.im;
        }
        A[e] = s;
    }
    __syncthreads();
    // C <- C^ ; then S^H
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) C[e] = SH[e];
    __syncthreads();
    for (int e = threadIdx.x; e < MAXN * MAXN; e += blockDim.x) {
        const int i = e / MAXN, j = e % MAXN;
        Z2 v{0.0, 0.0};
        if (i < N && j < N) v = zconj(A[j * N + i]);
        gst(SH + e, v);
    }
    if (threadIdx.x == 0) {
        st->halt = 0;
        st->reason = HALT_NONE;
        st->pb_mode = PB_FULL;
        *ru_skip = 0;
    }
}

// ---------------------------------------------------------------------------------------------
static size_t small_lds(int N) { return 2 * (size_t)N * N * sizeof(Z2); }

hipError_t small_setup() {
    const int bytes = (int)small_lds(MAXN);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_small_init, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small1, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small2, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small_ru, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    return hipSuccess;
}

static int small_threads(int N) { return N <= 16 ? 256 : 1024; }

hipError_t launch_state_init(SolveState* st, double tol, double ru_delta, const double* bnorm, int N,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, ru_delta, bnorm, N);
    return hipGetLastError();
}
hipError_t launch_identity(double2* M, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_identity, dim3(1), dim3(1024), 0, s, M, N);
    return hipGetLastError();
}
hipError_t launch_small_init(const double2* H, double2* C, double2* Cinv, SolveState* st, int N,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_small_init, dim3(1), dim3(small_threads(N)), small_lds(N), s, H, C, Cinv, st, N);
    return hipGetLastError();
}
hipError_t launch_small1(const double2* G, const double2* C, double2* beta, double2* betaC,
                         SolveState* st, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_small1, dim3(1), dim3(small_threads(N)), small_lds(N), s, G, C, beta, betaC, st, N);
    return hipGetLastError();
}
hipError_t launch_small2(const double2* H, double2* C, double2* Sinv, double2* SH, SolveState* st,
                         int N, hipStream_t s) {
    hipLaunchKernelGGL(k_small2, dim3(1), dim3(small_threads(N)), small_lds(N), s, H, C, Sinv, SH, st, N);
    return hipGetLastError();
}
hipError_t launch_small_ru(const double2* H, double2* C, double2* Chinv, double2* SH,
                           SolveState* st, double* true_relres, int* ru_skip, int conv_check,
                           int N, hipStream_t s) {
    hipLaunchKernelGGL(k_small_ru, dim3(1), dim3(small_threads(N)), small_lds(N), s, H, C, Chinv, SH,
                       st, true_relres, ru_skip, conv_check, N);
    return hipGetLastError();
}

}  // namespace bcg
