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

// the wide LDS layout (five N x N buffers: the old C in k_small2 and the ping-pong
// partners of the factorisations) for N <= 32
__host__ __device__ constexpr bool small_has_cold(int N) { return N <= 32; }

// e / N for 1 <= N <= 64 and 0 <= e < 65 N (the row of entry e of a row-major
// matrix with N columns) from a float reciprocal: (e + 1/2) / N lies at least
// 1/(2N) from an integer and the reciprocal and product roundings move it by under
// 2e-5, so the truncation is the integer quotient (checked for every such N and e)
__device__ __forceinline__ int row_of(int e, int N) {
    return (int)(((float)e + 0.5f) * __builtin_amdgcn_rcpf((float)N));
}
// offset of entry e in a global [64][64] matrix
__device__ __forceinline__ int gofs(int e, int N) {
    const int i = row_of(e, N);
    return i * MAXN + (e - i * N);
}
__device__ __forceinline__ bool strict_upper(int e, int N) {
    const int i = row_of(e, N);
    return e - i * N > i;
}

// A <- (M + M^H)/2 for the leading N x N block of a global [64][64] matrix
__device__ void load_herm(Z2* A, const double2* M, int N) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        const Z2 a = gld(M + i * MAXN + j), b = gld(M + j * MAXN + i);
        A[e] = Z2{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
    }
}

// leading N x N block of a global [64][64] matrix into LDS (ld = N)
__device__ void load_mat(Z2* A, const double2* M, int N) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) A[e] = gld(M + gofs(e, N));
}

// Z = L^{-1} for lower-triangular L with real positive diagonal, column by column
// (two barriers per column, all updates of a column in parallel).
__device__ void tri_inv_lower(const Z2* L, Z2* Zm, int N) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
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
            const int q = row_of(e, w), i = k + 1 + q, j = e - q * w;
            const Z2 p = zmul(L[i * N + k], Zm[k * N + j]);
            Zm[i * N + j].re -= p.re;
            Zm[i * N + j].im -= p.im;
        }
        __syncthreads();
    }
}

// Cholesky A = L L^H (in place, lower) and Z = L^{-1} together: step k scales
// column k of L and row k of Z (phase 1), then updates the trailing block of A and
// the rows below k of Z (phase 2); two barriers per column.  Phase 1 also copies
// the scaled column k into colk (LDS, N entries), which phase 2 reads: the lanes
// then touch consecutive entries instead of a column of A.  L has a positive real
// diagonal and a zeroed strict upper triangle.  A pivot d_k that is not positive,
// not finite, or (when diag != nullptr) not above 1e-14 of the column's own
// original diagonal is a breakdown: returns false on every thread (all threads
// read the same pivot after a barrier, so the decision is uniform).
__device__ bool chol_inv_lower(Z2* A, Z2* Zm, int N, const double* diag, Z2* colk) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        Zm[e] = Z2{i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const double d = A[k * N + k].re;
        const double floor_k = diag ? 1e-14 * diag[k] : 0.0;
        if (!(d > floor_k) || !isfinite(d)) return false;
        const double rs = 1.0 / sqrt(d);
        // phase 1: L[i][k] = A[i][k] / sqrt(d) (i > k);  Z[k][j] /= L[k][k] (j <= k)
        for (int e = threadIdx.x; e < N; e += blockDim.x) {
            if (e > k) {
                const Z2 v = A[e * N + k];
                const Z2 l{v.re * rs, v.im * rs};
                A[e * N + k] = l;
                colk[e] = l;
            } else {
                const Z2 v = Zm[k * N + e];
                Zm[k * N + e] = Z2{v.re * rs, v.im * rs};
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) A[k * N + k] = Z2{d * rs, 0.0};
        // phase 2: trailing update of A (j <= i, both > k) and Z[i][j] -= L[i][k] Z[k][j]
        const int m = N - k - 1;
        for (int e = threadIdx.x; e < m * m + m * (k + 1); e += blockDim.x) {
            if (e < m * m) {
                const int q = row_of(e, m), i = k + 1 + q, j = k + 1 + (e - q * m);
                if (j <= i) {
                    const Z2 p = zmul(colk[i], zconj(colk[j]));
                    A[i * N + j].re -= p.re;
                    A[i * N + j].im -= p.im;
                }
            } else {
                const int f = e - m * m;
                const int q = row_of(f, k + 1), i = k + 1 + q, j = f - q * (k + 1);
                const Z2 p = zmul(colk[i], Zm[k * N + j]);
                Zm[i * N + j].re -= p.re;
                Zm[i * N + j].im -= p.im;
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x)
        if (strict_upper(e, N)) A[e] = Z2{0.0, 0.0};
    __syncthreads();
    return true;
}

// chol_inv_lower with two buffers per matrix and 2 x 2 pivot blocks: step k reads
// (X, ZX) and writes (Y, ZY), then the roles swap, so one barrier per step and half
// the steps.  A step does two columns k, k + 1 of the right-looking factorisation at
// once (the same products as two single-column steps): with l00 = sqrt(a00),
// l10 = a10 / l00, d1 = a11 - |l10|^2 and l11 = sqrt(d1),
//   L[i][k] = a_ik / l00,  L[i][k+1] = (a_i,k+1 - L[i][k] conj(l10)) / l11,
//   A[i][j] -= L[i][k] conj(L[j][k]) + L[i][k+1] conj(L[j][k+1])   (i >= j > k + 1),
// and on the rows of Z = L^{-1}: Z[k] /= l00, Z[k+1] = (Z[k+1] - l10 Z[k]) / l11,
// Z[i] -= L[i][k] Z[k] + L[i][k+1] Z[k+1] (i > k + 1).  Every thread forms the
// factors of its own row and column itself.  An odd last column is a single step
// (the same formulas with a10 = 0, a11 = 1).  The breakdown test (either pivot, d_k
// or d1, not positive, not finite or, when diag != nullptr, not above 1e-14 of the
// column's original diagonal) follows the step's barrier; a failed step's outputs are
// discarded.  On return *L and *Zout point at the buffers holding L (lower, strict
// upper zeroed) and L^{-1}.  Only the lower triangles are written and read.
__device__ void chol_inv_lower_pp(Z2* X, Z2* Y, Z2* ZX, Z2* ZY, int N, const double* diag, bool& ok,
                                  Z2** L, Z2** Zout) {
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        ZX[e] = Z2{i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    for (int k = 0; k < N;) {
        const bool two = k + 1 < N;
        const int k1 = two ? k + 1 : k;   // column k + 1 (only read when two)
        const double a00 = X[k * N + k].re;
        const Z2 a10 = two ? X[k1 * N + k] : Z2{0.0, 0.0};
        const double a11 = two ? X[k1 * N + k1].re : 1.0;
        const double r0 = 1.0 / sqrt(a00);
        const Z2 l10{a10.re * r0, a10.im * r0};
        const double d1 = a11 - (l10.re * l10.re + l10.im * l10.im);
        const double r1 = 1.0 / sqrt(d1);
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int i = row_of(e, N), j = e - i * N;
            if (j > i) continue;   // strict upper triangles: never written or read
            const Z2 xe = X[e], ze = ZX[e];
            const Z2 zero{0.0, 0.0};
            const Z2 ai0 = i >= k ? X[i * N + k] : zero, ai1 = two && i >= k1 ? X[i * N + k1] : zero;
            const Z2 aj0 = j > k1 ? X[j * N + k] : zero, aj1 = j > k1 ? X[j * N + k1] : zero;
            // row k of Z is zero right of its diagonal (j = k + 1 lies in the unread upper part)
            const Z2 zk0 = j <= k ? ZX[k * N + j] : zero, zk1 = two ? ZX[k1 * N + j] : zero;
            // this thread's row and column of the two new L columns (i, j >= k)
            const Z2 li0{ai0.re * r0, ai0.im * r0}, lj0{aj0.re * r0, aj0.im * r0};
            const Z2 ti = zmul(li0, zconj(l10)), tj = zmul(lj0, zconj(l10));
            const Z2 li1{(ai1.re - ti.re) * r1, (ai1.im - ti.im) * r1};
            const Z2 lj1{(aj1.re - tj.re) * r1, (aj1.im - tj.im) * r1};
            // L part
            Z2 v = xe;
            if (j == k) {
                v = (i == k) ? Z2{a00 * r0, 0.0} : li0;
            } else if (two && j == k1) {
                v = (i == k1) ? Z2{d1 * r1, 0.0} : li1;
            } else if (j > k1) {
                const Z2 p = zmul(li0, zconj(lj0)), q = zmul(li1, zconj(lj1));
                v.re -= p.re + q.re;
                v.im -= p.im + q.im;
            }
            Y[e] = v;
            // Z part: rows k, k + 1 of the pivot block, then the rows below it
            Z2 z = ze;
            if (j <= k1) {
                const Z2 zn0{zk0.re * r0, zk0.im * r0};
                const Z2 t = zmul(l10, zn0);
                const Z2 zn1{(zk1.re - t.re) * r1, (zk1.im - t.im) * r1};
                if (i == k) {
                    z = zn0;
                } else if (two && i == k1) {
                    z = zn1;
                } else if (i > k1) {
                    const Z2 p = zmul(li0, zn0), q = zmul(li1, zn1);
                    z.re -= p.re + q.re;
                    z.im -= p.im + q.im;
                }
            }
            ZY[e] = z;
        }
        __syncthreads();
        const double f0 = diag ? 1e-14 * diag[k] : 0.0;
        const double f1 = (diag && two) ? 1e-14 * diag[k1] : 0.0;
        if (!(a00 > f0) || !isfinite(a00) || (two && (!(d1 > f1) || !isfinite(d1)))) {
            ok = false;
            *L = X;
            *Zout = ZX;
            return;
        }
        Z2* t = X;
        X = Y;
        Y = t;
        t = ZX;
        ZX = ZY;
        ZY = t;
        k += two ? 2 : 1;
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x)
        if (strict_upper(e, N)) X[e] = Z2{0.0, 0.0};
    __syncthreads();
    ok = true;
    *L = X;
    *Zout = ZX;
}

// In-place Gauss-Jordan inverse of a Hermitian positive-definite A (no pivoting
// needed: the pivots are the Cholesky pivots d_k > 0).  rowk, colk: LDS scratch of
// length N.  Returns false on a non-positive pivot.
__device__ bool gj_inverse_hpd(Z2* A, int N, Z2* rowk, Z2* colk) {
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const double p = A[k * N + k].re;
        if (!(p > 0.0) || !isfinite(p)) return false;
        const double pinv = 1.0 / p;
        for (int j = threadIdx.x; j < N; j += blockDim.x) {
            const Z2 v = (j == k) ? Z2{1.0, 0.0} : A[k * N + j];
            rowk[j] = Z2{v.re * pinv, v.im * pinv};
            colk[j] = (j == k) ? Z2{0.0, 0.0} : A[j * N + k];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int i = row_of(e, N), j = e - i * N;
            if (i == k) {
                A[e] = rowk[j];
            } else {
                const Z2 base = (j == k) ? Z2{0.0, 0.0} : A[e];
                const Z2 q = zmul(colk[i], rowk[j]);
                A[e] = Z2{base.re - q.re, base.im - q.im};
            }
        }
        __syncthreads();
    }
    return true;
}

// Gauss-Jordan inverse of a Hermitian positive-definite X with 2 x 2 pivot blocks
// (a 1 x 1 block last when N is odd): half the steps of gj_inverse_hpd, and with two
// buffers (step reads X, writes Y, then the roles swap) one barrier per step.  Step K = {k, k+1} with P = X[K][K] (Hermitian: P^{-1} from its
// determinant), writing into Y:
//   Y[K][K] = P^{-1},  Y[K][j] = P^{-1} X[K][j],  Y[i][K] = -X[i][K] P^{-1},
//   Y[i][j] = X[i][j] - X[i][K] P^{-1} X[K][j]      (i, j outside K).
// Returns the buffer holding the inverse; ok = false when a pivot block is not
// positive definite (p00 <= 0 or det <= 0, tested after the step's barrier).
__device__ Z2* gj_inverse_hpd_pp2(Z2* X, Z2* Y, int N, bool& ok) {
    __syncthreads();
    for (int k = 0; k < N;) {
        const int b = (k + 1 < N) ? 2 : 1;
        const double p00 = X[k * N + k].re;
        const double p11 = (b == 2) ? X[(k + 1) * N + k + 1].re : 1.0;
        const Z2 p01 = (b == 2) ? X[k * N + k + 1] : Z2{0.0, 0.0};
        const double det = p00 * p11 - (p01.re * p01.re + p01.im * p01.im);
        const double idet = 1.0 / det;
        const Z2 q00{p11 * idet, 0.0}, q11{p00 * idet, 0.0};
        const Z2 q01{-p01.re * idet, -p01.im * idet}, q10{-p01.re * idet, p01.im * idet};
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int i = row_of(e, N), j = e - i * N;
            const Z2 xe = X[e], a0 = X[i * N + k], r0 = X[k * N + j];
            const Z2 a1 = (b == 2) ? X[i * N + k + 1] : Z2{0.0, 0.0};
            const Z2 r1 = (b == 2) ? X[(k + 1) * N + j] : Z2{0.0, 0.0};
            const bool iK = i >= k && i < k + b, jK = j >= k && j < k + b;
            Z2 y;
            if (iK && jK) {
                y = (i == k) ? ((j == k) ? q00 : q01) : ((j == k) ? q10 : q11);
            } else if (iK) {
                const Z2 qa = (i == k) ? q00 : q10, qb = (i == k) ? q01 : q11;
                const Z2 u = zmul(qa, r0), v = zmul(qb, r1);
                y = Z2{u.re + v.re, u.im + v.im};
            } else if (jK) {
                const Z2 qa = (j == k) ? q00 : q01, qb = (j == k) ? q10 : q11;
                const Z2 u = zmul(a0, qa), v = zmul(a1, qb);
                y = Z2{-(u.re + v.re), -(u.im + v.im)};
            } else {
                const Z2 t0a = zmul(q00, r0), t0b = zmul(q01, r1), t1a = zmul(q10, r0), t1b = zmul(q11, r1);
                const Z2 t0{t0a.re + t0b.re, t0a.im + t0b.im}, t1{t1a.re + t1b.re, t1a.im + t1b.im};
                const Z2 u = zmul(a0, t0), v = zmul(a1, t1);
                y = Z2{xe.re - (u.re + v.re), xe.im - (u.im + v.im)};
            }
            Y[e] = y;
        }
        __syncthreads();
        if (!(p00 > 0.0) || !(det > 0.0) || !isfinite(det)) {
            ok = false;
            return X;
        }
        Z2* t = X;
        X = Y;
        Y = t;
        k += b;
    }
    ok = true;
    return X;
}

// relres[i] = sqrt((C^H H C)_ii) / bnorm[i].  A group of G lanes (G = 16, 32 or
// 64, the smallest power of two >= N) handles one column i, lane m forming
// conj(C[m][i]) (H C)[m][i]; the group sums its lanes with shuffles.  H must be
// exactly Hermitian (as load_herm leaves it): lane m reads row n of H, so the
// lanes of a group touch consecutive entries.
__device__ void residual_norms(const Z2* H, const Z2* C, int N, const double* bnorm, double* rel) {
    const int G = N <= 16 ? 16 : (N <= 32 ? 32 : 64);
    const int groups = blockDim.x / G;
    const int m = threadIdx.x % G, grp = threadIdx.x / G;
    for (int i0 = 0; i0 < N; i0 += groups) {
        const int i = i0 + grp;
        double t = 0.0;
        if (i < N && m <= i) {   // C upper: C[m][i] = 0 for m > i, C[n][i] = 0 for n > i
            Z2 hc{0.0, 0.0};
            for (int n = 0; n <= i; ++n) {   // H[m][n] = conj(H[n][m]) (exactly Hermitian), read by rows
                const Z2 q = zmul(zconj(H[n * N + m]), C[n * N + i]);
                hc.re += q.re;
                hc.im += q.im;
            }
            const Z2 c = C[m * N + i];
            t = c.re * hc.re + c.im * hc.im;
        }
        for (int off = G >> 1; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (m == 0 && i < N) rel[i] = sqrt(fmax(t, 0.0)) / bnorm[i];
    }
}

// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_state_init(SolveState* st, double tol, double ru_delta, int ru_window, const double* bnorm, int N) {
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
        st->best_relres = 1.0;
        st->best_it = 0;
        st->ru_window = ru_window;
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
    __shared__ double diag[MAXN];
    __shared__ double rel[MAXN];
    load_herm(A, H, N);
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) diag[k] = A[k * N + k].re;
    __shared__ Z2 colk[MAXN];
    if (!chol_inv_lower(A, Zm, N, diag, colk)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            st->pb_mode = PB_SKIP;
        }
        return;
    }
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        gst(C + i * MAXN + j, (j >= i) ? zconj(A[j * N + i]) : Z2{0.0, 0.0});      // C = L^H
        gst(Cinv + i * MAXN + j, (j >= i) ? zconj(Zm[j * N + i]) : Z2{0.0, 0.0});  // C^{-1} = (L^{-1})^H
    }
    // relative residual of column i = ||C[:, i]|| / ||b_i||  (R = Q C)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double s2 = 0.0;
        for (int m = 0; m <= i; ++m) {  // C[m][i] = conj(L[i][m]), nonzero for m <= i
            const Z2 v = A[i * N + m];
            s2 += v.re * v.re + v.im * v.im;
        }
        rel[i] = sqrt(s2) / st->bnorm[i];
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
        st->best_relres = mx;
        st->best_it = st->iters;
        st->halt = 0;
        st->reason = HALT_NONE;
        st->pb_mode = PB_FULL;
    }
}

// beta = G^{-1} (Gauss-Jordan on the Hermitian part of G), betaC = beta C
__global__ void __launch_bounds__(1024)
k_small1(const double2* __restrict__ G, const double2* __restrict__ C, double2* __restrict__ beta,
         double2* __restrict__ betaC, SolveState* st, int N) {
    if (st->halt) return;
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* Cm = sm + N * N;
    __shared__ Z2 rowk[MAXN], colk[MAXN];
    load_herm(A, G, N);
    load_mat(Cm, C, N);
    bool ok;
    Z2* Bi;  // G^{-1}
    if (small_has_cold(N)) {
        Bi = gj_inverse_hpd_pp2(A, sm + 2 * N * N, N, ok);
    } else {
        ok = gj_inverse_hpd(A, N, rowk, colk);
        Bi = A;
    }
    if (!ok) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_G;
        }
        return;
    }
    // beta is Hermitian: average the two triangles the elimination produced
    Z2 bv[4];   // N*N / blockDim <= 4 (the launcher guarantees it)
    int cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) {
        const int i = row_of(e, N), j = e - i * N;
        const Z2 a = Bi[e], b = Bi[j * N + i];
        bv[cnt] = Z2{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) {
        Bi[e] = bv[cnt];
        gst(beta + gofs(e, N), bv[cnt]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        Z2 s{0.0, 0.0};
        for (int m = 0; m <= j; ++m) {   // C upper triangular
            const Z2 p = zmul(Bi[i * N + m], Cm[m * N + j]);
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
    __shared__ double rel[MAXN];
    __shared__ int decision;
    load_herm(A, H, N);
    load_mat(W, C, N);
    if (small_has_cold(N)) load_mat(sm + 2 * N * N, C, N);
    __syncthreads();
    residual_norms(A, W, N, st->bnorm, rel);
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
        if (mx < st->best_relres) {
            st->best_relres = mx;
            st->best_it = st->iters;
        }
        // reliable update when the residual has dropped by ru_delta since the last one
        // (Alg. 3), or when it has stopped reaching new minima (adaptive trigger)
        const bool ru = (st->ru_delta > 0.0 && mx <= st->ru_delta * st->rho_ru) ||
                        (st->ru_window > 0 && st->iters - st->best_it >= st->ru_window);
        decision = conv ? HALT_CONVERGED : (ru ? HALT_RU : HALT_NONE);
        if (decision != HALT_NONE) {
            st->halt = 1;
            st->reason = decision;
            st->pb_mode = PB_X_ONLY;
        }
    }
    __syncthreads();
    if (decision != HALT_NONE) return;
    // Cholesky of H and L^{-1} together (W, which held C, becomes L^{-1}; with the
    // wide LDS layout the ping-pong variant, one barrier per step)
    Z2* Lm = A;
    Z2* Zm = W;
    bool ok;
    if (small_has_cold(N)) chol_inv_lower_pp(A, sm + 3 * N * N, W, sm + 4 * N * N, N, nullptr, ok, &Lm, &Zm);
    else {
        __shared__ Z2 colk[MAXN];
        ok = chol_inv_lower(A, W, N, nullptr, colk);
    }
    if (!ok) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            st->pb_mode = PB_X_ONLY;
        }
        return;
    }
    // C <- S C with S = L^H upper: (S C)[i][j] = sum_{m=i..j} conj(L[m][i]) C[m][j];
    // the old C is read from its LDS copy when the third buffer fits (N <= 32),
    // else from global memory; all reads finish before the writes
    const bool cl = small_has_cold(N);
    const Z2* Cold = sm + 2 * N * N;
    Z2 cn[4];   // N*N / blockDim <= 4 (the launcher guarantees it)
    int cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) {
        const int i = row_of(e, N), j = e - i * N;
        Z2 s2{0.0, 0.0};
        for (int m = i; m <= j; ++m) {
            const Z2 c = cl ? Cold[m * N + j] : gld(C + m * MAXN + j);
            const Z2 p = zmul(zconj(Lm[m * N + i]), c);
            s2.re += p.re;
            s2.im += p.im;
        }
        cn[cnt] = s2;
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) gst(C + gofs(e, N), cn[cnt]);
    // S^H = L; S^{-1} = (L^{-1})^H  (leading N x N blocks only)
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        gst(SH + i * MAXN + j, (j <= i) ? Lm[i * N + j] : Z2{0.0, 0.0});
        gst(Sinv + i * MAXN + j, (j >= i) ? zconj(Zm[j * N + i]) : Z2{0.0, 0.0});
    }
    if (threadIdx.x == 0) st->pb_mode = PB_FULL;
}

// End of a reliable update: with C^ in SH (upper) and C_k in C, S^ = C^ C_k^{-1},
// C <- C^, SH <- S^^H, and the iteration resumes.  A, W: LDS N x N scratch.
__device__ void ru_set_s(double2* __restrict__ C, double2* __restrict__ SH, Z2* A, Z2* W, SolveState* st,
                         int* __restrict__ ru_skip, int N) {
    // A <- C_k^H (lower), W <- (C_k^H)^{-1} = (C_k^{-1})^H
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        A[e] = (j <= i) ? zconj(gld(C + j * MAXN + i)) : Z2{0.0, 0.0};
    }
    __syncthreads();
    tri_inv_lower(A, W, N);
    // S^ = C^ C_k^{-1} (upper), C_k^{-1}[m][j] = conj(W[j][m])
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        Z2 s2{0.0, 0.0};
        for (int m = i; m <= j; ++m) {
            const Z2 p = zmul(gld(SH + i * MAXN + m), zconj(W[j * N + m]));
            s2.re += p.re;
            s2.im += p.im;
        }
        A[e] = s2;
    }
    __syncthreads();
    // C <- C^ ; then S^H
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int o = gofs(e, N);
        C[o] = SH[o];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        gst(SH + i * MAXN + j, zconj(A[j * N + i]));
    }
    if (threadIdx.x == 0) {
        st->halt = 0;
        st->reason = HALT_NONE;
        st->pb_mode = PB_FULL;
        *ru_skip = 0;
    }
}

// Reliable update from H = R^H R of the true residual R = B - A Y.  first_pass:
// stop after C^ (into SH) and C^{-1} (into Chinv), for CholQR2 (k_small_qr2
// finishes the update).
__global__ void __launch_bounds__(1024)
k_small_ru(const double2* __restrict__ H, double2* __restrict__ C, double2* __restrict__ Chinv,
           double2* __restrict__ SH, SolveState* st, double* __restrict__ true_relres,
           int* __restrict__ ru_skip, int conv_check, int first_pass, int N) {
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* W = sm + N * N;
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
        st->best_relres = mx;
        st->best_it = st->iters;
    }
    __syncthreads();
    if (done) return;
    load_herm(A, H, N);
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) diag[k] = A[k * N + k].re;
    __shared__ Z2 colk[MAXN];
    if (!chol_inv_lower(A, W, N, diag, colk)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            *ru_skip = 1;
        }
        return;
    }
    // C^ = L^H -> temporarily in SH; C^{-1} = (L^{-1})^H -> Chinv
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = row_of(e, N), j = e - i * N;
        gst(SH + i * MAXN + j, (j >= i) ? zconj(A[j * N + i]) : Z2{0.0, 0.0});
        gst(Chinv + i * MAXN + j, (j >= i) ? zconj(W[j * N + i]) : Z2{0.0, 0.0});
    }
    __syncthreads();
    if (first_pass) {
        if (threadIdx.x == 0) *ru_skip = 0;
        return;
    }
    ru_set_s(C, SH, A, W, st, ru_skip, N);
}

// Second pass of CholQR2 (Alg. 2 applied to Q1 = R C1^{-1}): H2 = Q1^H Q1 =
// C2^H C2; Cacc <- C2 C1 (C1 in Cacc), Cinv <- C1^{-1} C2^{-1}, C2inv <- C2^{-1}
// (for Q = Q1 C2^{-1}).  ru = 1: the pass of a reliable update (Cacc is SH,
// holding C^, and C holds C_k): the update is then finished with S^ = C^ C_k^{-1}.
// Does nothing when *skip is set (the reliable update found convergence or broke
// down); a breakdown pivot (below 1e-14 of the column's diagonal) halts the solve.
__global__ void __launch_bounds__(1024)
k_small_qr2(const double2* __restrict__ H2, double2* __restrict__ Cacc, double2* __restrict__ Cinv,
            double2* __restrict__ C2inv, double2* __restrict__ C, SolveState* st, int* __restrict__ skip,
            int ru, int N) {
    if (skip && *skip) return;
    extern __shared__ Z2 sm[];
    Z2* A = sm;
    Z2* W = sm + N * N;
    __shared__ double diag[MAXN];
    __shared__ Z2 colk[MAXN];
    load_herm(A, H2, N);
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) diag[k] = A[k * N + k].re;
    if (!chol_inv_lower(A, W, N, diag, colk)) {
        if (threadIdx.x == 0) {
            st->halt = 1;
            st->reason = HALT_BREAKDOWN_H;
            st->pb_mode = PB_SKIP;
            if (skip) *skip = 1;
        }
        return;
    }
    // C2[i][m] = conj(L[m][i]) (m >= i), C2^{-1}[m][j] = conj(Z[j][m]) (j >= m)
    Z2 cv[4], iv[4];   // N*N / blockDim <= 4 (the launcher guarantees it)
    int cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) {
        const int i = row_of(e, N), j = e - i * N;
        Z2 a{0.0, 0.0}, b{0.0, 0.0};
        for (int m = i; m <= j; ++m) {
            const Z2 p = zmul(zconj(A[m * N + i]), gld(Cacc + m * MAXN + j));    // (C2 C1)[i][j]
            const Z2 q = zmul(gld(Cinv + i * MAXN + m), zconj(W[j * N + m]));    // (C1^{-1} C2^{-1})[i][j]
            a.re += p.re;
            a.im += p.im;
            b.re += q.re;
            b.im += q.im;
        }
        cv[cnt] = a;
        iv[cnt] = b;
    }
    __syncthreads();
    cnt = 0;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x, ++cnt) {
        const int i = row_of(e, N), j = e - i * N;
        const int o = i * MAXN + j;
        gst(Cacc + o, j >= i ? cv[cnt] : Z2{0.0, 0.0});
        gst(Cinv + o, j >= i ? iv[cnt] : Z2{0.0, 0.0});
        gst(C2inv + o, j >= i ? zconj(W[j * N + i]) : Z2{0.0, 0.0});
    }
    __syncthreads();
    if (ru) ru_set_s(C, Cacc, A, W, st, skip, N);
}

// ---------------------------------------------------------------------------------------------
// ---------------------------------------------------------------------------------------------
// s-step block CG: the coefficients of one outer iteration (K = s N basis columns)
//   inputs (global [64][64]): Gv = V^H AV, Gvv = V^H V (its first N columns are
//   Gr = V^H R, as V_0 = R), and after the first outer iteration Ga = (A P')^H V,
//   Wp = P'^H A P' and Pv = P'^H V (first N columns: Pr = P'^H R)
//   first:  Bk = 0, W = Gv, g = Gr
//   else:   Bk = -Wp^{-1} Ga, W = Gv + Ga^H Bk, g = Gr + Bk^H Pr
//   out:    Bk (K x K), alpha = W^{-1} g and nalpha = -alpha (K x N)
// The inverses go through the Cholesky factor L and Z = L^{-1} (W^{-1} = Z^H Z).
// A non-positive pivot of Wp (status 1) or W (status 2) stops the kernel with
// *status set; the update kernels that follow take *status as their skip flag.
// LDS holds two K x K matrices (four for K <= 32, where the Cholesky factorisations
// take 2 x 2 pivots); every K^3 product reads LDS only, and its result
// goes to a global [64][64] array (nalpha or alpha before they receive their final
// values) and back into LDS after a barrier, which makes the workgroup's global
// writes visible to all of its threads.
// ---------------------------------------------------------------------------------------------
__device__ void load_full(Z2* A, const double2* M, int K) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) A[e] = gld(M + gofs(e, K));
}

// LDS matrices of k_sstep_coef: four for K <= 32 (the 2 x 2-pivot ping-pong
// Cholesky), two above
__host__ __device__ constexpr int sstep_bufs(int K) { return K <= 32 ? 4 : 2; }

// Cholesky W = L L^H of the Hermitian K x K matrix in b[0] and Z = L^{-1}: *Z gets
// the buffer holding Z and *spare a buffer free for other use.  False on a
// non-positive pivot (uniform over the workgroup).
__device__ bool sstep_chol(Z2* const* b, int K, Z2* colk, Z2** Z, Z2** spare) {
    if (sstep_bufs(K) == 4) {
        bool ok = false;
        Z2 *L = nullptr, *Zo = nullptr;
        chol_inv_lower_pp(b[0], b[2], b[1], b[3], K, nullptr, ok, &L, &Zo);
        *Z = Zo;
        *spare = L;
        return ok;
    }
    if (!chol_inv_lower(b[0], b[1], K, nullptr, colk)) return false;
    *Z = b[1];
    *spare = b[0];
    return true;
}

__global__ void __launch_bounds__(1024)
k_sstep_coef(const double2* __restrict__ Gv, const double2* __restrict__ Gvv, const double2* __restrict__ Ga,
             const double2* __restrict__ Wp, const double2* __restrict__ Pv, double2* __restrict__ Bk,
             double2* __restrict__ alpha, double2* __restrict__ nalpha, int* __restrict__ status, int K, int N,
             int first) {
    extern __shared__ Z2 sm[];
    Z2* b[4];
    for (int q = 0; q < 4; ++q) b[q] = sm + (q < sstep_bufs(K) ? q : 0) * K * K;
    __shared__ Z2 colk[MAXN];
    Z2 *Zm = nullptr, *S = nullptr;
    if (!first) {
        load_herm(b[0], Wp, K);
        __syncthreads();
        if (!sstep_chol(b, K, colk, &Zm, &S)) {
            if (threadIdx.x == 0) *status = 1;
            return;
        }
        load_full(S, Ga, K);
        __syncthreads();
        // Y = Z Ga (Z lower triangular) -> nalpha
        for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
            const int i = row_of(e, K), j = e - i * K;
            Z2 acc{0.0, 0.0};
            for (int l = 0; l <= i; ++l) {
                const Z2 p = zmul(Zm[i * K + l], S[l * K + j]);
                acc.re += p.re;
                acc.im += p.im;
            }
            gst(nalpha + i * MAXN + j, acc);
        }
        __syncthreads();
        load_full(S, nalpha, K);
        __syncthreads();
        // Bk = -Z^H Y
        for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
            const int i = row_of(e, K), j = e - i * K;
            Z2 acc{0.0, 0.0};
            for (int l = i; l < K; ++l) {
                const Z2 p = zmul(zconj(Zm[l * K + i]), S[l * K + j]);
                acc.re += p.re;
                acc.im += p.im;
            }
            gst(Bk + i * MAXN + j, Z2{-acc.re, -acc.im});
        }
        __syncthreads();
        Z2 *GaL = S, *BkL = Zm;
        load_full(GaL, Ga, K);
        load_full(BkL, Bk, K);
        __syncthreads();
        // W = Gv + Ga^H Bk -> nalpha;  g = Gr + Bk^H Pr -> alpha
        for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
            const int i = row_of(e, K), j = e - i * K;
            Z2 acc = gld(Gv + i * MAXN + j);
            for (int l = 0; l < K; ++l) {
                const Z2 p = zmul(zconj(GaL[l * K + i]), BkL[l * K + j]);
                acc.re += p.re;
                acc.im += p.im;
            }
            gst(nalpha + i * MAXN + j, acc);
        }
        for (int e = threadIdx.x; e < K * N; e += blockDim.x) {
            const int i = row_of(e, N), n = e - i * N;
            Z2 acc = gld(Gvv + i * MAXN + n);
            for (int l = 0; l < K; ++l) {
                const Z2 p = zmul(zconj(BkL[l * K + i]), gld(Pv + l * MAXN + n));
                acc.re += p.re;
                acc.im += p.im;
            }
            gst(alpha + i * MAXN + n, acc);
        }
        __syncthreads();
        load_herm(b[0], nalpha, K);
    } else {
        load_herm(b[0], Gv, K);
        for (int e = threadIdx.x; e < K * K; e += blockDim.x) gst(Bk + gofs(e, K), Z2{0.0, 0.0});
        for (int e = threadIdx.x; e < K * N; e += blockDim.x) {
            const int i = row_of(e, N), n = e - i * N;
            gst(alpha + i * MAXN + n, gld(Gvv + i * MAXN + n));
        }
    }
    __syncthreads();
    if (!sstep_chol(b, K, colk, &Zm, &S)) {
        if (threadIdx.x == 0) *status = 2;
        return;
    }
    // T = Z g (into S, K x N with leading dimension N), then alpha = Z^H T
    for (int e = threadIdx.x; e < K * N; e += blockDim.x) {
        const int i = row_of(e, N), n = e - i * N;
        Z2 acc{0.0, 0.0};
        for (int l = 0; l <= i; ++l) {
            const Z2 p = zmul(Zm[i * K + l], gld(alpha + l * MAXN + n));
            acc.re += p.re;
            acc.im += p.im;
        }
        S[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * N; e += blockDim.x) {
        const int i = row_of(e, N), n = e - i * N;
        Z2 acc{0.0, 0.0};
        for (int l = i; l < K; ++l) {
            const Z2 p = zmul(zconj(Zm[l * K + i]), S[l * N + n]);
            acc.re += p.re;
            acc.im += p.im;
        }
        gst(alpha + i * MAXN + n, acc);
        gst(nalpha + i * MAXN + n, Z2{-acc.re, -acc.im});
    }
}

static size_t small_lds(int N) { return (small_has_cold(N) ? 5 : 2) * (size_t)N * N * sizeof(Z2); }

hipError_t small_setup() {
    const int bytes = (int)(small_lds(32) > small_lds(MAXN) ? small_lds(32) : small_lds(MAXN));
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_small_init, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small1, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small2, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small_ru, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_small_qr2, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_sstep_coef, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(2 * MAXN * MAXN * sizeof(Z2)))) != hipSuccess)
        return e;
    return hipSuccess;
}

// threads of the single-workgroup N x N kernels: a request of 64, 256 or 1024 is
// honoured when every thread keeps at most four entries of an N x N matrix
static int small_threads(int N, int req) {
    if ((req == 64 || req == 256 || req == 1024) && N * N <= 4 * req) return req;
    return N <= 16 ? 256 : 1024;
}

hipError_t launch_state_init(SolveState* st, double tol, double ru_delta, int ru_window, const double* bnorm,
                             int N, hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, st, tol, ru_delta, ru_window, bnorm, N);
    return hipGetLastError();
}
hipError_t launch_identity(double2* M, int N, hipStream_t s) {
    hipLaunchKernelGGL(k_identity, dim3(1), dim3(1024), 0, s, M, N);
    return hipGetLastError();
}
hipError_t launch_small_init(const double2* H, double2* C, double2* Cinv, SolveState* st, int N,
                             int req, hipStream_t s) {
    hipLaunchKernelGGL(k_small_init, dim3(1), dim3(small_threads(N, req)), small_lds(N), s, H, C, Cinv, st, N);
    return hipGetLastError();
}
hipError_t launch_sstep_coef(const double2* Gv, const double2* Gvv, const double2* Ga, const double2* Wp,
                             const double2* Pv, double2* Bk, double2* alpha, double2* nalpha, int* status, int K,
                             int N, int first, hipStream_t s) {
    if (K < 1 || K > MAXN || N < 1 || N > K) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sstep_coef, dim3(1), dim3(small_threads(K, 0)), sstep_bufs(K) * (size_t)K * K * sizeof(Z2),
                       s, Gv, Gvv, Ga, Wp, Pv, Bk, alpha, nalpha, status, K, N, first);
    return hipGetLastError();
}
hipError_t launch_small1(const double2* G, const double2* C, double2* beta, double2* betaC,
                         SolveState* st, int N, int req, hipStream_t s) {
    hipLaunchKernelGGL(k_small1, dim3(1), dim3(small_threads(N, req)), small_lds(N), s, G, C, beta, betaC, st, N);
    return hipGetLastError();
}
hipError_t launch_small2(const double2* H, double2* C, double2* Sinv, double2* SH, SolveState* st,
                         int N, int req, hipStream_t s) {
    hipLaunchKernelGGL(k_small2, dim3(1), dim3(small_threads(N, req)), small_lds(N), s, H, C, Sinv, SH, st, N);
    return hipGetLastError();
}
hipError_t launch_small_ru(const double2* H, double2* C, double2* Chinv, double2* SH,
                           SolveState* st, double* true_relres, int* ru_skip, int conv_check,
                           int first_pass, int N, int req, hipStream_t s) {
    hipLaunchKernelGGL(k_small_ru, dim3(1), dim3(small_threads(N, req)), small_lds(N), s, H, C, Chinv, SH,
                       st, true_relres, ru_skip, conv_check, first_pass, N);
    return hipGetLastError();
}
hipError_t launch_small_qr2(const double2* H2, double2* Cacc, double2* Cinv, double2* C2inv, double2* C,
                            SolveState* st, int* skip, int ru, int N, int req, hipStream_t s) {
    hipLaunchKernelGGL(k_small_qr2, dim3(1), dim3(small_threads(N, req)), small_lds(N), s, H2, Cacc, Cinv, C2inv,
                       C, st, skip, ru, N);
    return hipGetLastError();
}

}  // namespace bcg
