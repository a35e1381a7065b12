// Pseudo-block CG (the prior work of Sec. 2): N independent CG recurrences that
// share every stencil application.  The hop kernels apply A to all N search
// directions at once (each link read once per site for the whole block); the
// scalar recurrences of the columns stay separate: per column
//   alpha_i = |r_i|^2 / p_i^H A p_i,  x_i += alpha_i p_i,  r_i -= alpha_i A p_i,
//   beta_i = |r_i,new|^2 / |r_i|^2,   p_i = r_i + beta_i p_i.
// A column whose iterated relative residual meets tol stops moving (alpha = 0)
// while the others go on.  FP64 storage, block vectors [N][3][Vh] pairs.
//
// Reductions are deterministic: one partial per (column, workgroup), summed in
// a fixed order by a single-workgroup kernel (16 lanes per column).
#include "device_common.h"
#include "internal.h"

namespace bcg {

static int pb_blocks(int Vh) {
    const int g = (Vh + 255) / 256;
    return g < NORM_BLOCKS ? g : NORM_BLOCKS;
}

// workgroup sum of v (256 threads); the total on thread 0
__device__ double pb_block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// partials[j][b] = Re sum over the sites of workgroup b of conj(P_j) AP_j; grid (blocks, N)
__global__ void __launch_bounds__(256)
k_pb_dot(const double2* __restrict__ P, const double2* __restrict__ AP, int Vh, double* __restrict__ partials,
         const PbState* __restrict__ st) {
    if (st->halt) return;
    const int j = blockIdx.y;
    __shared__ double red[4];
    double s = 0.0;
    if (st->active[j]) {
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < Vh; i += (long)gridDim.x * 256)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long o = ((long)j * 3 + c) * Vh + i;
                const double2 p = P[o], a = AP[o];
                s += p.x * a.x + p.y * a.y;
            }
    }
    s = pb_block_sum(s, red);
    if (threadIdx.x == 0) partials[(long)j * gridDim.x + blockIdx.x] = s;
}

// sum over b of partials[j][b] for column j = threadIdx.x / 16, in a fixed order: lane
// g of the column's 16 takes b = g, g + 16, ..., then an xor butterfly over the 16 lanes
// (1024 threads: up to 64 columns); every lane of the group ends with the total
__device__ double pb_column_sum(const double* __restrict__ partials, int nb, int N) {
    const int j = threadIdx.x >> 4, g = threadIdx.x & 15;
    double v = 0.0;
    if (j < N)
        for (int b = g; b < nb; b += 16) v += partials[(long)j * nb + b];
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    return v;
}

// alpha_j = rr_j / p_j^H A p_j for the active columns (0 for the others)
__global__ void __launch_bounds__(1024) k_pb_alpha(const double* __restrict__ partials, int nb, int N, PbState* st) {
    if (st->halt) return;
    const int j = threadIdx.x >> 4;
    const double pap = pb_column_sum(partials, nb, N);
    if (j < N && (threadIdx.x & 15) == 0) {
        double a = 0.0;
        if (st->active[j]) {
            if (!(pap > 0.0)) {
                st->halt = 1;
                st->reason = HALT_BREAKDOWN_G;
            } else {
                a = st->rr[j] / pap;
            }
        }
        st->alpha[j] = a;
    }
}

// x_j += alpha_j p_j, r_j -= alpha_j Ap_j; partials[j][b] = |r_j|^2 over workgroup b's sites
__global__ void __launch_bounds__(256)
k_pb_update1(double2* __restrict__ X, double2* __restrict__ R, const double2* __restrict__ P,
             const double2* __restrict__ AP, int Vh, double* __restrict__ partials, const PbState* __restrict__ st) {
    if (st->halt) return;
    const int j = blockIdx.y;
    __shared__ double red[4];
    double s = 0.0;
    if (st->active[j]) {
        const double a = st->alpha[j];
        for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < Vh; i += (long)gridDim.x * 256)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long o = ((long)j * 3 + c) * Vh + i;
                const double2 p = P[o], ap = AP[o];
                double2 x = X[o], r = R[o];
                x.x = fma(a, p.x, x.x);
                x.y = fma(a, p.y, x.y);
                r.x = fma(-a, ap.x, r.x);
                r.y = fma(-a, ap.y, r.y);
                X[o] = x;
                R[o] = r;
                s += r.x * r.x + r.y * r.y;
            }
    }
    s = pb_block_sum(s, red);
    if (threadIdx.x == 0) partials[(long)j * gridDim.x + blockIdx.x] = s;
}

// beta_j, the iterated residuals and the convergence of each column
__global__ void __launch_bounds__(1024) k_pb_beta(const double* __restrict__ partials, int nb, int N, PbState* st) {
    if (st->halt) return;
    __shared__ int still;
    if (threadIdx.x == 0) still = 0;
    __syncthreads();
    const int j = threadIdx.x >> 4;
    const double rr = pb_column_sum(partials, nb, N);
    if (j < N && (threadIdx.x & 15) == 0 && st->active[j]) {
        st->beta[j] = rr / st->rr[j];
        st->rr[j] = rr;
        st->relres[j] = sqrt(rr) / st->bnorm[j];
        st->col_iters[j] += 1;
        if (st->relres[j] <= st->tol) st->active[j] = 0;
        else atomicAdd(&still, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->iters += 1;
        if (still == 0) {
            st->halt = 1;
            st->reason = HALT_CONVERGED;
        }
    }
}

// p_j = r_j + beta_j p_j for the columns still active
__global__ void __launch_bounds__(256)
k_pb_update2(double2* __restrict__ P, const double2* __restrict__ R, int Vh, const PbState* __restrict__ st) {
    if (st->halt) return;
    const int j = blockIdx.y;
    if (!st->active[j]) return;
    const double b = st->beta[j];
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < Vh; i += (long)gridDim.x * 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long o = ((long)j * 3 + c) * Vh + i;
            const double2 r = R[o];
            double2 p = P[o];
            p.x = fma(b, p.x, r.x);
            p.y = fma(b, p.y, r.y);
            P[o] = p;
        }
}

// start (or restart from the true residual) the columns whose flag is set:
// rr_j = |r_j|^2 from the colnorm partials [b][N]; the others keep their state
__global__ void k_pb_start(const double* __restrict__ partials, int nb, int N, PbState* st,
                           const int* __restrict__ restart, double tol, int first) {
    const int j = threadIdx.x;
    if (threadIdx.x == 0) {
        st->halt = 0;
        st->reason = HALT_NONE;
        st->tol = tol;
        if (first) st->iters = 0;
    }
    if (j < N) {
        if (first || restart[j]) {
            double rr = 0.0;
            for (int b = 0; b < nb; ++b) rr += partials[(long)b * N + j];
            st->rr[j] = rr;
            if (first) {
                st->bnorm[j] = sqrt(rr);
                st->col_iters[j] = 0;
            }
            st->relres[j] = sqrt(rr) / st->bnorm[j];
            st->active[j] = 1;
        } else {
            st->active[j] = 0;
        }
        st->alpha[j] = 0.0;
        st->beta[j] = 0.0;
    }
}

hipError_t launch_pb_dot(const double2* P, const double2* AP, int N, int Vh, double* partials, const PbState* st,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_pb_dot, dim3(pb_blocks(Vh), N), dim3(256), 0, s, P, AP, Vh, partials, st);
    return hipGetLastError();
}
hipError_t launch_pb_alpha(const double* partials, int N, int Vh, PbState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_alpha, dim3(1), dim3(1024), 0, s, partials, pb_blocks(Vh), N, st);
    return hipGetLastError();
}
hipError_t launch_pb_update1(double2* X, double2* R, const double2* P, const double2* AP, int N, int Vh,
                             double* partials, const PbState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_update1, dim3(pb_blocks(Vh), N), dim3(256), 0, s, X, R, P, AP, Vh, partials, st);
    return hipGetLastError();
}
hipError_t launch_pb_beta(const double* partials, int N, int Vh, PbState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_beta, dim3(1), dim3(1024), 0, s, partials, pb_blocks(Vh), N, st);
    return hipGetLastError();
}
hipError_t launch_pb_update2(double2* P, const double2* R, int N, int Vh, const PbState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_update2, dim3(pb_blocks(Vh), N), dim3(256), 0, s, P, R, Vh, st);
    return hipGetLastError();
}
hipError_t launch_pb_start(const double* colnorm_partials, int N, int Vh, PbState* st, const int* restart,
                           double tol, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_pb_start, dim3(1), dim3(64), 0, s, colnorm_partials, pb_blocks(Vh), N, st, restart, tol,
                       first);
    return hipGetLastError();
}

}  // namespace bcg
