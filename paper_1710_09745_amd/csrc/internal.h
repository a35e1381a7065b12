// Host-side declarations shared by the library's translation units: the
// launchers of every gfx950 kernel and the constants of the solver's layouts.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace bcg {

// Timing events for the next kernel launch on the calling thread.  A launcher that
// finds them set issues its kernel with hipExtLaunchKernelGGL, so that the two events
// carry the start and end of that dispatch itself (no queue gap or end-of-kernel
// cache write-back between an event and the kernel), marks them used and clears
// them.  Set by the library's per-kernel profiler around single-launch calls.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
extern thread_local LaunchTiming g_launch_timing;

#define BCG_TIMED_LAUNCH(KERNEL, GRID, BLOCK, LDS, STREAM, ...)                                         \
    do {                                                                                               \
        if (::bcg::g_launch_timing.start != nullptr) {                                                 \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, ::bcg::g_launch_timing.start,      \
                                  ::bcg::g_launch_timing.stop, 0u, __VA_ARGS__);                       \
            ::bcg::g_launch_timing.used = true;                                                        \
            ::bcg::g_launch_timing.start = ::bcg::g_launch_timing.stop = nullptr;                      \
        } else {                                                                                       \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);                         \
        }                                                                                              \
    } while (0)

enum class Prec { FP64 = 0, FP32 = 1, FP16 = 2, BF16 = 3, FX16 = 4 };

constexpr int MAXN = 64;          // largest block size; N x N matrices use leading dimension 64
constexpr int GRAM_BLOCKS = 512;  // workgroups of a Gram reduction (= rows of its partials)
constexpr int NORM_BLOCKS = 512;  // workgroups of a column-norm reduction

struct HopShape {
    int tr;     // right-hand sides per lane (register tile)
    int tpb;    // site-parallel kernel: lane groups per workgroup sharing the same sites
    int pf;     // 1: two folded matrices in flight per loop trip
    int split;  // 1: lane-split kernel (runs of 16 sites), 2: lane-split, runs of 32 sites, 0: site-parallel
    int queue_wpc = 0;  // site-parallel kernel: > 0 = per-XCD task queues, this many workgroups per CU
};

// Per-XCD task queues of the site-parallel hop: ctr[0..7] queue counters, ctr[8] the
// count of finished workgroups (all reset to 0 by the last one); cells of bpc site blocks
struct HopQueue {
    int* ctr;
    int ncell;
    int bpc;
};

// bytes per stored complex number, and bytes of a [cols][K][Vh] allocation
// including the per-group FP32 scales of the 16-bit formats
inline int pd_bytes(Prec p) {
    switch (p) {
        case Prec::FP64: return 16;
        case Prec::FP32: return 8;
        default: return 4;
    }
}
inline size_t store_bytes(Prec p, long cols, int K, long Vh) {
    size_t b = (size_t)pd_bytes(p) * cols * K * Vh;
    if (p == Prec::FP16 || p == Prec::BF16 || p == Prec::FX16) b += (size_t)4 * cols * Vh;
    return b;
}

// padded block size used to instantiate the N-dependent kernels: 1, 2, 4, ..., 64
inline int pad_n(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// hop.hip ---------------------------------------------------------------------------------------
// FP64 folded links of one output parity from canonical device links
hipError_t pack_links(const void* fat, const void* lng, void* W, const Geom& g, int parity, int nl,
                      hipStream_t s);
// lower-precision folded links from the FP64 ones
hipError_t links_from64(Prec pd, const void* W64, void* Wd, int nl, long Vh, hipStream_t s);
// launch shape of the hop for N right-hand sides in precision p on lattice g;
// nonzero tr, tpb override the defaults, pf: 1 on, 2 off; kernel: 1 lane split,
// 2 site-parallel, 0 chosen by lattice size; fused (Gram epilogue) always takes
// the site-parallel kernel
// sched: 0 default, 1 static slab order, 2..5 per-XCD queues with 1, 2, 4, 8 workgroups per CU
HopShape hop_shape(Prec p, int N, int tr, int tpb, int pf, int kernel, const Geom& g, bool fused, int sched = 0);
// partial dot products written by the EPI_MASS_DOT hop (one right-hand side)
int hop_dot_blocks(const Geom& g);
// partials != nullptr (EPI_PLAIN only): also T^H T partials of the output, one per
// workgroup of the persistent grid hop_grid(g, h, true)
// queue: 9 zero-initialised ints of the context (per-XCD task queues), or nullptr
hipError_t launch_hop(Prec prec, int nl, const void* W, const void* in, void* out, const void* ctr,
                      double m2, int N, const Geom& g, int out_parity, int epi, const HopShape& h,
                      const int* halt, double* dot, double2* partials, int* queue, hipStream_t s);
// cells of the per-XCD queues for spb-site blocks (ctr == nullptr in the result: no queue)
HopQueue hop_queue_layout(const Geom& g, int spb, int* ctr);
size_t hop_tile_bytes(Prec prec, int N, const HopShape& h);
int hop_grid(const Geom& g, const HopShape& h, bool fused);
enum { EPI_PLAIN_ = 0, EPI_MASS_ = 1, EPI_MASS_DOT_ = 2 };

// blas.hip --------------------------------------------------------------------------------------
// partials[b][i*NB + j] = sum over the rows of workgroup b of conj(A[row,i]) B[row,j]
// mfma: matrix-core kernel for N > 8 (vector-ALU kernel otherwise); it forms the
// 16 x 16 tiles a <= b only and writes the others as their conjugate transpose, so
// it needs a Hermitian A^H B (the vector kernel forms every entry)
hipError_t launch_gram(Prec prec, const void* A, const void* B, int N, int Vh, double2* partials,
                       const int* halt, bool mfma, hipStream_t s);
// out[i*64 + j] = sum_b partials[b][i*NB + j]  (fixed order)
// number of partials launch_gram writes
int gram_parts(int N, int Vh, bool mfma);
// out[i*64 + j] = sum_b pa[b][i*NB + j] + alpha * sum_b pb[b][i*NB + j]  (fixed order; pb may be NULL)
hipError_t launch_gram_reduce(const double2* pa, int na, const double2* pb, int nb, double alpha, int N,
                              double2* out, const int* halt, hipStream_t s);
// LDS bytes of a fused Gram epilogue of the streaming passes (0: does not fit, use launch_gram)
size_t fused_tile_bytes(Prec prec, int N);
int fused_grid(int Vh);
// Q <- Q - AP beta    (beta: [64][64] FP64); partials != nullptr: also Qt^H Qt partials
// bps: 64-site blocks per time slice (workgroup order, xcd_task), 0 for the identity order
hipError_t launch_pass_a(Prec prec, void* Q, const void* AP, const double2* beta, int N, int Vh,
                         const int* halt, double2* partials, int cpt, int bps, int kernel, hipStream_t s);
// X += P betaC; Qn <- Qt Sinv; Pn <- Qn + P S^H, as selected by state->pb_mode;
// partials != nullptr: also Pn^H Pn partials
hipError_t launch_pass_b(Prec prec, double2* X, const void* Qt, const void* P, void* Qn, void* Pn,
                         const double2* betaC, const double2* Sinv, const double2* SH, int N,
                         int Vh, const SolveState* state, double2* partials, int cpt, int bps, int kernel,
                         hipStream_t s);
// Y <- Z + X M  (Z may be NULL = 0; X, Z may alias Y); X in precision px, Y/Z in py
hipError_t launch_bmul(Prec px, const void* X, Prec py, const void* Z, void* Y, const double2* M,
                       int N, int Vh, const int* skip, hipStream_t s);
// Y <- Z + X M with X of Nin columns in precision px (FP64 or FP32), Y and Z of Nout
// FP64 columns, M Nin x Nout (leading dimension 64)
hipError_t launch_bmul_rect(Prec px, const void* X, const double2* Z, double2* Y, const double2* M, int Nin,
                            int Nout, int Vh, const int* skip, hipStream_t s);
// Vn = a (AV - c V) - Vm (Vm may be NULL), FP64 or FP32 storage, n pairs: one
// Chebyshev basis step
hipError_t launch_cheb_step(Prec p, void* Vn, const void* AV, const void* V, const void* Vm, double a, double c,
                            long n, hipStream_t s);
// v = w / *nrm, FP64, n pairs (*nrm read on the device)
hipError_t launch_scale_inv(double2* v, const double2* w, const double* nrm, long n, hipStream_t s);
// canonical [N][Vh][3] complex128 <-> internal FP64 [N][3][Vh] pairs
hipError_t launch_canon_to_int(const double2* src, double2* dst, int N, int Vh, hipStream_t s);
hipError_t launch_int_to_canon(const double2* src, double2* dst, int N, int Vh, hipStream_t s);
// Y += X; X = 0 (FP64)
hipError_t launch_fold_x(double2* Y, double2* X, long n, hipStream_t s);
// R <- B - R (FP64)
hipError_t launch_residual(const double2* B, double2* R, long n, hipStream_t s);
// per-column ||V_i||^2 partials [NORM_BLOCKS][N]; then reduce into out[N] (sqrt if take_sqrt)
hipError_t launch_colnorm2(const double2* V, int N, int Vh, double* partials, hipStream_t s);
hipError_t launch_colnorm_reduce(const double* partials, int N, int Vh, double* out,
                                 int take_sqrt, hipStream_t s);
hipError_t launch_zero(void* p, long bytes, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, long bytes, hipStream_t s);

// CG baseline (one right-hand side, FP64)
struct CgState {
    int halt;
    int reason;
    int iters;
    int pad;
    double rr;      // ||r||^2
    double alpha;
    double beta;
    double bnorm;
    double tol;
    double relres;
    double rr_prev;   // ||r||^2 before the last update (beta of a reliable update)
    double ru_delta;  // > 0: reliable update when relres <= ru_delta * rho_ru (sloppy storage)
    double rho_ru;    // relres at the last reliable update
};
hipError_t launch_cg_alpha(const double* dot_partials, int nparts, CgState* st, hipStream_t s);
hipError_t launch_cg_update1(double2* x, double2* r, const double2* p, const double2* Ap, long n,
                             double* partials, CgState* st, hipStream_t s);
hipError_t launch_cg_beta(const double* partials, long n, CgState* st, hipStream_t s);
hipError_t launch_cg_update2(double2* p, const double2* r, long n, CgState* st, hipStream_t s);
// mixed precision (Sec. 6 applied to CG, the double-single baseline of Sec. 7.1): r, p, Ap
// in storage precision prec (one column, [3][Vh] groups), x FP64; partials count cg_parts(Vh)
hipError_t launch_cg_update1_s(Prec prec, double2* x, void* r, const void* p, const void* Ap, int Vh,
                               double* partials, CgState* st, hipStream_t s);
hipError_t launch_cg_update2_s(Prec prec, void* p, const void* r, int Vh, CgState* st, hipStream_t s);
// reliable update of CG from the norm partials of r = b - A y (FP64): ||r||^2, beta = ||r||^2 /
// rr_prev, rho_ru; conv_check and relres <= tol: reason HALT_DONE (halt kept), else resume
hipError_t launch_cg_ru(const double* partials, int Vh, CgState* st, int conv_check, hipStream_t s);
hipError_t launch_cg_set_ru(CgState* st, double ru_delta, hipStream_t s);
// rr = ||r||^2 from colnorm partials of a Vh-site field (restart keeps ||b|| and iters)
hipError_t launch_cg_init(const double* partials, int Vh, CgState* st, double tol, int restart,
                          hipStream_t s);

// pseudo.hip ------------------------------------------------------------------------------------
// N independent CG recurrences sharing the block hop (FP64)
struct PbState {
    int halt;
    int reason;
    int iters;        // lockstep iterations
    int pad;
    double tol;
    double rr[64];
    double alpha[64];
    double beta[64];
    double relres[64];
    double bnorm[64];
    int active[64];
    int col_iters[64];
};
hipError_t launch_pb_dot(const double2* P, const double2* AP, int N, int Vh, double* partials, const PbState* st,
                         hipStream_t s);
hipError_t launch_pb_alpha(const double* partials, int N, int Vh, PbState* st, hipStream_t s);
hipError_t launch_pb_update1(double2* X, double2* R, const double2* P, const double2* AP, int N, int Vh,
                             double* partials, const PbState* st, hipStream_t s);
hipError_t launch_pb_beta(const double* partials, int N, int Vh, PbState* st, hipStream_t s);
hipError_t launch_pb_update2(double2* P, const double2* R, int N, int Vh, const PbState* st, hipStream_t s);
// (re)start: colnorm_partials from launch_colnorm2 of R; first = 1 starts every column,
// otherwise the columns with restart[j] != 0 restart and the others stay finished
hipError_t launch_pb_start(const double* colnorm_partials, int N, int Vh, PbState* st, const int* restart,
                           double tol, int first, hipStream_t s);

// kernel attributes of blas.hip (dynamic LDS above the default limit), for the current device
hipError_t blas_setup();

// small.hip -------------------------------------------------------------------------------------
// kernel attributes of small.hip (dynamic LDS above the default limit), for the current device
hipError_t small_setup();
// initial thin QR of R from H = R^H R:  C (upper) and Cinv; relres, rho_ru; halts on breakdown
hipError_t launch_small_init(const double2* H, double2* C, double2* Cinv, SolveState* st, int N,
                             int req, hipStream_t s);
// s-step block CG coefficients (one workgroup): Bk, alpha = W^{-1} g, nalpha = -alpha from
// the Grams Gv = V^H AV, Gvv = V^H V and (first == 0) Ga = (AP')^H V, Wp = P'^H AP',
// Pv = P'^H V; *status = 1 / 2 on a non-positive pivot of Wp / W.  K = s N <= 64.
hipError_t launch_sstep_coef(const double2* Gv, const double2* Gvv, const double2* Ga, const double2* Wp,
                             const double2* Pv, double2* Bk, double2* alpha, double2* nalpha, int* status, int K,
                             int N, int first, hipStream_t s);
// beta = G^{-1}, betaC = beta C
hipError_t launch_small1(const double2* G, const double2* C, double2* beta, double2* betaC,
                         SolveState* st, int N, int req, hipStream_t s);
// residual test, S from H = S^H S, Sinv, S^H, C <- S C; sets pb_mode / halt
hipError_t launch_small2(const double2* H, double2* C, double2* Sinv, double2* SH, SolveState* st,
                         int N, int req, hipStream_t s);
// reliable update from H = R^H R of the true residual: true residuals; if conv_check and
// all <= tol: done; else C^ , C^-1, S^H = (C^ C^-1)^H, C <- C^, resume
// first_pass: stop after C^ (in SH) and C^{-1} (in Chinv) for CholQR2
hipError_t launch_small_ru(const double2* H, double2* C, double2* Chinv, double2* SH,
                           SolveState* st, double* true_relres, int* ru_skip, int conv_check,
                           int first_pass, int N, int req, hipStream_t s);
// second CholQR pass from H2 = Q1^H Q1: Cacc <- C2 Cacc, Cinv <- Cinv C2^{-1}, C2inv <- C2^{-1};
// ru: Cacc is the reliable update's C^ (in SH) and C holds C_k: finish the update (S^, C <- C^)
hipError_t launch_small_qr2(const double2* H2, double2* Cacc, double2* Cinv, double2* C2inv, double2* C,
                            SolveState* st, int* skip, int ru, int N, int req, hipStream_t s);
hipError_t launch_state_init(SolveState* st, double tol, double ru_delta, int ru_window,
                             const double* bnorm, int N, hipStream_t s);
hipError_t launch_identity(double2* M, int N, hipStream_t s);

// force.hip -------------------------------------------------------------------------------------
hipError_t launch_link_force(const double2* X, const double2* Lam, const double2* YX,
                             const double2* YL, int N, const Geom& g, int improved,
                             double2* gfat, double2* glong, hipStream_t s);

}  // namespace bcg
