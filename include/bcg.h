/*
 * bcg.h -- C ABI of the MI355X (gfx950) block conjugate-gradient library.
 *
 * The library solves A X = B for a block of N right-hand sides at once with
 * blockCGrQ: the block CG of O'Leary retooled by Dubrulle so that the residual
 * block is re-orthonormalised every iteration by a thin QR (Sec. 4, Alg. 1),
 * where the thin QR is CholQR (Sec. 6, Alg. 2) and, in mixed precision,
 * the residual is periodically replaced by the true one with the block
 * reliable update (Sec. 6, Alg. 3).
 *
 * Operator.  The improved staggered stencil of Sec. 3.2 (Eq. 2) with fat
 * (one-hop) links F and long (three-hop) links G, read with the standard
 * staggered phases and an anti-Hermitian hopping term:
 *   (D psi)(x) = sum_mu eta_mu(x) [ F_mu(x) psi(x+mu) - F_mu(x-mu)^H psi(x-mu)
 *                                 + G_mu(x) psi(x+3mu) - G_mu(x-3mu)^H psi(x-3mu) ]
 *   eta_0 = 1, eta_1 = (-1)^x0, eta_2 = (-1)^(x0+x1), eta_3 = (-1)^(x0+x1+x2),
 * periodic in all four directions.  The naive operator drops the G terms.
 * The solver inverts the even-even Schur block of the normal operator
 * (Sec. 3.2):
 *   A = 4 m^2 - D_eo D_oe      (Hermitian positive definite, lambda_min >= 4 m^2)
 *
 * Layouts (all complex128, C order, interleaved re/im):
 *   dims    = {Lx, Ly, Lz, Lt}, every extent even and >= 2, V = Lx Ly Lz Lt.
 *   lex(x)  = x0 + Lx*(x1 + Ly*(x2 + Lz*x3)); parity(x) = (x0+x1+x2+x3) mod 2.
 *   links   [4][V][3][3]: U_mu(x) at [mu][lex(x)], (U v)_a = sum_b U_ab v_b.
 *   vectors [nrhs][V/2][3]: nrhs colour-vector fields on one checkerboard,
 *           site index cb = lex(x) >> 1 (x0 is the fastest coordinate, so the
 *           even and odd sites each map one-to-one onto 0 .. V/2-1).
 *
 * Memory.  Vector and gradient arguments are DEVICE pointers owned by the
 * caller (e.g. the data of a torch tensor); the library never frees or keeps
 * them.  Links are copied into library-owned device storage by
 * bcg_load_links (from host or device memory).  Work buffers are allocated
 * by the library on first use for a given nrhs and precision and kept until
 * bcg_destroy.
 *
 * Streams.  Every kernel is launched on the context's stream (given to
 * bcg_create; NULL = the null stream).  bcg_apply, bcg_hop and
 * bcg_link_force only enqueue work (stream-ordered, asynchronous to the
 * host).  bcg_solve and bcg_solve_cg read convergence information and return
 * after the solve has completed on the stream.
 *
 * Errors.  Every function returns a bcg_status; nothing throws or aborts
 * across the ABI.  bcg_last_error gives a message for the last failure on a
 * context.  A context is not thread-safe: use one per host thread.
 */
#ifndef BCG_H
#define BCG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bcg_ctx bcg_ctx;

typedef enum {
    BCG_OK = 0,
    BCG_ERR_ARG = -1,            /* bad argument: null pointer, bad dims, nrhs out of range,
                                    zero right-hand-side column, unknown precision */
    BCG_ERR_HIP = -2,            /* a HIP runtime call failed */
    BCG_ERR_NOMEM = -3,          /* device or pinned host allocation failed */
    BCG_ERR_NOT_CONVERGED = -4,  /* max_iter reached (X holds the current iterate), or
                                    the solve stagnated (see bcg_set_stability; X holds
                                    the best iterate) */
    BCG_ERR_BREAKDOWN = -5,      /* a Cholesky factor met a non-positive pivot before
                                    convergence (R^H R singular, Sec. 4); X holds the
                                    best iterate (see bcg_set_stability) */
    BCG_ERR_STATE = -6           /* call out of order, e.g. solve before bcg_load_links */
} bcg_status;

/* Storage precision of the low-precision ("sloppy") block vectors and links.
 * Y (solution), X (update since the last reliable update), B, the true
 * residual, every N x N matrix and the Gram accumulation stay FP64. */
typedef enum {
    BCG_PREC_FP64 = 0,
    BCG_PREC_FP32 = 1,
    BCG_PREC_FP16 = 2,           /* FP16 components with one FP32 scale per site and column */
    BCG_PREC_BF16 = 3,           /* BF16 components with one FP32 scale per site and column */
    BCG_PREC_FIX16 = 4           /* 16-bit fixed-point components (q / 32767 of the largest
                                    component of the site and column, kept as an FP32 scale) */
} bcg_prec;

#define BCG_MAX_RHS 64           /* N <= 64 (Sec. 6: small N x N matrices) */

typedef struct {
    int iters;                   /* block iterations (solve) or summed CG iterations (solve_cg) */
    int reliable_updates;        /* reliable updates performed (Alg. 3) */
    int status;                  /* bcg_status of the solve */
    int restarts;                /* solve_cg: true-residual restarts; solve: unused (0) */
    double seconds;              /* wall time of the solve on the host */
    double max_true_rel_res;     /* max_i ||b_i - A x_i|| / ||b_i||, FP64 operator */
    double *true_rel_res;        /* optional caller array [nrhs] (host) or NULL */
} bcg_stats;

/* Create a context for one lattice.  dims: four even extents >= 2.
 * improved: 0 = naive operator (fat links only), 1 = fat + long links.
 * hip_stream: a hipStream_t (NULL = null stream).  *out receives the context. */
int bcg_create(bcg_ctx **out, const int dims[4], int improved, void *hip_stream);

/* Free every device, pinned and host allocation owned by the context. */
int bcg_destroy(bcg_ctx *ctx);

/* Load links in the canonical layout [4][V][3][3] complex128.  fat is
 * required; lng must be non-NULL iff the context is improved.  on_device:
 * 0 = host pointers, 1 = device pointers.  The data is copied; the staggered
 * phases and the hop signs are folded into library-owned copies for each
 * output parity and each storage precision.  Synchronous w.r.t. the inputs
 * (they may be freed on return). */
int bcg_load_links(bcg_ctx *ctx, const void *fat, const void *lng, int on_device);

/* Set the mass m of A = 4 m^2 - D_eo D_oe (any real m; m = 0 gives the
 * positive semi-definite -D_eo D_oe). */
int bcg_set_mass(bcg_ctx *ctx, double m);

/* Solver parameters.  tol > 0: stop when every column's relative residual
 * ||b_i - A x_i|| / ||b_i|| <= tol, tested on the iterated residual and then
 * confirmed with the FP64 true residual (a reliable update and further
 * iterations follow if a column misses).  max_iter >= 1.  sloppy_prec: a
 * bcg_prec.  ru_delta in [0, 1): reliable update when the maximum relative
 * iterated residual has dropped by this factor since the last one (0 = only
 * at exit; Sec. 7.1 uses 0.1). */
int bcg_set_solver(bcg_ctx *ctx, double tol, int max_iter, int sloppy_prec, double ru_delta);

/* out = A in for nrhs even fields (FP64 links, FP64 arithmetic).
 * in, out: device [nrhs][V/2][3] complex128, must not overlap. */
int bcg_apply(bcg_ctx *ctx, const void *in, void *out, int nrhs);

/* bcg_apply without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result as bcg_apply (the same kernels).  Instead of
 * the context's work buffers it uses a scratch array that the library keeps in
 * device memory for the life of the process, one per GPU, shared by every
 * context on that GPU: 3 regions of 16 MiB, so nrhs * V/2 * 48 bytes must not
 * exceed 16 MiB (nrhs * V/2 <= 349525, e.g. 16^4 with nrhs <= 10); larger
 * requests return BCG_ERR_ARG.  Nothing in the scratch needs to start at zero.
 * Calls that overlap in time on one GPU (from two contexts, or on two streams)
 * race on the scratch: order them on one stream or synchronise between them.
 * in, out: device [nrhs][V/2][3] complex128.  Stream-ordered; no kernel timing. */
int bcg_apply_noalloc(bcg_ctx *ctx, const void *in, void *out, int nrhs);

/* out = A in evaluated the way the solver's iteration evaluates A P in storage
 * precision prec (a bcg_prec): in is rounded to the storage format (one FP32
 * scale per site and column for the 16-bit formats), T = D_oe in and
 * A in = 4 m^2 in - D_eo T are computed with the links stored in that format,
 * in FP32 arithmetic for every format but FP64, and T and the result are
 * stored in the format before the result is widened to complex128.  The same
 * kernels and launch shapes as the solver's hops for nrhs columns.  FP64 is
 * bcg_apply.  in, out: device [nrhs][V/2][3] complex128, must not overlap.
 * Stream-ordered. */
int bcg_apply_prec(bcg_ctx *ctx, int prec, const void *in, void *out, int nrhs);

/* One checkerboard hop out = D_{p,1-p} in (p = out_parity: 1 gives D_oe,
 * 0 gives D_eo), FP64.  in: fields on parity 1-p, out: on parity p, both
 * device [nrhs][V/2][3] complex128, must not overlap. */
int bcg_hop(bcg_ctx *ctx, int out_parity, const void *in, void *out, int nrhs);

/* Solve A X = B with blockCGrQ (Alg. 1-3) for nrhs columns at once.
 * B, X: device [nrhs][V/2][3] complex128, must not overlap.  use_guess:
 * 1 = X holds the initial guess X0, 0 = start from X0 = 0.  stats may be
 * NULL.  Returns BCG_OK, BCG_ERR_NOT_CONVERGED or BCG_ERR_BREAKDOWN (X holds
 * the current iterate in both), or an argument / runtime error. */
int bcg_solve(bcg_ctx *ctx, const void *B, void *X, int nrhs, int use_guess, bcg_stats *stats);

/* The baseline: nrhs independent single right-hand-side CG solves, one after
 * the other (Sec. 7.1), on the same operator, tolerance and storage precision.
 * FP64 storage: plain CG, restarted from the true residual if the iterated one
 * met tol and the true one did not.  Any other storage (bcg_set_solver's
 * sloppy_prec): r, p, A p and the links in that storage and FP32 arithmetic,
 * the solution in FP64, and reliable updates as in Sec. 6 for one right-hand
 * side (every ru_delta drop of the relative residual and at convergence: the
 * update is folded into the FP64 solution, r = b - A x is recomputed with the
 * FP64 operator and the recurrence continues with the same search direction),
 * i.e. the double-single CG of Sec. 7.1.  stats->restarts counts the restarts
 * (FP64) or reliable updates (other storage).  Same arguments and returns as
 * bcg_solve with X0 = 0. */
int bcg_solve_cg(bcg_ctx *ctx, const void *B, void *X, int nrhs, bcg_stats *stats);

/* Pseudo-block CG, the prior work the paper contrasts with (Sec. 2): nrhs
 * independent CG recurrences advanced together, so that every application of
 * A serves all columns (each link read once per site for the whole block) while
 * every column keeps its own alpha_i, beta_i and Krylov space.  A column whose
 * iterated relative residual meets tol stops; when all have, the FP64 true
 * residuals are checked and the columns that miss restart from theirs.  Its
 * time against bcg_solve_cg isolates the gain of sharing the stencil, against
 * bcg_solve the gain of sharing the Krylov space.  FP64 storage only
 * (BCG_ERR_ARG otherwise).  stats->iters counts lockstep iterations (the
 * largest per-column count), stats->restarts the true-residual restarts.
 * Same arguments and returns as bcg_solve_cg. */
int bcg_solve_pseudo(bcg_ctx *ctx, const void *B, void *X, int nrhs, bcg_stats *stats);

/* s-step block CG, the extension Sec. 8 proposes so that a block solver needs
 * fewer than one reduction per iteration (Chronopoulos and Gear's s-step CG with
 * nrhs columns per direction).  Each outer iteration builds the basis
 * V = [R, p_1(A) R, ..., p_{s-1}(A) R] of s nrhs columns (p_j the Chebyshev
 * polynomials of the interval [lmin, lmax], two-term recurrence from A V_j),
 * reduces all of its inner products in one phase (V^H A V, V^H V and, against
 * the previous direction block P', (A P')^H V, P'^H A P', P'^H V), forms the
 * coefficients in one workgroup, then updates P = V + P' Bk (A-orthogonal to
 * P'), A P, X += P alpha and R -= A P alpha.  In exact arithmetic k outer
 * iterations give the iterate of k s block-CG iterations; in floating point the
 * basis loses conditioning as s grows and the iteration count rises.  The
 * iterated residual is tested at the top of each outer iteration; when it meets
 * tol the FP64 true residual is checked and, if a column misses, the recurrence
 * restarts from the true residual.  Storage follows bcg_set_solver's
 * sloppy_prec: FP64, or FP32 (the mixed precision of Sec. 6 carried over: V,
 * A V, P and A P stored in FP32 and the basis applied with the FP32 links in
 * FP32 arithmetic, while X, R, every Gram and the coefficients stay FP64, and a
 * reliable update replaces R by the FP64 true residual B - A X whenever the
 * largest iterated relative residual has dropped by ru_delta since the last
 * one, keeping the directions); 16-bit storage returns BCG_ERR_ARG.  tol,
 * max_iter (counted in s-steps, rounded down to whole outer iterations) and
 * ru_delta come from bcg_set_solver.
 *   s:    directions per outer iteration; s * nrhs <= 64 (BCG_ERR_ARG otherwise)
 *   lmin: lower end of the basis interval; <= 0 selects 4 m^2, the smallest
 *         possible eigenvalue of A
 *   lmax: upper end; <= 0 selects 1.1 times a 30-step power-iteration estimate
 *         of the largest eigenvalue from the first column (lmin < lmax required
 *         when both are given)
 * stats->iters counts s-steps (outer iterations times s), stats->restarts the
 * true-residual restarts, stats->reliable_updates the reliable updates.  Returns BCG_OK, BCG_ERR_NOT_CONVERGED or
 * BCG_ERR_BREAKDOWN (a direction Gram P^H A P not positive definite: the basis
 * lost rank; X holds the last iterate), or an argument / runtime error.  Same
 * vector arguments as bcg_solve with X0 = 0. */
int bcg_solve_sstep(bcg_ctx *ctx, const void *B, void *X, int nrhs, int s, double lmin, double lmax,
                    bcg_stats *stats);

/* Link force: the gradients w.r.t. the fat and long links of a loss L with
 * dL = -Re sum_i Lam_i^H dA X_i (X = A^{-1} B, Lam = A^{-1} dL/dX), in the
 * complex convention grad = dL/dRe + i dL/dIm and without projection:
 *   with Y_X = D_oe X, Y_L = D_oe Lam and, for a link W_mu(x) of hop length
 *   k (1 fat, 3 long), y = x + k mu:
 *   x even: grad W_mu(x) = +eta_mu(x) sum_i [ Lam_i(x) Y_X,i(y)^H + X_i(x) Y_L,i(y)^H ]
 *   x odd : grad W_mu(x) = -eta_mu(x) sum_i [ Y_X,i(x) Lam_i(y)^H + Y_L,i(x) X_i(y)^H ]
 * X, Lam: device [nrhs][V/2][3] even fields; grad_fat, grad_long: device
 * [4][V][3][3] complex128, overwritten (grad_long ignored and may be NULL for
 * the naive operator).  Stream-ordered. */
int bcg_link_force(bcg_ctx *ctx, const void *X, const void *Lam, int nrhs, void *grad_fat,
                   void *grad_long);

/* Progress callback: called on the host thread of bcg_solve / bcg_solve_cg each
 * time the solver reads its device state (every few to some tens of
 * iterations, and after each reliable update), with the iterations so far, the
 * reliable updates (solve_cg: true-residual restarts) and the current maximum
 * relative residual (iterated; the true one right after a reliable update).
 * fn = NULL turns it off.  The callback must not call into the context. */
typedef void (*bcg_monitor_fn)(void *user, int iters, int reliable_updates, double max_rel_res);
int bcg_set_monitor(bcg_ctx *ctx, bcg_monitor_fn fn, void *user);

/* Safeguards of the iteration in low storage precision.  The paper observes
 * that the double-half form of the solver breaks down and leaves more
 * frequent or adaptive reliable updates to future work (Sec. 8); these are
 * this library's versions of them.
 *   ru_window   > 0: also make a reliable update (Alg. 3) when the maximum
 *               relative iterated residual has not reached a new minimum for
 *               ru_window iterations (the iteration has stagnated, or its
 *               residual has drifted away from the true one); 0 = only the
 *               ru_delta rule of bcg_set_solver.  Default 100.
 *   stall_limit > 0: give up with BCG_ERR_NOT_CONVERGED after stall_limit
 *               reliable updates in a row whose true residual fails to halve
 *               the smallest maximum true relative residual seen so far (the
 *               start included); after such a stop, and after a breakdown, X
 *               holds the iterate with the smallest maximum true residual among
 *               those checked (a max_iter stop returns the current iterate).
 *               0 = never (and a breakdown returns the current iterate).
 *               Default 3.
 *   qr_passes   1: the initial and reliable-update thin QR is one CholQR
 *               (Alg. 2); 2: CholQR2 (Alg. 2 applied twice, the second pass on
 *               the Q of the first; C = C2 C1).  Default 1.
 * In exact arithmetic none of these changes the iterates: a reliable update
 * continues the recurrence (S = C^ C_k^{-1}) and CholQR2 returns the same
 * factors.  Returns BCG_ERR_ARG for negative values or qr_passes not 1 or 2. */
int bcg_set_stability(bcg_ctx *ctx, int ru_window, int stall_limit, int qr_passes);

/* Tuning options (launch shapes and kernel variants; results do not depend on
 * them beyond floating-point rounding order).  value 0 restores the default.
 *   BCG_OPT_HOP_TR        right-hand sides per lane in the hop (1, 2, 4, 8)
 *   BCG_OPT_HOP_TPB       lane groups per workgroup sharing sites (1, 2, 4)
 *   BCG_OPT_HOP_PIPELINE  1: two folded matrices in flight per loop trip, 2: one
 *   BCG_OPT_PASS_CPT      columns per lane in the streaming passes (1, 2, 4)
 *   BCG_OPT_FUSE_GRAM     1: Gram products fused into the epilogues of the hop
 *                         and the streaming passes (G = 4 m^2 P^H P + T^H T);
 *                         when the epilogue's Gram tile does not fit the LDS
 *                         budget for the chosen hop shape (e.g. FP64, N = 16
 *                         with two lane groups), the solver uses the separate
 *                         Gram kernels instead, with no error
 *   BCG_OPT_HOP_KERNEL    1: lane-split hop (the four lane groups of a wave take
 *                         one direction each for 16 sites), 2: site-parallel hop
 *                         (lane groups share sites, BCG_OPT_HOP_TPB), 3: lane-split
 *                         hop with two lane groups of 32 sites taking two
 *                         directions each; default by lattice size and storage
 *                         (3 in place of 1 below FP64 storage)
 *   BCG_OPT_GRAM_KERNEL   1: Gram products on the matrix cores (FP64 MFMA) for
 *                         N > 8, 2: on the vector ALUs
 *   BCG_OPT_SMALL_THREADS threads (64, 256, 1024) of the one-workgroup N x N
 *                         kernels, used when N^2 <= 4 x threads; 0 (default):
 *                         256 for N <= 16, else 1024
 *   BCG_OPT_SITE_ORDER    1: workgroups walk the lattice so that XCD x takes the
 *                         x-th eighth of every time slice and all XCDs sweep the
 *                         slices together, 2: plain lexicographic order
 *   BCG_OPT_PASS_KERNEL   1: passes A and B on the matrix cores (FP64 MFMA) for
 *                         16 < N <= 32 in FP32 / FP64 storage, pass A also for
 *                         32 < N <= 64 in FP64 storage, and both passes for
 *                         32 < N <= 64 in FP32 storage with FP32 MFMA for the FP32
 *                         products (FP64 MFMA for the X increment); otherwise vector
 *                         ALUs (pass B with its N x N coefficients staged in LDS);
 *                         2: vector kernels with LDS-staged coefficients (both
 *                         passes); 3: vector kernels reading the coefficients
 *                         with scalar loads
 *   BCG_OPT_GRAPH         1: the solver iterations run as replays of a captured
 *                         HIP graph of two iterations; 0 (default), 2: eager
 *                         launches (always eager while kernel profiling is on)
 *   BCG_OPT_HOP_SCHED     site-parallel hop: 1 static slab order; 2, 3, 4, 5:
 *                         per-XCD task queues (the workgroups of each XCD take
 *                         consecutive blocks of neighbouring lattice cells, then
 *                         help drain the other XCDs' queues) with 1, 2, 4 or 8
 *                         workgroups per CU in a persistent grid
 * Returns BCG_ERR_ARG for an unknown option. */
enum { BCG_OPT_HOP_TR = 0, BCG_OPT_HOP_TPB = 1, BCG_OPT_HOP_PIPELINE = 2, BCG_OPT_PASS_CPT = 3,
       BCG_OPT_FUSE_GRAM = 4, BCG_OPT_HOP_KERNEL = 5, BCG_OPT_GRAM_KERNEL = 6, BCG_OPT_SMALL_THREADS = 7,
       BCG_OPT_SITE_ORDER = 8, BCG_OPT_PASS_KERNEL = 9, BCG_OPT_GRAPH = 10, BCG_OPT_HOP_SCHED = 11,
       BCG_OPT_COUNT = 12 };
int bcg_set_option(bcg_ctx *ctx, int option, int value);

/* Per-kernel timing with HIP events on the context's stream.  mask: bit set of
 * BCG_K_* kernels to time (0 = off).  While on, each hop launch carries a start
 * and a stop event in its own dispatch (hipExtLaunchKernelGGL), which time the
 * kernel alone; the other classes, whose calls may launch several kernels, are
 * bracketed by two events recorded on the stream around the call.
 * bcg_kernel_time returns the number of timed launches and their summed
 * duration in milliseconds since the last bcg_profile_reset, after
 * synchronising the stream. */
enum {
    BCG_K_HOP_OE = 0, BCG_K_HOP_EO = 1, BCG_K_GRAM = 2, BCG_K_REDUCE = 3, BCG_K_SMALL = 4,
    BCG_K_PASS_A = 5, BCG_K_PASS_B = 6, BCG_K_CG_VEC = 7, BCG_K_CONVERT = 8, BCG_K_OTHER = 9,
    BCG_K_COUNT = 10
};
int bcg_set_profiling(bcg_ctx *ctx, unsigned mask);
int bcg_profile_reset(bcg_ctx *ctx);
int bcg_kernel_time(bcg_ctx *ctx, int kernel, long *launches, double *total_ms);

/* Message for the last error on ctx (static storage owned by the context;
 * valid until the next call on it).  ctx may be NULL for creation errors. */
const char *bcg_last_error(const bcg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* BCG_H */
