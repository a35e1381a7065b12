// C ABI of the block CG library: context, link loading, work buffers, the
// blockCGrQ driver loop (Alg. 1-3), the single right-hand-side CG baseline,
// the operator applications and the link force.
//
// The driver enqueues whole iterations without waiting: every iteration kernel
// first reads the device SolveState and does nothing once a single-workgroup
// N x N kernel has raised `halt` (convergence, a reliable-update trigger or a
// breakdown).  The host reads the state (one small device-to-host copy into
// pinned memory) only between chunks of iterations, sized from the observed
// convergence rate, and then carries out the reliable update (Alg. 3) or the
// final true-residual check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bcg.h"
#include "internal.h"

using namespace bcg;

namespace bcg {
thread_local LaunchTiming g_launch_timing;
}

namespace {

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct ProfEvent {
    int kid;
    hipEvent_t a, b;
};

}  // namespace

// Scratch of bcg_apply_noalloc: three regions (the input and the result in the
// internal layout, and the odd-parity intermediate), each of SCRATCH_REGION bytes,
// in a file-scope device array.  Every GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (kept per device in
// g_scratch, looked up by bcg_create).
constexpr size_t SCRATCH_REGION = (size_t)16 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[3 * SCRATCH_REGION];
static void* g_scratch[SCRATCH_MAX_DEVICES] = {};

struct bcg_ctx {
    Geom g{};
    int device = 0;
    int dims[4]{};
    int improved = 0;
    int nl = 8;
    long V = 0, Vh = 0;
    hipStream_t stream = nullptr;
    double mass = 0.0;
    double tol = 1e-10;
    int max_iter = 100000;
    Prec sloppy = Prec::FP64;
    double ru_delta = 0.1;
    int ru_window = 100;      // adaptive reliable-update trigger (bcg_set_stability)
    int stall_limit = 3;      // reliable updates in a row without progress before giving up
    int qr_passes = 1;        // 1: CholQR, 2: CholQR2 in the initial and reliable-update QR
    bool links = false;
    void* W64[2] = {nullptr, nullptr};
    void* Wsl[2] = {nullptr, nullptr};
    Prec wsl_prec = Prec::FP64;
    // device state
    SolveState* d_state = nullptr;
    SolveState* h_state = nullptr;  // pinned
    CgState* d_cg = nullptr;
    CgState* h_cg = nullptr;        // pinned
    PbState* d_pb = nullptr;
    PbState* h_pb = nullptr;        // pinned
    double2* mats = nullptr;        // small matrices, 10 x [64][64]
    double2* partials = nullptr;    // 3 x GRAM_BLOCKS x 64 x 64: general / T^H T / P^H P
    double2* part_tt = nullptr;
    double2* part_pp = nullptr;
    double* nparts = nullptr;       // NORM_BLOCKS x 64 norm partials, then the CG dot partials
    long dot_off = 0;               // offset of the CG dot partials in nparts
    double* d_vec = nullptr;        // bnorm[64], true_relres[64]
    int* d_flags = nullptr;         // [0] ru_skip, [64..127] pseudo-block restart flags
    int* hopq = nullptr;            // per-XCD task queues of the hop (16 ints, kept at zero between launches)
    int* h_flags = nullptr;         // pinned [64]
    double* h_vec = nullptr;        // pinned [128]
    Buf work[16];
    std::string err;
    // profiling
    unsigned prof_mask = 0;
    std::vector<ProfEvent> pending;
    std::vector<hipEvent_t> pool;
    long prof_n[BCG_K_COUNT]{};
    double prof_ms[BCG_K_COUNT]{};
    // tuning options (bcg_set_option), 0 = default
    int opt[BCG_OPT_COUNT]{};
    hipStream_t cap_stream = nullptr;  // graph capture of the iteration loop
    bcg_monitor_fn monitor = nullptr;   // progress callback (bcg_set_monitor)
    void* monitor_user = nullptr;
};

namespace {

// work buffer slots
enum { WB_B64, WB_Y, WB_X, WB_R64, WB_T64, WB_P0, WB_P1, WB_Q0, WB_Q1, WB_AP, WB_T, WB_A0, WB_A1, WB_A2, WB_A3,
       WB_YBEST };
// small matrix slots
enum { M_G, M_H, M_BETA, M_BETAC, M_C, M_CINV, M_SINV, M_SH, M_HR, M_ID, M_C2I, M_COUNT };

thread_local std::string g_create_err;

int fail(bcg_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return code;
}

#define HIPCK(call)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, BCG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define RETCK(call)                      \
    do {                                 \
        int r_ = (call);                 \
        if (r_ != BCG_OK) return r_;     \
    } while (0)

int ensure(bcg_ctx* ctx, int slot, size_t bytes) {
    Buf& b = ctx->work[slot];
    if (b.bytes >= bytes) return BCG_OK;
    if (b.p) {
        HIPCK(hipStreamSynchronize(ctx->stream));
        HIPCK(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return fail(ctx, BCG_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
    return BCG_OK;
}

void* W(bcg_ctx* ctx, int slot) { return ctx->work[slot].p; }
double2* Wd(bcg_ctx* ctx, int slot) { return (double2*)ctx->work[slot].p; }
double2* M(bcg_ctx* ctx, int m) { return ctx->mats + (size_t)m * MAXN * MAXN; }

// ---- profiling -----------------------------------------------------------------------------
hipEvent_t prof_event(bcg_ctx* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// two instantiated graphs (one per starting ping-pong buffer), destroyed with the
// solve once the stream they were launched on has drained
struct GraphPair {
    hipGraph_t g[2] = {nullptr, nullptr};
    hipGraphExec_t x[2] = {nullptr, nullptr};
    hipStream_t launched_on = nullptr;
    ~GraphPair() {
        if (x[0] || x[1]) (void)hipStreamSynchronize(launched_on);
        for (int i = 0; i < 2; ++i) {
            if (x[i]) (void)hipGraphExecDestroy(x[i]);
            if (g[i]) (void)hipGraphDestroy(g[i]);
        }
    }
};

// Per-kernel timing.  A scope that makes several launches is bracketed by two
// events on the stream.  A single-launch scope (the hops) hands its events to the
// launch itself (BCG_TIMED_LAUNCH), so that they time the dispatch and not the
// event packets and cache write-back around it.
struct Prof {
    bcg_ctx* ctx;
    int kid;
    hipEvent_t a = nullptr, b1 = nullptr;
    Prof(bcg_ctx* c, int k, bool single_launch = false) : ctx(c), kid(k) {
        if (ctx->prof_mask & (1u << kid)) {
            a = prof_event(ctx);
            if (a && single_launch) {
                b1 = prof_event(ctx);
                if (b1) {
                    g_launch_timing = LaunchTiming{a, b1, false};
                    return;
                }
            }
            if (a) (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~Prof() {
        if (b1) {
            const bool used = g_launch_timing.used;
            g_launch_timing = LaunchTiming{};
            if (used) {
                ctx->pending.push_back(ProfEvent{kid, a, b1});
            } else {
                ctx->pool.push_back(a);
                ctx->pool.push_back(b1);
            }
            return;
        }
        if (a) {
            hipEvent_t b = prof_event(ctx);
            if (b) {
                (void)hipEventRecord(b, ctx->stream);
                ctx->pending.push_back(ProfEvent{kid, a, b});
            } else {
                ctx->pool.push_back(a);
            }
        }
    }
};

void prof_collect(bcg_ctx* ctx) {
    for (auto& pe : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            ctx->prof_n[pe.kid] += 1;
            ctx->prof_ms[pe.kid] += ms;
        }
        ctx->pool.push_back(pe.a);
        ctx->pool.push_back(pe.b);
    }
    ctx->pending.clear();
}

int sync(bcg_ctx* ctx) {
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (!ctx->pending.empty()) prof_collect(ctx);
    return BCG_OK;
}

// ---- argument checks -----------------------------------------------------------------------
int check_nrhs(bcg_ctx* ctx, int nrhs) {
    if (nrhs < 1 || nrhs > BCG_MAX_RHS)
        return fail(ctx, BCG_ERR_ARG, "nrhs must be in [1, 64], got " + std::to_string(nrhs));
    return BCG_OK;
}

int check_ready(bcg_ctx* ctx) {
    if (!ctx->links) return fail(ctx, BCG_ERR_STATE, "links not loaded (call bcg_load_links first)");
    return BCG_OK;
}

// ---- building blocks -----------------------------------------------------------------------
long nvec(bcg_ctx* ctx, int N) { return (long)N * 3 * ctx->Vh; }

bool gram_mfma(bcg_ctx* ctx) { return ctx->opt[BCG_OPT_GRAM_KERNEL] != 2; }

// 64-site blocks per time slice for the XCD order of the streaming passes
int bps64(bcg_ctx* ctx) { return blocks_per_slice(ctx->g, 64); }

HopShape shape(bcg_ctx* ctx, Prec p, int N, bool fused) {
    return hop_shape(p, N, ctx->opt[BCG_OPT_HOP_TR], ctx->opt[BCG_OPT_HOP_TPB], ctx->opt[BCG_OPT_HOP_PIPELINE],
                     ctx->opt[BCG_OPT_HOP_KERNEL], ctx->g, fused, ctx->opt[BCG_OPT_HOP_SCHED]);
}

// The CG path's hop with the fused p^H A p: one column on the lane-split kernel, with
// the run length (16 or 32 sites) that the one-column shape picks; it writes one dot
// partial per workgroup of four runs.
HopShape dot_shape(bcg_ctx* ctx, Prec p) {
    const HopShape h = shape(ctx, p, 1, false);
    return HopShape{1, 1, h.pf, h.split == 2 ? 2 : 1};
}
int dot_parts(bcg_ctx* ctx, Prec p) {
    const long sites = dot_shape(ctx, p).split == 2 ? 128 : 64;
    return (int)((ctx->Vh + sites - 1) / sites);
}

int hop(bcg_ctx* ctx, Prec p, int out_parity, const void* in, void* out, const void* ctr, int N,
        int epi, const int* halt, double* dot = nullptr, double2* partials = nullptr) {
    const void* Wp = (p == Prec::FP64) ? ctx->W64[out_parity] : ctx->Wsl[out_parity];
    HopShape h = shape(ctx, p, N, partials != nullptr);
    if (epi == EPI_MASS_DOT_) h = dot_shape(ctx, p);
    Prof pr(ctx, out_parity == 1 ? BCG_K_HOP_OE : BCG_K_HOP_EO, true);
    HIPCK(launch_hop(p, ctx->nl, Wp, in, out, ctr, 4.0 * ctx->mass * ctx->mass, N, ctx->g,
                     out_parity, epi, h, halt, dot, partials, ctx->hopq, ctx->stream));
    return BCG_OK;
}

// the fused Gram epilogues fit in LDS for this precision and block size
// The fused epilogues save one read of a block vector per Gram but keep a Gram
// accumulator live through the streaming loop (lower occupancy); measured slower
// than the separate Gram kernels on MI355X, so they are opt-in (BCG_OPT_FUSE_GRAM).
bool fused_ok(bcg_ctx* ctx, Prec p, int N) {
    if (!ctx->opt[BCG_OPT_FUSE_GRAM]) return false;
    return hop_tile_bytes(p, N, shape(ctx, p, N, true)) > 0 && fused_tile_bytes(p, N) > 0;
}

int reduce(bcg_ctx* ctx, const double2* pa, int na, const double2* pb, int nb, double alpha, int N,
           double2* out, const int* halt) {
    Prof pr(ctx, BCG_K_REDUCE);
    HIPCK(launch_gram_reduce(pa, na, pb, nb, alpha, N, out, halt, ctx->stream));
    return BCG_OK;
}

// out = A in, FP64, internal layout; tmp: odd-parity scratch
int apply64(bcg_ctx* ctx, const void* in, void* out, void* tmp, int N, const int* halt) {
    RETCK(hop(ctx, Prec::FP64, 1, in, tmp, nullptr, N, EPI_PLAIN_, halt));
    RETCK(hop(ctx, Prec::FP64, 0, tmp, out, in, N, EPI_MASS_, halt));
    return BCG_OK;
}

// partials of A^H B into part (count gram_parts(N, Vh, gram_mfma(ctx)))
int gram_partials(bcg_ctx* ctx, Prec p, const void* A, const void* B, int N, double2* part, const int* halt) {
    Prof pr(ctx, BCG_K_GRAM);
    HIPCK(launch_gram(p, A, B, N, (int)ctx->Vh, part, halt, gram_mfma(ctx), ctx->stream));
    return BCG_OK;
}

// out = A^H B  (N x N, FP64, leading dimension 64) for a Hermitian A^H B (the
// matrix-core kernel forms the upper tiles only)
int gram(bcg_ctx* ctx, Prec p, const void* A, const void* B, int N, double2* out, const int* halt) {
    RETCK(gram_partials(ctx, p, A, B, N, ctx->partials, halt));
    return reduce(ctx, ctx->partials, gram_parts(N, (int)ctx->Vh, gram_mfma(ctx)), nullptr, 0, 0.0, N, out, halt);
}

// out = A^H B for any A, B (the vector-ALU Gram, which forms every tile)
int gram_general(bcg_ctx* ctx, Prec p, const void* A, const void* B, int N, double2* out) {
    {
        Prof pr(ctx, BCG_K_GRAM);
        HIPCK(launch_gram(p, A, B, N, (int)ctx->Vh, ctx->partials, nullptr, false, ctx->stream));
    }
    return reduce(ctx, ctx->partials, gram_parts(N, (int)ctx->Vh, false), nullptr, 0, 0.0, N, out, nullptr);
}

int colnorms(bcg_ctx* ctx, const double2* V, int N, double* out) {
    Prof pr(ctx, BCG_K_OTHER);
    HIPCK(launch_colnorm2(V, N, (int)ctx->Vh, ctx->nparts, ctx->stream));
    HIPCK(launch_colnorm_reduce(ctx->nparts, N, (int)ctx->Vh, out, 1, ctx->stream));
    return BCG_OK;
}

int read_state(bcg_ctx* ctx) {
    HIPCK(hipMemcpyAsync(ctx->h_state, ctx->d_state, sizeof(SolveState), hipMemcpyDeviceToHost,
                         ctx->stream));
    return sync(ctx);
}

int alloc_solve(bcg_ctx* ctx, int N, Prec ps) {
    const size_t n64 = (size_t)nvec(ctx, N) * 16, nsl = store_bytes(ps, N, 3, ctx->Vh);
    for (int s : {WB_B64, WB_Y, WB_X, WB_R64, WB_T64}) RETCK(ensure(ctx, s, n64));
    for (int s : {WB_P0, WB_P1, WB_Q0, WB_Q1, WB_AP, WB_T}) RETCK(ensure(ctx, s, nsl));
    return BCG_OK;
}

int ensure_sloppy_links(bcg_ctx* ctx, Prec ps) {
    if (ps == Prec::FP64) return BCG_OK;
    if (ctx->Wsl[0] && ctx->wsl_prec == ps) return BCG_OK;
    for (int p = 0; p < 2; ++p) {
        if (ctx->Wsl[p]) {
            HIPCK(hipStreamSynchronize(ctx->stream));
            HIPCK(hipFree(ctx->Wsl[p]));
            ctx->Wsl[p] = nullptr;
        }
        if (hipMalloc(&ctx->Wsl[p], store_bytes(ps, ctx->nl, 9, ctx->Vh)) != hipSuccess) {
            ctx->Wsl[p] = nullptr;
            return fail(ctx, BCG_ERR_NOMEM, "sloppy link allocation failed");
        }
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(links_from64(ps, ctx->W64[p], ctx->Wsl[p], ctx->nl, ctx->Vh, ctx->stream));
    }
    ctx->wsl_prec = ps;
    return BCG_OK;
}

void fill_stats(bcg_stats* st, int iters, int rus, int status, int restarts, double secs,
                const double* tr, int N) {
    if (!st) return;
    st->iters = iters;
    st->reliable_updates = rus;
    st->status = status;
    st->restarts = restarts;
    st->seconds = secs;
    double mx = 0.0;
    for (int i = 0; i < N; ++i) mx = std::fmax(mx, tr[i]);
    st->max_true_rel_res = mx;
    if (st->true_rel_res)
        for (int i = 0; i < N; ++i) st->true_rel_res[i] = tr[i];
}

// One CG solve per column with the vectors r, p, Ap and the links in the sloppy
// storage and reliable updates in FP64 (Sec. 6's scheme for one right-hand side:
// the double-single baseline of Sec. 7.1).  x holds the FP64 update since the last
// reliable update and y the solution; a reliable update (every ru_delta drop of the
// relative residual, and at convergence) folds x into y, recomputes r = b - A y with
// the FP64 operator and continues with beta = ||r_true||^2 / ||r_prev||^2 and the
// same search direction (CG's form of S = C^ C_k^{-1}).
int cg_mixed(bcg_ctx* ctx, const double2* B64, double2* Ys, const double* bn, int N, double* tr,
             int* total_iters, int* n_ru) {
    const Prec ps = ctx->sloppy;
    const int Vh = (int)ctx->Vh;
    const long n1 = 3L * Vh;
    hipStream_t s = ctx->stream;
    RETCK(ensure_sloppy_links(ctx, ps));
    const size_t b1 = store_bytes(ps, 1, 3, ctx->Vh);
    for (int slot : {WB_A0, WB_A1, WB_A2, WB_A3}) RETCK(ensure(ctx, slot, b1));
    void *r = W(ctx, WB_A0), *p = W(ctx, WB_A1), *Ap = W(ctx, WB_A2), *t = W(ctx, WB_A3);
    double2 *x = Wd(ctx, WB_X), *R64 = Wd(ctx, WB_R64), *T64 = Wd(ctx, WB_T64);
    CgState* st = ctx->d_cg;
    const int* halt = &st->halt;
    double* dot = ctx->nparts + ctx->dot_off;
    const int nparts = dot_parts(ctx, ps);
    HIPCK(launch_identity(M(ctx, M_ID), 1, s));
    int status = BCG_OK;
    for (int i = 0; i < N; ++i) {
        const double2* b = B64 + (long)i * n1;
        double2* y = Ys + (long)i * n1;
        HIPCK(launch_zero(x, n1 * 16, s));
        HIPCK(launch_zero(y, n1 * 16, s));
        HIPCK(launch_bmul(Prec::FP64, b, ps, nullptr, r, M(ctx, M_ID), 1, Vh, nullptr, s));
        HIPCK(launch_copy(r, p, (long)b1, s));
        HIPCK(launch_colnorm2(b, 1, Vh, ctx->nparts, s));
        HIPCK(launch_cg_init(ctx->nparts, Vh, st, ctx->tol, 0, s));
        HIPCK(launch_cg_set_ru(st, ctx->ru_delta, s));
        double rate = -0.02, last_log = 0.0;
        int last_it = 0, col_iters = 0;
        tr[i] = 1.0;
        for (;;) {
            HIPCK(hipMemcpyAsync(ctx->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            const CgState hc = *ctx->h_cg;
            col_iters = hc.iters;
            if (ctx->monitor) ctx->monitor(ctx->monitor_user, *total_iters + hc.iters, *n_ru, hc.relres);
            if (hc.halt && hc.reason == HALT_BREAKDOWN_G) {
                status = BCG_ERR_BREAKDOWN;
                fail(ctx, status, "CG breakdown: p^H A p <= 0");
                break;
            }
            if (hc.halt) {
                // reliable update (also the convergence check on the true residual)
                HIPCK(launch_fold_x(y, x, n1, s));
                RETCK(apply64(ctx, y, R64, T64, 1, nullptr));
                HIPCK(launch_residual(b, R64, n1, s));
                HIPCK(launch_colnorm2(R64, 1, Vh, ctx->nparts, s));
                HIPCK(launch_cg_ru(ctx->nparts, Vh, st, hc.reason == HALT_CONVERGED ? 1 : 0, s));
                HIPCK(hipMemcpyAsync(ctx->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
                RETCK(sync(ctx));
                tr[i] = ctx->h_cg->relres;
                if (ctx->h_cg->reason == HALT_DONE) break;
                *n_ru += 1;
                HIPCK(launch_bmul(Prec::FP64, R64, ps, nullptr, r, M(ctx, M_ID), 1, Vh, nullptr, s));
                HIPCK(launch_cg_update2_s(ps, p, r, Vh, st, s));
                last_log = std::log(std::fmax(ctx->h_cg->relres, 1e-300));
                last_it = ctx->h_cg->iters;
                if (ctx->h_cg->iters >= ctx->max_iter) {
                    status = BCG_ERR_NOT_CONVERGED;
                    fail(ctx, status, "max_iter reached in CG");
                    break;
                }
                continue;
            }
            if (hc.iters >= ctx->max_iter) {
                status = BCG_ERR_NOT_CONVERGED;
                fail(ctx, status, "max_iter reached in CG");
                break;
            }
            const double lg = std::log(std::fmax(hc.relres, 1e-300));
            if (hc.iters > last_it) {
                const double rr = (lg - last_log) / (hc.iters - last_it);
                if (rr < 0) rate = rr;
            }
            last_log = lg;
            last_it = hc.iters;
            double target = std::log(ctx->tol);
            if (ctx->ru_delta > 0.0) target = std::fmax(target, std::log(ctx->ru_delta * hc.rho_ru));
            int est = (int)std::ceil((target - lg) / (rate < -1e-6 ? rate : -1e-6));
            int chunk = est < 2 ? 2 : (est > 64 ? 64 : est);
            if (chunk > ctx->max_iter - hc.iters) chunk = ctx->max_iter - hc.iters;
            for (int k = 0; k < chunk; ++k) {
                RETCK(hop(ctx, ps, 1, p, t, nullptr, 1, EPI_PLAIN_, halt));
                RETCK(hop(ctx, ps, 0, t, Ap, p, 1, EPI_MASS_DOT_, halt, dot));
                Prof pr(ctx, BCG_K_CG_VEC);
                HIPCK(launch_cg_alpha(dot, nparts, st, s));
                HIPCK(launch_cg_update1_s(ps, x, r, p, Ap, Vh, ctx->nparts, st, s));
                HIPCK(launch_cg_beta(ctx->nparts, Vh, st, s));
                HIPCK(launch_cg_update2_s(ps, p, r, Vh, st, s));
            }
        }
        *total_iters += col_iters;
        if (status != BCG_OK) {
            // the column's current solution: fold the pending update and measure it
            HIPCK(launch_fold_x(y, x, n1, s));
            RETCK(apply64(ctx, y, R64, T64, 1, nullptr));
            HIPCK(launch_residual(b, R64, n1, s));
            HIPCK(launch_colnorm2(R64, 1, Vh, ctx->nparts, s));
            HIPCK(launch_colnorm_reduce(ctx->nparts, 1, Vh, ctx->d_vec + MAXN, 1, s));
            HIPCK(hipMemcpyAsync(ctx->h_vec, ctx->d_vec + MAXN, sizeof(double), hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            tr[i] = ctx->h_vec[0] / bn[i];
            for (int j = i + 1; j < N; ++j) {
                tr[j] = 1.0;
                HIPCK(launch_zero(Ys + (long)j * n1, n1 * 16, s));
            }
            break;
        }
    }
    return status;
}

}  // namespace

// =============================================================================================
extern "C" {

int bcg_create(bcg_ctx** out, const int dims[4], int improved, void* hip_stream) {
    bcg_ctx* ctx = nullptr;
    if (!out || !dims) return fail(nullptr, BCG_ERR_ARG, "null argument");
    *out = nullptr;
    long V = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || dims[d] % 2)
            return fail(nullptr, BCG_ERR_ARG, "every lattice extent must be even and >= 2");
        V *= dims[d];
    }
    if (V >= (1L << 30)) return fail(nullptr, BCG_ERR_ARG, "lattice too large for 32-bit site indices");
    if (improved != 0 && improved != 1) return fail(nullptr, BCG_ERR_ARG, "improved must be 0 or 1");
    int dev = 0;
    {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail(nullptr, BCG_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
        if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(nullptr, BCG_ERR_ARG, "device index out of range");
        // kernel attributes (dynamic LDS above the default limit), once per device
        static bool setup[SCRATCH_MAX_DEVICES] = {};
        if (!setup[dev]) {
            if ((e = small_setup()) != hipSuccess || (e = blas_setup()) != hipSuccess)
                return fail(nullptr, BCG_ERR_HIP, std::string("kernel setup: ") + hipGetErrorString(e));
            setup[dev] = true;
        }
        if (!g_scratch[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(nullptr, BCG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            g_scratch[dev] = p;
        }
    }
    ctx = new bcg_ctx();
    ctx->device = dev;
    for (int d = 0; d < 4; ++d) {
        ctx->dims[d] = dims[d];
        ctx->g.L[d] = dims[d];
    }
    ctx->V = V;
    ctx->Vh = V / 2;
    ctx->g.Vh = (int)ctx->Vh;
    ctx->g.slab = 1;
    ctx->improved = improved;
    ctx->nl = improved ? 16 : 8;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->dot_off = (long)NORM_BLOCKS * MAXN;
    bool ok = hipMalloc(&ctx->d_state, sizeof(SolveState)) == hipSuccess &&
              hipHostMalloc(&ctx->h_state, sizeof(SolveState)) == hipSuccess &&
              hipMalloc(&ctx->d_cg, sizeof(CgState)) == hipSuccess &&
              hipHostMalloc(&ctx->h_cg, sizeof(CgState)) == hipSuccess &&
              hipMalloc(&ctx->mats, sizeof(double2) * M_COUNT * MAXN * MAXN) == hipSuccess &&
              hipMalloc(&ctx->partials, sizeof(double2) * 3 * GRAM_BLOCKS * MAXN * MAXN) == hipSuccess &&
              hipMalloc(&ctx->nparts, sizeof(double) * ((long)NORM_BLOCKS * MAXN + hop_dot_blocks(ctx->g) + 1)) == hipSuccess &&
              hipMalloc(&ctx->d_vec, sizeof(double) * 4 * MAXN) == hipSuccess &&
              hipMalloc(&ctx->d_flags, sizeof(int) * 128) == hipSuccess &&
              hipMalloc(&ctx->d_pb, sizeof(PbState)) == hipSuccess &&
              hipMalloc(&ctx->hopq, sizeof(int) * 16) == hipSuccess &&
              hipMemset(ctx->hopq, 0, sizeof(int) * 16) == hipSuccess &&
              hipHostMalloc(&ctx->h_pb, sizeof(PbState)) == hipSuccess &&
              hipHostMalloc(&ctx->h_flags, sizeof(int) * MAXN) == hipSuccess &&
              hipHostMalloc(&ctx->h_vec, sizeof(double) * 4 * MAXN) == hipSuccess;
    if (!ok) {
        bcg_destroy(ctx);
        return fail(nullptr, BCG_ERR_NOMEM, "context allocation failed");
    }
    ctx->part_tt = ctx->partials + (size_t)GRAM_BLOCKS * MAXN * MAXN;
    ctx->part_pp = ctx->partials + (size_t)2 * GRAM_BLOCKS * MAXN * MAXN;
    *out = ctx;
    return BCG_OK;
}

int bcg_destroy(bcg_ctx* ctx) {
    if (!ctx) return BCG_OK;
    (void)hipStreamSynchronize(ctx->stream);
    prof_collect(ctx);
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    for (auto& b : ctx->work)
        if (b.p) (void)hipFree(b.p);
    for (int p = 0; p < 2; ++p) {
        if (ctx->W64[p]) (void)hipFree(ctx->W64[p]);
        if (ctx->Wsl[p]) (void)hipFree(ctx->Wsl[p]);
    }
    if (ctx->d_state) (void)hipFree(ctx->d_state);
    if (ctx->h_state) (void)hipHostFree(ctx->h_state);
    if (ctx->d_cg) (void)hipFree(ctx->d_cg);
    if (ctx->h_cg) (void)hipHostFree(ctx->h_cg);
    if (ctx->mats) (void)hipFree(ctx->mats);
    if (ctx->partials) (void)hipFree(ctx->partials);
    if (ctx->nparts) (void)hipFree(ctx->nparts);
    if (ctx->d_vec) (void)hipFree(ctx->d_vec);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->d_pb) (void)hipFree(ctx->d_pb);
    if (ctx->hopq) (void)hipFree(ctx->hopq);
    if (ctx->h_pb) (void)hipHostFree(ctx->h_pb);
    if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
    if (ctx->h_vec) (void)hipHostFree(ctx->h_vec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return BCG_OK;
}

int bcg_load_links(bcg_ctx* ctx, const void* fat, const void* lng, int on_device) {
    if (!ctx) return BCG_ERR_ARG;
    if (!fat) return fail(ctx, BCG_ERR_ARG, "fat links are required");
    if ((lng != nullptr) != (ctx->improved != 0))
        return fail(ctx, BCG_ERR_ARG, "long links must be given iff the context is improved");
    const size_t bytes = (size_t)4 * ctx->V * 9 * 16;
    const void* dfat = fat;
    const void* dlng = lng;
    void* tmp = nullptr;
    if (!on_device) {
        const size_t tot = bytes * (ctx->improved ? 2 : 1);
        if (hipMalloc(&tmp, tot) != hipSuccess) return fail(ctx, BCG_ERR_NOMEM, "link staging allocation failed");
        HIPCK(hipMemcpyAsync(tmp, fat, bytes, hipMemcpyHostToDevice, ctx->stream));
        dfat = tmp;
        if (ctx->improved) {
            HIPCK(hipMemcpyAsync((char*)tmp + bytes, lng, bytes, hipMemcpyHostToDevice, ctx->stream));
            dlng = (char*)tmp + bytes;
        }
    }
    const size_t wbytes = (size_t)ctx->nl * 9 * ctx->Vh * 16;
    for (int p = 0; p < 2; ++p) {
        if (!ctx->W64[p] && hipMalloc(&ctx->W64[p], wbytes) != hipSuccess) {
            if (tmp) (void)hipFree(tmp);
            return fail(ctx, BCG_ERR_NOMEM, "link allocation failed");
        }
        HIPCK(pack_links(dfat, dlng, ctx->W64[p], ctx->g, p, ctx->nl, ctx->stream));
    }
    ctx->wsl_prec = Prec::FP64;   // sloppy copies are rebuilt from the new links on demand
    if (ctx->Wsl[0]) {
        (void)hipFree(ctx->Wsl[0]);
        (void)hipFree(ctx->Wsl[1]);
        ctx->Wsl[0] = ctx->Wsl[1] = nullptr;
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (tmp) (void)hipFree(tmp);
    ctx->links = true;
    return BCG_OK;
}

int bcg_set_mass(bcg_ctx* ctx, double m) {
    if (!ctx) return BCG_ERR_ARG;
    if (!std::isfinite(m)) return fail(ctx, BCG_ERR_ARG, "mass must be finite");
    ctx->mass = m;
    return BCG_OK;
}

int bcg_set_solver(bcg_ctx* ctx, double tol, int max_iter, int sloppy_prec, double ru_delta) {
    if (!ctx) return BCG_ERR_ARG;
    if (!(tol > 0.0) || !(tol < 1.0)) return fail(ctx, BCG_ERR_ARG, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(ctx, BCG_ERR_ARG, "max_iter must be >= 1");
    if (sloppy_prec < 0 || sloppy_prec > 4) return fail(ctx, BCG_ERR_ARG, "unknown precision");
    if (!(ru_delta >= 0.0) || !(ru_delta < 1.0)) return fail(ctx, BCG_ERR_ARG, "ru_delta must be in [0, 1)");
    ctx->tol = tol;
    ctx->max_iter = max_iter;
    ctx->sloppy = (Prec)sloppy_prec;
    ctx->ru_delta = ru_delta;
    return BCG_OK;
}

int bcg_apply(bcg_ctx* ctx, const void* in, void* out, int nrhs) {
    if (!ctx) return BCG_ERR_ARG;
    if (!in || !out) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const size_t b = (size_t)nvec(ctx, nrhs) * 16;
    RETCK(ensure(ctx, WB_A0, b));
    RETCK(ensure(ctx, WB_A1, b));
    RETCK(ensure(ctx, WB_A2, b));
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)in, Wd(ctx, WB_A0), nrhs, (int)ctx->Vh, ctx->stream));
    }
    RETCK(apply64(ctx, W(ctx, WB_A0), W(ctx, WB_A1), W(ctx, WB_A2), nrhs, nullptr));
    Prof pr(ctx, BCG_K_CONVERT);
    HIPCK(launch_int_to_canon(Wd(ctx, WB_A1), (double2*)out, nrhs, (int)ctx->Vh, ctx->stream));
    return BCG_OK;
}

int bcg_apply_noalloc(bcg_ctx* ctx, const void* in, void* out, int nrhs) {
    if (!ctx) return BCG_ERR_ARG;
    if (!in || !out) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const size_t b = (size_t)nvec(ctx, nrhs) * 16;
    if (b > SCRATCH_REGION)
        return fail(ctx, BCG_ERR_ARG, "bcg_apply_noalloc: nrhs * V/2 * 48 bytes = " + std::to_string(b) +
                                          " exceeds the scratch region of " + std::to_string(SCRATCH_REGION) +
                                          " bytes (nrhs * V/2 <= 349525); use bcg_apply");
    char* base = (char*)g_scratch[ctx->device];
    if (!base) return fail(ctx, BCG_ERR_STATE, "scratch address not set for this device");
    double2* A0 = (double2*)base;
    double2* A1 = (double2*)(base + SCRATCH_REGION);
    double2* A2 = (double2*)(base + 2 * SCRATCH_REGION);
    // no kernel timing here: its events would be created on demand
    const unsigned mask = ctx->prof_mask;
    ctx->prof_mask = 0;
    int rc = BCG_OK;
    hipError_t e = launch_canon_to_int((const double2*)in, A0, nrhs, (int)ctx->Vh, ctx->stream);
    if (e == hipSuccess) {
        rc = apply64(ctx, A0, A1, A2, nrhs, nullptr);
        if (rc == BCG_OK) e = launch_int_to_canon(A1, (double2*)out, nrhs, (int)ctx->Vh, ctx->stream);
    }
    ctx->prof_mask = mask;
    if (rc != BCG_OK) return rc;
    if (e != hipSuccess) return fail(ctx, BCG_ERR_HIP, std::string("bcg_apply_noalloc: ") + hipGetErrorString(e));
    return BCG_OK;
}

int bcg_apply_prec(bcg_ctx* ctx, int prec, const void* in, void* out, int nrhs) {
    if (!ctx) return BCG_ERR_ARG;
    if (!in || !out) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    if (prec < 0 || prec > 4) return fail(ctx, BCG_ERR_ARG, "unknown precision");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const Prec ps = (Prec)prec;
    if (ps == Prec::FP64) return bcg_apply(ctx, in, out, nrhs);
    RETCK(alloc_solve(ctx, nrhs, ps));
    RETCK(ensure_sloppy_links(ctx, ps));
    const int Vh = (int)ctx->Vh;
    hipStream_t s = ctx->stream;
    double2* I64 = Wd(ctx, WB_B64);
    void *P = W(ctx, WB_P0), *T = W(ctx, WB_T), *AP = W(ctx, WB_AP);
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)in, I64, nrhs, Vh, s));
        HIPCK(launch_identity(M(ctx, M_ID), nrhs, s));
        HIPCK(launch_bmul(Prec::FP64, I64, ps, nullptr, P, M(ctx, M_ID), nrhs, Vh, nullptr, s));
    }
    RETCK(hop(ctx, ps, 1, P, T, nullptr, nrhs, EPI_PLAIN_, nullptr));
    RETCK(hop(ctx, ps, 0, T, AP, P, nrhs, EPI_MASS_, nullptr));
    Prof pr(ctx, BCG_K_CONVERT);
    HIPCK(launch_bmul(ps, AP, Prec::FP64, nullptr, I64, M(ctx, M_ID), nrhs, Vh, nullptr, s));
    HIPCK(launch_int_to_canon(I64, (double2*)out, nrhs, Vh, s));
    return BCG_OK;
}

int bcg_hop(bcg_ctx* ctx, int out_parity, const void* in, void* out, int nrhs) {
    if (!ctx) return BCG_ERR_ARG;
    if (!in || !out) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    if (out_parity != 0 && out_parity != 1) return fail(ctx, BCG_ERR_ARG, "out_parity must be 0 or 1");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const size_t b = (size_t)nvec(ctx, nrhs) * 16;
    RETCK(ensure(ctx, WB_A0, b));
    RETCK(ensure(ctx, WB_A1, b));
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)in, Wd(ctx, WB_A0), nrhs, (int)ctx->Vh, ctx->stream));
    }
    RETCK(hop(ctx, Prec::FP64, out_parity, W(ctx, WB_A0), W(ctx, WB_A1), nullptr, nrhs, EPI_PLAIN_, nullptr));
    Prof pr(ctx, BCG_K_CONVERT);
    HIPCK(launch_int_to_canon(Wd(ctx, WB_A1), (double2*)out, nrhs, (int)ctx->Vh, ctx->stream));
    return BCG_OK;
}

int bcg_link_force(bcg_ctx* ctx, const void* X, const void* Lam, int nrhs, void* grad_fat,
                   void* grad_long) {
    if (!ctx) return BCG_ERR_ARG;
    if (!X || !Lam || !grad_fat || (ctx->improved && !grad_long))
        return fail(ctx, BCG_ERR_ARG, "null pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const size_t b = (size_t)nvec(ctx, nrhs) * 16;
    for (int s : {WB_A0, WB_A1, WB_A2, WB_A3}) RETCK(ensure(ctx, s, b));
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)X, Wd(ctx, WB_A0), nrhs, (int)ctx->Vh, ctx->stream));
        HIPCK(launch_canon_to_int((const double2*)Lam, Wd(ctx, WB_A1), nrhs, (int)ctx->Vh, ctx->stream));
    }
    RETCK(hop(ctx, Prec::FP64, 1, W(ctx, WB_A0), W(ctx, WB_A2), nullptr, nrhs, EPI_PLAIN_, nullptr));
    RETCK(hop(ctx, Prec::FP64, 1, W(ctx, WB_A1), W(ctx, WB_A3), nullptr, nrhs, EPI_PLAIN_, nullptr));
    Prof pr(ctx, BCG_K_OTHER);
    HIPCK(launch_link_force(Wd(ctx, WB_A0), Wd(ctx, WB_A1), Wd(ctx, WB_A2), Wd(ctx, WB_A3), nrhs,
                            ctx->g, ctx->improved, (double2*)grad_fat, (double2*)grad_long,
                            ctx->stream));
    return BCG_OK;
}

// ---------------------------------------------------------------------------------------------
// blockCGrQ
// ---------------------------------------------------------------------------------------------
int bcg_solve(bcg_ctx* ctx, const void* B, void* Xout, int nrhs, int use_guess, bcg_stats* stats) {
    if (!ctx) return BCG_ERR_ARG;
    if (!B || !Xout) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const auto t0 = std::chrono::steady_clock::now();
    const int N = nrhs;
    const Prec ps = ctx->sloppy;
    RETCK(alloc_solve(ctx, N, ps));
    if (ctx->stall_limit > 0) RETCK(ensure(ctx, WB_YBEST, (size_t)nvec(ctx, N) * 16));
    RETCK(ensure_sloppy_links(ctx, ps));
    const int Vh = (int)ctx->Vh;
    const long n = nvec(ctx, N);
    hipStream_t s = ctx->stream;
    SolveState* st = ctx->d_state;
    const int* halt = &st->halt;
    double* d_bnorm = ctx->d_vec;
    double* d_true = ctx->d_vec + MAXN;
    int* ru_skip = ctx->d_flags;
    double2 *B64 = Wd(ctx, WB_B64), *Y = Wd(ctx, WB_Y), *X = Wd(ctx, WB_X), *R64 = Wd(ctx, WB_R64),
            *T64 = Wd(ctx, WB_T64);
    void* Pb[2] = {W(ctx, WB_P0), W(ctx, WB_P1)};
    void* Qb[2] = {W(ctx, WB_Q0), W(ctx, WB_Q1)};
    void *AP = W(ctx, WB_AP), *T = W(ctx, WB_T);

    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)B, B64, N, Vh, s));
    }
    RETCK(colnorms(ctx, B64, N, d_bnorm));
    HIPCK(hipMemcpyAsync(ctx->h_vec, d_bnorm, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    RETCK(sync(ctx));
    for (int i = 0; i < N; ++i)
        if (!(ctx->h_vec[i] > 0.0) || !std::isfinite(ctx->h_vec[i]))
            return fail(ctx, BCG_ERR_ARG, "right-hand side column " + std::to_string(i) + " is zero or not finite");

    HIPCK(launch_zero(X, n * 16, s));
    if (use_guess) {
        HIPCK(launch_canon_to_int((const double2*)Xout, Y, N, Vh, s));
        RETCK(apply64(ctx, Y, R64, T64, N, nullptr));
        HIPCK(launch_residual(B64, R64, n, s));
    } else {
        HIPCK(launch_zero(Y, n * 16, s));
        HIPCK(launch_copy(B64, R64, n * 16, s));
    }
    HIPCK(launch_state_init(st, ctx->tol, ctx->ru_delta, ctx->ru_window, d_bnorm, N, s));
    // the iterate with the smallest true residual so far, returned if the solve stalls
    double2* Ybest = ctx->stall_limit > 0 ? Wd(ctx, WB_YBEST) : nullptr;
    if (Ybest) HIPCK(launch_copy(Y, Ybest, n * 16, s));
    // thin QR of the initial residual (Alg. 2), Q = R C^{-1}, P = Q (S = I, P_0 = 0)
    RETCK(gram(ctx, Prec::FP64, R64, R64, N, M(ctx, M_H), nullptr));
    {
        Prof pr(ctx, BCG_K_SMALL);
        HIPCK(launch_small_init(M(ctx, M_H), M(ctx, M_C), M(ctx, M_CINV), st, N, ctx->opt[BCG_OPT_SMALL_THREADS], s));
    }
    int cur = 0;
    if (ctx->qr_passes == 2) {
        // CholQR2: Q1 = R C1^{-1} in FP64, Q1^H Q1 = C2^H C2, Q = Q1 C2^{-1}, C = C2 C1
        {
            Prof pr(ctx, BCG_K_OTHER);
            HIPCK(launch_bmul(Prec::FP64, R64, Prec::FP64, nullptr, T64, M(ctx, M_CINV), N, Vh, halt, s));
        }
        RETCK(gram(ctx, Prec::FP64, T64, T64, N, M(ctx, M_H), halt));
        {
            Prof pr(ctx, BCG_K_SMALL);
            HIPCK(launch_small_qr2(M(ctx, M_H), M(ctx, M_C), M(ctx, M_CINV), M(ctx, M_C2I), M(ctx, M_C), st,
                                   (int*)&st->halt, 0, N, ctx->opt[BCG_OPT_SMALL_THREADS], s));
        }
        Prof pr(ctx, BCG_K_OTHER);
        HIPCK(launch_bmul(Prec::FP64, T64, ps, nullptr, Qb[cur], M(ctx, M_C2I), N, Vh, halt, s));
        HIPCK(launch_copy(Qb[cur], Pb[cur], (long)store_bytes(ps, N, 3, ctx->Vh), s));
    } else {
        Prof pr(ctx, BCG_K_OTHER);
        HIPCK(launch_bmul(Prec::FP64, R64, ps, nullptr, Qb[cur], M(ctx, M_CINV), N, Vh, halt, s));
        HIPCK(launch_copy(Qb[cur], Pb[cur], (long)store_bytes(ps, N, 3, ctx->Vh), s));
    }
    // fused path: G = 4 m^2 P^H P + T^H T, with P^H P kept as partials from the
    // kernel that last wrote P (here the initial P = Q)
    const bool fuse = fused_ok(ctx, ps, N);
    const double m2 = 4.0 * ctx->mass * ctx->mass;
    int n_pp = gram_parts(N, Vh, gram_mfma(ctx));
    const int n_tt = hop_grid(ctx->g, shape(ctx, ps, N, true), true);
    const int n_h = fused_grid(Vh);
    if (fuse) RETCK(gram_partials(ctx, ps, Pb[cur], Pb[cur], N, ctx->part_pp, halt));
    RETCK(read_state(ctx));
    int status = BCG_OK;
    int n_ru = 0;
    int iters_done = 0;
    if (ctx->h_state->halt) {
        status = BCG_ERR_BREAKDOWN;
        fail(ctx, status, "initial residual block is rank deficient (dependent right-hand sides)");
    } else if (ctx->h_state->max_relres <= ctx->tol) {
        // X0 already solves the system
        status = BCG_OK;
    }

    // stagnation: reliable updates in a row that fail to halve the best true residual
    double best_true = ctx->h_state->max_relres;
    int n_stall = 0;
    bool want_best = false;   // stagnation or breakdown: return the best iterate, not the current one
    // convergence-rate bookkeeping for the chunk size
    double last_log = std::log(std::fmax(ctx->h_state->max_relres, 1e-300));
    int last_it = 0;
    double rate = -0.02;   // log-residual change per iteration, refined as the solve runs
    int iters_at_resume = 0;
    bool finished = (status != BCG_OK) || (ctx->h_state->max_relres <= ctx->tol);
    bool need_final_check = true;   // cleared when a reliable update has confirmed convergence

    // one iteration of Alg. 1 on the ping-pong buffers c (P, Q) -> 1 - c (P', Q')
    auto iteration = [&](int c) -> int {
        void *P = Pb[c], *Q = Qb[c], *Pn = Pb[1 - c], *Qn = Qb[1 - c];
        if (fuse) {
            RETCK(hop(ctx, ps, 1, P, T, nullptr, N, EPI_PLAIN_, halt, nullptr, ctx->part_tt));
            RETCK(hop(ctx, ps, 0, T, AP, P, N, EPI_MASS_, halt));
            RETCK(reduce(ctx, ctx->part_tt, n_tt, ctx->part_pp, n_pp, m2, N, M(ctx, M_G), halt));
        } else {
            RETCK(hop(ctx, ps, 1, P, T, nullptr, N, EPI_PLAIN_, halt));
            RETCK(hop(ctx, ps, 0, T, AP, P, N, EPI_MASS_, halt));
            RETCK(gram(ctx, ps, P, AP, N, M(ctx, M_G), halt));
        }
        {
            Prof pr(ctx, BCG_K_SMALL);
            HIPCK(launch_small1(M(ctx, M_G), M(ctx, M_C), M(ctx, M_BETA), M(ctx, M_BETAC), st, N, ctx->opt[BCG_OPT_SMALL_THREADS], s));
        }
        if (fuse) {
            {
                Prof pr(ctx, BCG_K_PASS_A);
                HIPCK(launch_pass_a(ps, Q, AP, M(ctx, M_BETA), N, Vh, halt, ctx->partials, ctx->opt[BCG_OPT_PASS_CPT], bps64(ctx),
                                      ctx->opt[BCG_OPT_PASS_KERNEL], s));
            }
            RETCK(reduce(ctx, ctx->partials, n_h, nullptr, 0, 0.0, N, M(ctx, M_H), halt));
        } else {
            {
                Prof pr(ctx, BCG_K_PASS_A);
                HIPCK(launch_pass_a(ps, Q, AP, M(ctx, M_BETA), N, Vh, halt, nullptr, ctx->opt[BCG_OPT_PASS_CPT], bps64(ctx),
                                      ctx->opt[BCG_OPT_PASS_KERNEL], s));
            }
            RETCK(gram(ctx, ps, Q, Q, N, M(ctx, M_H), halt));
        }
        {
            Prof pr(ctx, BCG_K_SMALL);
            HIPCK(launch_small2(M(ctx, M_H), M(ctx, M_C), M(ctx, M_SINV), M(ctx, M_SH), st, N, ctx->opt[BCG_OPT_SMALL_THREADS], s));
        }
        {
            Prof pr(ctx, BCG_K_PASS_B);
            HIPCK(launch_pass_b(ps, X, Q, P, Qn, Pn, M(ctx, M_BETAC), M(ctx, M_SINV), M(ctx, M_SH),
                                N, Vh, st, fuse ? ctx->part_pp : nullptr, ctx->opt[BCG_OPT_PASS_CPT], bps64(ctx),
                                ctx->opt[BCG_OPT_PASS_KERNEL], s));
        }
        return BCG_OK;
    };
    // HIP graph of two iterations starting on buffers c0 (so a replay ends where it
    // began), captured on a private stream and replayed on the solver stream; only
    // once the P^H P partials come from pass B (n_pp = n_h), so the kernel arguments
    // are the same on every replay.  A failed capture falls back to eager launches.
    GraphPair gp;
    gp.launched_on = s;
    bool use_graph = ctx->opt[BCG_OPT_GRAPH] == 1 && ctx->prof_mask == 0;
    auto capture = [&](int c0) {
        if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            ctx->cap_stream = nullptr;
            use_graph = false;
            return;
        }
        hipStream_t keep = ctx->stream;
        ctx->stream = s = ctx->cap_stream;
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            int rc = iteration(c0);
            if (rc == BCG_OK) rc = iteration(1 - c0);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(s, &g);
            if (e == hipSuccess && rc == BCG_OK && g) {
                gp.g[c0] = g;
                e = hipGraphInstantiate(&gp.x[c0], g, nullptr, nullptr, 0);
                if (e != hipSuccess) gp.x[c0] = nullptr;
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
            if (rc != BCG_OK) e = hipErrorUnknown;
        }
        ctx->stream = s = keep;
        if (e != hipSuccess || !gp.x[c0]) {
            use_graph = false;
            (void)hipGetLastError();
        }
    };
    while (!finished) {
        const SolveState& hs = *ctx->h_state;
        // chunk size from the estimated iterations to the next event
        const double cur_log = std::log(std::fmax(hs.max_relres, 1e-300));
        double target = std::log(ctx->tol);
        if (ctx->ru_delta > 0.0) target = std::fmax(target, std::log(ctx->ru_delta * hs.rho_ru));
        int est = (int)std::ceil((target - cur_log) / (rate < -1e-6 ? rate : -1e-6));
        int chunk = est < 2 ? 2 : (est > 48 ? 48 : est);
        if (chunk > ctx->max_iter - hs.iters) chunk = ctx->max_iter - hs.iters;
        if (chunk < 1) chunk = 1;
        int c = cur;
        int k = 0;
        if (use_graph && chunk >= 2 && (!fuse || n_pp == n_h)) {
            if (!gp.x[c]) capture(c);
            if (use_graph)
                for (; k + 2 <= chunk; k += 2) HIPCK(hipGraphLaunch(gp.x[c], s));
        }
        for (; k < chunk; ++k) {
            RETCK(iteration(c));
            n_pp = n_h;
            c = 1 - c;
        }
        RETCK(read_state(ctx));
        if (ctx->monitor) ctx->monitor(ctx->monitor_user, hs.iters, n_ru, hs.max_relres);
        const int active = hs.iters - iters_at_resume;
        const bool halted = hs.halt != 0;
        const int reason = hs.reason;
        const int full = (halted && (reason == HALT_CONVERGED || reason == HALT_RU || reason == HALT_BREAKDOWN_H))
                             ? active - 1 : active;
        cur = (cur + full) & 1;
        iters_at_resume = hs.iters;
        iters_done = hs.iters;
        {
            const double lg = std::log(std::fmax(hs.max_relres, 1e-300));
            if (hs.iters > last_it) {
                const double r = (lg - last_log) / (hs.iters - last_it);
                if (r < 0) rate = r;
                last_log = lg;
                last_it = hs.iters;
            }
        }
        if (halted && (reason == HALT_BREAKDOWN_G || reason == HALT_BREAKDOWN_H)) {
            status = BCG_ERR_BREAKDOWN;
            want_best = true;
            fail(ctx, status, "Cholesky breakdown before convergence (rank-deficient block)");
            break;
        }
        if (!halted) {
            if (hs.iters >= ctx->max_iter) {
                status = BCG_ERR_NOT_CONVERGED;
                fail(ctx, status, "max_iter reached");
                break;
            }
            continue;
        }
        // reliable update (Alg. 3), also the convergence check on the true residual
        HIPCK(launch_fold_x(Y, X, n, s));
        RETCK(apply64(ctx, Y, R64, T64, N, nullptr));
        HIPCK(launch_residual(B64, R64, n, s));
        RETCK(gram(ctx, Prec::FP64, R64, R64, N, M(ctx, M_HR), nullptr));
        const bool qr2 = ctx->qr_passes == 2;
        {
            Prof pr(ctx, BCG_K_SMALL);
            HIPCK(launch_small_ru(M(ctx, M_HR), M(ctx, M_C), M(ctx, M_CINV), M(ctx, M_SH), st, d_true,
                                  ru_skip, reason == HALT_CONVERGED ? 1 : 0, qr2 ? 1 : 0, N,
                                  ctx->opt[BCG_OPT_SMALL_THREADS], s));
        }
        if (qr2) {
            // second CholQR pass on Q1 = R C^_1^{-1} (FP64), then S^ = C^ C_k^{-1}
            {
                Prof pr(ctx, BCG_K_OTHER);
                HIPCK(launch_bmul(Prec::FP64, R64, Prec::FP64, nullptr, T64, M(ctx, M_CINV), N, Vh, ru_skip, s));
            }
            RETCK(gram(ctx, Prec::FP64, T64, T64, N, M(ctx, M_HR), ru_skip));
            {
                Prof pr(ctx, BCG_K_SMALL);
                HIPCK(launch_small_qr2(M(ctx, M_HR), M(ctx, M_SH), M(ctx, M_CINV), M(ctx, M_C2I), M(ctx, M_C), st,
                                       ru_skip, 1, N, ctx->opt[BCG_OPT_SMALL_THREADS], s));
            }
        }
        {
            Prof pr(ctx, BCG_K_OTHER);
            if (qr2) HIPCK(launch_bmul(Prec::FP64, T64, ps, nullptr, Qb[1 - cur], M(ctx, M_C2I), N, Vh, ru_skip, s));
            else HIPCK(launch_bmul(Prec::FP64, R64, ps, nullptr, Qb[1 - cur], M(ctx, M_CINV), N, Vh, ru_skip, s));
            HIPCK(launch_bmul(ps, Pb[cur], ps, Qb[1 - cur], Pb[1 - cur], M(ctx, M_SH), N, Vh, ru_skip, s));
        }
        if (fuse) {
            RETCK(gram_partials(ctx, ps, Pb[1 - cur], Pb[1 - cur], N, ctx->part_pp, ru_skip));
            n_pp = gram_parts(N, Vh, gram_mfma(ctx));
        }
        RETCK(read_state(ctx));
        if (hs.reason == HALT_DONE) {
            finished = true;
            need_final_check = false;
            break;
        }
        if (hs.halt) {
            status = BCG_ERR_BREAKDOWN;
            want_best = true;
            fail(ctx, status, "Cholesky breakdown in the reliable update (rank-deficient residual)");
            break;
        }
        // hs.max_relres is now the maximum true relative residual of Y
        n_stall = (hs.max_relres <= 0.5 * best_true) ? 0 : n_stall + 1;
        if (hs.max_relres < best_true) {
            best_true = hs.max_relres;
            if (Ybest) HIPCK(launch_copy(Y, Ybest, n * 16, s));
        }
        if (ctx->stall_limit > 0 && n_stall >= ctx->stall_limit) {
            status = BCG_ERR_NOT_CONVERGED;
            want_best = true;
            fail(ctx, status, "stagnated: " + std::to_string(n_stall) +
                                  " reliable updates in a row did not halve the true residual (max relative " +
                                  std::to_string(best_true) + ")");
            n_ru += 1;
            break;
        }
        cur = 1 - cur;
        n_ru += 1;
        last_log = std::log(std::fmax(hs.max_relres, 1e-300));
        last_it = hs.iters;
        if (hs.iters >= ctx->max_iter) {
            status = BCG_ERR_NOT_CONVERGED;
            fail(ctx, status, "max_iter reached");
            break;
        }
    }
    // the solution: Y (+ X if the loop ended without folding it)
    if (status != BCG_OK || need_final_check) {
        HIPCK(launch_fold_x(Y, X, n, s));
        RETCK(apply64(ctx, Y, R64, T64, N, nullptr));
        HIPCK(launch_residual(B64, R64, n, s));
        RETCK(colnorms(ctx, R64, N, d_true));
        // relative: divide on the host below
    }
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_int_to_canon(Y, (double2*)Xout, N, Vh, s));
    }
    HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(ctx->h_vec + MAXN, d_bnorm, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    RETCK(sync(ctx));
    double tr[MAXN];
    double tr_max = 0.0;
    for (int i = 0; i < N; ++i) {
        tr[i] = ctx->h_vec[i];
        if (status != BCG_OK || need_final_check) tr[i] /= ctx->h_vec[MAXN + i];
        tr_max = std::fmax(tr_max, tr[i]);
    }
    if (want_best && Ybest && !(tr_max <= best_true)) {
        // a failed solve returns the iterate with the smallest true residual seen
        HIPCK(launch_copy(Ybest, Y, n * 16, s));
        RETCK(apply64(ctx, Y, R64, T64, N, nullptr));
        HIPCK(launch_residual(B64, R64, n, s));
        RETCK(colnorms(ctx, R64, N, d_true));
        {
            Prof pr(ctx, BCG_K_CONVERT);
            HIPCK(launch_int_to_canon(Y, (double2*)Xout, N, Vh, s));
        }
        HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
        RETCK(sync(ctx));
        for (int i = 0; i < N; ++i) tr[i] = ctx->h_vec[i] / ctx->h_vec[MAXN + i];
    }
    if (status == BCG_OK && need_final_check) {
        // only reached when the loop ended without a true-residual check (X0 already solved it)
        for (int i = 0; i < N; ++i)
            if (tr[i] > ctx->tol) status = BCG_ERR_NOT_CONVERGED;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, iters_done, n_ru, status, 0, secs, tr, N);
    return status;
}

// ---------------------------------------------------------------------------------------------
// N independent CG solves, one after the other (the baseline)
// ---------------------------------------------------------------------------------------------
int bcg_solve_cg(bcg_ctx* ctx, const void* B, void* Xout, int nrhs, bcg_stats* stats) {
    if (!ctx) return BCG_ERR_ARG;
    if (!B || !Xout) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    const auto t0 = std::chrono::steady_clock::now();
    const int N = nrhs;
    const int Vh = (int)ctx->Vh;
    const long n1 = 3L * Vh;
    hipStream_t s = ctx->stream;
    RETCK(alloc_solve(ctx, N, Prec::FP64));
    double2 *B64 = Wd(ctx, WB_B64), *Xs = Wd(ctx, WB_Y), *R64 = Wd(ctx, WB_R64), *T64 = Wd(ctx, WB_T64);
    double2 *r = Wd(ctx, WB_P0), *p = Wd(ctx, WB_Q0), *Ap = Wd(ctx, WB_AP), *t = Wd(ctx, WB_T);
    CgState* st = ctx->d_cg;
    const int* halt = &st->halt;
    double* dot = ctx->nparts + ctx->dot_off;
    double* d_true = ctx->d_vec + MAXN;
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)B, B64, N, Vh, s));
    }
    RETCK(colnorms(ctx, B64, N, ctx->d_vec));
    HIPCK(hipMemcpyAsync(ctx->h_vec, ctx->d_vec, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    RETCK(sync(ctx));
    double bn[MAXN];
    for (int i = 0; i < N; ++i) {
        bn[i] = ctx->h_vec[i];
        if (!(bn[i] > 0.0) || !std::isfinite(bn[i]))
            return fail(ctx, BCG_ERR_ARG, "right-hand side column " + std::to_string(i) + " is zero or not finite");
    }
    int status = BCG_OK;
    int total_iters = 0, restarts = 0;
    double tr[MAXN];
    const int nparts = dot_parts(ctx, Prec::FP64);
    if (ctx->sloppy != Prec::FP64) {
        status = cg_mixed(ctx, B64, Xs, bn, N, tr, &total_iters, &restarts);
        if (status == BCG_ERR_HIP || status == BCG_ERR_NOMEM) return status;
    }
    for (int i = 0; i < N && status == BCG_OK && ctx->sloppy == Prec::FP64; ++i) {
        const double2* b = B64 + (long)i * n1;
        double2* x = Xs + (long)i * n1;
        HIPCK(launch_zero(x, n1 * 16, s));
        HIPCK(launch_copy(b, r, n1 * 16, s));
        HIPCK(launch_copy(b, p, n1 * 16, s));
        HIPCK(launch_colnorm2(b, 1, Vh, ctx->nparts, s));
        HIPCK(launch_cg_init(ctx->nparts, Vh, st, ctx->tol, 0, s));
        double rate = -0.02, last_log = 0.0;
        int last_it = 0;
        for (;;) {
            HIPCK(hipMemcpyAsync(ctx->h_cg, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            const CgState hc = *ctx->h_cg;
            if (ctx->monitor) ctx->monitor(ctx->monitor_user, total_iters + hc.iters, restarts, hc.relres);
            if (hc.halt) {
                if (hc.reason == HALT_BREAKDOWN_G) {
                    status = BCG_ERR_BREAKDOWN;
                    fail(ctx, status, "CG breakdown: p^H A p <= 0");
                    break;
                }
                // converged on the iterated residual: check the true residual
                RETCK(apply64(ctx, x, R64, T64, 1, nullptr));
                HIPCK(launch_residual(b, R64, n1, s));
                HIPCK(launch_colnorm2(R64, 1, Vh, ctx->nparts, s));
                HIPCK(launch_colnorm_reduce(ctx->nparts, 1, Vh, d_true + i, 1, s));
                HIPCK(hipMemcpyAsync(ctx->h_vec, d_true + i, sizeof(double), hipMemcpyDeviceToHost, s));
                RETCK(sync(ctx));
                tr[i] = ctx->h_vec[0] / bn[i];
                if (tr[i] <= ctx->tol) break;
                // restart from the true residual
                HIPCK(launch_copy(R64, r, n1 * 16, s));
                HIPCK(launch_copy(R64, p, n1 * 16, s));
                HIPCK(launch_cg_init(ctx->nparts, Vh, st, ctx->tol, 1, s));
                restarts += 1;
                continue;
            }
            if (hc.iters >= ctx->max_iter) {
                status = BCG_ERR_NOT_CONVERGED;
                fail(ctx, status, "max_iter reached in CG");
                break;
            }
            const double lg = std::log(std::fmax(hc.relres, 1e-300));
            if (hc.iters > last_it) {
                const double rr = (lg - last_log) / (hc.iters - last_it);
                if (rr < 0) rate = rr;
            }
            last_log = lg;
            last_it = hc.iters;
            int est = (int)std::ceil((std::log(ctx->tol) - lg) / (rate < -1e-6 ? rate : -1e-6));
            int chunk = est < 2 ? 2 : (est > 64 ? 64 : est);
            if (chunk > ctx->max_iter - hc.iters) chunk = ctx->max_iter - hc.iters;
            for (int k = 0; k < chunk; ++k) {
                RETCK(hop(ctx, Prec::FP64, 1, p, t, nullptr, 1, EPI_PLAIN_, halt));
                RETCK(hop(ctx, Prec::FP64, 0, t, Ap, p, 1, EPI_MASS_DOT_, halt, dot));
                Prof pr(ctx, BCG_K_CG_VEC);
                HIPCK(launch_cg_alpha(dot, nparts, st, s));
                HIPCK(launch_cg_update1(x, r, p, Ap, n1, ctx->nparts, st, s));
                HIPCK(launch_cg_beta(ctx->nparts, n1, st, s));
                HIPCK(launch_cg_update2(p, r, n1, st, s));
            }
        }
        total_iters += ctx->h_cg->iters;
        if (status != BCG_OK) {
            for (int j = i; j < N; ++j) tr[j] = 1.0;
        }
    }
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_int_to_canon(Xs, (double2*)Xout, N, Vh, s));
    }
    RETCK(sync(ctx));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, total_iters, 0, status, restarts, secs, tr, N);
    return status;
}

// ---------------------------------------------------------------------------------------------
// Pseudo-block CG: N independent CG recurrences sharing every application of A
// ---------------------------------------------------------------------------------------------
int bcg_solve_pseudo(bcg_ctx* ctx, const void* B, void* Xout, int nrhs, bcg_stats* stats) {
    if (!ctx) return BCG_ERR_ARG;
    if (!B || !Xout) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    if (ctx->sloppy != Prec::FP64) return fail(ctx, BCG_ERR_ARG, "the pseudo-block solver runs in FP64 storage");
    const auto t0 = std::chrono::steady_clock::now();
    const int N = nrhs;
    const int Vh = (int)ctx->Vh;
    const long n = nvec(ctx, N);
    hipStream_t s = ctx->stream;
    RETCK(alloc_solve(ctx, N, Prec::FP64));
    double2 *B64 = Wd(ctx, WB_B64), *X = Wd(ctx, WB_Y), *R = Wd(ctx, WB_R64), *T64 = Wd(ctx, WB_T64),
            *Rt = Wd(ctx, WB_X);
    double2 *P = Wd(ctx, WB_P0), *AP = Wd(ctx, WB_AP), *T = Wd(ctx, WB_T);
    PbState* st = ctx->d_pb;
    const int* halt = &st->halt;
    int* d_restart = ctx->d_flags + 64;
    double* d_true = ctx->d_vec + MAXN;
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)B, B64, N, Vh, s));
    }
    RETCK(colnorms(ctx, B64, N, ctx->d_vec));
    HIPCK(hipMemcpyAsync(ctx->h_vec, ctx->d_vec, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    RETCK(sync(ctx));
    double bn[MAXN];
    for (int i = 0; i < N; ++i) {
        bn[i] = ctx->h_vec[i];
        if (!(bn[i] > 0.0) || !std::isfinite(bn[i]))
            return fail(ctx, BCG_ERR_ARG, "right-hand side column " + std::to_string(i) + " is zero or not finite");
    }
    HIPCK(launch_zero(X, n * 16, s));
    HIPCK(launch_copy(B64, R, n * 16, s));
    HIPCK(launch_copy(B64, P, n * 16, s));
    HIPCK(launch_colnorm2(R, N, Vh, ctx->nparts, s));
    HIPCK(launch_pb_start(ctx->nparts, N, Vh, st, d_restart, ctx->tol, 1, s));
    int status = BCG_OK, restarts = 0;
    double tr[MAXN];
    double rate = -0.02, last_log = 0.0;
    int last_it = 0;
    for (;;) {
        HIPCK(hipMemcpyAsync(ctx->h_pb, st, sizeof(PbState), hipMemcpyDeviceToHost, s));
        RETCK(sync(ctx));
        const PbState& hp = *ctx->h_pb;
        double mx = 0.0;
        for (int i = 0; i < N; ++i) mx = std::fmax(mx, hp.active[i] ? hp.relres[i] : 0.0);
        if (ctx->monitor) ctx->monitor(ctx->monitor_user, hp.iters, restarts, mx);
        if (hp.halt && hp.reason == HALT_BREAKDOWN_G) {
            status = BCG_ERR_BREAKDOWN;
            fail(ctx, status, "pseudo-block CG breakdown: p^H A p <= 0");
            break;
        }
        if (hp.halt) {
            // every column met tol on its iterated residual: check the true residuals
            RETCK(apply64(ctx, X, Rt, T64, N, nullptr));
            HIPCK(launch_residual(B64, Rt, n, s));
            RETCK(colnorms(ctx, Rt, N, d_true));
            HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            bool all = true;
            for (int i = 0; i < N; ++i) {
                tr[i] = ctx->h_vec[i] / bn[i];
                ctx->h_flags[i] = tr[i] > ctx->tol ? 1 : 0;
                all = all && !ctx->h_flags[i];
            }
            if (all) break;
            if (hp.iters >= ctx->max_iter) {
                status = BCG_ERR_NOT_CONVERGED;
                fail(ctx, status, "max_iter reached in pseudo-block CG");
                break;
            }
            // restart the columns that missed from their true residual
            for (int i = 0; i < N; ++i)
                if (ctx->h_flags[i]) {
                    HIPCK(launch_copy(Rt + (long)i * 3 * Vh, R + (long)i * 3 * Vh, 3L * Vh * 16, s));
                    HIPCK(launch_copy(Rt + (long)i * 3 * Vh, P + (long)i * 3 * Vh, 3L * Vh * 16, s));
                }
            HIPCK(hipMemcpyAsync(d_restart, ctx->h_flags, sizeof(int) * N, hipMemcpyHostToDevice, s));
            HIPCK(launch_colnorm2(R, N, Vh, ctx->nparts, s));
            HIPCK(launch_pb_start(ctx->nparts, N, Vh, st, d_restart, ctx->tol, 0, s));
            restarts += 1;
            continue;
        }
        if (hp.iters >= ctx->max_iter) {
            status = BCG_ERR_NOT_CONVERGED;
            fail(ctx, status, "max_iter reached in pseudo-block CG");
            break;
        }
        const double lg = std::log(std::fmax(mx, 1e-300));
        if (hp.iters > last_it) {
            const double r = (lg - last_log) / (hp.iters - last_it);
            if (r < 0) rate = r;
        }
        last_log = lg;
        last_it = hp.iters;
        int est = (int)std::ceil((std::log(ctx->tol) - lg) / (rate < -1e-6 ? rate : -1e-6));
        int chunk = est < 2 ? 2 : (est > 48 ? 48 : est);
        if (chunk > ctx->max_iter - hp.iters) chunk = ctx->max_iter - hp.iters;
        for (int k = 0; k < chunk; ++k) {
            RETCK(hop(ctx, Prec::FP64, 1, P, T, nullptr, N, EPI_PLAIN_, halt));
            RETCK(hop(ctx, Prec::FP64, 0, T, AP, P, N, EPI_MASS_, halt));
            Prof pr(ctx, BCG_K_CG_VEC);
            HIPCK(launch_pb_dot(P, AP, N, Vh, ctx->nparts, st, s));
            HIPCK(launch_pb_alpha(ctx->nparts, N, Vh, st, s));
            HIPCK(launch_pb_update1(X, R, P, AP, N, Vh, ctx->nparts, st, s));
            HIPCK(launch_pb_beta(ctx->nparts, N, Vh, st, s));
            HIPCK(launch_pb_update2(P, R, N, Vh, st, s));
        }
    }
    if (status != BCG_OK) {
        RETCK(apply64(ctx, X, Rt, T64, N, nullptr));
        HIPCK(launch_residual(B64, Rt, n, s));
        RETCK(colnorms(ctx, Rt, N, d_true));
        HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    }
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_int_to_canon(X, (double2*)Xout, N, Vh, s));
    }
    RETCK(sync(ctx));
    if (status != BCG_OK)
        for (int i = 0; i < N; ++i) tr[i] = ctx->h_vec[i] / bn[i];
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, ctx->h_pb->iters, 0, status, restarts, secs, tr, N);
    return status;
}

// ---------------------------------------------------------------------------------------------
// s-step block CG: s block Krylov directions per outer iteration, one reduction phase
// ---------------------------------------------------------------------------------------------
int bcg_solve_sstep(bcg_ctx* ctx, const void* B, void* Xout, int nrhs, int s_steps, double lmin, double lmax,
                    bcg_stats* stats) {
    if (!ctx) return BCG_ERR_ARG;
    if (!B || !Xout) return fail(ctx, BCG_ERR_ARG, "null vector pointer");
    RETCK(check_nrhs(ctx, nrhs));
    RETCK(check_ready(ctx));
    if (s_steps < 1 || (long)s_steps * nrhs > BCG_MAX_RHS)
        return fail(ctx, BCG_ERR_ARG, "s * nrhs must be in [1, 64], got s = " + std::to_string(s_steps));
    if (!std::isfinite(lmin) || !std::isfinite(lmax) || (lmax > 0.0 && lmin >= lmax))
        return fail(ctx, BCG_ERR_ARG, "the basis interval needs finite lmin < lmax");
    // storage of V, AV, P and AP: FP64, or FP32 with FP64 reliable updates (16-bit
    // storage keeps one scale array after all columns of a block, so the sub-blocks
    // of the basis would not be blocks of their own)
    const Prec ps = ctx->sloppy;
    if (ps != Prec::FP64 && ps != Prec::FP32)
        return fail(ctx, BCG_ERR_ARG, "the s-step solver stores its blocks in FP64 or FP32");
    const auto t0 = std::chrono::steady_clock::now();
    const int N = nrhs, S = s_steps, K = S * N;
    const int Vh = (int)ctx->Vh;
    const long n = nvec(ctx, N), n1 = 3L * Vh;
    hipStream_t s = ctx->stream;
    RETCK(alloc_solve(ctx, N, ps));
    RETCK(ensure_sloppy_links(ctx, ps));
    // three slots of K columns for the basis V, the previous directions P' and the
    // new ones (and the same for AV, AP', AP): V always sits next to P', so that
    // U = [V | P'] (or [P' | V]) is one block of 2K columns
    const long nK = nvec(ctx, K);
    const size_t eb = ps == Prec::FP64 ? 16 : 8;  // bytes per stored complex entry
    for (int slot : {WB_P0, WB_P1}) RETCK(ensure(ctx, slot, (size_t)3 * nK * eb));
    double2 *B64 = Wd(ctx, WB_B64), *X = Wd(ctx, WB_Y), *R = Wd(ctx, WB_R64), *T64 = Wd(ctx, WB_T64),
            *Rt = Wd(ctx, WB_X);
    char *PS = (char*)W(ctx, WB_P0), *APS = (char*)W(ctx, WB_P1);
    void* Ts = W(ctx, WB_T);  // odd-parity scratch of the stored-precision apply
    auto at = [&](char* base, long pairs) -> char* { return base + (size_t)pairs * eb; };
    double2 *Bk = M(ctx, M_CINV), *alpha = M(ctx, M_SINV), *nalpha = M(ctx, M_SH);
    // K <= 32: two Hermitian Grams of U (2K <= 64 columns) hold every product as a
    // block; above, five Grams of K columns
    const bool wide = 2 * K <= MAXN;
    double2 *GU = M(ctx, M_G), *GUU = M(ctx, M_H);
    double2 *Gv5 = M(ctx, M_G), *Gvv5 = M(ctx, M_H), *Ga5 = M(ctx, M_BETA), *Wp5 = M(ctx, M_BETAC),
            *Pv5 = M(ctx, M_C);
    int* d_status = ctx->d_flags + 1;
    double* d_rn = ctx->d_vec + 2 * MAXN;   // iterated residual norms
    double* d_lam = ctx->d_vec + 3 * MAXN;  // power-iteration estimate
    double* d_true = ctx->d_vec + MAXN;
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_canon_to_int((const double2*)B, B64, N, Vh, s));
    }
    RETCK(colnorms(ctx, B64, N, ctx->d_vec));
    HIPCK(hipMemcpyAsync(ctx->h_vec, ctx->d_vec, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    RETCK(sync(ctx));
    double bn[MAXN];
    for (int i = 0; i < N; ++i) {
        bn[i] = ctx->h_vec[i];
        if (!(bn[i] > 0.0) || !std::isfinite(bn[i]))
            return fail(ctx, BCG_ERR_ARG, "right-hand side column " + std::to_string(i) + " is zero or not finite");
    }
    // the basis interval: lmin defaults to 4 m^2 (the bound of A = 4 m^2 + D_oe^H D_oe),
    // lmax to 1.1 times a 30-step power-iteration estimate from the first column
    if (!(lmin > 0.0)) lmin = 4.0 * ctx->mass * ctx->mass;
    if (!(lmax > 0.0)) {
        for (int slot : {WB_A0, WB_A1}) RETCK(ensure(ctx, slot, (size_t)n1 * 16));
        double2 *pv = Wd(ctx, WB_A0), *pw = Wd(ctx, WB_A1);
        HIPCK(launch_scale_inv(pv, B64, ctx->d_vec, n1, s));
        for (int it = 0; it < 30; ++it) {
            RETCK(apply64(ctx, pv, pw, T64, 1, nullptr));
            RETCK(colnorms(ctx, pw, 1, d_lam));
            HIPCK(launch_scale_inv(pv, pw, d_lam, n1, s));
        }
        HIPCK(hipMemcpyAsync(ctx->h_vec, d_lam, sizeof(double), hipMemcpyDeviceToHost, s));
        RETCK(sync(ctx));
        lmax = 1.1 * ctx->h_vec[0];
        if (!(lmax > lmin) || !std::isfinite(lmax)) lmax = 2.0 * lmin + 1.0;
    }
    const double cc = 0.5 * (lmax + lmin), hh = 0.5 * (lmax - lmin);
    HIPCK(launch_zero(X, n * 16, s));
    HIPCK(launch_copy(B64, R, n * 16, s));
    HIPCK(hipMemsetAsync(d_status, 0, sizeof(int), s));
    if (ps != Prec::FP64) HIPCK(launch_identity(M(ctx, M_ID), N, s));
    const int max_outer = std::max(1, ctx->max_iter / S);
    // reliable updates (FP32 storage): R <- B - A X in FP64 whenever the largest
    // iterated relative residual has dropped by ru_delta since the last one
    const double ru_delta = ps == Prec::FP64 ? 0.0 : ctx->ru_delta;
    double rho_ru = 1.0;
    int status = BCG_OK, outer = 0, restarts = 0, rus = 0;
    int pslot = -1;  // slot of P' (-1: none, the first outer iteration after a (re)start)
    bool first = true;
    double tr[MAXN];
    for (;;) {
        RETCK(colnorms(ctx, R, N, d_rn));
        HIPCK(hipMemcpyAsync(ctx->h_vec, d_rn, sizeof(double) * N, hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(ctx->h_flags, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
        RETCK(sync(ctx));
        if (ctx->h_flags[0] != 0) {
            status = BCG_ERR_BREAKDOWN;
            fail(ctx, status, ctx->h_flags[0] == 1 ? "s-step breakdown: P'^H A P' not positive definite"
                                                   : "s-step breakdown: P^H A P not positive definite");
            break;
        }
        double mx = 0.0;
        for (int i = 0; i < N; ++i) mx = std::fmax(mx, ctx->h_vec[i] / bn[i]);
        if (ctx->monitor) ctx->monitor(ctx->monitor_user, outer * S, restarts, mx);
        if (mx <= ctx->tol) {
            // converged on the iterated residual: check the true residual
            RETCK(apply64(ctx, X, Rt, T64, N, nullptr));
            HIPCK(launch_residual(B64, Rt, n, s));
            RETCK(colnorms(ctx, Rt, N, d_true));
            HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            double tm = 0.0;
            for (int i = 0; i < N; ++i) {
                tr[i] = ctx->h_vec[i] / bn[i];
                tm = std::fmax(tm, tr[i]);
            }
            if (tm <= ctx->tol) break;
            // restart the recurrence from the true residual
            HIPCK(launch_copy(Rt, R, n * 16, s));
            first = true;
            pslot = -1;
            restarts += 1;
            rho_ru = tm;
        } else if (ru_delta > 0.0 && mx <= ru_delta * rho_ru) {
            // reliable update: the directions P', AP' are kept; the reduced products
            // with the new residual enter through P'^H V and V^H V
            RETCK(apply64(ctx, X, R, T64, N, nullptr));
            HIPCK(launch_residual(B64, R, n, s));
            RETCK(colnorms(ctx, R, N, d_rn));
            HIPCK(hipMemcpyAsync(ctx->h_vec, d_rn, sizeof(double) * N, hipMemcpyDeviceToHost, s));
            RETCK(sync(ctx));
            rho_ru = 0.0;
            for (int i = 0; i < N; ++i) rho_ru = std::fmax(rho_ru, ctx->h_vec[i] / bn[i]);
            rus += 1;
        }
        if (outer >= max_outer) {
            status = BCG_ERR_NOT_CONVERGED;
            fail(ctx, status, "max_iter reached in s-step block CG");
            break;
        }
        // slots: V next to P' (the middle slot unless P' is there), the new
        // directions in the remaining one; the first directions are V itself
        const int vslot = first ? 1 : (pslot == 1 ? 0 : 1);
        const int nslot = first ? vslot : 3 - pslot - vslot;
        char *V = at(PS, vslot * nK), *AV = at(APS, vslot * nK);
        char *Pn = at(PS, nslot * nK), *APn = at(APS, nslot * nK);
        char *Pp = first ? nullptr : at(PS, pslot * nK), *APp = first ? nullptr : at(APS, pslot * nK);
        // basis V = [R, p_1(A) R, ...] (Chebyshev polynomials of [lmin, lmax]) and AV = A V,
        // each block rounded to the storage precision as it is formed
        if (ps == Prec::FP64) {
            HIPCK(launch_copy(R, V, n * 16, s));
        } else {
            Prof pr(ctx, BCG_K_CONVERT);
            HIPCK(launch_bmul(Prec::FP64, R, ps, nullptr, V, M(ctx, M_ID), N, Vh, nullptr, s));
        }
        for (int j = 0; j < S; ++j) {
            if (ps == Prec::FP64) {
                RETCK(apply64(ctx, at(V, j * n), at(AV, j * n), T64, N, nullptr));
            } else {
                RETCK(hop(ctx, ps, 1, at(V, j * n), Ts, nullptr, N, EPI_PLAIN_, nullptr));
                RETCK(hop(ctx, ps, 0, Ts, at(AV, j * n), at(V, j * n), N, EPI_MASS_, nullptr));
            }
            if (j + 1 < S) {
                Prof pr(ctx, BCG_K_OTHER);
                HIPCK(launch_cheb_step(ps, at(V, (j + 1) * n), at(AV, j * n), at(V, j * n),
                                       j ? at(V, (j - 1) * n) : nullptr, (j ? 2.0 : 1.0) / hh, cc, n, s));
            }
        }
        // one reduction phase
        const double2 *Gv, *Gvv, *Ga = nullptr, *Wpm = nullptr, *Pv = nullptr;
        if (first) {
            RETCK(gram(ctx, ps, V, AV, K, Gv5, nullptr));
            RETCK(gram(ctx, ps, V, V, K, Gvv5, nullptr));
            Gv = Gv5;
            Gvv = Gvv5;
        } else if (wide) {
            // U^H A U and U^H U for U = the two adjacent slots of V and P'
            const int lo = std::min(vslot, pslot);
            const int vo = vslot < pslot ? 0 : K, po = K - vo;
            RETCK(gram(ctx, ps, at(PS, lo * nK), at(APS, lo * nK), 2 * K, GU, nullptr));
            RETCK(gram(ctx, ps, at(PS, lo * nK), at(PS, lo * nK), 2 * K, GUU, nullptr));
            Gv = GU + vo * MAXN + vo;
            Ga = GU + po * MAXN + vo;   // P'^H A V = (A P')^H V
            Wpm = GU + po * MAXN + po;
            Gvv = GUU + vo * MAXN + vo;
            Pv = GUU + po * MAXN + vo;
        } else {
            // the Hermitian V^H AV, V^H V, P'^H AP' on the matrix cores, the general
            // (AP')^H V and P'^H V on the vector ALUs
            RETCK(gram(ctx, ps, V, AV, K, Gv5, nullptr));
            RETCK(gram(ctx, ps, V, V, K, Gvv5, nullptr));
            RETCK(gram_general(ctx, ps, APp, V, K, Ga5));
            RETCK(gram(ctx, ps, Pp, APp, K, Wp5, nullptr));
            RETCK(gram_general(ctx, ps, Pp, V, K, Pv5));
            Gv = Gv5;
            Gvv = Gvv5;
            Ga = Ga5;
            Wpm = Wp5;
            Pv = Pv5;
        }
        {
            Prof pr(ctx, BCG_K_SMALL);
            HIPCK(launch_sstep_coef(Gv, Gvv, Ga, Wpm, Pv, Bk, alpha, nalpha, d_status, K, N, first ? 1 : 0, s));
        }
        {
            // P = V + P' Bk, AP = AV + AP' Bk, X += P alpha, R -= AP alpha
            Prof pr(ctx, BCG_K_PASS_B);
            if (!first) {
                HIPCK(launch_bmul(ps, Pp, ps, V, Pn, Bk, K, Vh, d_status, s));
                HIPCK(launch_bmul(ps, APp, ps, AV, APn, Bk, K, Vh, d_status, s));
            }
            HIPCK(launch_bmul_rect(ps, Pn, X, X, alpha, K, N, Vh, d_status, s));
            HIPCK(launch_bmul_rect(ps, APn, R, R, nalpha, K, N, Vh, d_status, s));
        }
        pslot = nslot;
        first = false;
        outer += 1;
    }
    if (status != BCG_OK) {
        RETCK(apply64(ctx, X, Rt, T64, N, nullptr));
        HIPCK(launch_residual(B64, Rt, n, s));
        RETCK(colnorms(ctx, Rt, N, d_true));
        HIPCK(hipMemcpyAsync(ctx->h_vec, d_true, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    }
    {
        Prof pr(ctx, BCG_K_CONVERT);
        HIPCK(launch_int_to_canon(X, (double2*)Xout, N, Vh, s));
    }
    RETCK(sync(ctx));
    if (status != BCG_OK)
        for (int i = 0; i < N; ++i) tr[i] = ctx->h_vec[i] / bn[i];
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, outer * S, rus, status, restarts, secs, tr, N);
    return status;
}

int bcg_set_monitor(bcg_ctx* ctx, bcg_monitor_fn fn, void* user) {
    if (!ctx) return BCG_ERR_ARG;
    ctx->monitor = fn;
    ctx->monitor_user = user;
    return BCG_OK;
}

int bcg_set_stability(bcg_ctx* ctx, int ru_window, int stall_limit, int qr_passes) {
    if (!ctx) return BCG_ERR_ARG;
    if (ru_window < 0 || stall_limit < 0) return fail(ctx, BCG_ERR_ARG, "ru_window and stall_limit must be >= 0");
    if (qr_passes != 1 && qr_passes != 2) return fail(ctx, BCG_ERR_ARG, "qr_passes must be 1 or 2");
    ctx->ru_window = ru_window;
    ctx->stall_limit = stall_limit;
    ctx->qr_passes = qr_passes;
    return BCG_OK;
}

int bcg_set_option(bcg_ctx* ctx, int option, int value) {
    if (!ctx) return BCG_ERR_ARG;
    if (option < 0 || option >= BCG_OPT_COUNT) return fail(ctx, BCG_ERR_ARG, "unknown option");
    ctx->opt[option] = value;
    if (option == BCG_OPT_SITE_ORDER) ctx->g.slab = (value == 2) ? 0 : 1;
    return BCG_OK;
}

int bcg_set_profiling(bcg_ctx* ctx, unsigned mask) {
    if (!ctx) return BCG_ERR_ARG;
    ctx->prof_mask = mask;
    return BCG_OK;
}

int bcg_profile_reset(bcg_ctx* ctx) {
    if (!ctx) return BCG_ERR_ARG;
    RETCK(sync(ctx));
    for (int k = 0; k < BCG_K_COUNT; ++k) {
        ctx->prof_n[k] = 0;
        ctx->prof_ms[k] = 0.0;
    }
    return BCG_OK;
}

int bcg_kernel_time(bcg_ctx* ctx, int kernel, long* launches, double* total_ms) {
    if (!ctx) return BCG_ERR_ARG;
    if (kernel < 0 || kernel >= BCG_K_COUNT || !launches || !total_ms)
        return fail(ctx, BCG_ERR_ARG, "bad kernel id or null output");
    RETCK(sync(ctx));
    *launches = ctx->prof_n[kernel];
    *total_ms = ctx->prof_ms[kernel];
    return BCG_OK;
}

const char* bcg_last_error(const bcg_ctx* ctx) {
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

}  // extern "C"
