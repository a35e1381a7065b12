"""GPU parity of blockCGrQ and the CG baseline against the CPU oracle.

The solution of A X = B is unique, so the bar is the true relative residual of
every column computed with the oracle's FP64 operator (<= 1e-10 in FP64 mode,
<= 1e-8 in mixed precision) plus the distance to the oracle's own solution
(solved to 1e-12), bounded by the condition number.  The first iterates are
unique too (the CholQR factors have positive real diagonals), so X after k
iterations is compared with the oracle's X after k iterations."""
import numpy as np
import pytest
import torch

import oracle
from paper_1710_09745_amd import bcg, synth

from gpu_util import DEV, col_rel_err, context, inputs, kappa_bound, to_dev, true_rel_res

pytestmark = pytest.mark.gpu


def test_config1_solve_matches_oracle_and_dense_solve():
    c = synth.CONFIGS[1]
    fat, lng, B = synth.config_inputs(1)
    ctx = context(c["dims"], False, fat, lng, c["mass"], tol=c["tol"])
    X, info = ctx.solve(to_dev(B))
    X = X.cpu().numpy()
    op = oracle.Operator(c["dims"], fat, lng, c["mass"])
    assert true_rel_res(op, B, X).max() <= c["tol"]
    assert max(info["true_rel_res"]) <= c["tol"]
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-12)
    from test_oracle_operator import dense_A
    A = dense_A(op)
    kappa = np.linalg.cond(A)
    Xd = oracle.from_mat(np.linalg.solve(A, oracle.to_mat(B)), op.Vh)
    err = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    print(f"config 1: iters={info['iters']} rus={info['reliable_updates']} "
          f"||X-X_oracle||/||X_oracle||={err:.2e} kappa={kappa:.1f}")
    assert err <= kappa * c["tol"]
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) <= kappa * c["tol"]


@pytest.mark.parametrize("dims,improved,m,n", [((6, 6, 6, 6), True, 0.1, 5),
                                               ((8, 8, 8, 8), True, 0.1, 16),
                                               ((4, 6, 4, 8), False, 0.2, 1),
                                               ((8, 8, 8, 8), True, 0.2, 64)])
def test_solve_matches_oracle(dims, improved, m, n):
    fat, lng, B = inputs(dims, improved, n, 4000 + n)
    ctx = context(dims, improved, fat, lng, m, tol=1e-10)
    X, info = ctx.solve(to_dev(B))
    X = X.cpu().numpy()
    op = oracle.Operator(dims, fat, lng, m)
    res = true_rel_res(op, B, X)
    assert res.max() <= 1e-10
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3, atol=1e-14)
    Xo, io = oracle.block_cg_rq(op.apply, B, 1e-12)
    err = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    kappa = kappa_bound(op)
    print(f"iters gpu={info['iters']} oracle={io.iters} err={err:.2e} kappa<={kappa:.0f}")
    assert err <= kappa * 1e-10


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_iterates_match_oracle(k):
    dims = (6, 4, 6, 6)
    fat, lng, B = inputs(dims, True, 6, 5000)
    m = 0.1
    ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=k)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    assert info["rc"] == bcg.ERR_NOT_CONVERGED and info["iters"] == k
    op = oracle.Operator(dims, fat, lng, m)
    Xo, io = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k)
    assert col_rel_err(X.cpu().numpy(), Xo).max() <= 1e-10


def test_cg_baseline_matches_oracle():
    dims = (6, 6, 6, 6)
    fat, lng, B = inputs(dims, True, 3, 6000)
    m = 0.1
    ctx = context(dims, True, fat, lng, m, tol=1e-10)
    X, info = ctx.solve_cg(to_dev(B))
    X = X.cpu().numpy()
    op = oracle.Operator(dims, fat, lng, m)
    assert true_rel_res(op, B, X).max() <= 1e-10
    its = 0
    kappa = kappa_bound(op)
    for i in range(3):
        xo, io = oracle.cg(op.apply, B[i], 1e-10)
        its += io.iters
        assert np.linalg.norm(X[i] - xo) / np.linalg.norm(xo) <= kappa * 2e-10
    print(f"cg iters gpu={info['iters']} oracle={its}")
    assert abs(info["iters"] - its) <= 3 * 3


@pytest.mark.parametrize("prec", ["fp32", "fix16"])
def test_mixed_cg_baseline_meets_tolerance(prec):
    """Double-single (and 16-bit) CG with reliable updates: every column reaches
    1e-8 by the oracle's FP64 operator, in about the FP64 CG iteration count."""
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 3, 6050)
    m = 0.05
    op = oracle.Operator(dims, fat, lng, m)
    c64 = context(dims, True, fat, lng, m, tol=1e-8)
    _, i64 = c64.solve_cg(to_dev(B))
    ctx = context(dims, True, fat, lng, m, tol=1e-8, prec=prec)
    X, info = ctx.solve_cg(to_dev(B))
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"{prec} CG: iters={info['iters']} reliable updates={info['restarts']} (fp64 CG {i64['iters']}) "
          f"max res={res.max():.2e}")
    assert res.max() <= 1e-8
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3)
    assert info["restarts"] >= 3
    assert info["iters"] <= 1.5 * i64["iters"] + 30


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
def test_cg_hop_run_lengths_agree(prec, tol):
    """The CG baseline's hop with its fused p^H A p on runs of 32 sites (128-site
    workgroups and half as many dot partials; the default below FP64 on large
    lattices, chosen here explicitly) and on runs of 16 sites: both meet the
    tolerance by the oracle's operator, in the same iteration counts, and in FP64 the
    solutions agree to the rounding bound."""
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 2, 6070)
    m = 0.1
    op = oracle.Operator(dims, fat, lng, m)
    out = {}
    for kernel in (1, 3):
        ctx = context(dims, True, fat, lng, m, tol=tol, prec=prec)
        ctx.set_option("hop_kernel", kernel)
        print(f"[case] CG {prec} hop_kernel={kernel}", flush=True)
        X, info = ctx.solve_cg(to_dev(B))
        X = X.cpu().numpy()
        assert true_rel_res(op, B, X).max() <= tol
        out[kernel] = (X, info["iters"])
    assert abs(out[1][1] - out[3][1]) <= 4
    if prec == "fp64":
        assert col_rel_err(out[3][0], out[1][0]).max() <= kappa_bound(op) * 2e-10


@pytest.mark.parametrize("k", [1, 3, 7])
def test_pseudo_block_iterates_match_oracle_cg(k):
    """Pseudo-block CG after k lockstep iterations: every column is the oracle's
    textbook CG iterate after k iterations (the recurrences are independent)."""
    dims = (6, 4, 6, 6)
    fat, lng, B = inputs(dims, True, 5, 6010)
    m = 0.1
    ctx = context(dims, True, fat, lng, m, tol=1e-14, max_iter=k)
    X, info = ctx.solve_pseudo(to_dev(B), raise_on_error=False)
    assert info["rc"] == bcg.ERR_NOT_CONVERGED and info["iters"] == k
    op = oracle.Operator(dims, fat, lng, m)
    Xo = np.stack([oracle.cg(op.apply, B[i], 1e-14, max_iter=k)[0] for i in range(B.shape[0])])
    assert col_rel_err(X.cpu().numpy(), Xo).max() <= 1e-10


@pytest.mark.parametrize("dims,n", [((8, 8, 8, 8), 8), ((6, 6, 6, 8), 17)])
def test_pseudo_block_solve_matches_cg(dims, n):
    """Converged pseudo-block solve: every column meets 1e-10 by the oracle's
    operator, each in the iteration count of its own CG (the columns finish at
    different iterations), and agrees with the CG baseline to kappa * tol."""
    fat, lng, B = inputs(dims, True, n, 6020 + n)
    m = 0.1
    ctx = context(dims, True, fat, lng, m, tol=1e-10)
    X, info = ctx.solve_pseudo(to_dev(B))
    Xc, ic = ctx.solve_cg(to_dev(B))
    op = oracle.Operator(dims, fat, lng, m)
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"pseudo-block: lockstep iters={info['iters']} restarts={info['restarts']}; "
          f"CG total {ic['iters']} (mean {ic['iters'] / n:.1f}) max res={res.max():.2e}")
    assert res.max() <= 1e-10
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3, atol=1e-14)
    assert info["iters"] >= ic["iters"] / n - 2 and info["iters"] <= ic["iters"]
    kappa = kappa_bound(op)
    assert col_rel_err(X.cpu().numpy(), Xc.cpu().numpy()).max() <= kappa * 2e-10


def test_n1_block_equals_cg():
    dims = (6, 6, 4, 4)
    fat, lng, B = inputs(dims, True, 1, 6100)
    ctx = context(dims, True, fat, lng, 0.15, tol=1e-11, ru_delta=0.0)
    Xb, ib = ctx.solve(to_dev(B))
    Xc, ic = ctx.solve_cg(to_dev(B))
    assert abs(ib["iters"] - ic["iters"]) <= 2
    assert col_rel_err(Xb.cpu().numpy(), Xc.cpu().numpy()).max() <= 1e-9


def test_solve_is_deterministic():
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 8, 6200)
    ctx = context(dims, True, fat, lng, 0.1, tol=1e-10)
    X1, i1 = ctx.solve(to_dev(B))
    X2, i2 = ctx.solve(to_dev(B))
    assert i1["iters"] == i2["iters"]
    assert torch.equal(X1, X2)


def test_initial_guess():
    dims = (6, 6, 6, 6)
    fat, lng, B = inputs(dims, True, 4, 6300)
    ctx = context(dims, True, fat, lng, 0.1, tol=1e-10)
    X, info = ctx.solve(to_dev(B))
    X2, info2 = ctx.solve(to_dev(B), X0=X)
    assert info2["iters"] <= 1
    op = oracle.Operator(dims, fat, lng, 0.1)
    assert true_rel_res(op, B, X2.cpu().numpy()).max() <= 1e-10


def test_error_paths():
    dims = (4, 4, 4, 4)
    fat, lng, B = inputs(dims, True, 4, 6400)
    ctx = bcg.Context(dims, improved=True, device=DEV)
    with pytest.raises(bcg.BcgError) as e:
        ctx.solve(to_dev(B))
    assert e.value.code == bcg.ERR_STATE
    ctx.load_links(fat, lng)
    ctx.set_mass(0.1)
    ctx.set_solver(tol=1e-10, max_iter=1000)
    Bz = B.copy()
    Bz[2] = 0
    with pytest.raises(bcg.BcgError) as e:
        ctx.solve(to_dev(Bz))
    assert e.value.code == bcg.ERR_ARG
    Bd = B.copy()
    Bd[3] = Bd[1]
    with pytest.raises(bcg.Breakdown):
        ctx.solve(to_dev(Bd))
    ctx.set_solver(tol=1e-10, max_iter=2)
    with pytest.raises(bcg.NotConverged):
        ctx.solve(to_dev(B))
    big = torch.zeros((65, ctx.Vh, 3), dtype=torch.complex128, device=DEV)
    with pytest.raises(bcg.BcgError) as e:
        ctx.apply(big)
    assert e.value.code == bcg.ERR_ARG
    with pytest.raises(bcg.BcgError) as e:
        ctx.set_solver(tol=0.0)
    assert e.value.code == bcg.ERR_ARG


def test_mixed_fp32_reaches_tolerance():
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 8, 6500)
    m = 0.05
    c64 = context(dims, True, fat, lng, m, tol=1e-8, prec="fp64")
    X64, i64 = c64.solve(to_dev(B))
    c32 = context(dims, True, fat, lng, m, tol=1e-8, prec="fp32")
    X32, i32 = c32.solve(to_dev(B))
    op = oracle.Operator(dims, fat, lng, m)
    r32 = true_rel_res(op, B, X32.cpu().numpy())
    d = np.linalg.norm((X32 - X64).cpu().numpy()) / np.linalg.norm(X64.cpu().numpy())
    print(f"fp64 iters={i64['iters']} fp32 iters={i32['iters']} rus={i32['reliable_updates']} "
          f"max res={r32.max():.2e} ||X32-X64||/||X64||={d:.2e}")
    assert r32.max() <= 1e-8
    assert i32["reliable_updates"] >= 1


def test_config2_full_size_solve_and_cg():
    c = synth.CONFIGS[2]
    fat, lng, B = synth.config_inputs(2)
    ctx = context(c["dims"], True, fat, lng, c["mass"], tol=c["tol"])
    X, info = ctx.solve(to_dev(B))
    op = oracle.Operator(c["dims"], fat, lng, c["mass"])
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"config 2 block: iters={info['iters']} rus={info['reliable_updates']} "
          f"t={info['seconds']:.3f}s max res={res.max():.2e}")
    assert res.max() <= c["tol"]
    Xc, ic = ctx.solve_cg(to_dev(B[:2].copy()))
    resc = true_rel_res(op, B[:2], Xc.cpu().numpy())
    print(f"config 2 cg (2 columns): iters={ic['iters']} t={ic['seconds']:.3f}s max res={resc.max():.2e}")
    assert resc.max() <= c["tol"]


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fix16"])
def test_mixed_16bit_reaches_tolerance(prec):
    """16-bit storage (FP16, BF16 or 16-bit fixed point) with one FP32 scale per site
    and column (vectors) or per folded link matrix, FP32 arithmetic, FP64 Gram /
    CholQR / reliable updates."""
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 8, 6600)
    m = 0.1
    c16 = context(dims, True, fat, lng, m, tol=1e-8, prec=prec, max_iter=20000)
    X16, i16 = c16.solve(to_dev(B))
    op = oracle.Operator(dims, fat, lng, m)
    r16 = true_rel_res(op, B, X16.cpu().numpy())
    c64 = context(dims, True, fat, lng, m, tol=1e-8, prec="fp64")
    X64, i64 = c64.solve(to_dev(B))
    d = np.linalg.norm((X16 - X64).cpu().numpy()) / np.linalg.norm(X64.cpu().numpy())
    print(f"{prec}: iters={i16['iters']} rus={i16['reliable_updates']} (fp64 iters={i64['iters']}) "
          f"max res={r16.max():.2e} ||X16-X64||/||X64||={d:.2e}")
    assert r16.max() <= 1e-8
    assert i16["reliable_updates"] >= 1


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fix16"])
def test_sloppy_iterates_track_fp64(prec):
    """The first iterations in reduced storage stay close to the FP64 iterates
    (error of the order of the storage precision times the small growth of a
    few iterations)."""
    dims = (6, 6, 6, 6)
    fat, lng, B = inputs(dims, True, 4, 6700)
    m = 0.2
    # fix16: half a step of q / 32767 relative to the largest component of the group
    eps = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "fix16": 2.0 ** -16}[prec]
    c = context(dims, True, fat, lng, m, tol=1e-14, prec=prec, ru_delta=0.0, max_iter=3)
    Xs, _ = c.solve(to_dev(B), raise_on_error=False)
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    err = col_rel_err(Xs.cpu().numpy(), Xo).max()
    print(f"{prec}: 3-iteration error {err:.2e} (storage eps {eps:.1e})")
    assert err <= 200 * eps


@pytest.mark.parametrize("prec,n", [("fp64", 16), ("fp64", 5), ("fp32", 8), ("bf16", 3)])
def test_fused_gram_path_matches_oracle(prec, n):
    """Gram products fused into the hop and pass epilogues (G = 4 m^2 P^H P + T^H T)."""
    dims = (8, 8, 6, 6)
    fat, lng, B = inputs(dims, True, n, 6800 + n)
    m = 0.1
    tol = 1e-10 if prec == "fp64" else 1e-8
    ctx = context(dims, True, fat, lng, m, tol=tol, prec=prec)
    ctx.set_option("fuse_gram", 1)
    if n > 8:
        # the default two lane groups per workgroup would need more LDS than the fused
        # epilogue may take (the solver would then quietly use the separate Grams)
        ctx.set_option("hop_tpb", 4)
    ctx.set_profiling(["gram"])
    X, info = ctx.solve(to_dev(B))
    gram_launches, _ = ctx.kernel_time("gram")
    ctx.set_profiling([])
    # fused: separate Gram kernels only for the initial QR and the reliable updates
    assert gram_launches < info["iters"], f"fused path not taken ({gram_launches} Gram launches)"
    op = oracle.Operator(dims, fat, lng, m)
    assert true_rel_res(op, B, X.cpu().numpy()).max() <= tol
    if prec == "fp64":
        ctx2 = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=4)
        ctx2.set_option("fuse_gram", 1)
        if n > 8:
            ctx2.set_option("hop_tpb", 4)
        X4, _ = ctx2.solve(to_dev(B), raise_on_error=False)
        Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=4)
        assert col_rel_err(X4.cpu().numpy(), Xo).max() <= 1e-10


@pytest.mark.parametrize("kernel,tr,tpb,pf,cpt", [(2, 1, 4, 1, 1), (2, 2, 2, 0, 2), (2, 8, 1, 1, 4), (2, 4, 4, 1, 2),
                                                  (2, 8, 2, 1, 4), (1, 1, 0, 0, 1), (1, 2, 0, 1, 2), (1, 8, 0, 1, 4),
                                                  (0, 0, 0, 0, 0), (3, 8, 0, 1, 4), (3, 4, 0, 0, 2), (3, 1, 0, 1, 1)])
def test_launch_shapes_match_oracle(kernel, tr, tpb, pf, cpt):
    """The hop kernels (direction split with runs of 16 or 32 sites, site-parallel)
    with every register tile, lane-group and pipelining choice, and every pass
    column tile, give the same operator and iterates."""
    dims = (6, 6, 6, 6)
    n = 9
    fat, lng, B = inputs(dims, True, n, 6900)
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    for prec, tol in [("fp64", 1e-12), ("fp32", 1e-5)]:
        ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3, prec=prec)
        for name, v in [("hop_kernel", kernel), ("hop_tr", tr), ("hop_tpb", tpb), ("hop_pipeline", pf),
                        ("pass_cpt", cpt)]:
            ctx.set_option(name, v)
        assert col_rel_err(ctx.apply(to_dev(B)).cpu().numpy(), op.apply(B)).max() <= 1e-12
        X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
        Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
        assert col_rel_err(X3.cpu().numpy(), Xo).max() <= (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec,tol_x", [("fp32", 1e-4), ("bf16", 5e-2)])
def test_single_column_sloppy_iterates_match_oracle(prec, tol_x):
    """One right-hand side in reduced storage with the lane-split hop on runs of 32
    sites (the default for N = 1 below FP64 on large lattices, chosen here
    explicitly): the first iterates stay within the storage precision of the
    oracle's."""
    dims = (6, 6, 6, 8)
    fat, lng, B = inputs(dims, True, 1, 6950)
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3, prec=prec)
    ctx.set_option("hop_kernel", 3)
    X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
    assert col_rel_err(X3.cpu().numpy(), Xo).max() <= tol_x


@pytest.mark.parametrize("n", [16, 24, 40, 64])
def test_gram_kernels_match_oracle(n):
    """Matrix-core (FP64 MFMA, Hermitian upper tiles) and vector-ALU Gram kernels
    give the same iterates as the oracle, for one, two and four 16-column tiles
    (ragged N included)."""
    dims = (6, 6, 6, 8)
    fat, lng, B = inputs(dims, True, n, 7000 + n)
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    for kernel in (1, 2):
        ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3)
        ctx.set_option("gram_kernel", kernel)
        X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
        assert col_rel_err(X3.cpu().numpy(), Xo).max() <= 1e-10, f"gram_kernel={kernel}"
    for prec in ("fp32", "bf16"):
        ctx = context(dims, True, fat, lng, m, tol=1e-8, prec=prec)
        X, info = ctx.solve(to_dev(B))
        assert true_rel_res(op, B, X.cpu().numpy()).max() <= 1e-8


@pytest.mark.parametrize("n,threads", [(4, 64), (16, 64), (16, 1024), (32, 256), (64, 1024), (1, 0), (7, 0)])
def test_small_kernel_threads_match_oracle(n, threads):
    """The one-workgroup N x N kernels give the same iterates with one, four or
    sixteen waves (a request that would exceed four entries per thread falls back;
    threads = 0 is the default choice by N)."""
    dims = (6, 6, 6, 8)
    fat, lng, B = inputs(dims, True, n, 7100 + n)
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3)
    ctx.set_option("small_threads", threads)
    X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
    assert col_rel_err(X3.cpu().numpy(), Xo).max() <= 1e-10


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dims", [(8, 8, 8, 6), (6, 6, 6, 8), (4, 8, 8, 8)])
def test_site_orders_match_oracle(order, dims):
    """Slab and lexicographic workgroup orders cover every site exactly once: the
    operator and the first iterates match the oracle for lattices whose time slice
    is and is not a whole number of eight-way blocks."""
    n = 6
    fat, lng, B = inputs(dims, True, n, 7200 + dims[0])
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    for prec, tol_x in (("fp64", 1e-10), ("fp32", 1e-4)):
        ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3, prec=prec)
        ctx.set_option("site_order", order)
        assert col_rel_err(ctx.apply(to_dev(B)).cpu().numpy(), op.apply(B)).max() <= 1e-12
        X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
        assert col_rel_err(X3.cpu().numpy(), Xo).max() <= tol_x


@pytest.mark.parametrize("n", [5, 16, 17, 32, 40, 64])
def test_pass_kernels_match_oracle(n):
    """Matrix-core (FP64 MFMA, transposed column tiles, triangular K-steps skipped;
    used for 16 < N <= 32, pass A in FP64 also for 32 < N <= 64, and the FP32-MFMA
    forms for FP32 at 32 < N <= 64), LDS-staged vector and scalar-load vector passes A
    and B give the oracle's iterates (FP64, FP32) and converged solves (FP32, FP16,
    BF16)."""
    dims = (6, 6, 6, 8)
    fat, lng, B = inputs(dims, True, n, 7300 + n)
    m = 0.15
    op = oracle.Operator(dims, fat, lng, m)
    Xo, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=3)
    for prec, tol_x in (("fp64", 1e-10), ("fp32", 1e-4)):
        for kernel in (1, 2, 3):
            ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=0.0, max_iter=3, prec=prec)
            ctx.set_option("pass_kernel", kernel)
            X3, _ = ctx.solve(to_dev(B), raise_on_error=False)
            assert col_rel_err(X3.cpu().numpy(), Xo).max() <= tol_x, f"{prec} pass_kernel={kernel}"
    for prec in ("fp32", "fp16", "bf16", "fix16"):
        for kernel in (1, 3):
            ctx = context(dims, True, fat, lng, m, tol=1e-8, prec=prec)
            ctx.set_option("pass_kernel", kernel)
            X, info = ctx.solve(to_dev(B))
            assert true_rel_res(op, B, X.cpu().numpy()).max() <= 1e-8, f"{prec} pass_kernel={kernel}"


@pytest.mark.parametrize("dims,n", [((6, 6, 6, 8), 4), ((8, 8, 8, 8), 16), ((6, 6, 6, 8), 33)])
def test_graph_replays_match_eager(dims, n):
    """The iteration loop replayed from a captured HIP graph (many replays per solve,
    with eager work and host synchronisations between them) gives bit-identical
    iterates to eager launches, on two solves in a row with different column counts,
    and the solution still meets the oracle's residual bound."""
    precs = (("fp64", 1e-10), ("fp32", 1e-8), ("bf16", 1e-8)) if n <= 16 else (("fp64", 1e-10), ("fp32", 1e-8))
    _graph_vs_eager(dims, n, precs)


@pytest.mark.skip(reason="BF16 storage does not converge here: on 4x4x4x8 with 33 columns (768 rows) the "
                         "BF16 iteration diverges after its second reliable update (oracle BF16 emulation: "
                         "iterated residual > 1e8), and the reliable-update CholQR of the diverged residual "
                         "broke down; test_gpu_stability.py checks that the solver now stops cleanly")
def test_graph_replays_match_eager_bf16_n33():
    _graph_vs_eager((4, 4, 4, 8), 33, (("bf16", 1e-8),))


def _graph_vs_eager(dims, n, precs):
    fat, lng, B = inputs(dims, True, n, 7400 + n)
    m = 0.12
    op = oracle.Operator(dims, fat, lng, m)
    for prec, tol in precs:
        out = {}
        for graph in (2, 1):
            ctx = context(dims, True, fat, lng, m, tol=tol, prec=prec)
            ctx.set_option("graph", graph)
            X1, i1 = ctx.solve(to_dev(B))
            X2, i2 = ctx.solve(to_dev(B[: max(1, n // 2)]))
            out[graph] = (X1.cpu().numpy(), i1["iters"], X2.cpu().numpy(), i2["iters"])
        e, g = out[2], out[1]
        assert e[1] == g[1] and e[3] == g[3], f"{prec}: iterations eager {e[1]},{e[3]} graph {g[1]},{g[3]}"
        assert np.array_equal(e[0], g[0]) and np.array_equal(e[2], g[2]), prec
        assert true_rel_res(op, B, g[0]).max() <= tol
