"""GPU parity of the s-step block CG (bcg_solve_sstep) against the oracle's
sstep_block_cg.

* iterates after k outer iterations, for s = 1 ... 8 and s * N up to 64, on a
  lattice with a ragged site tail: both sides use the same Chebyshev interval, so
  the only differences are rounding orders (the oracle's W stays below 1.5e5 in
  condition on these cases and its iterates move by about 1e-13 under a 1e-13
  perturbation of B, so 1e-10 leaves a wide margin);
* converged solves with the library's own interval (4 m^2 and a power-iteration
  estimate of the largest eigenvalue): true residual by the oracle's FP64 operator,
  distance to the blockCGrQ solution, s-step counts against block CG's;
* argument errors and determinism.
"""
import numpy as np
import pytest

import oracle
from paper_1710_09745_amd import bcg

from gpu_util import col_rel_err, context, elem_rel_err, inputs, kappa_bound, to_dev, true_rel_res

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 6, 6)   # V/2 = 432 sites: six full 64-site blocks and a ragged tail
MASS = 0.1


def interval(op, B, iters=60):
    """(4 m^2, 1.1 lambda_max) with lambda_max from an oracle power iteration."""
    v = B[:1].copy()
    lam = 0.0
    for _ in range(iters):
        w = op.apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return 4 * op.mass * op.mass, 1.1 * lam


@pytest.fixture(scope="module")
def prob():
    fat, lng, B = inputs(DIMS, True, 32, 7000)
    op = oracle.Operator(DIMS, fat, lng, MASS)
    return fat, lng, B, op, interval(op, B)


@pytest.mark.parametrize("s,n,k", [(1, 5, 3), (2, 5, 2), (3, 4, 2), (2, 1, 3), (5, 3, 2),
                                   (4, 16, 1), (4, 16, 2), (2, 32, 2), (8, 8, 2)])
def test_iterates_match_oracle(prob, s, n, k):
    fat, lng, B, op, lam = prob
    Bn = B[:n]
    ctx = context(DIMS, True, fat, lng, MASS, tol=1e-14, max_iter=k * s)
    print(f"[case] s-step s={s} n={n} outer={k}", flush=True)
    X, info = ctx.solve_sstep(to_dev(Bn), s, lam[0], lam[1], raise_on_error=False)
    assert info["rc"] == bcg.ERR_NOT_CONVERGED and info["iters"] == k * s
    Xo, io = oracle.sstep_block_cg(op.apply, Bn, s, 1e-14, lam, max_outer=k)
    assert io.outer == k
    Xg = X.cpu().numpy()
    assert col_rel_err(Xg, Xo).max() <= 1e-10
    assert elem_rel_err(Xg, Xo).max() <= 1e-10
    # the library's true residuals of the returned iterate
    assert np.allclose(info["true_rel_res"], true_rel_res(op, Bn, Xg), rtol=1e-6)


@pytest.mark.parametrize("dims,n,s", [((8, 8, 8, 8), 8, 2), ((8, 8, 8, 8), 8, 4), ((6, 6, 6, 8), 16, 3)])
def test_solve_converges(dims, n, s):
    fat, lng, B = inputs(dims, True, n, 7100 + n + s)
    m = 0.1
    ctx = context(dims, True, fat, lng, m, tol=1e-10)
    print(f"[case] s-step solve s={s} n={n}", flush=True)
    X, info = ctx.solve_sstep(to_dev(B), s)
    Xb, ib = ctx.solve(to_dev(B))
    op = oracle.Operator(dims, fat, lng, m)
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"s-step s={s}: {info['iters']} steps ({info['iters'] // s} outer), restarts {info['restarts']}; "
          f"block CG {ib['iters']} iterations; max res {res.max():.2e}")
    assert res.max() <= 1e-10
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3, atol=1e-14)
    # the s-step space after k outer iterations is block CG's after k s iterations:
    # neither stops much earlier than the other in floating point (rounding delays
    # both by a few per cent), and rounding costs the s-step form at most a factor
    assert 0.9 * ib["iters"] - s <= info["iters"] <= 2.5 * ib["iters"]
    kappa = kappa_bound(op)
    assert col_rel_err(X.cpu().numpy(), Xb.cpu().numpy()).max() <= kappa * 2e-10


def test_arguments(prob):
    fat, lng, B, op, lam = prob
    ctx = context(DIMS, True, fat, lng, MASS, tol=1e-10)
    Bd = to_dev(B[:16])
    for s, lo, hi in [(0, 0.0, 0.0), (5, 0.0, 0.0), (2, 2.0, 1.0), (2, float("nan"), 1.0)]:
        X, info = ctx.solve_sstep(Bd, s, lo, hi, raise_on_error=False)
        assert info["rc"] == bcg.ERR_ARG, (s, lo, hi)


def test_deterministic(prob):
    fat, lng, B, op, lam = prob
    ctx = context(DIMS, True, fat, lng, MASS, tol=1e-12)
    X1, i1 = ctx.solve_sstep(to_dev(B[:8]), 3)
    X2, i2 = ctx.solve_sstep(to_dev(B[:8]), 3)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(X1.cpu().numpy(), X2.cpu().numpy())


def test_restart_from_true_residual():
    """At tol 1e-14 the iterated residual passes tol before the true one can: the
    true-residual check restarts the recurrence (as in the oracle's pin on the same
    4^4 problem), and the solve ends within a few ulps of the attainable accuracy."""
    dims = (4, 4, 4, 4)
    fat, lng, B = inputs(dims, False, 4, 7300)
    ctx = context(dims, False, fat, lng, 0.1, tol=1e-14, max_iter=400)
    print("[case] s-step restart s=2 n=4 tol=1e-14", flush=True)
    X, info = ctx.solve_sstep(to_dev(B), 2, raise_on_error=False)
    op = oracle.Operator(dims, fat, lng, 0.1)
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"s-step restarts {info['restarts']}, rc {info['rc']}, steps {info['iters']}, max res {res.max():.2e}")
    assert info["restarts"] >= 1
    assert info["rc"] in (bcg.OK, bcg.ERR_NOT_CONVERGED)
    assert res.max() <= 5e-14
    if info["rc"] == bcg.OK:
        assert res.max() <= 1.01e-14


@pytest.mark.parametrize("s,n,k", [(1, 4, 3), (2, 4, 3), (3, 5, 2), (2, 16, 2), (3, 11, 2), (4, 16, 2)])
def test_fp32_iterates_track_oracle(prob, s, n, k):
    """FP32 storage of V, A V, P and A P (FP32 links and arithmetic in the basis
    apply; FP64 X, R and Grams), no reliable updates: the iterate after k outer
    iterations stays within a small multiple of FP32's unit roundoff of the oracle's
    emulation of the same storage (its apply rounds the input, the odd-parity
    intermediate and the output to binary32, the GPU's also rounds inside the stencil
    sums), and of the FP64 iterate.  K = s N up to 32 takes the two Grams of
    [V | P'], above it the five K-column Grams (two of them on the vector ALUs)."""
    from test_oracle_sstep import _fp32_storage

    fat, lng, B, op, lam = prob
    Bn = B[:n]
    ctx = context(DIMS, True, fat, lng, MASS, tol=1e-14, prec="fp32", ru_delta=0.0, max_iter=k * s)
    print(f"[case] s-step fp32 s={s} n={n} outer={k}", flush=True)
    X, info = ctx.solve_sstep(to_dev(Bn), s, lam[0], lam[1], raise_on_error=False)
    assert info["rc"] == bcg.ERR_NOT_CONVERGED and info["iters"] == k * s
    rnd, As = _fp32_storage(op)
    Xe, _ = oracle.sstep_block_cg(op.apply, Bn, s, 1e-14, lam, max_outer=k, sloppy=rnd, apply_sloppy=As)
    Xo, _ = oracle.sstep_block_cg(op.apply, Bn, s, 1e-14, lam, max_outer=k)
    Xg = X.cpu().numpy()
    eps = 2.0 ** -24
    e_emul, e64 = col_rel_err(Xg, Xe).max(), col_rel_err(Xg, Xo).max()
    print(f"fp32 s-step: error against the emulated oracle {e_emul:.2e}, against FP64 {e64:.2e}")
    assert e_emul <= 200 * eps
    assert e64 <= 200 * eps


@pytest.mark.parametrize("s", [1, 2])
def test_fp32_solve_with_reliable_updates(s):
    """FP32 storage with reliable updates every 10x drop reaches 1e-8 by the oracle's
    FP64 operator; the step count stays within the bound the oracle shows for the
    s-step recurrence in FP32 storage against blockCGrQ in the same storage."""
    dims = (8, 8, 8, 8)
    fat, lng, B = inputs(dims, True, 8, 6500)
    m = 0.05
    ctx = context(dims, True, fat, lng, m, tol=1e-8, prec="fp32", ru_delta=0.1, max_iter=20000)
    print(f"[case] s-step fp32 solve s={s} n=8 8^4", flush=True)
    X, info = ctx.solve_sstep(to_dev(B), s)
    Xb, ib = ctx.solve(to_dev(B))
    op = oracle.Operator(dims, fat, lng, m)
    res = true_rel_res(op, B, X.cpu().numpy())
    print(f"fp32 s-step s={s}: {info['iters']} steps, {info['reliable_updates']} reliable updates, "
          f"restarts {info['restarts']}; blockCGrQ fp32 {ib['iters']} iterations; max res {res.max():.2e}")
    assert res.max() <= 1e-8
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3, atol=1e-14)
    assert info["reliable_updates"] >= 1
    assert info["iters"] <= 1.8 * ib["iters"] + s


def test_16bit_storage_refused(prob):
    fat, lng, B, op, lam = prob
    for prec in ("fp16", "bf16", "fix16"):
        ctx = context(DIMS, True, fat, lng, MASS, tol=1e-10, prec=prec)
        X, info = ctx.solve_sstep(to_dev(B[:4]), 2, raise_on_error=False)
        assert info["rc"] == bcg.ERR_ARG
