"""GPU parity of the low-precision safeguards: adaptive reliable updates, the
stagnation exit and CholQR2 (bcg_set_stability), against the CPU oracle run
with the same rules."""
import numpy as np
import pytest

import oracle
from paper_1710_09745_amd import bcg, synth

from gpu_util import col_rel_err, context, inputs, to_dev, true_rel_res

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forced_reliable_updates_match_oracle(prec):
    """ru_window = 1 forces a reliable update after every iteration that does not
    reach a new minimum of the iterated residual; the iterates still match the
    oracle's under the same rule (the updates continue the recurrence)."""
    dims = (4, 4, 4, 6)
    fat, lng, B = inputs(dims, True, 4, 31)
    m, k = 0.08, 12
    op = oracle.Operator(dims, fat, lng, m)
    Xo, io = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k, ru_window=1, ru_delta=1e-300)
    assert io.reliable_updates >= 4
    ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=1e-300, max_iter=k, prec=prec)
    ctx.set_stability(ru_window=1, stall_limit=0)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    assert info["rc"] == bcg.ERR_NOT_CONVERGED and info["iters"] == k
    assert info["reliable_updates"] == io.reliable_updates
    assert col_rel_err(X.cpu().numpy(), Xo).max() <= (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec,n", [("fp64", 5), ("fp64", 24), ("fp32", 16)])
def test_cholqr2_matches_oracle(prec, n):
    """CholQR2 in the initial and reliable-update QR: iterates through several
    reliable updates match the oracle's CholQR2 run; converged solves meet the
    residual bound by the oracle's operator."""
    dims = (6, 6, 4, 6)
    fat, lng, B = inputs(dims, True, n, 8200 + n)
    m = 0.1
    op = oracle.Operator(dims, fat, lng, m)
    k = 10
    Xo, io = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k, ru_window=1, ru_delta=1e-300, qr_passes=2)
    assert io.reliable_updates >= 2
    ctx = context(dims, True, fat, lng, m, tol=1e-14, ru_delta=1e-300, max_iter=k, prec=prec)
    ctx.set_stability(ru_window=1, stall_limit=0, qr_passes=2)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    assert info["iters"] == k
    if prec == "fp64":
        assert info["reliable_updates"] == io.reliable_updates
    assert col_rel_err(X.cpu().numpy(), Xo).max() <= (1e-10 if prec == "fp64" else 1e-4)
    tol = 1e-10 if prec == "fp64" else 1e-8
    ctx = context(dims, True, fat, lng, m, tol=tol, prec=prec)
    ctx.set_stability(qr_passes=2)
    X, info = ctx.solve(to_dev(B))
    assert true_rel_res(op, B, X.cpu().numpy()).max() <= tol


def _bf16_problem():
    dims, m, n = (4, 4, 4, 8), 0.02, 8
    r = synth.make_rng(11)
    fat = synth.fat_links(r, dims)
    lng = synth.long_links(r, dims)
    B = synth.rhs(synth.make_rng(12), n, dims)
    return dims, m, fat, lng, B


def test_bf16_stagnation_exits_with_best_iterate():
    """The double-half breakdown (Sec. 8) at m = 0.02: BF16 storage cannot reach
    1e-8 on this operator (the oracle's BF16 emulation stagnates near 0.75).
    The solver must stop by itself with NOT_CONVERGED well before max_iter and
    return the iterate with the smallest true residual it checked; FP32 storage
    converges on the same problem."""
    dims, m, fat, lng, B = _bf16_problem()
    op = oracle.Operator(dims, fat, lng, m)
    c32 = context(dims, True, fat, lng, m, tol=1e-8, prec="fp32", max_iter=3000)
    X32, i32 = c32.solve(to_dev(B))
    assert true_rel_res(op, B, X32.cpu().numpy()).max() <= 1e-8
    ctx = context(dims, True, fat, lng, m, tol=1e-8, prec="bf16", max_iter=20000)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    msg = ctx.lib.bcg_last_error(ctx.h).decode()
    print(f"bf16: rc={info['rc']} ({msg}) iters={info['iters']} rus={info['reliable_updates']} best max true "
          f"res={info['max_true_rel_res']:.3e} (fp32 converged in {i32['iters']})")
    # stops by stagnation (or a reliable-update QR breakdown), never by max_iter
    assert info["rc"] in (bcg.ERR_NOT_CONVERGED, bcg.ERR_BREAKDOWN) and info["iters"] < 5000
    if info["rc"] == bcg.ERR_NOT_CONVERGED:
        assert "stagnated" in msg
    res = true_rel_res(op, B, X.cpu().numpy())
    assert np.allclose(res, info["true_rel_res"], rtol=1e-6)
    assert res.max() <= 1.0 + 1e-12      # never worse than the start (X = 0)


def test_diverging_bf16_block_stops_cleanly():
    """BF16 storage with 33 columns on a 768-row problem (4^3 x 8): the oracle's
    BF16 emulation diverges after its second reliable update (the iterated
    residual grows past 1e8).  The solver must stop by itself with a
    NOT_CONVERGED or BREAKDOWN status and a finite best iterate, never hang."""
    dims, n = (4, 4, 4, 8), 33
    fat, lng, B = inputs(dims, True, n, 7400 + n)
    m = 0.12
    op = oracle.Operator(dims, fat, lng, m)
    ctx = context(dims, True, fat, lng, m, tol=1e-8, prec="bf16", max_iter=20000)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    print(f"bf16 n=33: rc={info['rc']} iters={info['iters']} rus={info['reliable_updates']} "
          f"max true res={info['max_true_rel_res']:.3e}")
    assert info["rc"] in (bcg.OK, bcg.ERR_NOT_CONVERGED, bcg.ERR_BREAKDOWN)
    assert info["iters"] < 5000
    Xh = X.cpu().numpy()
    assert np.all(np.isfinite(Xh))
    res = true_rel_res(op, B, Xh)
    assert np.allclose(res, info["true_rel_res"], rtol=1e-6)
    if info["rc"] == bcg.OK:
        assert res.max() <= 1e-8
