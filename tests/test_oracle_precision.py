"""Pins of the oracle's low-precision emulation and of its safeguards for it.

* rounding: every emulated format against an independent conversion (torch's
  binary16 / bfloat16 casts) and against its round-trip bound relative to the
  group's largest component;
* CholQR2 (Alg. 2 applied twice) against Householder QR, and its orthogonality
  against single CholQR on an ill-conditioned block (the loss of orthogonality
  of CholQR grows like kappa^2 u, that of CholQR2 stays at u);
* adaptive reliable updates: in exact arithmetic a reliable update continues
  the recurrence (S = C^ C_k^{-1}), so forcing one every few iterations leaves
  the iterates of an FP64 solve unchanged to rounding;
* the double-half breakdown the paper reports (Sec. 8), reproduced with BF16
  storage emulation: without a safeguard the iteration spins, with the
  stagnation exit it stops in bounded iterations with the best iterate, while
  FP32 storage converges on the same problem.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import rounding
from paper_1710_09745_amd import synth

from test_oracle_solver import small_problem


def _groups(fmt, a, axes):
    return rounding.round_groups(a, fmt, axes)


@pytest.mark.parametrize("fmt,tdtype", [("fp16", torch.float16), ("bf16", torch.bfloat16)])
def test_16bit_rounding_matches_torch_casts(fmt, tdtype):
    r = synth.make_rng(21)
    v = synth.gaussian_complex(r, (3, 50, 3)) * np.exp(r.uniform(-8, 8, (3, 50, 1)))
    got = _groups(fmt, v, 1)
    s = np.maximum(np.abs(v.real.astype(np.float32)).max(-1, keepdims=True),
                   np.abs(v.imag.astype(np.float32)).max(-1, keepdims=True)).astype(np.float32)
    re = torch.from_numpy(v.real.astype(np.float32) * (np.float32(1) / s))
    im = torch.from_numpy(v.imag.astype(np.float32) * (np.float32(1) / s))
    ref_re = re.to(tdtype).float().numpy() * s
    ref_im = im.to(tdtype).float().numpy() * s
    assert np.array_equal(got.real, ref_re.astype(np.float64))
    assert np.array_equal(got.imag, ref_im.astype(np.float64))


def test_bf16_ties_to_even():
    x = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9], dtype=np.float32)
    got = rounding._to_bf16(x)
    assert list(got) == [1.0, 1.0 + 2.0 ** -6, 1.0]


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16", "fix16"])
def test_rounding_bounds(fmt):
    r = synth.make_rng(22)
    v = synth.gaussian_complex(r, (4, 200, 3)) * np.exp(r.uniform(-5, 5, (4, 200, 1)))
    got = _groups(fmt, v, 1)
    if fmt == "fp32":
        # each real relative to itself
        for a, b in ((got.real, v.real), (got.imag, v.imag)):
            assert np.all(np.abs(a - b) <= 2.0 ** -24 * np.abs(b) * (1 + 1e-12))
        return
    s = np.maximum(np.abs(v.real).max(-1, keepdims=True), np.abs(v.imag).max(-1, keepdims=True))
    u = rounding.UNIT_ROUNDOFF[fmt]
    # 16-bit rounding of x/s plus the binary32 steps (division, scale, product)
    bound = (u + 4 * 2.0 ** -24) * s
    assert np.all(np.abs(got.real - v.real) <= bound)
    assert np.all(np.abs(got.imag - v.imag) <= bound)
    # the bound is reached to within a factor of two (the format is not finer than claimed)
    assert np.abs(got - v).max() >= 0.25 * u * s.min()


def test_link_rounding_groups_per_matrix():
    r = synth.make_rng(23)
    U = synth.fat_links(r, (2, 2, 2, 2))
    U[1, 3] *= 1e4   # one large matrix does not coarsen its neighbours
    got = rounding.round_links(U, "bf16")
    rel = np.abs(got - U).max(axis=(-2, -1)) / np.abs(U).max(axis=(-2, -1))
    assert rel.max() <= 2.0 ** -8 * 1.01


def test_cholqr2_matches_householder_and_is_orthogonal():
    r = synth.make_rng(24)
    L, n = 400, 8
    U, _ = np.linalg.qr(synth.gaussian_complex(r, (L, n)))
    W, _ = np.linalg.qr(synth.gaussian_complex(r, (n, n)))
    M = (U * np.logspace(0, -6, n)[None, :]) @ W          # kappa(M) = 1e6
    Q1, R1 = oracle.thin_qr(M)
    Q2, R2 = oracle.thin_qr2(M)
    e1 = np.abs(Q1.conj().T @ Q1 - np.eye(n)).max()
    e2 = np.abs(Q2.conj().T @ Q2 - np.eye(n)).max()
    assert e1 > 1e-8          # CholQR: orthogonality lost like kappa^2 u
    assert e2 < 1e-13         # CholQR2: orthogonal to rounding
    q, rr = np.linalg.qr(M)
    ph = np.diag(rr) / np.abs(np.diag(rr))
    q = q * ph[None, :]
    rr = ph.conj()[:, None] * rr
    assert np.abs(Q2 - q).max() <= 1e-8
    assert np.abs(R2 - rr).max() <= 1e-12 * np.abs(rr).max()
    assert np.abs(np.tril(R2, -1)).max() <= 1e-20 and np.all(np.diag(R2).real > 0)
    assert np.abs(Q2 @ R2 - M).max() <= 1e-13 * np.abs(M).max()


def test_cholqr2_solve_equals_cholqr_solve():
    op, B = small_problem((4, 4, 4, 4), True, 0.1, 5)
    X1, i1 = oracle.block_cg_rq(op.apply, B, 1e-11, ru_delta=0.1)
    X2, i2 = oracle.block_cg_rq(op.apply, B, 1e-11, qr_passes=2, ru_delta=0.1)
    assert i2.reliable_updates >= 3
    assert abs(i1.iters - i2.iters) <= 1
    assert np.linalg.norm(X1 - X2) / np.linalg.norm(X1) <= 1e-9


@pytest.mark.parametrize("window,min_updates", [(1, 4), (3, 1)])
def test_forced_reliable_updates_do_not_change_fp64_iterates(window, min_updates):
    """ru_window forces a reliable update whenever the residual has not reached a
    new minimum for `window` iterations (window = 1: every iteration that fails
    to improve).  Each update continues the recurrence, so the iterates stay
    those of the plain solve (S = C^ C_k^{-1}, the reading of Alg. 3)."""
    op, B = small_problem((4, 4, 4, 6), True, 0.08, 4, seed=31)
    k = 12
    X0, _ = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k)
    # a tiny ru_delta is never met; the window alone triggers the updates
    X1, i1 = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k, ru_window=window, ru_delta=1e-300)
    assert i1.reliable_updates >= min_updates
    assert np.linalg.norm(X1 - X0) / np.linalg.norm(X0) <= 1e-12


def test_window_triggers_on_stagnation():
    """A sloppy operator that is wrong by a constant factor makes the iterated
    residual stop falling; the window then forces reliable updates."""
    op, B = small_problem((4, 4, 4, 4), True, 0.1, 3, seed=33)
    wrong = oracle.Operator(op.dims, op.fat * 1.3, op.lng * 1.3, op.mass)
    tr = []
    _, info = oracle.block_cg_rq(op.apply, B, 1e-10, max_iter=400, ru_delta=0.1, apply_sloppy=wrong.apply,
                                 ru_window=20, trace=tr)
    assert info.reliable_updates >= 2


def _bf16_problem():
    dims, m, n = (4, 4, 4, 8), 0.02, 8
    r = synth.make_rng(11)
    fat = synth.fat_links(r, dims)
    lng = synth.long_links(r, dims)
    B = synth.rhs(synth.make_rng(12), n, dims)
    op = oracle.Operator(dims, fat, lng, m)
    return op, B


def _sloppy_run(op, B, fmt, **kw):
    ops = oracle.Operator(op.dims, rounding.round_links(op.fat, fmt), rounding.round_links(op.lng, fmt), op.mass)
    tr = []
    X, info = oracle.block_cg_rq(op.apply, B, 1e-8, ru_delta=0.1, sloppy=rounding.vector_rounder(fmt, op.Vh),
                                 apply_sloppy=ops.apply, trace=tr, **kw)
    return X, info, tr


@pytest.mark.slow
def test_bf16_storage_stagnates_and_stall_exit_stops_it():
    """The double-half breakdown of Sec. 8 on a 4^3 x 8 lattice at m = 0.02 (the
    32^3 x 64 workload's mass): with BF16 vectors and links the first reliable
    update finds a true residual far above the iterated one, and afterwards
    the iterated residual never falls by the factor ru_delta asks for, so no
    further update fires and the solve would run to max_iter.  The adaptive
    window makes the updates happen; the stall limit then ends the solve, with
    the best iterate returned.  FP32 storage converges on the same problem."""
    op, B = _bf16_problem()
    _, i32, _ = _sloppy_run(op, B, "fp32", ru_window=100, stall_limit=3, max_iter=3000)
    assert i32.converged and i32.true_rel_res.max() <= 1e-8
    # no safeguard: spins until max_iter with at most a couple of updates
    _, i0, tr0 = _sloppy_run(op, B, "bf16", max_iter=600)
    assert not i0.converged and i0.iters == 600 and i0.reliable_updates <= 2
    first_ru = next(t for t in tr0 if t.get("ru"))
    assert first_ru["true_rel"].max() > 2 * first_ru["relres"].max()   # iterated residual drifted off
    # safeguards: stops by itself, well before max_iter, on the best iterate
    X, i1, tr1 = _sloppy_run(op, B, "bf16", ru_window=100, stall_limit=3, max_iter=3000)
    assert i1.stalled and not i1.converged and i1.iters < 1500
    trues = [t["true_rel"].max() for t in tr1 if "true_rel" in t]
    assert np.isclose(i1.true_rel_res.max(), min([1.0] + trues), rtol=1e-6)
    res = np.linalg.norm(oracle.to_mat(B - op.apply(X)), axis=0) / np.linalg.norm(oracle.to_mat(B), axis=0)
    assert np.allclose(res, i1.true_rel_res, rtol=1e-10)
