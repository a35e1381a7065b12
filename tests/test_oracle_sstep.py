"""Pins of the oracle's s-step block CG.

* brute force on tiny inputs: after k outer iterations the iterate is the Galerkin
  solution over the block Krylov space K_{ks}(A, B) (X = Qb (Qb^H A Qb)^{-1} Qb^H B
  with Qb an orthonormal basis from a block Arnoldi process with full
  re-orthogonalisation on the dense A), for s = 1 ... 4;
* invariance: the Chebyshev and the monomial basis, and different Chebyshev
  intervals, give the same iterates (the search space does not depend on the
  basis polynomials);
* special case: s = 1 is block CG, so its iterates match blockCGrQ's iteration by
  iteration;
* solves reach the dense solution; the true-residual restart path is taken when
  the iterated residual meets tol before the true one does.
"""
import numpy as np
import pytest

import oracle
from paper_1710_09745_amd import synth

from test_oracle_operator import dense_A


def problem(dims=(4, 4, 4, 4), improved=False, m=0.1, n=4, seed=21):
    r = synth.make_rng(seed)
    fat = synth.fat_links(r, dims)
    lng = synth.long_links(r, dims) if improved else None
    op = oracle.Operator(dims, fat, lng, m)
    B = synth.rhs(synth.make_rng(seed + 1), n, dims)
    return op, B


def spectrum(Ad):
    ev = np.linalg.eigvalsh(Ad)
    return float(ev[0]), float(ev[-1])


def galerkin(Ad, Bm, dim_blocks):
    """Galerkin solution over K_m(A, B), m = dim_blocks blocks, from an orthonormal
    block Arnoldi basis (two Gram-Schmidt passes per block)."""
    Q0, _ = np.linalg.qr(Bm)
    blocks = [Q0]
    for _ in range(dim_blocks - 1):
        Wb = Ad @ blocks[-1]
        for _ in range(2):
            for Qj in blocks:
                Wb = Wb - Qj @ (Qj.conj().T @ Wb)
        Qn, _ = np.linalg.qr(Wb)
        blocks.append(Qn)
    Qb = np.hstack(blocks)
    y = np.linalg.solve(Qb.conj().T @ Ad @ Qb, Qb.conj().T @ Bm)
    return Qb @ y


@pytest.fixture(scope="module")
def p1():
    op, B = problem()
    Ad = dense_A(op)
    return op, B, Ad, spectrum(Ad)


@pytest.mark.parametrize("s,k", [(1, 3), (2, 1), (2, 3), (3, 2), (4, 1), (4, 2)])
def test_iterates_are_block_krylov_galerkin(p1, s, k):
    op, B, Ad, lam = p1
    X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=k)
    assert info.outer == k and info.iters == k * s and not info.converged
    Xg = galerkin(Ad, oracle.to_mat(B), k * s)
    Xm = oracle.to_mat(X)
    assert np.linalg.norm(Xm - Xg) <= 1e-9 * np.linalg.norm(Xg)


def test_basis_does_not_change_iterates(p1):
    op, B, Ad, lam = p1
    ref, _ = oracle.sstep_block_cg(op.apply, B, 3, 1e-14, lam, max_outer=2)
    for basis, lm in [("monomial", lam), ("chebyshev", (0.5 * lam[0], 1.2 * lam[1])),
                      ("chebyshev", (lam[0], 0.9 * lam[1]))]:
        X, _ = oracle.sstep_block_cg(op.apply, B, 3, 1e-14, lm, max_outer=2, basis=basis)
        assert np.linalg.norm(oracle.to_mat(X - ref)) <= 1e-8 * np.linalg.norm(oracle.to_mat(ref))


def test_s1_matches_block_cg_rq(p1):
    op, B, Ad, lam = p1
    for k in (1, 2, 5):
        X1, _ = oracle.sstep_block_cg(op.apply, B, 1, 1e-14, lam, max_outer=k)
        X2, info = oracle.block_cg_rq(op.apply, B, 1e-14, max_iter=k)
        assert info.iters == k
        assert np.linalg.norm(oracle.to_mat(X1 - X2)) <= 1e-10 * np.linalg.norm(oracle.to_mat(X2))


@pytest.mark.parametrize("s", [1, 2, 4])
@pytest.mark.parametrize("improved,n", [(False, 4), (True, 3)])
def test_solve_reaches_dense_solution(s, improved, n):
    op, B = problem(improved=improved, n=n, m=0.2 if improved else 0.1, seed=31)
    Ad = dense_A(op)
    lam = spectrum(Ad)
    X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-10, lam)
    assert info.converged and info.true_rel_res.max() <= 1e-10
    Xd = np.linalg.solve(Ad, oracle.to_mat(B))
    kappa = lam[1] / lam[0]
    assert np.linalg.norm(oracle.to_mat(X) - Xd) <= 2e-10 * kappa * np.linalg.norm(Xd)
    # the iterate after k outer iterations minimises the A-norm error over the
    # same space as k s block-CG iterations, so it cannot stop much earlier; in
    # floating point the s-step recurrence loses A-orthogonality to the older
    # blocks and needs more steps (up to 2x here at s = 4 on the naive operator)
    _, i1 = oracle.block_cg_rq(op.apply, B, 1e-10)
    assert i1.iters - s <= info.iters <= 2.5 * i1.iters


@pytest.mark.parametrize("s", [1, 2])
def test_restart_from_true_residual(p1, s):
    op, B, Ad, lam = p1
    # at tol 1e-14 the iterated residual passes tol before the true one can (its
    # attainable accuracy is a few ulps times the condition): the true-residual
    # check must restart the recurrence, which then converges
    X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=400 // s)
    assert info.restarts >= 1
    assert info.converged and info.true_rel_res.max() <= 1e-14
    r = np.linalg.norm(oracle.to_mat(B) - Ad @ oracle.to_mat(X), axis=0) / np.linalg.norm(oracle.to_mat(B), axis=0)
    assert r.max() <= 2e-14


def test_zero_column_and_bad_s(p1):
    op, B, Ad, lam = p1
    Bz = B.copy()
    Bz[2] = 0
    with pytest.raises(ValueError):
        oracle.sstep_block_cg(op.apply, Bz, 2, 1e-10, lam)
    with pytest.raises(ValueError):
        oracle.sstep_block_cg(op.apply, B, 0, 1e-10, lam)


def _fp32_storage(op):
    """The emulated FP32 storage of the solver's sloppy path: links, the apply's
    input, its odd-parity intermediate and its output rounded to binary32."""
    from oracle import rounding
    lng = rounding.round_links(op.lng, "fp32") if op.improved else None
    ops = oracle.Operator(tuple(int(d) for d in op.dims), rounding.round_links(op.fat, "fp32"), lng, op.mass)

    def apply_sloppy(v):
        P = rounding.round_groups(v, "fp32", 1)
        T = rounding.round_groups(ops.hop(1, P), "fp32", 1)
        return rounding.round_groups(4 * op.mass * op.mass * P - ops.hop(0, T), "fp32", 1)

    return rounding.vector_rounder("fp32", op.Vh), apply_sloppy


def test_reliable_update_is_a_no_op_in_fp64(p1):
    """R replaced by B - A X at (almost) every outer iteration: in exact arithmetic the
    replacement is the identity, so the iterates agree with the plain recurrence's."""
    op, B, Ad, lam = p1
    for s in (1, 3):
        ref, _ = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=6)
        X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=6, ru_delta=0.9999)
        assert info.reliable_updates >= 1
        assert np.linalg.norm(oracle.to_mat(X - ref)) <= 1e-10 * np.linalg.norm(oracle.to_mat(ref))


@pytest.mark.parametrize("improved,n,m,s", [(False, 4, 0.1, 1), (False, 4, 0.1, 2), (False, 4, 0.1, 4),
                                             (True, 4, 0.05, 1), (True, 4, 0.05, 2)])
def test_fp32_storage_with_reliable_updates(improved, n, m, s):
    """FP32 storage of V, AV, P, AP and FP32 links in the basis: with reliable updates
    every 10x drop the solve reaches 1e-8 by the FP64 operator without a restart.  It
    needs more steps than blockCGrQ in the same storage (the s-step recurrence works on
    the raw residual block, not on an orthonormal one: 1.0-1.2x on the naive operator,
    1.3x at s = 1 and 1.7x at s = 2 on the improved one), and fewer than the same solve
    without reliable updates, whose iterated residual drifts from the true one until a
    restart is needed."""
    op, B = problem(improved=improved, n=n, m=m, seed=31)
    Ad = dense_A(op)
    lam = spectrum(Ad)
    rnd, As = _fp32_storage(op)
    X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-8, lam, max_outer=2000 // s, sloppy=rnd,
                                    apply_sloppy=As, ru_delta=0.1)
    assert info.converged and info.restarts == 0 and info.reliable_updates >= 1
    r = np.linalg.norm(oracle.to_mat(B) - Ad @ oracle.to_mat(X), axis=0) / np.linalg.norm(oracle.to_mat(B), axis=0)
    assert r.max() <= 1e-8
    _, ib = oracle.block_cg_rq(op.apply, B, 1e-8, ru_delta=0.1, sloppy=rnd, apply_sloppy=As)
    assert info.iters <= 1.8 * ib.iters + s
    _, i0 = oracle.sstep_block_cg(op.apply, B, s, 1e-8, lam, max_outer=2000 // s, sloppy=rnd, apply_sloppy=As)
    assert i0.restarts >= 1 and i0.iters > info.iters


@pytest.mark.parametrize("s", [1, 2, 3])
def test_fp32_storage_iterates_stay_near_fp64(p1, s):
    """A few outer iterations in emulated FP32 storage move the iterate by a small
    multiple of FP32's unit roundoff from the FP64 iterate, and by more than FP64
    rounding: the storage rounding is applied, and nothing else changes."""
    op, B, Ad, lam = p1
    rnd, As = _fp32_storage(op)
    ref, _ = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=2)
    X, info = oracle.sstep_block_cg(op.apply, B, s, 1e-14, lam, max_outer=2, sloppy=rnd, apply_sloppy=As)
    assert info.outer == 2 and info.reliable_updates == 0
    err = np.linalg.norm(oracle.to_mat(X - ref)) / np.linalg.norm(oracle.to_mat(ref))
    assert 1e-12 < err <= 200 * 2.0 ** -24
