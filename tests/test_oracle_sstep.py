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
