"""GPU parity of the link force and of the autograd backward of the block solve
against the CPU oracle, and a central finite-difference check of the full
16^4, N = 8 workload (the loss L = Re sum_i b_i^H A^{-1} b_i)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1710_09745_amd import bcg, synth

from gpu_util import DEV, context, inputs, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,improved,n", [((4, 4, 4, 4), True, 3), ((6, 4, 6, 8), False, 5),
                                             ((8, 8, 6, 6), True, 9)])
def test_link_force_matches_oracle(dims, improved, n):
    fat, lng, X = inputs(dims, improved, n, 7000 + n)
    Lam = synth.rhs(synth.make_rng(7100 + n), n, dims)
    ctx = context(dims, improved, fat, lng, 0.1)
    gf, gl = ctx.link_force(to_dev(X), to_dev(Lam))
    op = oracle.Operator(dims, fat, lng, 0.1)
    rf, rl = op.link_force(X, Lam)
    assert np.abs(gf.cpu().numpy() - rf).max() <= 1e-12 * np.abs(rf).max()
    if improved:
        assert np.abs(gl.cpu().numpy() - rl).max() <= 1e-12 * np.abs(rl).max()


def test_autograd_backward_matches_oracle():
    dims = (4, 4, 4, 6)
    m = 0.2
    fat, lng, B = inputs(dims, True, 3, 7200)
    ctx = context(dims, True, fat, lng, m, tol=1e-12)
    Bt = to_dev(B).requires_grad_(True)
    ft = to_dev(fat).requires_grad_(True)
    lt = to_dev(lng).requires_grad_(True)
    X = bcg.BlockSolve.apply(Bt, ft, lt, ctx)
    loss = torch.real(torch.sum(Bt.conj() * X))
    loss.backward()
    op = oracle.Operator(dims, fat, lng, m)
    from test_oracle_operator import dense_A
    Xo = oracle.from_mat(np.linalg.solve(dense_A(op), oracle.to_mat(B)), op.Vh)
    rf, rl = op.link_force(Xo, Xo)
    assert np.abs(Bt.grad.cpu().numpy() - 2 * Xo).max() <= 1e-9 * np.abs(Xo).max()
    assert np.abs(ft.grad.cpu().numpy() - rf).max() <= 1e-9 * np.abs(rf).max()
    assert np.abs(lt.grad.cpu().numpy() - rl).max() <= 1e-9 * np.abs(rl).max()


@pytest.mark.parametrize("cols", [(0, 2), (1,), ()])
def test_autograd_backward_with_unused_columns(cols):
    """A loss that depends on some columns only: dL/dX is zero for the others, their
    Lam is zero (no solve of a zero right-hand side) and the link gradients are the
    oracle's link force of the used columns."""
    dims = (4, 4, 4, 6)
    m = 0.2
    fat, lng, B = inputs(dims, True, 3, 7250)
    ctx = context(dims, True, fat, lng, m, tol=1e-12)
    Bt = to_dev(B).requires_grad_(True)
    ft = to_dev(fat).requires_grad_(True)
    lt = to_dev(lng).requires_grad_(True)
    X = bcg.BlockSolve.apply(Bt, ft, lt, ctx)
    mask = torch.zeros(3, dtype=torch.float64, device=DEV)
    for c in cols:
        mask[c] = 1.0
    loss = torch.sum(mask[:, None, None] * torch.real(Bt.conj() * X))
    loss.backward()
    op = oracle.Operator(dims, fat, lng, m)
    from test_oracle_operator import dense_A
    Xo = oracle.from_mat(np.linalg.solve(dense_A(op), oracle.to_mat(B)), op.Vh)
    keep = list(cols)
    gB = np.zeros_like(B)
    gB[keep] = 2 * Xo[keep]
    assert np.abs(Bt.grad.cpu().numpy() - gB).max() <= 1e-9 * np.abs(Xo).max()
    if keep:
        rf, rl = op.link_force(Xo[keep], Xo[keep])
    else:
        rf, rl = np.zeros_like(fat), np.zeros_like(lng)
    scale = max(np.abs(rf).max(), 1.0)
    assert np.abs(ft.grad.cpu().numpy() - rf).max() <= 1e-9 * scale
    assert np.abs(lt.grad.cpu().numpy() - rl).max() <= 1e-9 * max(np.abs(rl).max(), 1.0)


def test_config5_backward_finite_differences():
    """Full 16^4, N = 8 workload: directional derivative of the loss along random
    complex directions of all fat links, all long links and B at once, central
    differences h = 1e-6 in FP64.  The loss is evaluated with the variational
    estimator 2 Re(b^H x) - x^H A x, whose error is quadratic in the solve error."""
    c = synth.CONFIGS[5]
    dims, m = c["dims"], c["mass"]
    fat, lng, B = synth.config_inputs(5)
    ctx = context(dims, True, fat, lng, m, tol=1e-11)
    Bt = to_dev(B).requires_grad_(True)
    ft = to_dev(fat).requires_grad_(True)
    lt = to_dev(lng).requires_grad_(True)
    X = bcg.BlockSolve.apply(Bt, ft, lt, ctx)
    loss = torch.real(torch.sum(Bt.conj() * X))
    loss.backward()
    r = synth.make_rng(synth.seed_for(5, 3))
    Vf = synth.gaussian_complex(r, fat.shape)
    Vl = synth.gaussian_complex(r, lng.shape)
    VB = synth.gaussian_complex(r, B.shape)
    an = (np.real(np.vdot(ft.grad.cpu().numpy(), Vf)) + np.real(np.vdot(lt.grad.cpu().numpy(), Vl))
          + np.real(np.vdot(Bt.grad.cpu().numpy(), VB)))

    def L(t):
        ctx.load_links(to_dev(fat + t * Vf), to_dev(lng + t * Vl))
        b = to_dev(B + t * VB)
        x, _ = ctx.solve(b)
        ax = ctx.apply(x)
        return float(2 * torch.real(torch.sum(b.conj() * x)) - torch.real(torch.sum(x.conj() * ax)))

    h = 1e-6
    fd = (L(h) - L(-h)) / (2 * h)
    print(f"config 5: analytic {an:.12e} fd {fd:.12e} rel {abs(fd - an) / abs(an):.2e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    # the oracle's gradient at the GPU solution (link force is linear in X, Lam)
    op = oracle.Operator(dims, fat, lng, m)
    Xh = X.detach().cpu().numpy()
    rf, rl = op.link_force(Xh, Xh)
    assert np.abs(ft.grad.cpu().numpy() - rf).max() <= 1e-8 * np.abs(rf).max()
    assert np.abs(lt.grad.cpu().numpy() - rl).max() <= 1e-8 * np.abs(rl).max()
