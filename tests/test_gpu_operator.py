"""GPU parity of the multi-right-hand-side hop and A = 4 m^2 - D_eo D_oe against the
CPU oracle, element by element (per-column relative error and largest elementwise
error relative to the column's largest element both <= 1e-12, FP64), on
lattices that span several workgroups and leave ragged site and right-hand-side
tails, and on sampled sites of the full 16^4 and 32^3 x 64 workloads."""
import numpy as np
import pytest
import torch

import oracle
from paper_1710_09745_amd import synth

from gpu_util import (DEV, col_rel_err, config_inputs_cached, context, elem_rel_err, emulated_sloppy_apply,
                      inputs, site_scaled_err, to_dev)

pytestmark = pytest.mark.gpu

CASES = [((2, 2, 2, 2), False, 1), ((4, 4, 4, 4), False, 4), ((4, 4, 4, 4), True, 3),
         ((6, 6, 6, 6), True, 5), ((8, 6, 4, 10), True, 17), ((6, 4, 6, 8), False, 9),
         ((8, 8, 8, 8), True, 64), ((10, 6, 6, 6), True, 2), ((8, 8, 8, 8), True, 33)]


@pytest.mark.parametrize("dims,improved,n", CASES)
def test_apply_matches_oracle(dims, improved, n):
    fat, lng, B = inputs(dims, improved, n, 1000 + n)
    m = 0.07
    ctx = context(dims, improved, fat, lng, m)
    op = oracle.Operator(dims, fat, lng, m)
    out = ctx.apply(to_dev(B)).cpu().numpy()
    ref = op.apply(B)
    assert col_rel_err(out, ref).max() <= 1e-12
    assert elem_rel_err(out, ref).max() <= 1e-12


@pytest.mark.parametrize("dims,improved,n", CASES[:6])
def test_hops_match_oracle(dims, improved, n):
    fat, lng, B = inputs(dims, improved, n, 2000 + n)
    ctx = context(dims, improved, fat, lng, 0.1)
    op = oracle.Operator(dims, fat, lng, 0.1)
    for p in (0, 1):
        out = ctx.hop(p, to_dev(B)).cpu().numpy()
        ref = op.hop(p, B)
        assert col_rel_err(out, ref).max() <= 1e-12
        assert elem_rel_err(out, ref).max() <= 1e-12


def test_free_field_plane_wave_on_gpu():
    dims = (6, 6, 6, 6)
    m = 0.13
    ctx = context(dims, True, synth.unit_links(dims), synth.unit_links(dims), m)
    c = np.stack(np.meshgrid(*[np.arange(L) for L in dims[::-1]], indexing="ij"), -1).reshape(-1, 4)[:, ::-1]
    even = np.nonzero(c.sum(1) % 2 == 0)[0]
    p = 2 * np.pi * np.array([1, 2, 0, 5]) / np.array(dims)
    f = np.exp(1j * (c[even] @ p))[:, None] * np.array([1.0, 0.5j, -0.25])[None, :]
    lam = 4 * m * m + 4 * np.sum((np.sin(p) + np.sin(3 * p)) ** 2)
    out = ctx.apply(to_dev(f[None])).cpu().numpy()[0]
    assert np.abs(out - lam * f).max() <= 1e-12 * lam


@pytest.mark.parametrize("config,n", [(2, 16), (3, 4)])
def test_full_size_apply_sampled_sites(config, n):
    c = synth.CONFIGS[config]
    dims = c["dims"]
    fat, lng, B = synth.config_inputs(config, nrhs=n)
    ctx = context(dims, True, fat, lng, c["mass"])
    out = ctx.apply(to_dev(B))
    op = oracle.Operator(dims, fat, lng, c["mass"])
    sites = synth.make_rng(77).choice(synth.volume(dims) // 2, size=48, replace=False)
    sites = np.concatenate([sites, [0, synth.volume(dims) // 2 - 1]])
    ref = op.apply_sites(B, sites)
    got = out[:, torch.from_numpy(sites).to(DEV)].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= 1e-12


def test_gauge_covariance_on_gpu():
    dims = (6, 4, 4, 6)
    fat, lng, B = inputs(dims, True, 3, 3001)
    g = synth.gauge_transform(synth.make_rng(3002), dims)
    from test_oracle_operator import gauge_rotate, parity_split
    f2, l2 = gauge_rotate(dims, fat, lng, g)
    even, _ = parity_split(dims)
    c1 = context(dims, True, fat, lng, 0.05)
    c2 = context(dims, True, f2, l2, 0.05)
    gB = np.einsum("sab,nsb->nsa", g[even], B)
    lhs = c2.apply(to_dev(gB)).cpu().numpy()
    rhs = np.einsum("sab,nsb->nsa", g[even], c1.apply(to_dev(B)).cpu().numpy())
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# allowed deviation from the emulation, relative to the site's largest component:
# the kernels sum the 48 complex products of a hop in FP32 (a few 2^-24 of the
# largest term, which can exceed the result by an order of magnitude) and may round
# T or the result to the neighbouring stored value where the emulation (FP64
# arithmetic) rounds the other way; a flipped T propagates through the eight
# one-hop terms of D_eo.  For the 16-bit formats that is a few storage steps (for
# 16-bit fixed point, whose step 1/32767 is within 16x of the FP32 error of the
# sums, eight), for FP32 a few 1e-6.  A wrong neighbour or link gives O(1).
SLOPPY_TOL = {"fp32": 1e-5, "fp16": 4 * 2.0 ** -11, "bf16": 4 * 2.0 ** -8, "fix16": 8.0 / 32767}


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fix16"])
@pytest.mark.parametrize("kernel,tr,tpb,n", [(2, 8, 2, 17), (2, 8, 2, 33), (2, 4, 2, 6), (1, 8, 0, 17),
                                             (2, 8, 4, 16), (1, 4, 0, 3)])
def test_sloppy_apply_matches_emulation(prec, kernel, tr, tpb, n):
    """A P in reduced storage, as the solver's iteration forms it, against the
    oracle's emulation of the same storage, element by element.  16x16x8x4 has
    time slices of 1024 even sites, so the site-parallel hop with two lane groups
    (128 sites per workgroup) takes the XCD slab order, as on 32^3 x 64; ragged N
    leaves partial register tiles."""
    dims = (16, 16, 8, 4)
    fat, lng, B = inputs(dims, True, n, 9000 + n)
    m = 0.05
    ctx = context(dims, True, fat, lng, m)
    for name, v in [("hop_kernel", kernel), ("hop_tr", tr), ("hop_tpb", tpb)]:
        ctx.set_option(name, v)
    op = oracle.Operator(dims, fat, lng, m)
    got = ctx.apply_prec(prec, to_dev(B)).cpu().numpy()
    ref = emulated_sloppy_apply(op, prec, B)
    err = site_scaled_err(got, ref)
    print(f"{prec} kernel={kernel} tr={tr} tpb={tpb} n={n}: max site-scaled error {err:.2e}")
    assert err <= SLOPPY_TOL[prec]


@pytest.mark.parametrize("prec,n", [("fp32", 16), ("fix16", 32), ("bf16", 32)])
def test_full_size_sloppy_apply_sampled_sites(prec, n):
    """The 32^3 x 64 operator in reduced storage with the default launch shape
    (site-parallel, 8 columns per lane, two lane groups, slab order) at sampled
    sites against the oracle's FP64 operator: the difference is the storage
    rounding only (a wrong neighbour or link would be O(1))."""
    c = synth.CONFIGS[3]
    dims = c["dims"]
    fat, lng, B = config_inputs_cached(3, n)
    ctx = context(dims, True, fat, lng, c["mass"])
    out = ctx.apply_prec(prec, to_dev(B))
    op = oracle.Operator(dims, fat, lng, c["mass"])
    sites = synth.make_rng(78).choice(synth.volume(dims) // 2, size=40, replace=False)
    sites = np.concatenate([sites, [0, 1, synth.volume(dims) // 2 - 1]])
    ref = op.apply_sites(B, sites)
    got = out[:, torch.from_numpy(sites).to(DEV)].cpu().numpy()
    del out
    err = site_scaled_err(got, ref)
    bound = {"fp32": 1e-5, "fix16": 2e-3, "bf16": 0.1}[prec]
    print(f"{prec} n={n}: max site-scaled error vs FP64 {err:.2e} (bound {bound:g})")
    assert err <= bound


@pytest.mark.parametrize("dims,n", [((16, 16, 8, 4), 17), ((6, 6, 6, 8), 5), ((8, 8, 8, 8), 33), ((16, 16, 16, 16), 16)])
def test_hop_task_queues_match_static_order(dims, n):
    """The site-parallel hop with per-XCD task queues (persistent grid of 1, 2, 4 or 8
    workgroups per CU; workgroups drain their own XCD's queue, then the others')
    computes every site exactly as the static walk does: bit-identical FP64 and FP32
    results, FP64 within 1e-12 of the oracle; repeated launches reuse the
    self-resetting counters."""
    fat, lng, B = inputs(dims, True, n, 9700 + n)
    m = 0.05
    op = oracle.Operator(dims, fat, lng, m)
    ref = op.apply(B)
    ctx = context(dims, True, fat, lng, m)
    ctx.set_option("hop_kernel", 2)
    ctx.set_option("hop_sched", 1)
    x = to_dev(B)
    a64 = ctx.apply(x)
    a32 = ctx.apply_prec("fp32", x)
    assert col_rel_err(a64.cpu().numpy(), ref).max() <= 1e-12
    for sched in (2, 3, 4, 5):
        ctx.set_option("hop_sched", sched)
        for _ in range(3):
            assert torch.equal(ctx.apply(x), a64), f"sched={sched}"
            assert torch.equal(ctx.apply_prec("fp32", x), a32), f"sched={sched}"
