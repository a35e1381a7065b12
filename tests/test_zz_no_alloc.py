"""bcg_apply_noalloc (no device allocation in the library) against bcg_apply,
through the C ABI: two calls in a row, the second with a smaller input, and
the size limit of its scratch."""
import numpy as np
import pytest
import torch

from paper_1710_09745_amd import bcg

from gpu_util import DEV, context, inputs, to_dev

pytestmark = pytest.mark.gpu


def test_noalloc_apply_matches_apply_twice():
    dims = (8, 8, 6, 10)
    fat, lng, B = inputs(dims, True, 9, 9500)
    ctx = context(dims, True, fat, lng, 0.07)
    ref1 = ctx.apply(to_dev(B)).cpu().numpy()
    ref2 = ctx.apply(to_dev(B[:3])).cpu().numpy()
    out1 = torch.full((9, ctx.Vh, 3), float("nan"), dtype=torch.complex128, device=DEV)
    out2 = torch.full((3, ctx.Vh, 3), float("nan"), dtype=torch.complex128, device=DEV)
    ctx.apply_noalloc(to_dev(B), out1)
    got1 = out1.cpu().numpy()
    ctx.apply_noalloc(to_dev(B[:3].copy()), out2)
    got2 = out2.cpu().numpy()
    # the same kernels on the same inputs: identical to the last bit
    assert np.array_equal(got1, ref1)
    assert np.array_equal(got2, ref2)


def test_noalloc_apply_rejects_oversized_requests():
    dims = (16, 16, 16, 16)
    fat, lng, B = inputs(dims, True, 11, 9600)
    ctx = context(dims, True, fat, lng, 0.05)
    x = to_dev(B)
    out = torch.empty_like(x)
    with pytest.raises(bcg.BcgError) as e:
        ctx.apply_noalloc(x, out)
    assert e.value.code == bcg.ERR_ARG and "scratch" in str(e.value)
    # ten columns of 16^4 fit, and match bcg_apply
    ctx.apply_noalloc(x[:10], out[:10])
    assert torch.equal(out[:10], ctx.apply(x[:10]))
