"""Full-size solves of the 32^3 x 64 workloads in reduced storage, checked with
the CPU oracle's FP64 operator: every column's true relative residual
||b_i - A x_i|| / ||b_i|| <= 1e-8 (mixed-precision bar), and the distance to
the FP64-storage GPU solution printed next to it.

* FP32 vectors and links with FP64 reliable updates, N = 16 (the kernel-sweep
  workload);
* 16-bit storage (16-bit fixed point, FP16) with one FP32 scale per site and
  column, N = 32;
* BF16 storage, N = 32: the iteration cannot reach 1e-8 at m = 0.02 (see
  test_gpu_stability.py); the solver must stop by itself and return its best
  iterate, whose residual is checked with the oracle's operator.
"""
import numpy as np
import pytest

import oracle
from paper_1710_09745_amd import bcg, synth

from gpu_util import config_inputs_cached, context, to_dev, true_rel_res

pytestmark = pytest.mark.gpu

C3 = synth.CONFIGS[3]


@pytest.fixture(scope="module")
def op3():
    fat, lng, _ = config_inputs_cached(3, 1)
    return oracle.Operator(C3["dims"], fat, lng, C3["mass"])


def _solve(prec, n, max_iter=20000):
    fat, lng, B = config_inputs_cached(3, n)
    ctx = context(C3["dims"], True, fat, lng, C3["mass"], tol=C3["tol"], prec=prec, max_iter=max_iter)
    X, info = ctx.solve(to_dev(B), raise_on_error=False)
    Xh = X.cpu().numpy()
    ctx.close()
    return B, Xh, info


def test_config3_fp32_n16_meets_tolerance(op3):
    B, X, info = _solve("fp32", 16)
    res = true_rel_res(op3, B, X)
    print(f"32^3x64 fp32 N=16: rc={info['rc']} iters={info['iters']} rus={info['reliable_updates']} "
          f"max true res (oracle) {res.max():.3e} (library {info['max_true_rel_res']:.3e})")
    assert info["rc"] == bcg.OK
    assert res.max() <= 1e-8
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3)


@pytest.fixture(scope="module")
def x64_n32():
    B, X, info = _solve("fp64", 32)
    assert info["rc"] == bcg.OK
    return X


@pytest.mark.parametrize("prec", ["fix16", "fp16"])
def test_config4_16bit_n32_meets_tolerance(op3, x64_n32, prec):
    B, X, info = _solve(prec, 32)
    res = true_rel_res(op3, B, X)
    d = np.linalg.norm(X - x64_n32) / np.linalg.norm(x64_n32)
    print(f"32^3x64 {prec} N=32: rc={info['rc']} iters={info['iters']} rus={info['reliable_updates']} "
          f"max true res (oracle) {res.max():.3e}; ||X - X_fp64gpu|| / ||X_fp64gpu|| = {d:.2e}")
    assert info["rc"] == bcg.OK
    assert res.max() <= 1e-8
    # both solutions are within 1e-8 residual of A^{-1} B; their distance is bounded
    # by 2e-8 kappa with kappa <= lambda_max / (4 m^2) < 1e5 here
    assert d <= 2e-3


def test_config4_bf16_stops_by_itself(op3):
    B, X, info = _solve("bf16", 32, max_iter=100000)
    res = true_rel_res(op3, B, X)
    print(f"32^3x64 bf16 N=32: rc={info['rc']} iters={info['iters']} rus={info['reliable_updates']} "
          f"best max true res (oracle) {res.max():.3e}")
    assert info["rc"] in (bcg.OK, bcg.ERR_NOT_CONVERGED, bcg.ERR_BREAKDOWN)
    assert info["iters"] < 20000
    assert np.allclose(res, info["true_rel_res"], rtol=1e-3)
    if info["rc"] == bcg.OK:
        assert res.max() <= 1e-8
