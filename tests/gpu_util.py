"""Helpers shared by the GPU parity tests: contexts on cuda:0 and seeded inputs."""
import numpy as np
import torch

import oracle
from paper_1710_09745_amd import bcg, synth

DEV = torch.device("cuda:0")


def inputs(dims, improved, nrhs, seed):
    r = synth.make_rng(seed)
    fat = synth.fat_links(r, dims)
    lng = synth.long_links(r, dims) if improved else None
    B = synth.rhs(synth.make_rng(seed + 1), nrhs, dims)
    return fat, lng, B


def context(dims, improved, fat, lng, mass, tol=1e-10, prec="fp64", ru_delta=0.1, max_iter=100000):
    print(f"[case] dims={dims} improved={improved} mass={mass} prec={prec}", flush=True)
    ctx = bcg.Context(dims, improved=improved, device=DEV)
    ctx.load_links(fat, lng)
    ctx.set_mass(mass)
    ctx.set_solver(tol=tol, max_iter=max_iter, prec=prec, ru_delta=ru_delta)
    return ctx


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def col_rel_err(got, ref):
    n = ref.shape[0]
    d = np.linalg.norm((got - ref).reshape(n, -1), axis=1)
    r = np.linalg.norm(ref.reshape(n, -1), axis=1)
    return d / r


def elem_rel_err(got, ref):
    """Largest elementwise error of each column, relative to that column's largest
    element: localises a wrong site, colour or column that a norm could average out."""
    n = ref.shape[0]
    d = np.abs(got - ref).reshape(n, -1).max(axis=1)
    r = np.abs(ref).reshape(n, -1).max(axis=1)
    return d / r


def true_rel_res(op: oracle.Operator, B, X):
    n = B.shape[0]
    R = B - op.apply(X)
    return np.linalg.norm(R.reshape(n, -1), axis=1) / np.linalg.norm(B.reshape(n, -1), axis=1)


def kappa_bound(op: oracle.Operator, iters=60, seed=5):
    """Upper estimate of the condition number of A: lambda_max by power iteration
    (times 1.05 for safety) over the lower bound lambda_min >= 4 m^2."""
    v = synth.rhs(synth.make_rng(seed), 1, tuple(int(d) for d in op.dims))
    lam = 0.0
    for _ in range(iters):
        w = op.apply(v)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return 1.05 * lam / (4 * op.mass * op.mass)


def emulated_sloppy_apply(op: oracle.Operator, fmt, B):
    """The oracle's A B as the solver's iteration forms it in storage format fmt:
    input, links, T = D_oe B and the result rounded to the format (oracle.rounding),
    arithmetic in FP64."""
    from oracle import rounding
    lng = rounding.round_links(op.lng, fmt) if op.improved else None
    ops = oracle.Operator(tuple(int(d) for d in op.dims), rounding.round_links(op.fat, fmt), lng, op.mass)
    P = rounding.round_groups(B, fmt, 1)
    T = rounding.round_groups(ops.hop(1, P), fmt, 1)
    AP = 4 * op.mass * op.mass * P - ops.hop(0, T)
    return rounding.round_groups(AP, fmt, 1)


def site_scaled_err(got, ref):
    """max over elements of |got - ref| / (largest component of ref at that site and column)."""
    s = np.maximum(np.abs(ref.real).max(-1, keepdims=True), np.abs(ref.imag).max(-1, keepdims=True))
    d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
    return float((d / s).max())


_LINKS = {}


def config_inputs_cached(config, nrhs):
    """synth.config_inputs(config, nrhs=nrhs) with the links drawn once per process
    (the 32^3 x 64 links take a while to draw); the right-hand sides are the same
    draws as synth.config_inputs gives."""
    if config not in _LINKS:
        fat, lng, _ = synth.config_inputs(config, nrhs=1)
        _LINKS[config] = (fat, lng)
    fat, lng = _LINKS[config]
    c = synth.CONFIGS[config]
    B = synth.rhs(synth.make_rng(synth.seed_for(config, 1)), nrhs, c["dims"])
    return fat, lng, B
