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
