"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module draws random numbers and nothing else: gauge links, right-hand
sides and gauge transformations in the canonical host layouts.  It holds no
part of the solver's arithmetic (no stencil, no phases, no Krylov step), so
both the HIP path and the CPU oracle can take their inputs from here without
sharing any of the method.

Canonical layouts (complex128, C order):
  links   [4][V][3][3]   U_mu(x) at [mu][lex(x)], lex = x + Lx*(y + Ly*(z + Lz*t))
  vectors [N][V/2][3]    one checkerboard (parity) of N colour-vector fields,
                         site index cb = lex >> 1
  gauge   [V][3][3]      one SU(3) matrix per site

The workload stands in for the paper's HISQ ensembles (Table 1) and its
diluted noise sources (Sec. 7.1), which are not available: Haar-random SU(3)
long links, fat links with iid Gaussian entries of standard deviation 1/3 in
real and imaginary part, and iid standard-normal complex right-hand sides; for
the diluted-source workload also smooth SU(3) links (exp(i eps H), closer to
smeared ensembles).
"""
from __future__ import annotations

import numpy as np

# Seed recipe: 171000 + 10*config + stream, stream 0 links, 1 right-hand sides,
# 2 gauge transformation, 3 finite-difference directions, 4 extra.
SEED_BASE = 171000


def seed_for(config: int, stream: int) -> int:
    return SEED_BASE + 10 * int(config) + int(stream)


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def check_dims(dims) -> None:
    if len(dims) != 4:
        raise ValueError("dims must have four entries (Lx, Ly, Lz, Lt)")
    for d in dims:
        if int(d) < 2 or int(d) % 2:
            raise ValueError(f"every extent must be even and >= 2, got {tuple(dims)}")


def gaussian_complex(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """Real and imaginary parts iid N(0, scale^2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * scale


def haar_su3(rng: np.random.Generator, shape) -> np.ndarray:
    """Haar-distributed SU(3) matrices of the given batch shape.

    QR of a complex Ginibre matrix with the phases of R's diagonal moved into
    Q (Mezzadri 2007) gives Haar U(3); dividing by a cube root of the
    determinant lands in SU(3).
    """
    z = gaussian_complex(rng, tuple(shape) + (3, 3), 1.0 / np.sqrt(2.0))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    ph = d / np.abs(d)
    q = q * ph[..., None, :]
    det = np.linalg.det(q)
    q = q / np.power(det, 1.0 / 3.0)[..., None, None]
    return np.ascontiguousarray(q)


def fat_links(rng: np.random.Generator, dims, scale: float = 1.0 / 3.0) -> np.ndarray:
    """Fat (one-hop) links: general complex 3x3, entries N(0,1)*scale in Re and Im."""
    return np.ascontiguousarray(gaussian_complex(rng, (4, volume(dims), 3, 3), scale))


def long_links(rng: np.random.Generator, dims) -> np.ndarray:
    """Long (three-hop) links: Haar SU(3)."""
    return haar_su3(rng, (4, volume(dims)))


def smooth_su3(rng: np.random.Generator, shape, eps: float) -> np.ndarray:
    """SU(3) matrices exp(i eps H) with H traceless Hermitian, H = (G + G^H)/2 minus
    its trace part for a complex Ginibre G (entries of variance 1/2 in Re and Im):
    eps = 0 is the unit matrix, eps around 0.6 gives an average Re tr U / 3 of about
    0.8, the range of smeared (fat) links, and large eps approaches Haar."""
    g = gaussian_complex(rng, tuple(shape) + (3, 3), 1.0 / np.sqrt(2.0))
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1) / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    e = np.exp(1j * float(eps) * w)
    return np.ascontiguousarray((v * e[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2)))


def smooth_links(rng: np.random.Generator, dims, eps: float):
    """Fat and long links as independent smooth SU(3) fields (smooth_su3): a
    stand-in for the smeared links of a physical ensemble, whose staggered spectrum
    has the clustered low modes that the Haar / Gaussian links lack."""
    fat = smooth_su3(rng, (4, volume(dims)), eps)
    lng = smooth_su3(rng, (4, volume(dims)), eps)
    return fat, lng


def unit_links(dims) -> np.ndarray:
    v = volume(dims)
    u = np.zeros((4, v, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def rhs(rng: np.random.Generator, nrhs: int, dims) -> np.ndarray:
    """N right-hand sides on one checkerboard, [N][V/2][3] complex128."""
    return np.ascontiguousarray(gaussian_complex(rng, (int(nrhs), volume(dims) // 2, 3)))


def gauge_transform(rng: np.random.Generator, dims) -> np.ndarray:
    """One Haar SU(3) matrix per site, [V][3][3]."""
    return haar_su3(rng, (volume(dims),))


# The five workloads: (lattice, improved, mass, N, storage, tolerance).
CONFIGS = {
    1: dict(dims=(4, 4, 4, 4), improved=False, mass=0.1, nrhs=4, prec="fp64", tol=1e-10),
    2: dict(dims=(16, 16, 16, 16), improved=True, mass=0.05, nrhs=16, prec="fp64", tol=1e-10),
    3: dict(dims=(32, 32, 32, 64), improved=True, mass=0.02, nrhs=16, prec="fp32", tol=1e-8),
    4: dict(dims=(32, 32, 32, 64), improved=True, mass=0.02, nrhs=32, prec="fp16", tol=1e-8),
    5: dict(dims=(16, 16, 16, 16), improved=True, mass=0.05, nrhs=8, prec="fp64", tol=1e-10),
}


def config_inputs(config: int, dims=None, nrhs=None):
    """Links and right-hand sides for one workload (optionally at other sizes).

    Config 1 uses Haar SU(3) links for the naive operator; the others use
    Gaussian fat links plus Haar long links.
    Returns (fat, long_or_None, B).
    """
    c = CONFIGS[config]
    dims = tuple(dims) if dims is not None else c["dims"]
    nrhs = int(nrhs) if nrhs is not None else c["nrhs"]
    check_dims(dims)
    lr = make_rng(seed_for(config, 0))
    if c["improved"]:
        fat = fat_links(lr, dims)
        lng = long_links(lr, dims)
    else:
        fat = long_links(lr, dims)
        lng = None
    b = rhs(make_rng(seed_for(config, 1)), nrhs, dims)
    return fat, lng, b


def diluted_noise_sources(dims, n_sources: int, n_subsets: int, rng: np.random.Generator) -> np.ndarray:
    """Stochastic-trace sources split into disjoint-support pieces, as in the
    paper's measurement workload (Sec. 7.1: 24 noise sources, each partitioned
    into 8 disjoint subsets): n_sources fields on the even checkerboard with
    complex Z4 noise (1, i, -1, -i) in every colour component, each split into
    n_subsets pieces by the site's corner of the 2^3 spatial unit cube,
    (x mod 2) + 2 (y mod 2) + 4 (z mod 2) (n_subsets = 8; with fewer, that index
    mod n_subsets).  Returns [n_sources * n_subsets][V/2][3], piece s of source k
    at k * n_subsets + s."""
    check_dims(dims)
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    vh = volume(dims) // 2
    lex = np.arange(volume(dims))
    x = lex % Lx
    y = (lex // Lx) % Ly
    z = (lex // (Lx * Ly)) % Lz
    t = lex // (Lx * Ly * Lz)
    even = ((x + y + z + t) % 2) == 0
    cb = lex[even] >> 1
    corner = ((x[even] & 1) + 2 * (y[even] & 1) + 4 * (z[even] & 1)) % n_subsets
    cls = np.empty(vh, dtype=np.int64)
    cls[cb] = corner
    noise = np.exp(0.5j * np.pi * rng.integers(0, 4, size=(n_sources, vh, 3)))
    out = np.zeros((n_sources * n_subsets, vh, 3), dtype=np.complex128)
    for k in range(n_sources):
        for s in range(n_subsets):
            sel = cls == s
            out[k * n_subsets + s, sel] = noise[k, sel]
    return out
