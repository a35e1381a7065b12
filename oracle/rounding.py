"""Emulated low-precision storage for the oracle's mixed-precision runs.

TEST INFRASTRUCTURE (part of the oracle; the solver library never uses it).

Sec. 6 of the paper keeps the Krylov block vectors and the links of the
iteration in a low ("sloppy") precision and recovers accuracy with reliable
updates in full precision (Alg. 3).  These functions round FP64 data the way
such a storage format would, so that ``block_cg_rq(..., sloppy=...,
apply_sloppy=...)`` shows on the CPU what the format does to the iteration.

Formats (one group = the 3 colour components of a vector at one site and
column, or the 9 entries of one link matrix):

* ``fp32``  : every real rounded to IEEE binary32 (round to nearest even);
* ``fp16``  : the group divided by s = max |Re|, |Im| over the group, each real
              rounded to IEEE binary16, then multiplied back by s (s in binary32);
* ``bf16``  : the same with bfloat16 (binary32 with the low 16 bits of the
              significand rounded away, round to nearest even);
* ``fix16`` : the same with 16-bit fixed point, q = nearest integer to 32767 x.

The scaled formats round x/s in binary32 first (the division is done in
single precision), then to the 16-bit format.
"""
from __future__ import annotations

import numpy as np

FORMATS = ("fp64", "fp32", "fp16", "bf16", "fix16")

# unit roundoff of each format relative to the group's largest component
# (fp32 / fp64 relative to the value itself)
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8,
                 "fix16": 0.5 / 32767.0}


def _to_bf16(x32: np.ndarray) -> np.ndarray:
    """binary32 -> nearest bfloat16 (ties to even), returned as binary32 values."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _round_reals(x32: np.ndarray, fmt: str) -> np.ndarray:
    if fmt == "fp16":
        return x32.astype(np.float16).astype(np.float32)
    if fmt == "bf16":
        return _to_bf16(x32)
    if fmt == "fix16":
        return (np.rint(x32.astype(np.float64) * 32767.0) / 32767.0).astype(np.float32)
    raise ValueError(fmt)


def round_groups(a, fmt: str, group_axes) -> np.ndarray:
    """Round complex array ``a`` as stored in ``fmt``; the reals of one group
    (the trailing ``group_axes`` axes, real and imaginary parts together) share
    one scale in the 16-bit formats."""
    a = np.asarray(a, dtype=np.complex128)
    if fmt == "fp64":
        return a.copy()
    if fmt == "fp32":
        return a.astype(np.complex64).astype(np.complex128)
    if fmt not in FORMATS:
        raise ValueError(f"unknown format {fmt!r}")
    re = a.real.astype(np.float32)
    im = a.imag.astype(np.float32)
    axes = tuple(range(a.ndim - group_axes, a.ndim))
    s = np.maximum(np.abs(re).max(axis=axes, keepdims=True), np.abs(im).max(axis=axes, keepdims=True))
    inv = np.where(s > 0, np.float32(1.0) / np.where(s > 0, s, np.float32(1.0)), np.float32(0.0))
    qr = _round_reals(re * inv, fmt).astype(np.float64) * s.astype(np.float64)
    qi = _round_reals(im * inv, fmt).astype(np.float64) * s.astype(np.float64)
    # decoded values are formed in binary32, as a kernel would
    qr = qr.astype(np.float32).astype(np.float64)
    qi = qi.astype(np.float32).astype(np.float64)
    return qr + 1j * qi


def vector_rounder(fmt: str, vh: int):
    """Rounding of an L x N block-vector matrix (L = 3 vh) for block_cg_rq's
    ``sloppy`` argument: one group per (site, column)."""
    if fmt == "fp64":
        return None

    def rnd(M):
        n = M.shape[1]
        v = np.ascontiguousarray(M.T).reshape(n, vh, 3)
        r = round_groups(v, fmt, 1)
        return np.ascontiguousarray(r.reshape(n, -1).T)

    return rnd


def round_links(U, fmt: str) -> np.ndarray:
    """Links [4][V][3][3] as stored in ``fmt`` (one group per 3 x 3 matrix)."""
    return round_groups(U, fmt, 2)
