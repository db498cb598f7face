"""Helpers of the GPU parity tests: device inputs and the library's packed
layouts rearranged into per-site records (the layouts are part of the ABI
documented in the library's device header)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09224_amd import inputs

FMT_NAME = {0: "f64", 1: "f32", 2: "half16", 3: "int20", 4: "int30", 5: "int24"}
GFMT_NAME = {0: "f64", 1: "f32", 2: "fix16", 3: "fix32", 4: "sx24"}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_09224_amd import hisq
    hisq.load()
    return hisq


def spinor_records(packed, n, fmt):
    """packed uint8 (numpy) SoA field -> per-site records as the oracle codecs use"""
    b = np.ascontiguousarray(packed[: n * {0: 48, 1: 24, 2: 16, 3: 16, 4: 24, 5: 20}[fmt]])
    if fmt == 0:
        a = b.view(np.float64).reshape(3, n, 2)
        return (a[..., 0] + 1j * a[..., 1]).T.copy()
    if fmt == 1:
        p0 = b[: 16 * n].view(np.float32).reshape(n, 4)
        p1 = b[16 * n: 24 * n].view(np.float32).reshape(n, 2)
        r = np.concatenate([p0, p1], axis=1).reshape(n, 3, 2)
        return (r[..., 0] + 1j * r[..., 1]).astype(np.complex64)
    if fmt == 2:
        w = b.view(np.uint32).reshape(n, 4)
        q = np.empty((n, 6), dtype=np.int16)
        for k in range(3):
            q[:, 2 * k] = (w[:, k] & 0xFFFF).astype(np.uint16).view(np.int16)
            q[:, 2 * k + 1] = (w[:, k] >> 16).astype(np.uint16).view(np.int16)
        return q, w[:, 3].copy().view(np.float32)
    if fmt == 3:
        return b.view(np.uint32).reshape(n, 4).copy()
    if fmt == 4:
        p0 = b[: 16 * n].view(np.uint32).reshape(n, 4)
        p1 = b[16 * n: 24 * n].view(np.uint32).reshape(n, 2)
        return np.concatenate([p0, p1], axis=1)
    if fmt == 5:
        p0 = b[: 16 * n].view(np.uint32).reshape(n, 4)
        p1 = b[16 * n: 20 * n].view(np.uint32).reshape(n, 1)
        return np.concatenate([p0, p1], axis=1)
    raise ValueError(fmt)


def gauge_reals(packed, dims, gfmt):
    """packed link field -> canonical-order array [4, V, 18] of the stored
    integers (fixed point) or reals (IEEE); SX24: [4, V, 15], the five words
    of each of the three row records"""
    V = oracle.volume(dims)
    vh = V // 2
    b = np.ascontiguousarray(packed)
    mb = {0: 144, 1: 72, 2: 36, 3: 72, 4: 60}[gfmt]
    dt = {0: np.float64, 1: np.float32, 2: np.int16, 3: np.int32, 4: np.uint32}[gfmt]
    out = np.zeros((4, V, 15 if gfmt == 4 else 18), dtype=dt)
    for mu in range(4):
        for p in range(2):
            sub = b[(2 * mu + p) * mb * vh:(2 * mu + p + 1) * mb * vh]
            if gfmt == 0:
                r = sub.view(np.float64).reshape(9, vh, 2).transpose(1, 0, 2).reshape(vh, 18)
            elif gfmt == 4:
                p0 = sub[: 48 * vh].view(np.uint32).reshape(3, vh, 4)
                p1 = sub[48 * vh: 60 * vh].view(np.uint32).reshape(3, vh, 1)
                r = np.concatenate([p0, p1], axis=2).transpose(1, 0, 2).reshape(vh, 15)
            elif gfmt in (1, 3):
                p0 = sub[: 64 * vh].view(dt).reshape(4, vh, 4).transpose(1, 0, 2).reshape(vh, 16)
                p1 = sub[64 * vh: 72 * vh].view(dt).reshape(vh, 2)
                r = np.concatenate([p0, p1], axis=1)
            else:
                p0 = sub[: 32 * vh].view(dt).reshape(2, vh, 8).transpose(1, 0, 2).reshape(vh, 16)
                p1 = sub[32 * vh: 36 * vh].view(dt).reshape(vh, 2)
                r = np.concatenate([p0, p1], axis=1)
            out[mu, oracle.parity_sites(dims, p)] = r
    return out


def make_fields(dims, kind="near_unit", seed=inputs.GAUGE_SEED, device="cuda"):
    fat, lng = inputs.make_links(dims, kind, seed, device=device)
    return fat, lng


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def format_bounds():
    """{triplet: (Dslash bound, normal-operator bound)}: max-norm relative
    errors against the unquantised FP64 operator, written by
    golden/make_format_bounds.py from the oracle alone"""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "format_bounds.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, d, n = [part.split() for part in line.split("|")]
        out[name[0]] = (float(d[1]), float(n[1]))
    return out


def long8_records(packed, dims, gfmt):
    """packed eight-parameter long field -> canonical-order [4, V, 8]: float64
    parameters (F64) or the stored int32 (FIX32), as oracle.long_recon8_encode"""
    V = oracle.volume(dims)
    vh = V // 2
    b = np.ascontiguousarray(packed)
    mb = {0: 64, 3: 32}[gfmt]
    dt = {0: np.float64, 3: np.int32}[gfmt]
    out = np.zeros((4, V, 8), dtype=dt)
    for mu in range(4):
        for p in range(2):
            sub = b[(2 * mu + p) * mb * vh:(2 * mu + p + 1) * mb * vh].view(dt)
            per = 16 // np.dtype(dt).itemsize                  # parameters per 16-byte plane entry
            r = sub.reshape(8 // per, vh, per).transpose(1, 0, 2).reshape(vh, 8)
            out[mu, oracle.parity_sites(dims, p)] = r
    return out
