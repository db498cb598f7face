"""Seeded synthetic lattice inputs: gauge links, staggered phases and sources.

This module generates the *inputs* of the HISQ operator and its solvers and
nothing else: it holds none of the operator, solver or storage-format
arithmetic, so both the FP64 CPU oracle (test infrastructure) and the HIP
library can be fed from it.

The paper measures on thermalised gauge ensembles that are not available
here; these generators stand in for them with the same shapes and value
structure:

* ``kind="haar"``: every SU(3) factor is Haar random (QR of a complex Gaussian
  matrix, phase-fixed, then divided by a cube root of its determinant).  Rough
  links, dense low spectrum.
* ``kind="near_unit"``: every factor is ``exp(i * eps * H)`` with ``H`` a
  random traceless Hermitian matrix (``eps = 0.3``).  Smooth links.

Fat links are ``F = 0.6 U + 0.4 U'`` (a non-unitary, smeared-like link) and
long (Naik) links are ``L = -(1/24) U1 U2 U3``.  The staggered phases
``eta_mu(x)`` and the antiperiodic temporal boundary are folded into ``F`` and
``L`` here, so the operator itself sees plain matrices.

Conventions (these are also the library's canonical host/device layouts):

* ``dims = (X, Y, Z, T)``, every extent even and >= 4;
* lexicographic site index ``i = ((t*Z + z)*Y + y)*X + x``;
* parity ``(x+y+z+t) % 2``; checkerboard index ``cb = i // 2``;
* links: complex128 ``[4, V, 3, 3]`` (direction, site, row, column);
* full-lattice spinor: complex128 ``[V, 3]``; one-parity spinor:
  complex128 ``[V/2, 3]`` in checkerboard order.

Seeds: gauge ``1000 + k``, source ``2000 + k``, right-hand side j ``3000 + j``
for workload k.
"""
from __future__ import annotations

import math

import torch

__all__ = [
    "volume", "coords", "parity_of_sites", "cb_sites", "eta_phases",
    "haar_su3", "near_unit_su3", "make_links", "gaussian_spinor",
    "unit_links", "random_su3_field", "GAUGE_SEED", "SOURCE_SEED", "RHS_SEED",
]

GAUGE_SEED = 1000
SOURCE_SEED = 2000
RHS_SEED = 3000

# Sites generated per chunk; fixed so that a seed gives the same field
# whatever the lattice size or device memory.
_CHUNK = 1 << 18


def volume(dims) -> int:
    X, Y, Z, T = dims
    return X * Y * Z * T


def _check_dims(dims):
    if len(dims) != 4 or any(int(d) < 4 or int(d) % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even integers >= 4, got {dims}")


def coords(dims, device="cpu"):
    """(x, y, z, t) int64 tensors of length V in lexicographic order."""
    _check_dims(dims)
    X, Y, Z, T = dims
    i = torch.arange(volume(dims), device=device, dtype=torch.int64)
    x = i % X
    y = (i // X) % Y
    z = (i // (X * Y)) % Z
    t = i // (X * Y * Z)
    return x, y, z, t


def parity_of_sites(dims, device="cpu"):
    x, y, z, t = coords(dims, device)
    return (x + y + z + t) % 2


def cb_sites(dims, parity, device="cpu"):
    """Lexicographic indices of the sites of one parity, in checkerboard order."""
    par = parity_of_sites(dims, device)
    idx = torch.nonzero(par == parity).flatten()
    return idx


def eta_phases(dims, device="cpu"):
    """Staggered phases with the temporal boundary sign, for fat and long links.

    Returns ``(eta_fat, eta_long)``, float64 ``[4, V]`` of +-1:
    ``eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z)``;
    the one-hop link ``F_3(x)`` also changes sign when ``t = T-1`` and the
    three-hop link ``L_3(x)`` when ``t >= T-3`` (antiperiodic in time).
    """
    x, y, z, t = coords(dims, device)
    T = dims[3]
    one = torch.ones_like(x, dtype=torch.float64)
    sgn = lambda n: 1.0 - 2.0 * (n % 2).to(torch.float64)  # noqa: E731
    eta = torch.stack([one, sgn(x), sgn(x + y), sgn(x + y + z)])
    eta_f = eta.clone()
    eta_l = eta.clone()
    eta_f[3] = eta_f[3] * torch.where(t == T - 1, -1.0, 1.0).to(torch.float64)
    eta_l[3] = eta_l[3] * torch.where(t >= T - 3, -1.0, 1.0).to(torch.float64)
    return eta_f, eta_l


def _cgauss(shape, gen, device):
    """Complex Gaussian with E|z|^2 = 1 (real and imaginary parts N(0, 1/2))."""
    re = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    return torch.complex(re, im) * math.sqrt(0.5)


def _mm3(a, b):
    """Batched 3x3 complex product written out elementwise (no batched GEMM)."""
    return (a.unsqueeze(-1) * b.unsqueeze(-3)).sum(-2)


def _dagger(a):
    return a.conj().transpose(-1, -2)


def haar_su3(n, gen, device="cpu"):
    """n Haar-random SU(3) matrices (Mezzadri's QR recipe, det fixed to 1)."""
    z = _cgauss((n, 3, 3), gen, device)
    q, r = torch.linalg.qr(z)
    d = torch.diagonal(r, dim1=-2, dim2=-1)
    q = q * (d / d.abs()).unsqueeze(-2)          # Q diag(R_ii/|R_ii|): Haar U(3)
    det = torch.linalg.det(q)
    q = q * torch.exp(-1j * torch.angle(det) / 3.0).reshape(n, 1, 1)  # -> SU(3)
    return q


def _expm_i(h, eps):
    """exp(i*eps*h) for Hermitian 3x3 h by scaling (2^-4), Taylor (order 14)
    and four squarings; accurate to ~1e-15 for |eps*lambda| up to ~10."""
    a = (1j * eps / 16.0) * h
    eye = torch.eye(3, dtype=h.dtype, device=h.device).expand_as(h)
    e = eye.clone()
    for k in range(14, 0, -1):                  # Horner: I + a/1 (I + a/2 (...))
        e = eye + _mm3(a, e) / k
    for _ in range(4):
        e = _mm3(e, e)
    return e


def near_unit_su3(n, gen, device="cpu", eps=0.3):
    """n matrices exp(i*eps*H), H traceless Hermitian with E|G_ij|^2 = 1."""
    g = _cgauss((n, 3, 3), gen, device)
    h = 0.5 * (g + _dagger(g))
    tr = torch.diagonal(h, dim1=-2, dim2=-1).sum(-1) / 3.0
    h = h - tr.reshape(n, 1, 1) * torch.eye(3, dtype=h.dtype, device=device)
    return _expm_i(h, eps)


def random_su3_field(n, seed, device="cpu"):
    """n Haar SU(3) matrices from a given seed (gauge transformations in tests)."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((n, 3, 3), dtype=torch.complex128, device=device)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = haar_su3(e - s, gen, device)
    return out


def make_links(dims, kind="near_unit", seed=GAUGE_SEED, device="cpu", eps=0.3,
               fold_phases=True):
    """Fat and long links, complex128 ``[4, V, 3, 3]`` each.

    ``F = 0.6 U + 0.4 U'`` and ``L = -(1/24) U1 U2 U3`` with every factor drawn
    from ``kind`` ('haar' or 'near_unit'); phases folded in unless
    ``fold_phases`` is False.
    """
    _check_dims(dims)
    V = volume(dims)
    if kind == "haar":
        draw = lambda n, g: haar_su3(n, g, device)  # noqa: E731
    elif kind == "near_unit":
        draw = lambda n, g: near_unit_su3(n, g, device, eps)  # noqa: E731
    else:
        raise ValueError(f"unknown link kind {kind!r}")
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    fat = torch.empty((4, V, 3, 3), dtype=torch.complex128, device=device)
    lng = torch.empty((4, V, 3, 3), dtype=torch.complex128, device=device)
    for mu in range(4):
        for s in range(0, V, _CHUNK):
            e = min(V, s + _CHUNK)
            n = e - s
            u0, u1 = draw(n, gen), draw(n, gen)
            fat[mu, s:e] = 0.6 * u0 + 0.4 * u1
            w1, w2, w3 = draw(n, gen), draw(n, gen), draw(n, gen)
            lng[mu, s:e] = (-1.0 / 24.0) * _mm3(_mm3(w1, w2), w3)
    if fold_phases:
        eta_f, eta_l = eta_phases(dims, device)
        fat *= eta_f.reshape(4, V, 1, 1)
        lng *= eta_l.reshape(4, V, 1, 1)
    return fat, lng


def unit_links(dims, device="cpu", c1=1.0, c3=-1.0 / 24.0):
    """Free field: F = c1 * eta, L = c3 * eta (phases and boundary folded in)."""
    V = volume(dims)
    eye = torch.eye(3, dtype=torch.complex128, device=device)
    eta_f, eta_l = eta_phases(dims, device)
    fat = c1 * eta_f.reshape(4, V, 1, 1).to(torch.complex128) * eye
    lng = c3 * eta_l.reshape(4, V, 1, 1).to(torch.complex128) * eye
    return fat.contiguous(), lng.contiguous()


def gaussian_spinor(n_sites, seed, device="cpu", nrhs=None):
    """Complex Gaussian colour vectors, complex128 ``[n_sites, 3]`` (or
    ``[nrhs, n_sites, 3]``), unit variance per complex component."""
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    shape = (n_sites, 3) if nrhs is None else (nrhs, n_sites, 3)
    return _cgauss(shape, gen, device)
