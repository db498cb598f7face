"""Pins of the oracle's two-row long-link storage (Sec. 1, compression of
special unitary matrices): the rebuilt third row, the split of a long link
into coefficient, phase and SU(3) factor, and the round trip."""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_09224_amd import inputs


def test_third_row_of_random_su3():
    u = inputs.haar_su3(500, torch.Generator().manual_seed(5)).numpy()
    r3 = oracle.su3_third_row(u[:, :2, :])
    assert np.abs(r3 - u[:, 2, :]).max() < 1e-13


def test_third_row_closed_forms():
    a, b = 0.7, -1.9
    d = np.diag([np.exp(1j * a), np.exp(1j * b), np.exp(-1j * (a + b))])
    assert np.abs(oracle.su3_third_row(d[:2]) - [0, 0, np.exp(-1j * (a + b))]).max() < 1e-15
    # cyclic permutation matrix (det +1): rows e2, e3 -> third row e1
    p = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=np.complex128)
    assert np.array_equal(oracle.su3_third_row(p[:2]), np.array([1, 0, 0], dtype=np.complex128))
    # a U(3) matrix with det = e^{i phi}: the rebuilt row misses it by exactly that phase
    phi = 0.3
    w = inputs.haar_su3(1, torch.Generator().manual_seed(6)).numpy()[0]
    w[2] *= np.exp(1j * phi)
    assert abs(np.linalg.det(w) - np.exp(1j * phi)) < 1e-13
    assert np.abs(oracle.su3_third_row(w[:2]) * np.exp(1j * phi) - w[2]).max() < 1e-13


def test_long_phases_match_free_field():
    """the free long link is c3 * phase * 1"""
    dims = (4, 6, 4, 8)
    _, lng = inputs.unit_links(dims, c3=-1.0 / 24.0)
    ph = oracle.long_phases(dims)
    assert np.array_equal(lng.numpy()[:, :, 0, 0].real, -ph / 24.0)
    # antiperiodic time: only the temporal link of the last three slices flips
    X, Y, Z, T = dims
    i = np.arange(oracle.volume(dims))
    t = i // (X * Y * Z)
    x, y, z = i % X, (i // X) % Y, (i // (X * Y)) % Z
    eta3 = np.where((x + y + z) % 2 == 1, -1.0, 1.0)
    assert np.array_equal(ph[3] * eta3, np.where(t >= T - 3, -1.0, 1.0))


@pytest.mark.parametrize("kind", ["near_unit", "haar"])
def test_split_recovers_construction(kind):
    dims = (4, 4, 4, 6)
    _, lng = inputs.make_links(dims, kind, seed=17)
    c, u = oracle.long_link_split(lng.numpy(), dims)
    assert abs(c + 1.0 / 24.0) < 1e-14
    assert np.abs(np.linalg.det(u.reshape(-1, 3, 3)) - 1).max() < 1e-12
    # round trip in FP64 with two rows: the field itself
    back = oracle.long_recon_roundtrip(lng.numpy(), dims, "f64", 64)
    assert np.abs(back - lng.numpy()).max() < 1e-14


def test_split_rejects():
    dims = (4, 4, 4, 4)
    fat, lng = inputs.make_links(dims, "near_unit", seed=18)
    with pytest.raises(ValueError):
        oracle.long_link_split(fat.numpy(), dims)          # fat links are not SU(3) multiples
    bad = lng.numpy().copy()
    bad[2, 5] *= -1.0                                        # one sign off the phase pattern
    with pytest.raises(ValueError):
        oracle.long_link_split(bad, dims)
    bad = lng.numpy().copy()
    bad[1, 7] *= np.exp(0.1j)                                # det phase
    with pytest.raises(ValueError):
        oracle.long_link_split(bad, dims)


def test_recon_dslash_equals_full_dslash():
    dims = (4, 6, 4, 8)
    fat, lng = inputs.make_links(dims, "haar", seed=19)
    psi = inputs.gaussian_spinor(oracle.volume(dims), 21).numpy()
    for parity in (0, 1):
        a = oracle.emulated_dslash(fat.numpy(), lng.numpy(), psi, dims, parity, "f64", "f64", 64, long_recon=12)
        b = oracle.dslash(fat.numpy(), lng.numpy(), psi, dims, parity)
        assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()
    # with 16-bit rows the long-link contribution carries the 16-bit error only
    a = oracle.emulated_dslash(fat.numpy(), lng.numpy(), psi, dims, 0, "fix16", "f64", 64, long_recon=12)
    b = oracle.emulated_dslash(fat.numpy(), lng.numpy(), psi, dims, 0, "fix16", "f64", 64)
    assert 0 < np.abs(a - b).max() < 1e-4 * np.abs(b).max()


# ---------------------------------------------------------------------------
# eight-parameter storage
# ---------------------------------------------------------------------------

def test_eight_params_rebuild_random_su3():
    """parameters taken from random special unitary matrices rebuild them:
    Haar (rough) and near-unit ones, to within FP64 rounding amplified by the
    conditioning, 1/min(N, |u20|^2) with N = |u01|^2 + |u02|^2 (the 2x2
    system's determinant) and |u20| the root of a difference of norms"""
    for u in (inputs.haar_su3(4000, torch.Generator().manual_seed(8)).numpy(),
              oracle.long_link_split(inputs.make_links((4, 4, 4, 4), "near_unit", seed=19)[1].numpy(),
                                     (4, 4, 4, 4))[1].reshape(-1, 3, 3)):
        back = oracle.su3_from_eight(oracle.su3_eight_params(u))
        n = np.minimum(np.abs(u[:, 0, 1]) ** 2 + np.abs(u[:, 0, 2]) ** 2, np.abs(u[:, 2, 0]) ** 2)
        err = np.abs(back - u).max(axis=(1, 2))
        assert (err <= 1e-13 / n).all(), float((err * n).max())
        assert np.median(err) < 1e-14
        assert np.abs(np.linalg.det(back) - 1).max() < 1e-12


def test_eight_params_closed_forms():
    """the rotation in the (1,3) plane, a1 = cos(a), a3 = u20 = i sin(a):
    parameters (0, 0, 0, sin(a), 0, 0, 0, tan(pi/8)) and back; a phase of
    pi on a1 is v = tan(pi/4) = 1"""
    a = 0.4
    w = np.array([[np.cos(a), 0, 1j * np.sin(a)], [0, 1, 0], [1j * np.sin(a), 0, np.cos(a)]], dtype=np.complex128)
    assert abs(np.linalg.det(w) - 1) < 1e-15
    pw = oracle.su3_eight_params(w)
    assert np.allclose(pw, [0, 0, 0, np.sin(a), 0, 0, 0, np.tan(np.pi / 8)], atol=1e-16)
    assert np.abs(oracle.su3_from_eight(pw) - w).max() < 1e-15
    d = np.diag([-1.0, -1.0, 1.0]).astype(np.complex128) @ w
    pd = oracle.su3_eight_params(d)
    assert pd[6] == pytest.approx(1.0, abs=1e-15)
    assert np.abs(oracle.su3_from_eight(pd) - d).max() < 1e-15


def test_eight_params_degenerate_column():
    """u20 = 0: |u20| is the root of a difference of norms that rounding
    leaves at about 1e-16, so the rebuild is only good to about sqrt(eps)
    there (the known weak point of eight-parameter storage)"""
    a = 0.4
    u = np.array([[np.cos(a), np.sin(a), 0], [-np.sin(a), np.cos(a), 0], [0, 0, 1]], dtype=np.complex128)
    p = oracle.su3_eight_params(u)
    assert np.allclose(p, [np.sin(a), 0, 0, 0, -np.sin(a), 0, 0, 0], atol=1e-16)
    err = np.abs(oracle.su3_from_eight(p) - u).max()
    assert err < 4 * np.sqrt(np.finfo(float).eps), err


def test_phase_param_is_tan_quarter_angle():
    """the fixed operation sequence computes tan(arg(z)/4): closed forms and
    random arguments (including both signs of zero and the negative axis)"""
    z = np.array([1, 1j, -1, -1j, 1 + 1j, -1 + 0j, complex(-1, -0.0), 0, 3 - 4j], dtype=np.complex128)
    want = np.array([0, np.tan(np.pi / 8), 1, -np.tan(np.pi / 8), np.tan(np.pi / 16), 1, -1, 0,
                     np.tan(np.arctan2(-4, 3) / 4)])
    assert np.abs(oracle.phase_param(z) - want).max() < 2e-16
    rng = np.random.default_rng(3)
    zr = (rng.standard_normal(20000) + 1j * rng.standard_normal(20000)) * 10.0 ** rng.uniform(-3, 3, 20000)
    assert np.abs(oracle.phase_param(zr) - np.tan(np.angle(zr) / 4)).max() < 4e-16


def test_eight_param_long_links_round_trip():
    """FP64 storage of the eight parameters gives the long links back (to the
    rebuild's conditioning); FIX32 within the stored quantum amplified by it"""
    dims = (4, 4, 4, 6)
    _, lng = inputs.make_links(dims, "near_unit", seed=23)
    lng = lng.numpy()
    c, u = oracle.long_link_split(lng, dims)
    kappa = 1.0 / np.minimum(np.abs(u[..., 0, 1]) ** 2 + np.abs(u[..., 0, 2]) ** 2, np.abs(u[..., 2, 0]) ** 2)
    back = oracle.long_recon8_roundtrip(lng, dims, "f64")
    assert (np.abs(back - lng).max(axis=(-1, -2)) <= 1e-13 * abs(c) * kappa).all()
    back = oracle.long_recon8_roundtrip(lng, dims, "fix32")
    rel = np.abs(back - lng).max(axis=(-1, -2)) / abs(c)
    assert (rel <= 64 * 2.0 ** -31 * kappa).all()
    assert np.median(rel) <= 8 * 2.0 ** -31
    with pytest.raises(ValueError):
        oracle.long_recon8_encode(lng, dims, "fix16")
