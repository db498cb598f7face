"""Storage-format codecs of the oracle: error bounds and exact symmetries."""
import numpy as np
import pytest

import oracle
import pins


def rand6(n, seed, dtype, spread=True):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 6))
    if spread:  # per-site magnitudes over many decades
        v *= 10.0 ** rng.uniform(-20, 20, size=(n, 1))
    return v.astype(dtype)


def test_int20_error_bound(oracle_lib):
    v = rand6(20000, 1, np.float32)
    back = oracle.int20_decode(oracle.int20_encode(v, oracle_lib), oracle_lib)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float64)
    err = np.abs(back.astype(np.float64) - v)
    # q_unit = 2^(E-127) <= 2 t, t = fl(M/(2^19-1)); rounding error <= q_unit/2
    assert (err <= m / 524287.0 * (1 + 2.0 ** -22)).all()
    assert (err <= m * 2.0 ** -18).all()


def test_int30_error_bound(oracle_lib):
    v = rand6(20000, 2, np.float64)
    back = oracle.int30_decode(oracle.int30_encode(v, oracle_lib), oracle_lib)
    m = np.abs(v).max(axis=1, keepdims=True)
    err = np.abs(back - v)
    assert (err <= m / 536870911.0 * (1 + 2.0 ** -50)).all()


def test_half16_error_bound(oracle_lib):
    v = rand6(20000, 3, np.float32, spread=False) * np.float32(7.5)
    q, nm = oracle.half16_encode(v, oracle_lib)
    back = oracle.half16_decode(q, nm, oracle_lib)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float64)
    err = np.abs(back.astype(np.float64) - v)
    assert (err <= 0.5 * m / 32767.0 * (1 + 1e-5) + m * 2.0 ** -23).all()
    assert (np.abs(q).max(axis=1) == 32767).all()          # the max component maps to full scale


@pytest.mark.parametrize("fmt", ["int20", "int30"])
def test_shared_exponent_sign_and_scale(fmt, oracle_lib):
    dt = np.float32 if fmt == "int20" else np.float64
    enc = getattr(oracle, fmt + "_encode")
    v = rand6(3000, 4, dt, spread=False)
    w = enc(v, oracle_lib)
    wn = enc(-v, oracle_lib)
    back, backn = [getattr(oracle, fmt + "_decode")(a, oracle_lib) for a in (w, wn)]
    assert np.array_equal(backn, -back)                    # rint is odd-symmetric
    for k in (-7, 1, 5):
        ws = enc(v * dt(2.0 ** k), oracle_lib)
        ebits = (lambda a: a[:, 3] >> 24) if fmt == "int20" else (lambda a: (a[:, 5] >> 20) & 0xff)
        assert np.array_equal(ebits(ws).astype(np.int64), ebits(w).astype(np.int64) + k)
        if fmt == "int20":
            assert np.array_equal(ws[:, :3], w[:, :3]) and np.array_equal(ws[:, 3] & 0xffffff, w[:, 3] & 0xffffff)
        else:
            assert np.array_equal(ws[:, :5], w[:, :5]) and np.array_equal(ws[:, 5] & 0xfffff, w[:, 5] & 0xfffff)


def test_int20_exact_on_grid(oracle_lib):
    # values that are integer multiples of the site quantum round-trip exactly
    rng = np.random.default_rng(5)
    q = rng.integers(-2 ** 18, 2 ** 18 + 1, size=(2000, 6))
    q[:, 0] = 2 ** 18
    v = (q * 2.0 ** -18 * 2.0 ** rng.integers(-30, 30, size=(2000, 1))).astype(np.float32)
    back = oracle.int20_decode(oracle.int20_encode(v, oracle_lib), oracle_lib)
    assert np.array_equal(back, v)


def test_half16_scale_invariance(oracle_lib):
    v = rand6(2000, 6, np.float32, spread=False)
    q, nm = oracle.half16_encode(v, oracle_lib)
    q2, nm2 = oracle.half16_encode(v * np.float32(8.0), oracle_lib)
    assert np.array_equal(q, q2) and np.array_equal(nm2, nm * np.float32(8.0))
    qn, _ = oracle.half16_encode(-v, oracle_lib)
    assert np.array_equal(qn, -q)


@pytest.mark.parametrize("bits", [16, 32])
def test_fixed_gauge_bound(bits, oracle_lib):
    rng = np.random.default_rng(7)
    u = (rng.standard_normal((500, 3, 3)) + 1j * rng.standard_normal((500, 3, 3))) * 0.3
    q, absmax = oracle.fix_encode(u, bits, lib=oracle_lib)
    Q = 2.0 ** (bits - 1) - 1
    assert np.abs(q.astype(np.int64)).max() == Q
    back = oracle.fix_decode(q, absmax, 64, shape=u.shape, lib=oracle_lib)
    d = back - u
    err = max(np.abs(d.real).max(), np.abs(d.imag).max())
    assert err <= 0.5 * absmax / Q * (1 + 1e-12) + absmax * 2.0 ** -52



def test_half16_decode_exact_definition(oracle_lib):
    ok, detail = pins.check_half16_decode_exact(oracle_lib)
    assert ok, detail
    # the rounding order the definition excludes differs at M = 513
    r = np.float32(1.0) / np.float32(32767.0)
    assert np.float32(513.0) * r != np.float32(np.float32(513.0) / np.float32(32767.0))
