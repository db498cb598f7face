"""The oracle's shared-exponent generator (the family of Sec. 4 with component
width B): B = 20 and B = 30 reproduce the pinned 20- and 30-bit codecs bit for
bit, B = 24 matches hand-derived records, error bounds and exact symmetries,
and plausible mistakes planted in a copy of the generator are caught."""
import os
import types

import numpy as np
import pytest

import oracle
from pins import _read_golden


def spread(n, seed, dtype, decades=30):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 6)) * 10.0 ** rng.uniform(-decades, decades, size=(n, 1))
    v[::53] = 0.0                        # all-zero sites
    v[1::53, 3] = 0.0                    # partially zero sites
    return v.astype(dtype)


def golden_failures(mod, name, bits):
    bad = []
    words = mod.shared_exponent_words(bits)
    dt = np.float32 if bits <= 24 else np.float64
    for vin, wout in _read_golden(name):
        v = np.array([float(s) for s in vin], dtype=dt)[None, :]
        want = np.array([int(s, 16) for s in wout], dtype=np.uint32)
        assert want.size == words
        w = mod.shared_exponent_encode(v, bits)[0]
        if not np.array_equal(w, want):
            bad.append((vin, [hex(int(a)) for a in w]))
        back = mod.shared_exponent_decode(want[None, :], bits)[0]
        # the exponent field sits just above the six components
        k, off = divmod(6 * bits, 32)
        E = (int(want[k]) >> off) & 0xFF
        if np.abs(back.astype(np.float64) - v[0]).max() > 2.0 ** (E - 128):
            bad.append(("decode", vin, back))
    return bad


def generator_failures(mod):
    """every pin of the generator; returns the names of those that fail"""
    failed = []
    if golden_failures(mod, "int20_appendix_a.txt", 20):
        failed.append("golden20")
    if golden_failures(mod, "int30_listing3.txt", 30):
        failed.append("golden30")
    if golden_failures(mod, "int24_generated.txt", 24):
        failed.append("golden24")
    v = spread(4000, 11, np.float32)
    back = mod.shared_exponent_decode(mod.shared_exponent_encode(v, 24), 24).astype(np.float64)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float64)
    if not (np.abs(back - v) <= m / (2.0 ** 23 - 1) * (1 + 2.0 ** -23)).all():
        failed.append("bound24")
    return failed


def test_generator_reproduces_int20(oracle_lib):
    v = spread(30000, 1, np.float32)
    w = oracle.shared_exponent_encode(v, 20)
    assert w.shape == (30000, 4)
    assert np.array_equal(w, oracle.int20_encode(v, oracle_lib))
    assert np.array_equal(oracle.shared_exponent_decode(w, 20), oracle.int20_decode(w, oracle_lib))
    assert not golden_failures(oracle, "int20_appendix_a.txt", 20)


def test_generator_reproduces_int30(oracle_lib):
    v = spread(30000, 2, np.float64, decades=40)        # within the range of E <= 254
    w = oracle.shared_exponent_encode(v, 30)
    assert w.shape == (30000, 6)
    assert np.array_equal(w, oracle.int30_encode(v, oracle_lib))
    assert np.array_equal(oracle.shared_exponent_decode(w, 30), oracle.int30_decode(w, oracle_lib))
    assert not golden_failures(oracle, "int30_listing3.txt", 30)


def test_int24_hand_derived_records():
    assert oracle.shared_exponent_words(24) == 5
    assert not golden_failures(oracle, "int24_generated.txt", 24)


def test_int24_error_bound_and_range():
    v = spread(40000, 3, np.float32)
    w = oracle.int24_encode(v)
    back = oracle.int24_decode(w).astype(np.float64)
    m = np.abs(v).max(axis=1, keepdims=True).astype(np.float64)
    # quantum 2^(E-127) <= 2 t, t = fl(M/(2^23-1)): rounding error <= t
    assert (np.abs(back - v) <= m / (2.0 ** 23 - 1) * (1 + 2.0 ** -23)).all()
    # the largest component uses the top of the 24-bit range: 2^21 <= |q| <= 2^23 - 1
    E = (w[:, 4] >> 16) & 0xFF
    assert not (w[:, 4] >> 24).any()
    nz = m[:, 0] > 0
    qmax = m[nz, 0] / 2.0 ** (E[nz].astype(np.float64) - 127)
    assert (qmax >= 2.0 ** 21 * (1 - 2.0 ** -20)).all() and (qmax <= 2.0 ** 23).all()
    # zero sites: E = 1 and nothing else set
    z = ~nz
    assert (w[z, :4] == 0).all() and (w[z, 4] == 0x10000).all()


def test_int24_sign_and_scale():
    v = spread(3000, 4, np.float32, decades=3)
    w = oracle.int24_encode(v)
    assert np.array_equal(oracle.int24_decode(oracle.int24_encode(-v)), -oracle.int24_decode(w))
    for k in (-9, 1, 6):
        ws = oracle.int24_encode(v * np.float32(2.0 ** k))
        # only the exponent field moves, by k
        assert np.array_equal(ws[:, :4], w[:, :4]) and np.array_equal(ws[:, 4] & 0xFFFF, w[:, 4] & 0xFFFF)
        nz = np.abs(v).max(axis=1) > 0
        assert np.array_equal(((ws[nz, 4] >> 16) & 0xFF).astype(np.int64), ((w[nz, 4] >> 16) & 0xFF).astype(np.int64) + k)


def test_int24_finer_than_int20():
    v = spread(5000, 5, np.float32, decades=2)
    e32 = lambda f: np.abs(f.astype(np.float64) - v).sum()
    e20 = e32(oracle.int20_decode(oracle.int20_encode(v)))
    e24 = e32(oracle.int24_decode(oracle.int24_encode(v)))
    # four more bits: about 16 times smaller rounding error, and still above zero
    assert 8 * e24 < e20 and e24 > 0


GENERATOR_MUTATIONS = {
    "split_low_bits_first": ("words[:, k] |= (val >> np.uint64(spill)) << np.uint64(off)",
                             "words[:, k] |= val << np.uint64(off)"),
    "exponent_not_rounded_up": ("ex.astype(np.int64) + 127", "ex.astype(np.int64) + 126"),
    "scale_2_to_B": ("t = m / ft(2 ** (bits - 1) - 1)", "t = m / ft(2 ** bits - 1)"),
    "truncate_not_round": ("q = np.rint(a * inv[:, None])", "q = np.trunc(a * inv[:, None])"),
    "no_sign_extension": ("q = np.where(q >= 2 ** (bits - 1), q - 2 ** bits, q)", "q = q"),
    "exponent_below_components": ("[((f * bits) // 32, (f * bits) % 32, bits if f < 6 else 8) for f in range(7)]",
                                  "[((p // 32), p % 32, bits if f < 6 else 8) for f, p in "
                                  "enumerate([8 + bits * i for i in range(6)] + [0])]"),
}


@pytest.mark.parametrize("name", sorted(GENERATOR_MUTATIONS))
def test_generator_mutation_is_caught(name):
    old, new = GENERATOR_MUTATIONS[name]
    path = os.path.join(os.path.dirname(oracle.__file__), "__init__.py")
    src = open(path).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found in the oracle"
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = path
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    with np.errstate(all="ignore"):
        try:
            failed = generator_failures(mod)
        except Exception as e:                       # a crash counts as caught
            failed = [repr(e)]
    assert failed, f"mutation {name} passed every generator pin"


def test_unmutated_generator_passes_all():
    assert generator_failures(oracle) == []
