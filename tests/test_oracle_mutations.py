"""The pins are strong enough: each plausible mistake planted in a copy of
the oracle (on the CPU) makes at least one pin fail."""
import os
import tempfile

import pytest

import oracle
import pins

MUTATIONS = {
    "backward_fat_sign": ("add_mdv(acc, -1.0, link(fat", "add_mdv(acc, +1.0, link(fat"),
    "backward_fat_index": ("link(fat, mu, xm1, V)", "link(fat, mu, x, V)"),
    "backward_long_index": ("link(lng, mu, xm3, V)", "link(lng, mu, xm1, V)"),
    "dagger_missing_conj": ("acc += conj(U[3 * b + a]) * v[b]", "acc += U[3 * b + a] * v[b]"),
    "dagger_missing_transpose": ("acc += conj(U[3 * b + a]) * v[b]", "acc += conj(U[3 * a + b]) * v[b]"),
    "forward_transposed": ("acc += U[3 * a + b] * v[b]", "acc += U[3 * b + a] * v[b]"),
    "naik_hop_two": ("long xp3 = hop_site(x, mu, +3, d);", "long xp3 = hop_site(x, mu, +2, d);"),
    "naik_back_dropped": ("add_mdv(acc, -1.0, link(lng, mu, xm3, V), in + 3 * xm3);", ""),
    "naik_fwd_wrong_spinor": ("link(lng, mu, x, V), in + 3 * xp3", "link(lng, mu, x, V), in + 3 * xp1"),
    "normal_op_sign": ("c * in[3 * x + a] - out[3 * x + a]", "c * in[3 * x + a] + out[3 * x + a]"),
    "cg_residual_sign": ("r[k] -= alpha * ap[k]; }", "r[k] += alpha * ap[k]; }"),
    "cg_beta_inverted": ("double beta = rr_new / rr;", "double beta = rr / rr_new;"),
    "ms_zeta_shift_sign": ("(1.0 + a * s)", "(1.0 - a * s)"),
    "ms_beta_not_squared": ("double bi = bb * (znew / z[i]) * (znew / z[i]);", "double bi = bb * (znew / z[i]);"),
    "ms_alpha_ratio_inverted": ("double ai = a * znew / z[i];", "double ai = a * z[i] / znew;"),
    "int20_split_offset": ("o[0] = u[0] | ((u[1] >> 8) << 20);", "o[0] = u[0] | ((u[1] >> 8) << 19);"),
    "int20_exponent_not_rounded_up": ("uint32_t e = ((f32_bits(t) >> 23) & 0xffu) + 1u;",
                                      "uint32_t e = ((f32_bits(t) >> 23) & 0xffu) + 0u;"),
    "int30_scale_2_30": ("double t = m / 536870911.0;", "double t = m / 1073741823.0;"),
    "half16_scale_2_15": ("float c = 32767.0f / m;", "float c = 32768.0f / m;"),
    "half16_decode_reciprocal": ("float d = norm[s] / 32767.0f;", "float d = norm[s] * (1.0f / 32767.0f);"),
    "fix16_truncate": ("q[k] = (int16_t)llrint(u[k] * c);", "q[k] = (int16_t)(u[k] * c);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found in the oracle"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "hisq_oracle_mut.c")
        with open(path, "w") as fh:
            fh.write(src.replace(old, new))
        lib = oracle.load(oracle.build(out=os.path.join(d, "libmut.so"), src=path))
        failed = []
        for check in pins.ALL:
            try:
                ok, _ = check(lib)
            except Exception:
                ok = False
            if not ok:
                failed.append(check.__name__)
                break
        assert failed, f"no pin caught mutation {name}"
