"""Regression of the oracle against its own committed snapshot (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _snap():
    with open(os.path.join(HERE, "golden", "oracle_snapshot.json")) as f:
        return json.load(f)


def test_snapshot_unchanged(orc):
    s = _snap()
    n = 1 << 20
    u = orc.philox_generate(42, 0, orc.UNIFORM_F32, n)
    b = orc.philox_generate(42, 0, orc.BITS_U32, n)
    assert [int(x) for x in b[:16]] == s["philox_seed42_u32_first16"]
    assert hashlib.sha256(u.tobytes()).hexdigest() == s["philox_seed42_f32_n2^20_sha256"]
    assert hashlib.sha256(b.tobytes()).hexdigest() == s["philox_seed42_bits_n2^20_sha256"]
    st = orc.mrg_seed(42)
    y, st2 = orc.mrg_words(st, 16)
    assert [int(x) for x in y] == s["mrg_seed42_y_first16"]
    assert [int(x) for x in orc.mrg_skip(st, 1 << 76)] == s["mrg_seed42_state_after_2^76"]
    z = orc.philox_generate(42, 0, orc.GAUSSIAN_F32, 8)
    assert np.array_equal(z, np.array(s["philox_seed42_gauss_fp64_first8"]))


def test_snapshot_new_kinds_unchanged(orc):
    """Uniform int32 and the inverse-CDF Gaussians (R23, R24)."""
    s = _snap()
    i = orc.philox_generate(42, 0, orc.UNIFORM_I32, 4096, -1000.0, 1000.0)
    assert [int(x) for x in i[:16]] == s["philox_seed42_i32_-1000_1000_first16"]
    assert hashlib.sha256(i.tobytes()).hexdigest() == s["philox_seed42_i32_-1000_1000_n4096_sha256"]
    for kind, name in ((orc.GAUSSIAN_ICDF_F32, "icdf_f32"), (orc.GAUSSIAN_ICDF_F64, "icdf_f64")):
        zp = orc.philox_generate(42, 0, kind, 4096)
        zm, _ = orc.mrg_generate(orc.mrg_seed(42), kind, 4096)
        assert [float(x) for x in zp[:8]] == s[f"philox_seed42_{name}_first8"]
        assert hashlib.sha256(zp.tobytes()).hexdigest() == s[f"philox_seed42_{name}_n4096_sha256"]
        assert hashlib.sha256(zm.tobytes()).hexdigest() == s[f"mrg_seed42_{name}_n4096_sha256"]
