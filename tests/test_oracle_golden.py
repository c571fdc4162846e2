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
