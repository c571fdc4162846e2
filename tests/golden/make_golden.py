"""Writes tests/golden/oracle_snapshot.json from the oracle alone.

The paper prints no generated values, so these fixtures are not external
pins: they freeze the oracle's outputs so that any later change to its
arithmetic shows up as a test failure and must be justified.

Run: python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def main():
    n = 1 << 20
    snap = {}
    u = oracle.philox_generate(42, 0, oracle.UNIFORM_F32, n)
    b = oracle.philox_generate(42, 0, oracle.BITS_U32, n)
    b2 = oracle.philox_generate(42, n, oracle.BITS_U32, n)
    snap["philox_seed42_u32_first16"] = [int(x) for x in b[:16]]
    snap["philox_seed42_f32_first8"] = [float(x) for x in u[:8]]
    snap["philox_seed42_f32_n2^20_sha256"] = digest(u)
    snap["philox_seed42_bits_n2^20_sha256"] = digest(b)
    snap["philox_seed42_bits_after_f32_n2^20_sha256"] = digest(b2)
    st = oracle.mrg_seed(42)
    y, st2 = oracle.mrg_words(st, 16)
    snap["mrg_seed42_y_first16"] = [int(x) for x in y]
    snap["mrg_seed42_state_after16"] = [int(x) for x in st2]
    j = oracle.mrg_skip(st, 1 << 76)
    snap["mrg_seed42_state_after_2^76"] = [int(x) for x in j]
    z = oracle.philox_generate(42, 0, oracle.GAUSSIAN_F32, 8)
    snap["philox_seed42_gauss_fp64_first8"] = [float(x) for x in z]
    i = oracle.philox_generate(42, 0, oracle.UNIFORM_I32, 4096, -1000.0, 1000.0)
    snap["philox_seed42_i32_-1000_1000_first16"] = [int(x) for x in i[:16]]
    snap["philox_seed42_i32_-1000_1000_n4096_sha256"] = digest(i)
    for kind, name in ((oracle.GAUSSIAN_ICDF_F32, "icdf_f32"), (oracle.GAUSSIAN_ICDF_F64, "icdf_f64")):
        zp = oracle.philox_generate(42, 0, kind, 4096)
        zm, _ = oracle.mrg_generate(oracle.mrg_seed(42), kind, 4096)
        snap[f"philox_seed42_{name}_first8"] = [float(x) for x in zp[:8]]
        snap[f"philox_seed42_{name}_n4096_sha256"] = digest(zp)
        snap[f"mrg_seed42_{name}_n4096_sha256"] = digest(zm)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_snapshot.json")
    with open(path, "w") as f:
        json.dump(snap, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
