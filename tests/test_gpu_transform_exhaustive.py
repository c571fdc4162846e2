"""Exhaustive GPU checks of the FP32 Gaussian transforms, input by input:
every one of the 2^24 values of u1 for the Box-Muller radius r(u1), every
one of the 2^24 values of u2 for the rotation (cos, sin)(2 pi u2), and every
one of the 2^24 inputs of the inverse-CDF Gaussian FP32, each against the
oracle.

A Gaussian FP32 pair is (RN32(r c), RN32(r s)) of the two FP64 factors the
probe returns, so the factors' worst relative errors bound all 2^48 word
pairs at once: an output is within 1/2 ulp (its one rounding) plus
2^24 (max rel. error of r + max rel. error of cos/sin) ulp of the exact
transform, since |z| / ulp32(z) < 2^24.  The oracle's own factors are
pinned against mpmath far below that (tests/test_oracle_dists.py)."""
import concurrent.futures

import numpy as np
import pytest

import oracle
import paper_2109_01329_amd as mr
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

N24 = 1 << 24
THREADS = 16


def _probe(which: int, count: int, dtype):
    import torch
    out = torch.empty(count, dtype=dtype, device="cuda")
    mr.bench_transform_f32(which, 0, N24, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _rel(got: np.ndarray, want: np.ndarray):
    """Worst relative error where want != 0, and whether every exact zero
    of want is reproduced as an exact zero."""
    nz = want != 0.0
    rel = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    i = int(np.argmax(rel))
    return float(rel[i]), int(np.nonzero(nz)[0][i]), bool(np.all(got[~nz] == 0.0))


def test_box_muller_factors_every_input():
    print("exhaustive Box-Muller factors: 2^24 radii, 2^24 rotations", flush=True)
    words = np.arange(N24, dtype=np.uint32) << np.uint32(8)
    r_want, s_want, c_want = oracle.box_muller_factors(words)
    r = _probe(0, N24, _dtype("f64"))
    cs = _probe(1, 2 * N24, _dtype("f64"))
    c, s = cs[0::2], cs[1::2]
    er, kr, zr = _rel(r, r_want)
    ec, kc, zc = _rel(c, c_want)
    es, ks, zs = _rel(s, s_want)
    bound = 0.5 + 2.0**24 * (er + max(ec, es))
    print(f"radius worst rel {er:.3e} (2^{np.log2(er):.2f}) at u1 = ({kr} + 1) 2^-24; "
          f"cos {ec:.3e} (2^{np.log2(ec):.2f}) at k = {kc}; "
          f"sin {es:.3e} (2^{np.log2(es):.2f}) at k = {ks}; "
          f"composed bound {bound:.3f} ulp", flush=True)
    # exact zeros: r at u1 = 1, cos at u2 = 1/4, 3/4, sin at u2 = 0, 1/2
    assert r_want[N24 - 1] == 0.0 and r[N24 - 1] == 0.0
    assert zr and zc and zs
    assert np.count_nonzero(c_want == 0.0) == 2 and np.count_nonzero(s_want == 0.0) == 2
    assert bound <= 2.0, "the factors no longer compose to within 2 ulp"
    # what the kernels are built to: each factor within 2^-28
    assert er < 2.0**-28 and ec < 2.0**-28 and es < 2.0**-28


def test_gaussian_f32_zero_radius_in_a_generate():
    """u1 = 1 (the word's top 24 bits all ones) gives z0 = z1 = +-0 in a
    real generate: find the first Gaussian pair of seed 42 whose first word
    is such, generate around it, compare with the oracle."""
    seed, chunk = 42, 1 << 24
    pos = None
    for start in range(0, 1 << 28, chunk):
        w = oracle.philox_words(seed, start, chunk)
        hit = np.nonzero((w[0::2] >> np.uint32(8)) == 0xFFFFFF)[0]
        if hit.size:
            pos = start + 2 * int(hit[0])
            break
    assert pos is not None
    print(f"u1 = 1 at word position {pos}", flush=True)
    lo = max(0, pos - 64)
    e = mr.Engine(mr.PHILOX4X32_10, seed, lo)
    n = pos - lo + 66
    got, _ = gh.generate(e, mr.GAUSSIAN_F32, n)
    want = oracle.philox_generate(seed, lo, oracle.GAUSSIAN_F32, n)
    k = pos - lo
    assert want[k] == 0.0 and want[k + 1] == 0.0
    assert got[k] == 0.0 and got[k + 1] == 0.0
    assert gh.gauss_errors(got, want).max() <= 1.0


def test_icdf_f32_every_input():
    print("exhaustive inverse-CDF Gaussian FP32: 2^24 inputs", flush=True)
    g = _probe(2, N24, _dtype("f32"))
    words = np.arange(N24, dtype=np.uint32) << np.uint32(8)
    parts = np.array_split(np.arange(N24), THREADS)

    def part(idx):
        return oracle.apply(oracle.GAUSSIAN_ICDF_F32, oracle.PHILOX, words[idx], idx.size,
                            0.0, 1.0)

    with concurrent.futures.ThreadPoolExecutor(max_workers=THREADS) as ex:
        d = np.concatenate(list(ex.map(part, parts)))
    err = np.abs(g.astype(np.float64) - d) / gh.ulp32(d)
    i = int(np.argmax(err))
    print(f"inverse-CDF FP32 worst {err[i]:.3f} ulp at k = {i} (u = ({i} + 1/2) 2^-24)",
          flush=True)
    assert err[i] <= 2.0


def _dtype(name: str):
    import torch
    return torch.float64 if name == "f64" else torch.float32
