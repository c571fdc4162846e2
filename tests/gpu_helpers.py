"""Helpers for the GPU parity tests: device buffers at chosen byte offsets,
oracle expectations computed element by element, and the FP32 ulp measure.
The HIP path is reached only through the C ABI binding."""
from __future__ import annotations

import math

import numpy as np

import oracle
import paper_2109_01329_amd as mr

NP_DTYPE = {mr.BITS_U32: np.uint32, mr.UNIFORM_F32: np.float32,
            mr.UNIFORM_F64: np.float64, mr.GAUSSIAN_F32: np.float32,
            mr.GAUSSIAN_F64: np.float64, mr.UNIFORM_I32: np.int32,
            mr.GAUSSIAN_ICDF_F32: np.float32, mr.GAUSSIAN_ICDF_F64: np.float64}


def device_buffer(nbytes: int):
    import torch
    return torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")


def fetch(buf, byte_off: int, kind: int, n: int) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    raw = buf[byte_off: byte_off + n * mr.ELEM_BYTES[kind]].cpu().numpy()
    return raw.view(NP_DTYPE[kind])


def generate(engine: mr.Engine, kind: int, n: int, byte_off: int = 0,
             p0=None, p1=None, fill: int = 0xA5):
    """Generate into a fresh buffer at byte offset `byte_off`; returns the
    outputs and the buffer (so guard bytes can be checked)."""
    buf = device_buffer(n * mr.ELEM_BYTES[kind] + byte_off + 64)
    buf.fill_(fill)
    base = int(buf.data_ptr())
    engine.generate(kind, n, base + byte_off, p0, p1)
    return fetch(buf, byte_off, kind, n), buf


def guards_intact(buf, byte_off: int, nbytes: int, fill: int = 0xA5) -> bool:
    import torch
    torch.cuda.synchronize()
    a = buf.cpu().numpy()
    return bool(np.all(a[:byte_off] == fill) and np.all(a[byte_off + nbytes:] == fill))


def oracle_philox(seed: int, pos: int, kind: int, n: int, p0=None, p1=None):
    return oracle.philox_generate(seed, pos, kind, n, p0, p1)


def oracle_mrg(state, kind: int, n: int, p0=None, p1=None):
    out, _ = oracle.mrg_generate(state, kind, n, p0, p1)
    return out


def oracle_request(engine: int, seed: int, offset: int, kind: int, n: int, p0=None, p1=None):
    """Outputs of a batch request: engine created from (seed, offset), then
    n outputs of `kind`."""
    if engine == mr.PHILOX4X32_10:
        return oracle_philox(seed, offset, kind, n, p0, p1)
    state = oracle.mrg_skip(oracle.mrg_seed(seed), offset)
    return oracle_mrg(state, kind, n, p0, p1)


def ulp32(x: np.ndarray) -> np.ndarray:
    """2^(floor(log2 |x|) - 23) for normal FP32 magnitudes, 2^-149 below."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    _, e = np.frexp(ax)                      # ax = m 2^e, m in [1/2, 1)
    u = np.ldexp(1.0, e - 24)
    return np.where(ax >= 2.0**-126, u, 2.0**-149)


def gauss_errors(g: np.ndarray, d: np.ndarray, mean: float = 0.0, sd: float = 1.0):
    """Error of FP32 Gaussians g against the oracle's FP64 values d, in units
    of the tolerance.  For (mean, sd) = (0, 1) the unit is 2 ulp32(d) and an
    exact zero must be reproduced as +-0.  Otherwise the result is
    fma(z32, RN32(sd), RN32(mean)) with z32 within 2 ulp of z, so the bound is
    2 ulp32(z) |sd| + |z| |sd - RN32(sd)| + |mean - RN32(mean)| + ulp32(g)/2."""
    g = g.astype(np.float64)
    if mean == 0.0 and sd == 1.0:
        tol = 2.0 * ulp32(d)
        err = np.abs(g - d)
        zero = d == 0.0
        err = np.where(zero, np.where(g == 0.0, 0.0, np.inf), err)
        return err / np.where(zero, 1.0, tol)
    z = (d - mean) / sd
    sd32 = float(np.float32(sd))
    m32 = float(np.float32(mean))
    tol = (2.0 * ulp32(z) * abs(sd) + np.abs(z) * abs(sd - sd32) + abs(mean - m32)
           + 0.5 * ulp32(g) + 1e-300)
    return np.abs(g - d) / tol


def ulp64(x: np.ndarray) -> np.ndarray:
    """2^(floor(log2 |x|) - 52) for normal FP64 magnitudes, 2^-1074 below."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    _, e = np.frexp(ax)
    return np.where(ax >= 2.0**-1022, np.ldexp(1.0, np.maximum(e - 53, -1074)), 2.0**-1074)


def gauss64_errors(g: np.ndarray, d: np.ndarray, mean: float = 0.0, sd: float = 1.0):
    """Error of FP64 Gaussians g against the oracle's values d, in units of
    the tolerance: 8 ulp64 of z (both sides evaluate log, sqrt and a
    sin/cos with exact quarter-turn reduction, each within a few ulp of the
    exact transform; the oracle is pinned within 4) scaled by |sd|, plus
    2 ulp64 of the result for the final scaling (fma on the device, multiply
    and add in the oracle).  z = 0 (u1 = 1) must give exactly the mean."""
    z = (d - mean) / sd
    tol = 8.0 * ulp64(z) * abs(sd) + 2.0 * ulp64(d)
    err = np.abs(g - d)
    exact = z == 0.0
    err = np.where(exact, np.where(g == d, 0.0, np.inf), err)
    return err / np.where(exact, 1.0, tol)


def assert_match(kind: int, got: np.ndarray, want: np.ndarray, p0=None, p1=None):
    assert got.shape == want.shape
    if kind in (mr.GAUSSIAN_F64, mr.GAUSSIAN_ICDF_F64):
        e = gauss64_errors(got, want, 0.0 if p0 is None else p0, 1.0 if p1 is None else p1)
        bad = np.nonzero(e > 1.0)[0]
        assert bad.size == 0, (f"{bad.size} FP64 Gaussians outside tolerance; first at "
                               f"{bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}")
        return float(e.max()) if e.size else 0.0
    if kind in (mr.GAUSSIAN_F32, mr.GAUSSIAN_ICDF_F32):
        e = gauss_errors(got, want, 0.0 if p0 is None else p0, 1.0 if p1 is None else p1)
        bad = np.nonzero(e > 1.0)[0]
        assert bad.size == 0, (f"{bad.size} Gaussians outside tolerance; first at {bad[:5]}: "
                               f"got {got[bad[:5]]} want {want[bad[:5]]}")
        return float(e.max()) if e.size else 0.0
    if got.dtype.kind == "f":
        same = got.view(np.uint32 if got.dtype == np.float32 else np.uint64) == \
            want.view(np.uint32 if want.dtype == np.float32 else np.uint64)
    else:
        same = got == want
    bad = np.nonzero(~same)[0]
    assert bad.size == 0, (f"{bad.size} mismatches; first at {bad[:5]}: got {got[bad[:5]]} "
                           f"want {want[bad[:5]]}")
    return 0.0
