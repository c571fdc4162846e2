"""CPU oracle for the mirng hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and it shares no code with the library: the definitions live in
``oracle.c`` (plain C, compiled with gcc, no FMA contraction) and are reached
through ctypes here.

Every function states the definition it follows; see ``oracle.c`` for the
sources ([S11] Philox, [L99] MRG32k3a, [L02] substreams, [BM58] Box-Muller)
and for the paper's range transform (arXiv:2109.01329, Sec. 4.3).

Parity status: every function is pinned by tests under ``tests/`` except
the Philox-4x32 multipliers, which are pinned only by the published
definition on the CPU, and additionally by an opaque comparison against an
installed vendor generator where a GPU runtime is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BITS_U32, UNIFORM_F32, UNIFORM_F64, GAUSSIAN_F32, GAUSSIAN_F64 = 1, 2, 3, 4, 5
UNIFORM_I32, GAUSSIAN_ICDF_F32, GAUSSIAN_ICDF_F64 = 6, 7, 8
PHILOX, MRG = 1, 2

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no FMA
    contraction).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off",
            "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        L.orc_philox4x32.argtypes = [_u32p, _u32p, ctypes.c_int, _u32p]
        L.orc_philox4x64.argtypes = [_u64p, _u64p, ctypes.c_int, _u64p]
        L.orc_philox_constants.argtypes = [_u64p]
        L.orc_philox_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                       ctypes.c_uint64, _u32p]
        L.orc_mrg_constants.argtypes = [_u64p]
        L.orc_mrg_seed.argtypes = [ctypes.c_uint64, _u64p]
        L.orc_mrg_step.argtypes = [_u64p]
        L.orc_mrg_step.restype = ctypes.c_uint32
        L.orc_mrg_words.argtypes = [_u64p, ctypes.c_uint64, _u32p]
        L.orc_mrg_skip.argtypes = [_u64p, _u64p]
        L.orc_u01_f32.argtypes = [ctypes.c_uint32]
        L.orc_u01_f32.restype = ctypes.c_float
        L.orc_u01_f64_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_u01_f64_words.restype = ctypes.c_double
        L.orc_u01_f64_mrg.argtypes = [ctypes.c_uint32]
        L.orc_u01_f64_mrg.restype = ctypes.c_double
        L.orc_range_f32.argtypes = [ctypes.c_float, ctypes.c_double, ctypes.c_double]
        L.orc_range_f32.restype = ctypes.c_float
        L.orc_range_f64.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_range_f64.restype = ctypes.c_double
        L.orc_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.orc_box_muller64.argtypes = [ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.orc_gauss64_uniforms.argtypes = [ctypes.c_int, _u32p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        L.orc_uniform_i32.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double]
        L.orc_uniform_i32.restype = ctypes.c_int32
        L.orc_normal_quantile.argtypes = [ctypes.c_double]
        L.orc_normal_quantile.restype = ctypes.c_double
        L.orc_icdf_uniform.argtypes = [ctypes.c_int, ctypes.c_int, _u32p]
        L.orc_icdf_uniform.restype = ctypes.c_double
        L.orc_apply.argtypes = [ctypes.c_int, ctypes.c_int, _u32p, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.orc_words_consumed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        L.orc_words_consumed.restype = ctypes.c_uint64
        L.orc_philox_generate.argtypes = [ctypes.c_uint64, _u64p, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double,
                                          ctypes.c_uint64, _u32p, ctypes.c_void_p]
        L.orc_mrg_generate.argtypes = [_u64p, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, _u32p,
                                       ctypes.c_void_p]
    return _lib


# ---------------------------------------------------------------- helpers

def _limbs(value: int, count: int) -> np.ndarray:
    """Little-endian 64-bit limbs of a non-negative integer."""
    if value < 0:
        raise ValueError("negative")
    arr = np.zeros(count, dtype=np.uint64)
    for i in range(count):
        arr[i] = (value >> (64 * i)) & 0xFFFFFFFFFFFFFFFF
    return arr


def _ptr(a: np.ndarray, typ):
    return a.ctypes.data_as(typ)


OUT_DTYPE = {BITS_U32: np.uint32, UNIFORM_F32: np.float32,
             UNIFORM_F64: np.float64, GAUSSIAN_F32: np.float64, GAUSSIAN_F64: np.float64,
             UNIFORM_I32: np.int32, GAUSSIAN_ICDF_F32: np.float64,
             GAUSSIAN_ICDF_F64: np.float64}

PHILOX_POS_MOD = 1 << 130


# ---------------------------------------------------------------- Philox

def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    """One Philox-4x32 bijection ([S11]); returns 4 uint32 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c, _u32p), _ptr(k, _u32p), rounds, _ptr(out, _u32p))
    return out


def philox4x64(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox-4x64 instance of the same round body (used only to pin it)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(c, _u64p), _ptr(k, _u64p), rounds, _ptr(out, _u64p))
    return out


def philox_constants() -> dict:
    a = np.zeros(8, dtype=np.uint64)
    lib().orc_philox_constants(_ptr(a, _u64p))
    v = [int(x) for x in a]
    return {"M32": (v[0], v[1]), "W32": (v[2], v[3]),
            "M64": (v[4], v[5]), "W64": (v[6], v[7])}


def philox_words(seed: int, pos: int, n: int) -> np.ndarray:
    """Words pos .. pos+n-1 (mod 2^130) of the Philox engine with key
    (lo32(seed), hi32(seed))."""
    p = _limbs(pos % PHILOX_POS_MOD, 3)
    out = np.zeros(n, dtype=np.uint32)
    lib().orc_philox_words(seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF,
                           _ptr(p, _u64p), n, _ptr(out, _u32p))
    return out


def words_consumed(kind: int, engine: int, n: int) -> int:
    return int(lib().orc_words_consumed(kind, 1 if engine == MRG else 0, n))


def apply(kind: int, engine: int, words: np.ndarray, n: int,
          p0: float, p1: float) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.size < words_consumed(kind, engine, n):
        raise ValueError("not enough words")
    out = np.zeros(n, dtype=OUT_DTYPE[kind])
    lib().orc_apply(kind, 1 if engine == MRG else 0, _ptr(w, _u32p), n, p0, p1,
                    out.ctypes.data_as(ctypes.c_void_p))
    return out


def default_params(kind: int):
    if kind == UNIFORM_I32:
        return (0.0, float(2**31))
    return (0.0, 1.0)


def philox_generate(seed: int, pos: int, kind: int, n: int,
                    p0: float | None = None, p1: float | None = None) -> np.ndarray:
    """Plain generate on a Philox engine at word position `pos`.
    Gaussian results are the FP64 transform (z * stddev + mean)."""
    if p0 is None:
        p0, p1 = default_params(kind)
    nw = words_consumed(kind, PHILOX, n)
    scratch = np.zeros(max(nw, 1), dtype=np.uint32)
    out = np.zeros(n, dtype=OUT_DTYPE[kind])
    p = _limbs(pos % PHILOX_POS_MOD, 3)
    lib().orc_philox_generate(seed & 0xFFFFFFFFFFFFFFFF, _ptr(p, _u64p), kind, p0, p1, n,
                              _ptr(scratch, _u32p), out.ctypes.data_as(ctypes.c_void_p))
    return out


# ---------------------------------------------------------------- MRG32k3a

def mrg_constants() -> dict:
    a = np.zeros(6, dtype=np.uint64)
    lib().orc_mrg_constants(_ptr(a, _u64p))
    v = [int(x) for x in a]
    return {"m1": v[0], "m2": v[1], "a12": v[2], "a13": v[3], "a21": v[4], "a23": v[5]}


def mrg_seed(seed: int) -> np.ndarray:
    st = np.zeros(6, dtype=np.uint64)
    lib().orc_mrg_seed(seed & 0xFFFFFFFFFFFFFFFF, _ptr(st, _u64p))
    return st


def mrg_words(state, n: int):
    """Step n times from `state` (6 words); returns (outputs y, new state)."""
    st = np.array(state, dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint32)
    lib().orc_mrg_words(_ptr(st, _u64p), n, _ptr(out, _u32p))
    return out, st


def mrg_skip(state, n: int) -> np.ndarray:
    """State after n steps (0 <= n < 2^192), by the polynomial method."""
    st = np.array(state, dtype=np.uint64)
    lim = _limbs(n, 3)
    lib().orc_mrg_skip(_ptr(st, _u64p), _ptr(lim, _u64p))
    return st


def mrg_generate(state, kind: int, n: int, p0: float | None = None,
                 p1: float | None = None):
    """Plain generate on an MRG32k3a state; returns (outputs, new state)."""
    if p0 is None:
        p0, p1 = default_params(kind)
    st = np.array(state, dtype=np.uint64)
    nw = words_consumed(kind, MRG, n)
    scratch = np.zeros(max(nw, 1), dtype=np.uint32)
    out = np.zeros(n, dtype=OUT_DTYPE[kind])
    lib().orc_mrg_generate(_ptr(st, _u64p), kind, p0, p1, n, _ptr(scratch, _u32p),
                           out.ctypes.data_as(ctypes.c_void_p))
    return out, st


# ---------------------------------------------------------------- distributions

def u01_f32(w: int) -> float:
    return float(lib().orc_u01_f32(w))


def u01_f64_words(w_lo: int, w_hi: int) -> float:
    return float(lib().orc_u01_f64_words(w_lo, w_hi))


def u01_f64_mrg(y: int) -> float:
    return float(lib().orc_u01_f64_mrg(y))


def box_muller(w_a: int, w_b: int):
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().orc_box_muller(w_a, w_b, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def box_muller64(u1: float, u2: float):
    """Gaussian FP64 pair from FP64 uniforms (R21)."""
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().orc_box_muller64(u1, u2, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def gauss64_uniforms(engine: int, words) -> tuple:
    """The (u1, u2) of one Gaussian FP64 pair: four Philox words or two MRG
    outputs (R21)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    u1, u2 = ctypes.c_double(), ctypes.c_double()
    lib().orc_gauss64_uniforms(1 if engine == MRG else 0, _ptr(w, _u32p), ctypes.byref(u1),
                               ctypes.byref(u2))
    return u1.value, u2.value


def box_muller_factors(words: np.ndarray):
    """(r, sin, cos) factors of Box-Muller for each word taken as u1 (r) and
    as u2 (sin, cos); FP64."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    n = w.size
    r = np.zeros(n); s = np.zeros(n); c = np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    L = lib()
    L.orc_box_muller_factors.argtypes = [_u32p, ctypes.c_uint64, dp, dp, dp]
    L.orc_box_muller_factors(_ptr(w, _u32p), n, _ptr(r, dp), _ptr(s, dp), _ptr(c, dp))
    return r, s, c


def uniform_i32(w: int, a: float, b: float) -> int:
    """R23: a + floor(w (b - a) / 2^32) in exact integer arithmetic."""
    return int(lib().orc_uniform_i32(w, a, b))


def normal_quantile(u: float) -> float:
    """R24: the z with Phi(z) = u, by bisection on erf / erfc."""
    return float(lib().orc_normal_quantile(u))


def icdf_uniform(kind: int, engine: int, words) -> float:
    """R24: the uniform in (0, 1) behind one inverse-CDF Gaussian output."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    return float(lib().orc_icdf_uniform(kind, 1 if engine == MRG else 0, _ptr(w, _u32p)))
