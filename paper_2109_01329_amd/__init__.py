"""mirng: bulk Philox4x32-10 / MRG32k3a generation on one MI355X (gfx950).

Python binding of libmirng.so (C ABI in include/mirng.h).  This module only
marshals arguments: every step of generation runs in the library's HIP
kernels.  PyTorch is used, when given, only for device memory (tensor data
pointers) and streams.  If the shared library is missing the import of the
binding fails loudly; there is no fallback implementation.

Build the library with ``python -m paper_2109_01329_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmirng.so")

PHILOX4X32_10, MRG32K3A = 1, 2
BITS_U32, UNIFORM_F32, UNIFORM_F64, GAUSSIAN_F32, GAUSSIAN_F64 = 1, 2, 3, 4, 5
UNIFORM_I32, GAUSSIAN_ICDF_F32, GAUSSIAN_ICDF_F64 = 6, 7, 8

STATUS = {0: "MIRNG_OK", 1: "MIRNG_E_INVALID_ARG", 2: "MIRNG_E_UNSUPPORTED",
          3: "MIRNG_E_ALLOC", 4: "MIRNG_E_LAUNCH", 5: "MIRNG_E_DEVICE",
          6: "MIRNG_E_CAPACITY"}

ELEM_BYTES = {BITS_U32: 4, UNIFORM_F32: 4, UNIFORM_F64: 8, GAUSSIAN_F32: 4, GAUSSIAN_F64: 8,
              UNIFORM_I32: 4, GAUSSIAN_ICDF_F32: 4, GAUSSIAN_ICDF_F64: 8}


class MirngError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class Distribution(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("p0", ctypes.c_double), ("p1", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [("engine_type", ctypes.c_int32), ("words", ctypes.c_uint32 * 6),
                ("reserved", ctypes.c_uint32), ("pos", ctypes.c_uint64 * 3)]


class Request(ctypes.Structure):
    _fields_ = [("engine_type", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("dist", Distribution), ("seed", ctypes.c_uint64),
                ("offset", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("out", ctypes.c_void_p)]


class PhiloxConfig(ctypes.Structure):
    _fields_ = [("walk", ctypes.c_int32), ("block", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("blocks_per_lane", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class BatchConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("max_engines", ctypes.c_int32),
                ("capacity_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("refused", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("samples", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("max_inflight_bytes", ctypes.c_uint64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("span_s", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: (float(getattr(self, f)) if t is ctypes.c_double else int(getattr(self, f)))
                for f, t in self._fields_}


# numpy view of mirng_request (64 bytes, same field order and offsets)
REQUEST_FIELDS = [("engine_type", "<i4"), ("reserved", "<i4"), ("kind", "<i4"),
                  ("dist_reserved", "<i4"), ("p0", "<f8"), ("p1", "<f8"), ("seed", "<u8"),
                  ("offset", "<u8"), ("n", "<u8"), ("out", "<u8")]


def request_dtype():
    import numpy as np
    dt = np.dtype(REQUEST_FIELDS)
    assert dt.itemsize == ctypes.sizeof(Request) == 64
    return dt


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmirng.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_2109_01329_amd.build`")
    # Streams and device buffers come from PyTorch, which ships its own HIP
    # runtime: load it first so that libmirng.so binds to that same runtime
    # (two runtimes in one process do not share streams or allocations).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    E = ctypes.c_void_p
    vp = ctypes.c_void_p
    u64 = ctypes.c_uint64
    sig = {
        "mirng_engine_create": ([ctypes.c_int32, u64, u64, ctypes.POINTER(E)], ctypes.c_int),
        "mirng_engine_destroy": ([E], ctypes.c_int),
        "mirng_skip_ahead": ([E, u64], ctypes.c_int),
        "mirng_skip_ahead_multi": ([E, ctypes.POINTER(u64), ctypes.c_size_t], ctypes.c_int),
        "mirng_engine_get_state": ([E, ctypes.POINTER(State)], ctypes.c_int),
        "mirng_engine_set_state": ([E, ctypes.POINTER(State)], ctypes.c_int),
        "mirng_generate": ([E, ctypes.POINTER(Distribution), u64, vp, vp], ctypes.c_int),
        "mirng_generate_substreams": ([E, ctypes.POINTER(Distribution), u64, u64, u64, vp, vp],
                                      ctypes.c_int),
        "mirng_generate_streams": ([E, ctypes.POINTER(Distribution), u64, u64, u64, vp, vp],
                                   ctypes.c_int),
        "mirng_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "mirng_philox_config_get": ([ctypes.POINTER(PhiloxConfig)], ctypes.c_int),
        "mirng_philox_config_set": ([ctypes.POINTER(PhiloxConfig)], ctypes.c_int),
        "mirng_philox_config_get_kind": ([ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(PhiloxConfig)], ctypes.c_int),
        "mirng_philox_config_set_kind": ([ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(PhiloxConfig)], ctypes.c_int),
        "mirng_philox_phase": ([ctypes.c_int32, u64, vp], ctypes.c_uint32),
        "mirng_philox_candidates": ([ctypes.POINTER(PhiloxConfig), ctypes.c_int32],
                                    ctypes.c_int32),
        "mirng_abi_version": ([], ctypes.c_int32),
        "mirng_device_init": ([], ctypes.c_int),
        "mirng_batcher_create": ([ctypes.POINTER(vp)], ctypes.c_int),
        "mirng_batcher_destroy": ([vp], ctypes.c_int),
        "mirng_batcher_stage": ([vp, ctypes.c_size_t, ctypes.POINTER(vp)], ctypes.c_int),
        "mirng_generate_batch": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "mirng_batcher_statuses": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "mirng_generate_batch_noalloc": ([vp, ctypes.c_size_t, vp, ctypes.POINTER(BatchConfig),
                                          vp], ctypes.c_int),
        "mirng_batcher_config_get": ([vp, ctypes.POINTER(BatchConfig)], ctypes.c_int),
        "mirng_batcher_config_set": ([vp, ctypes.POINTER(BatchConfig)], ctypes.c_int),
        "mirng_words_consumed": ([ctypes.c_int32, ctypes.c_int32, u64], u64),
        "mirng_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)], ctypes.c_int),
        "mirng_server_destroy": ([vp], ctypes.c_int),
        "mirng_server_submit": ([vp, vp, ctypes.POINTER(u64)], ctypes.c_int),
        "mirng_server_poll": ([vp, u64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "mirng_server_wait": ([vp, u64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "mirng_server_drain": ([vp], ctypes.c_int),
        "mirng_server_stats_get": ([vp, ctypes.POINTER(ServerStats)], ctypes.c_int),
        "mirng_bench_server_replay": ([vp, vp, vp, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
        "mirng_server_engine_create": ([vp, ctypes.c_int32, u64, u64,
                                        ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
        "mirng_server_submit_engine": ([vp, ctypes.c_uint32, ctypes.POINTER(Distribution), u64,
                                        vp, ctypes.POINTER(u64)], ctypes.c_int),
        "mirng_server_engine_skip_ahead": ([vp, ctypes.c_uint32, ctypes.POINTER(u64),
                                            ctypes.c_size_t], ctypes.c_int),
        "mirng_server_engine_get_state": ([vp, ctypes.c_uint32, ctypes.POINTER(State)],
                                          ctypes.c_int),
        "mirng_server_engine_set_state": ([vp, ctypes.c_uint32, ctypes.POINTER(State)],
                                          ctypes.c_int),
        "mirng_autotune_philox": ([ctypes.c_int32, u64, u64, vp, vp, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PhiloxConfig),
                                   ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "mirng_autotune_batch": ([vp, vp, ctypes.c_size_t, vp, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.POINTER(BatchConfig),
                                  ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "mirng_bench_store": ([vp, u64, ctypes.c_int32, vp], ctypes.c_int),
        "mirng_bench_philox_nostore": ([u64, ctypes.c_uint32, ctypes.c_uint32, vp, vp],
                                       ctypes.c_int),
        "mirng_bench_valu": ([ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, vp, vp],
                             ctypes.c_int),
        "mirng_bench_transform_f32": ([ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, vp, vp],
                                      ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int, where: str) -> None:
    if status != 0:
        raise MirngError(status, where)


def _limbs(n: int):
    if n < 0 or n >= 1 << 192:
        raise ValueError("count must be in [0, 2^192)")
    return (ctypes.c_uint64 * 3)(*[(n >> (64 * i)) & (2**64 - 1) for i in range(3)])


def _ptr(out) -> int:
    """Device pointer of a torch tensor, or an int taken as a pointer."""
    if out is None:
        return 0
    if isinstance(out, int):
        return out
    return int(out.data_ptr())


def _stream(stream) -> int:
    """hipStream_t of a torch stream (current stream when None), or an int."""
    if isinstance(stream, int):
        return stream
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def device_init() -> None:
    """Set up the current device (resident tables) ahead of the first call."""
    _check(lib().mirng_device_init(), "device_init")


def words_consumed(engine_type: int, kind: int, n: int) -> int:
    return int(lib().mirng_words_consumed(engine_type, kind, n))


def default_params(kind: int) -> tuple:
    """Parameters used when none are given: (0, 1) (the unit range, or mean
    0 and stddev 1), and [0, 2^31) for uniform int32."""
    return (0.0, float(2**31)) if kind == UNIFORM_I32 else (0.0, 1.0)


def distribution(kind: int, p0: float | None = None, p1: float | None = None) -> Distribution:
    d0, d1 = default_params(kind)
    if p0 is None:
        p0 = d0
    if p1 is None:
        p1 = d1
    return Distribution(kind, 0, float(p0), float(p1))


class Engine:
    """An engine (Philox4x32-10 or MRG32k3a) at a position in its stream."""

    def __init__(self, engine_type: int, seed: int, offset: int = 0):
        if not 0 <= offset < 2**64:
            raise ValueError("offset must lie in [0, 2^64); reach larger positions with "
                             "skip_ahead")
        h = ctypes.c_void_p()
        _check(lib().mirng_engine_create(engine_type, seed & (2**64 - 1), offset,
                                         ctypes.byref(h)), "engine_create")
        self._h = h
        self.engine_type = engine_type

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mirng_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def skip_ahead(self, n: int) -> None:
        if n < 2**64:
            _check(lib().mirng_skip_ahead(self._h, n), "skip_ahead")
        else:
            _check(lib().mirng_skip_ahead_multi(self._h, _limbs(n), 3), "skip_ahead_multi")

    def get_state(self) -> State:
        s = State()
        _check(lib().mirng_engine_get_state(self._h, ctypes.byref(s)), "get_state")
        return s

    def set_state(self, s: State) -> None:
        _check(lib().mirng_engine_set_state(self._h, ctypes.byref(s)), "set_state")

    @property
    def position(self) -> int:
        s = self.get_state()
        return s.pos[0] | (s.pos[1] << 64) | (s.pos[2] << 128)

    def generate(self, kind: int, n: int, out, p0: float | None = None,
                 p1: float | None = None, stream=None) -> None:
        """Enqueue n outputs of `kind` into `out` (torch CUDA tensor or device
        pointer) on `stream`; asynchronous."""
        d = distribution(kind, p0, p1)
        _check(lib().mirng_generate(self._h, ctypes.byref(d), n, _ptr(out), _stream(stream)),
               "generate")

    def generate_substreams(self, kind: int, first: int, count: int, n_each: int, out,
                            p0: float | None = None, p1: float | None = None,
                            stream=None) -> None:
        d = distribution(kind, p0, p1)
        _check(lib().mirng_generate_substreams(self._h, ctypes.byref(d), first, count, n_each,
                                               _ptr(out), _stream(stream)),
               "generate_substreams")

    def generate_streams(self, kind: int, first: int, count: int, n_each: int, out,
                         p0: float | None = None, p1: float | None = None,
                         stream=None) -> None:
        """As generate_substreams with streams 2^127 steps apart."""
        d = distribution(kind, p0, p1)
        _check(lib().mirng_generate_streams(self._h, ctypes.byref(d), first, count, n_each,
                                            _ptr(out), _stream(stream)),
               "generate_streams")


def philox_phase(kind: int, position: int, out) -> int:
    """Phase (0..3) of a Philox launch of `kind` at word `position` into
    `out`: the position of its first 16-byte slot modulo 4."""
    return int(lib().mirng_philox_phase(kind, position % 2**64, _ptr(out)))


def philox_config(kind: int | None = None, phase: int = 1) -> PhiloxConfig:
    """The process-wide launch shape, or (with `kind`) the shape Philox
    generate calls of that distribution use at `phase`."""
    c = PhiloxConfig()
    if kind is None:
        _check(lib().mirng_philox_config_get(ctypes.byref(c)), "philox_config_get")
    else:
        _check(lib().mirng_philox_config_get_kind(kind, phase, ctypes.byref(c)),
               "philox_config_get_kind")
    return c


def set_philox_config(c: PhiloxConfig | None = None, kind: int | None = None,
                      phase: int = -1, **fields) -> PhiloxConfig:
    """Install a launch shape (fields not given keep their current value);
    returns the previous one.  Without `kind` it is the process-wide shape
    and every kind's own shape is dropped; with `kind`, that kind's own at
    `phase` (0..3) or at every phase (-1)."""
    prev = philox_config(kind, phase if phase >= 0 else 1)
    new = PhiloxConfig.from_buffer_copy(c if c is not None else prev)
    for k, v in fields.items():
        setattr(new, k, int(v))
    if kind is None:
        _check(lib().mirng_philox_config_set(ctypes.byref(new)), "philox_config_set")
    else:
        _check(lib().mirng_philox_config_set_kind(kind, phase, ctypes.byref(new)),
               "philox_config_set_kind")
    return prev


def philox_candidates() -> list:
    """The launch shapes the Philox autotuner times, in its order."""
    total = int(lib().mirng_philox_candidates(None, 0))
    arr = (PhiloxConfig * total)()
    lib().mirng_philox_candidates(arr, total)
    return [PhiloxConfig.from_buffer_copy(c) for c in arr]


def clear_philox_config(kind: int, phase: int = -1) -> None:
    """Drop `kind`'s own launch shape at `phase` (every phase for -1): it
    follows the process-wide one there."""
    _check(lib().mirng_philox_config_set_kind(kind, phase, None), "philox_config_set_kind")


class TuningCache:
    """Tuned launch shapes in a JSON file, keyed by GPU architecture, engine,
    distribution and size class (the bit length of the output count), so
    that a process can reuse a shape timed earlier instead of re-timing."""

    def __init__(self, path: str):
        import json
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key: str):
        return self.entries.get(key)

    def put(self, key: str, value: dict) -> None:
        import json
        self.entries[key] = value
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def size_class(n: int) -> int:
    return int(n).bit_length()


def autotune_philox(kind: int, n: int, out, stream=None, prewarm_ms: int = 300,
                    rounds: int = 5, reps: int = 10, cache: TuningCache | None = None,
                    offset: int = 1):
    """Time the candidate Philox launch shapes on `n` outputs of `kind` into
    `out` (overwritten) from engine word position `offset`, install the
    fastest as `kind`'s own shape at the phase of that position and output
    (philox_phase) and return (shape, ms).  With a cache, a shape stored for
    the same architecture, kind, phase and size class is installed without
    timing, and a newly timed one is stored."""
    phase = philox_phase(kind, offset, out)
    key = (f"{_arch()}/philox4x32_10/{kind}/phase{phase}/{size_class(n)}"
           if cache is not None else None)
    if key is not None and cache.get(key) is not None:
        hit = cache.get(key)
        set_philox_config(kind=kind, phase=phase, **hit["config"])
        return philox_config(kind, phase), float(hit["ms"])
    c = PhiloxConfig()
    ms = ctypes.c_float()
    _check(lib().mirng_autotune_philox(kind, offset % 2**64, n, _ptr(out), _stream(stream),
                                       prewarm_ms, rounds, reps, ctypes.byref(c),
                                       ctypes.byref(ms)), "autotune_philox")
    if key is not None:
        cache.put(key, {"config": c.as_dict(), "ms": float(ms.value)})
    return c, float(ms.value)


class Batcher:
    """Batched generation of many independent requests in one launch.

    Requests are numpy records of `request_dtype()` (field `out` is a device
    pointer).  `stage(count)` returns a record array in pinned host memory
    that `generate` sends without a host copy."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().mirng_batcher_create(ctypes.byref(h)), "batcher_create")
        self._h = h
        self._staged = None

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mirng_batcher_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self) -> BatchConfig:
        c = BatchConfig()
        _check(lib().mirng_batcher_config_get(self._h, ctypes.byref(c)), "batcher_config_get")
        return c

    def set_config(self, c: BatchConfig | None = None, **fields) -> BatchConfig:
        prev = self.config
        new = BatchConfig.from_buffer_copy(c if c is not None else prev)
        for k, v in fields.items():
            setattr(new, k, int(v))
        _check(lib().mirng_batcher_config_set(self._h, ctypes.byref(new)), "batcher_config_set")
        return prev

    def stage(self, count: int):
        import numpy as np
        ptr = ctypes.c_void_p()
        _check(lib().mirng_batcher_stage(self._h, count, ctypes.byref(ptr)), "batcher_stage")
        buf = (ctypes.c_char * (64 * max(count, 1))).from_address(ptr.value)
        arr = np.frombuffer(buf, dtype=request_dtype(), count=count)
        self._staged = arr
        return arr

    def generate(self, reqs, stream=None) -> None:
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=request_dtype())
        _check(lib().mirng_generate_batch(self._h, reqs.ctypes.data, len(reqs), _stream(stream)),
               "generate_batch")

    def autotune(self, reqs, stream=None, prewarm_ms: int = 300, rounds: int = 5,
                 reps: int = 10, cache: TuningCache | None = None):
        """Time the candidate batch launch shapes on this batch (its outputs
        are overwritten), install the fastest and return (shape, ms).  With a
        cache, keyed by architecture and the size classes of the request
        count and of the total output count."""
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=request_dtype())
        key = None
        if cache is not None:
            key = (f"{_arch()}/batch/{size_class(len(reqs))}/"
                   f"{size_class(int(reqs['n'].sum()))}")
            hit = cache.get(key)
            if hit is not None:
                self.set_config(**hit["config"])
                return self.config, float(hit["ms"])
        c = BatchConfig()
        ms = ctypes.c_float()
        _check(lib().mirng_autotune_batch(self._h, reqs.ctypes.data, len(reqs), _stream(stream),
                                          prewarm_ms, rounds, reps, ctypes.byref(c),
                                          ctypes.byref(ms)), "autotune_batch")
        if key is not None:
            cache.put(key, {"config": c.as_dict(), "ms": float(ms.value)})
        return c, float(ms.value)

    def statuses(self, count: int):
        import numpy as np
        out = np.zeros(count, dtype=np.int32)
        _check(lib().mirng_batcher_statuses(self._h, out.ctypes.data, count), "batcher_statuses")
        return out


class Server:
    """Serving loop: requests are submitted one at a time and completed
    asynchronously by continuous batching over `streams` HIP streams, with
    at most `capacity_bytes` of admitted, unfinished output."""

    def __init__(self, streams: int = 2, capacity_bytes: int = 32 * 10**9,
                 max_batch: int = 65536, max_engines: int = 0):
        cfg = ServerConfig(streams, max_engines, capacity_bytes, max_batch)
        h = ctypes.c_void_p()
        _check(lib().mirng_server_create(ctypes.byref(cfg), ctypes.byref(h)), "server_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mirng_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req) -> int:
        """Queue one request (a record of `request_dtype()`); returns its ticket."""
        import numpy as np
        r = np.ascontiguousarray(np.asarray(req, dtype=request_dtype()).reshape(1))
        t = ctypes.c_uint64()
        _check(lib().mirng_server_submit(self._h, r.ctypes.data, ctypes.byref(t)), "server_submit")
        return int(t.value)

    def engine_create(self, engine_type: int, seed: int, offset: int = 0) -> int:
        """A resident engine in the server's device table; returns its index."""
        e = ctypes.c_uint32()
        _check(lib().mirng_server_engine_create(self._h, engine_type, seed & (2**64 - 1), offset,
                                                ctypes.byref(e)), "server_engine_create")
        return int(e.value)

    def submit_engine(self, engine: int, kind: int, n: int, out, p0: float | None = None,
                      p1: float | None = None) -> int:
        """Queue n outputs of `kind` on resident engine `engine`, continuing
        it; returns the ticket."""
        d = distribution(kind, p0, p1)
        t = ctypes.c_uint64()
        _check(lib().mirng_server_submit_engine(self._h, engine, ctypes.byref(d), n, _ptr(out),
                                                ctypes.byref(t)), "server_submit_engine")
        return int(t.value)

    def engine_skip_ahead(self, engine: int, n: int) -> None:
        _check(lib().mirng_server_engine_skip_ahead(self._h, engine, _limbs(n), 3),
               "server_engine_skip_ahead")

    def engine_state(self, engine: int) -> State:
        st = State()
        _check(lib().mirng_server_engine_get_state(self._h, engine, ctypes.byref(st)),
               "server_engine_get_state")
        return st

    def engine_set_state(self, engine: int, st: State) -> None:
        _check(lib().mirng_server_engine_set_state(self._h, engine, ctypes.byref(st)),
               "server_engine_set_state")

    def poll(self, ticket: int):
        """(done, status) of a ticket, without blocking."""
        d, s = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().mirng_server_poll(self._h, ticket, ctypes.byref(d), ctypes.byref(s)),
               "server_poll")
        return bool(d.value), int(s.value)

    def wait(self, ticket: int):
        """Block until the ticket completes; returns (status, latency_ms)."""
        s, lat = ctypes.c_int32(), ctypes.c_double()
        _check(lib().mirng_server_wait(self._h, ticket, ctypes.byref(s), ctypes.byref(lat)),
               "server_wait")
        return int(s.value), float(lat.value)

    def drain(self) -> None:
        _check(lib().mirng_server_drain(self._h), "server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().mirng_server_stats_get(self._h, ctypes.byref(st)), "server_stats")
        return st.as_dict()

    def replay(self, reqs, arrival_s, engines=None):
        """Submit reqs[i] at arrival_s[i] seconds from now (native open-loop
        load generator), on resident engine engines[i] when `engines` is
        given; returns (tickets, submission statuses)."""
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=request_dtype())
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        assert len(arr) == len(reqs)
        eng = None
        if engines is not None:
            eng = np.ascontiguousarray(engines, dtype=np.uint32)
            assert len(eng) == len(reqs)
        tickets = np.zeros(len(reqs), dtype=np.uint64)
        st = np.zeros(len(reqs), dtype=np.int32)
        _check(lib().mirng_bench_server_replay(self._h, reqs.ctypes.data,
                                               None if eng is None else eng.ctypes.data,
                                               arr.ctypes.data, len(reqs), tickets.ctypes.data,
                                               st.ctypes.data), "server_replay")
        return tickets, st


# Limits of the allocation-free batch (the C header's MIRNG_NOALLOC_* values).
NOALLOC_MAX_REQUESTS = 16384
NOALLOC_MAX_WAVES = 65536


def generate_batch_noalloc(reqs, statuses, config: BatchConfig | None = None,
                           stream=None) -> None:
    """Batched generation through the allocation-free entry point: `reqs`
    is a host record array of `request_dtype()`, `statuses` a device int32
    buffer of len(reqs) that receives each request's status on `stream`."""
    import numpy as np
    reqs = np.ascontiguousarray(reqs, dtype=request_dtype())
    cfg = ctypes.byref(config) if config is not None else None
    _check(lib().mirng_generate_batch_noalloc(reqs.ctypes.data, len(reqs), _ptr(statuses), cfg,
                                              _stream(stream)), "generate_batch_noalloc")


def make_requests(count: int):
    """Zeroed request records (engine, distribution defaults left to fill)."""
    import numpy as np
    return np.zeros(count, dtype=request_dtype())


# ------------------------------------------------------------ measurement

def bench_store(out, nbytes: int, nontemporal: bool = True, stream=None) -> None:
    _check(lib().mirng_bench_store(_ptr(out), nbytes, 1 if nontemporal else 0,
                                   _stream(stream)), "bench_store")


def bench_philox_nostore(nblocks: int, sink, k0: int = 1, k1: int = 2, stream=None) -> None:
    _check(lib().mirng_bench_philox_nostore(nblocks, k0, k1, _ptr(sink), _stream(stream)),
           "bench_philox_nostore")


def bench_valu(op: int, threads: int, iters: int, sink, stream=None) -> None:
    _check(lib().mirng_bench_valu(op, threads, iters, _ptr(sink), _stream(stream)),
           "bench_valu")


def bench_transform_f32(which: int, first: int, n: int, out, stream=None) -> None:
    """Test-only FP32 transform pieces on the 24-bit inputs first .. first + n - 1
    (0: Box-Muller radius, 1: (cos, sin) pairs, 2: inverse-CDF Gaussian)."""
    _check(lib().mirng_bench_transform_f32(which, first, n, _ptr(out), _stream(stream)),
           "bench_transform_f32")
