"""Seeded synthetic workload descriptions shared by tests, bench and oracle
checks.  Holds none of the generators' arithmetic: only the sizes, seeds,
offsets and request mixes, drawn from numpy's default_rng with fixed
meta-seeds (1329 + k for workload k).

Shapes follow the paper's two workloads (arXiv:2109.01329):
  * the RNG burner: Philox4x32x10 uniform FP32 batches of 1 .. 10^8
    (Sec. 5.1 and Sec. 7);
  * FastCaloSim: three uniforms per calorimeter hit, hits per event ranging
    from a few to O(10^4) secondaries (Sec. 5.2) -- here a lognormal hit
    count per event plus one Gaussian per hit.
"""
from __future__ import annotations

import dataclasses

import numpy as np

META_SEED = 1329

PHILOX, MRG = 1, 2
BITS_U32, UNIFORM_F32, UNIFORM_F64, GAUSSIAN_F32, GAUSSIAN_F64 = 1, 2, 3, 4, 5
UNIFORM_I32, GAUSSIAN_ICDF_F32, GAUSSIAN_ICDF_F64 = 6, 7, 8
KINDS = (UNIFORM_F32, UNIFORM_F64, GAUSSIAN_F32, BITS_U32)
EXTRA_KINDS = (GAUSSIAN_F64, UNIFORM_I32, GAUSSIAN_ICDF_F32, GAUSSIAN_ICDF_F64)
ENGINES = (PHILOX, MRG)
KIND_NAME = {BITS_U32: "bits_u32", UNIFORM_F32: "uniform_f32",
             UNIFORM_F64: "uniform_f64", GAUSSIAN_F32: "gaussian_f32",
             GAUSSIAN_F64: "gaussian_f64", UNIFORM_I32: "uniform_i32",
             GAUSSIAN_ICDF_F32: "gaussian_icdf_f32", GAUSSIAN_ICDF_F64: "gaussian_icdf_f64"}
ENGINE_NAME = {PHILOX: "philox4x32_10", MRG: "mrg32k3a"}
ELEM_BYTES = {BITS_U32: 4, UNIFORM_F32: 4, UNIFORM_F64: 8, GAUSSIAN_F32: 4, GAUSSIAN_F64: 8,
              UNIFORM_I32: 4, GAUSSIAN_ICDF_F32: 4, GAUSSIAN_ICDF_F64: 8}


def rng(k: int) -> np.random.Generator:
    return np.random.default_rng(META_SEED + k)


# --- small single-engine case: Philox, seed 42, offset 0, n = 2^20 -------
SMALL = dict(engine=PHILOX, seed=42, offset=0, n=1 << 20)


# --- plain bulk case: both engines x four outputs, n = 2^28 --------------
BULK_N = 1 << 28


def bulk_draws(count: int = 3):
    """(engine, kind, seed, offset) cells of the bulk case: seeds uniform in
    [0, 2^64), offsets uniform in [0, 2^40); `count` draws per cell."""
    g = rng(2)
    cells = []
    for engine in ENGINES:
        for kind in KINDS:
            for _ in range(count):
                seed = int(g.integers(0, 2**64, dtype=np.uint64))
                offset = int(g.integers(0, 2**40, dtype=np.uint64))
                cells.append((engine, kind, seed, offset))
    return cells


def extra_draws():
    """(engine, kind, seed, offset) cells of the kinds outside the bulk mix
    (Gaussian FP64, uniform int32, inverse-CDF Gaussians), one per engine
    and kind, drawn like the bulk cells (meta-seed 6 for Gaussian FP64,
    8 for the others)."""
    cells = []
    for k, kinds in ((6, (GAUSSIAN_F64,)), (8, EXTRA_KINDS[1:])):
        g = rng(k)
        for kind in kinds:
            for engine in ENGINES:
                seed = int(g.integers(0, 2**64, dtype=np.uint64))
                offset = int(g.integers(0, 2**40, dtype=np.uint64))
                cells.append((engine, kind, seed, offset))
    return cells


# --- MRG32k3a substreams: 65536 x 4096 uniform FP64 ----------------------
SUBSTREAMS = dict(count=65536, per_stream=4096,
                  check_streams=(0, 1, 2, 3, 4095, 32768, 65534, 65535),
                  check_len=1024)


def substream_seed() -> int:
    return int(rng(3).integers(0, 2**64, dtype=np.uint64))


# --- batched calorimeter-shaped events ----------------------------------
@dataclasses.dataclass
class EventBatch:
    hits: np.ndarray          # hits per event (int64)
    seed32: int = 42          # low key word shared by all events

    @property
    def n_events(self) -> int:
        return int(self.hits.size)

    @property
    def total_samples(self) -> int:
        return int(4 * self.hits.sum())


def calo_events(n_events: int = 20000, median: float = 2000.0,
                sigma: float = 1.0, k: int = 4) -> EventBatch:
    """Hits per event h = max(1, round(exp(ln(median) + sigma N(0,1))))."""
    g = rng(k)
    z = g.standard_normal(n_events)
    h = np.maximum(1, np.rint(np.exp(np.log(median) + sigma * z))).astype(np.int64)
    return EventBatch(hits=h)


# --- FastCaloSim-shaped scenarios (Sec. 5.2 of the paper) ------------------
@dataclasses.dataclass
class CaloScenario:
    name: str
    hits: np.ndarray          # hits per event
    seed32: int = 42
    min_per_event: int = 0    # least uniforms an event draws (the paper's 200,000 variant)
    layout: str = "aos"       # "aos": one request per event, a hit's 3 uniforms adjacent;
                              # "soa": one request per event and quantity, 3 arrays

    @property
    def n_events(self) -> int:
        return int(self.hits.size)

    @property
    def uniforms(self) -> np.ndarray:
        """Uniforms per event: three per hit, at least min_per_event."""
        return np.maximum(3 * self.hits, self.min_per_event)

    def requests(self):
        """One Philox uniform FP32 request per row, on the event's key
        (event << 32) | seed32: (seed, offset in words, n, first output
        element).  AoS: one request per event at offset 0, outputs
        contiguous per event.  SoA: quantity q of event e is h_e outputs at
        offset q h_e, stored in array q (elements [q H, (q + 1) H), H the
        total hits) at that event's place among the events."""
        e = np.arange(self.n_events, dtype=np.uint64)
        seeds = (e << np.uint64(32)) | np.uint64(self.seed32)
        if self.layout == "aos":
            n = self.uniforms.astype(np.uint64)
            first = np.concatenate([[0], np.cumsum(n)])[:-1].astype(np.uint64)
            return seeds, np.zeros_like(n), n, first
        h = self.hits.astype(np.uint64)
        total = np.uint64(h.sum())
        place = np.concatenate([[0], np.cumsum(h)])[:-1].astype(np.uint64)
        rows = [(seeds, np.uint64(q) * h, h, np.uint64(q) * total + place) for q in range(3)]
        return tuple(np.stack([r[i] for r in rows], axis=1).reshape(-1) for i in range(4))


SCENARIOS = ("single_electron", "ttbar", "single_electron_min200k", "single_electron_soa")


def calo_scenario(name: str, n_events: int | None = None, k: int = 7) -> CaloScenario:
    """Single-electron events: 4000-6500 hits each (10^4 events, as in the
    paper's results); ttbar events: 600-800 times as many hits (500
    events).  Hit counts uniform over those ranges.  Variants of the
    single-electron shape: every event draws at least 200,000 uniforms
    (the paper's stated minimum), or the three quantities of a hit go to
    three separate arrays (SoA)."""
    g = rng(k)
    if name.startswith("single_electron"):
        n = 10000 if n_events is None else n_events
        hits = g.integers(4000, 6501, n)
    elif name == "ttbar":
        n = 500 if n_events is None else n_events
        hits = (g.integers(4000, 6501, n) * g.uniform(600.0, 800.0, n)).astype(np.int64)
    else:
        raise ValueError(name)
    sc = CaloScenario(name, hits.astype(np.int64))
    if name == "single_electron_min200k":
        sc.min_per_event = 200000
    elif name == "single_electron_soa":
        sc.layout = "soa"
    elif name != "single_electron" and name != "ttbar":
        raise ValueError(name)
    return sc


# --- served request trace ------------------------------------------------
@dataclasses.dataclass
class Trace:
    arrival_s: np.ndarray     # scheduled arrival times (seconds, from 0)
    n: np.ndarray             # samples per request
    engine: np.ndarray        # PHILOX / MRG
    kind: np.ndarray          # distribution kind
    seed: np.ndarray          # uint64
    offset: np.ndarray        # uint64 in [0, 2^40)


def request_trace(rate_per_s: float, count: int, k: int = 5,
                  log10_min: float = 3.0, log10_max: float = 8.0) -> Trace:
    """Open-loop Poisson arrivals at `rate_per_s`; sizes floor(10^U(a,b));
    engine and distribution uniform over the 2 x 4 mix."""
    g = rng(k)
    gaps = g.exponential(1.0 / rate_per_s, count)
    arrival = np.cumsum(gaps) - gaps[0]
    n = np.floor(10.0 ** g.uniform(log10_min, log10_max, count)).astype(np.int64)
    engine = g.choice(np.array(ENGINES), count)
    kind = g.choice(np.array(KINDS), count)
    seed = g.integers(0, 2**64, count, dtype=np.uint64)
    offset = g.integers(0, 2**40, count, dtype=np.uint64)
    return Trace(arrival, n, engine, kind, seed, offset)
