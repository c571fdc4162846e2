// Batched generation: many independent requests of uneven sizes in two
// persistent launches, one for Philox4x32-10 and one for MRG32k3a requests
// (the inter-event batching the paper defers for its calorimeter
// application, arXiv:2109.01329 Sec. 7).
//
// plan:  one thread per request validates it (the ABI's rules), derives
//        its Philox slot run (as the plain path does on the host) or its
//        MRG32k3a start state (seed state jumped by the offset through the
//        A^(2^k) table), and counts its Philox tiles of 64 slots or MRG
//        chunks; each workgroup scans both counts over its 1024 requests.
// scan:  one workgroup scans the per-chunk totals (only for batches of more
//        than 64 chunks; smaller ones are scanned by every generating wave in
//        registers).
// start: one thread per Philox wave finds the request holding the wave's
//        first tile (a table read by the generating waves).
// philox main: a fixed grid of waves; wave w takes a contiguous range of
//        tiles (tiles of one request are adjacent, requests in table order),
//        reads the request holding its first tile from the start table and
//        walks forward, running the plain kernel's slot walk on each request
//        segment.
// mrg main: a fixed grid of 256-thread groups, each over a contiguous range
//        of chunks found the same way, running the plain kernel's LDS passes
//        on each chunk.
// Every value depends only on its request and position, never on the
// tiling, the grid or the neighbouring requests.
#include "internal.hpp"
#include "mrg.hpp"
#include "philox.hpp"
#include "transforms.hpp"

namespace mirng {
namespace {

constexpr uint32_t kChunk = 1024;

// p <- (p + n) mod 2^130 over little-endian 64-bit limbs.
__device__ __forceinline__ void add130(uint64_t p[3], const uint64_t n[3])
{
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint64_t s1 = p[i] + n[i];
        const uint64_t c1 = s1 < n[i] ? 1u : 0u;
        const uint64_t s2 = s1 + carry;
        carry = c1 | (s2 < carry ? 1u : 0u);
        p[i] = s2;
    }
    p[2] &= 3u;
}

// MRG32k3a state v <- A^n v for an n of `limbs` 64-bit limbs, through the
// resident A^(2^k) table.
__device__ __forceinline__ void mrg_jump_limbs(uint32_t v[6], const uint64_t *n, int limbs,
                                               const uint32_t *pow2)
{
    for (int l = 0; l < limbs; ++l)
        for (int k = 0; k < 64; ++k)
            if ((n[l] >> k) & 1u) apply_mat(pow2 + (64 * l + k) * kMatWords, v);
}

// Validation and planning of one request: its Philox tiles or MRG chunks.
// The start is (seed, offset) of the request, or, when `ref` names a
// resident engine, entry ref.slot of the device engine table advanced by
// ref.skip words (Philox, modulo 2^130) or steps (MRG, a 192-bit jump).
__device__ void plan_one(const mirng_request &q, const EngineRef &ref,
                         const mirng_state *engines, BatchDesc &d, int32_t &st, int nt,
                         const uint32_t *pow2, uint64_t &tiles, uint64_t &mchunks)
{
    st = MIRNG_OK;
    tiles = 0;
    mchunks = 0;
    d = BatchDesc{};
    d.engine = (uint32_t)q.engine_type;
    if (q.engine_type != MIRNG_PHILOX4X32_10 && q.engine_type != MIRNG_MRG32K3A) {
        st = MIRNG_E_UNSUPPORTED;
        return;
    }
    const int kind = q.dist.kind;
    if (q.reserved != 0 || q.dist.reserved != 0) { st = MIRNG_E_INVALID_ARG; return; }
    const double p0 = q.dist.p0, p1 = q.dist.p1;
    st = check_params(kind, p0, p1);
    if (st != MIRNG_OK) return;
    if (q.n == 0) return;
    const uint64_t esz = (uint64_t)elem_bytes(kind);
    const uint64_t addr = (uint64_t)(uintptr_t)q.out;
    if (addr == 0 || addr % esz) { st = MIRNG_E_INVALID_ARG; return; }
    if (q.n >= (1ull << 32)) { st = MIRNG_E_CAPACITY; return; }
    const bool resident = (ref.flags & kRefEngine) != 0;
    mirng_state e{};
    if (resident) {
        e = engines[ref.slot];
        if (e.engine_type != q.engine_type) { st = MIRNG_E_INVALID_ARG; return; }
    }

    const Epilogue ep = epilogue_of(kind, p0, p1, nt);
    SlotRun &r = d.run;
    r.n = q.n;
    r.ep = ep;
    r.pad = 0;
    d.kind = (uint32_t)kind;

    if (q.engine_type == MIRNG_MRG32K3A) {
        uint32_t v[6];
        if (resident) {
#pragma unroll
            for (int i = 0; i < 6; ++i) v[i] = e.words[i];
            mrg_jump_limbs(v, ref.skip, 3, pow2);
        } else {
            v[0] = (uint32_t)((q.seed & 0xFFFFFFFFull) % kM1);
            v[1] = 1u;
            v[2] = 1u;
            v[3] = (uint32_t)((q.seed >> 32) % kM2);
            v[4] = 1u;
            v[5] = 1u;
            mrg_jump_limbs(v, &q.offset, 1, pow2);   // steps from the seed state
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) d.mst[i] = v[i];
        const uint64_t per = (uint64_t)kMrgThreads * kBatchMrgPasses * (esz == 8 ? 16 : 32);
        r.out_base = (char *)q.out;
        mchunks = (q.n + per - 1) / per;
        d.mchunks = (uint32_t)mchunks;
        return;
    }

    // Philox: key and 130-bit word position of output 0
    uint64_t p[3] = {q.offset, 0, 0};
    if (resident) {
        r.k0 = e.words[0];
        r.k1 = e.words[1];
        p[0] = e.pos[0];
        p[1] = e.pos[1];
        p[2] = e.pos[2] & 3u;
        add130(p, ref.skip);
    } else {
        r.k0 = (uint32_t)q.seed;
        r.k1 = (uint32_t)(q.seed >> 32);
    }
    const uint32_t head = (uint32_t)((addr & 15u) / esz);
    const uint32_t wpe = (uint32_t)philox_words_per_elem(kind);
    const uint32_t epv = (uint32_t)(16 / esz);
    // position of slot 0: p, or p - head * wpe (mod 2^130) when slot 0 starts
    // on the 16-byte grid before the output
    uint64_t g[3] = {p[0], p[1], p[2]};
    if (paired(kind) && (head & 1u)) {
        // pairs would straddle the 16-byte grid: slots (two FP32 pairs or
        // one FP64 pair) start at the output itself
        r.head = 0;
        d.nunits = (uint32_t)((q.n + epv - 1) / epv);
        r.full_lo = 0;
        r.full_count = (uint32_t)(q.n / epv);
        r.out_base = (char *)q.out;
    } else {
        const uint64_t dq = (uint64_t)head * wpe;
        const uint64_t b0 = p[0] < dq ? 1u : 0u;
        g[0] = p[0] - dq;
        const uint64_t b1 = p[1] < b0 ? 1u : 0u;
        g[1] = p[1] - b0;
        g[2] = (p[2] - b1) & 3u;
        r.head = head;
        d.nunits = (uint32_t)((head + q.n + epv - 1) / epv);
        const uint64_t lo = head ? 1 : 0;
        const uint64_t hi = (head + q.n) / epv;
        r.full_lo = (uint32_t)lo;
        r.full_count = (uint32_t)(hi > lo ? hi - lo : 0);
        r.out_base = (char *)q.out - (addr & 15u);
        // slot 0's place in its 1 KiB block: the tiles follow that grid
        d.slot0 = (uint32_t)(((uint64_t)(uintptr_t)r.out_base >> 4) & 63u);
    }
    // block index floor(g / 4) (128 bits) and phase g mod 4
    const uint64_t b_lo = (g[0] >> 2) | (g[1] << 62);
    const uint64_t b_hi = (g[1] >> 2) | (g[2] << 62);
    r.base[0] = (uint32_t)b_lo;
    r.base[1] = (uint32_t)(b_lo >> 32);
    r.base[2] = (uint32_t)b_hi;
    r.base[3] = (uint32_t)(b_hi >> 32);
    d.phase = (uint32_t)(g[0] & 3u);
    tiles = ((uint64_t)d.slot0 + d.nunits + 63) / 64;
}

// Inclusive scan over a workgroup of kChunk threads (16 waves).
__device__ uint64_t block_scan(uint64_t v, uint64_t *wsum)
{
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t t = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v += t;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    if (wid == 0) {
        uint64_t w = lane < (blockDim.x >> 6) ? wsum[lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t t = __shfl_up(w, off);
            if (lane >= (uint32_t)off) w += t;
        }
        if (lane < (blockDim.x >> 6)) wsum[lane] = w;
    }
    __syncthreads();
    if (wid > 0) v += wsum[wid - 1];
    __syncthreads();
    return v;
}

// The whole 64-byte request in one round of four 16-byte loads (field by
// field, the validation's early exits would fetch it in six dependent
// rounds).
__device__ __forceinline__ mirng_request load_request(const mirng_request *p)
{
    static_assert(sizeof(mirng_request) == 64, "request layout");
    const uint4 *src = reinterpret_cast<const uint4 *>(p);
    uint4 w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = src[i];
    // keeps the compiler from sinking each load into the branch that first
    // needs it
#pragma unroll
    for (int i = 0; i < 4; ++i)
        asm volatile("" : "+v"(w[i].x), "+v"(w[i].y), "+v"(w[i].z), "+v"(w[i].w));
    mirng_request q;
    __builtin_memcpy(&q, w, sizeof(q));
    return q;
}

__global__ __launch_bounds__(kChunk) void batch_plan_kernel(BatchArgs a)
{
    __shared__ uint64_t wsum[kChunk / 64];
    const uint32_t r = blockIdx.x * kChunk + threadIdx.x;
    uint64_t tiles = 0, mchunks = 0;
    if (r < a.count) {
        int32_t st;
        BatchDesc d;
        const mirng_request q = load_request(&a.reqs[r]);
        EngineRef ref{};
        if (a.refs) ref = a.refs[r];
        plan_one(q, ref, a.engines, d, st, a.nt, a.pow2, tiles, mchunks);
        a.status[r] = st;
        if (st != MIRNG_OK) {
            d.nunits = 0;
            d.mchunks = 0;
            tiles = 0;
            mchunks = 0;
        }
        a.desc[r] = d;
    }
    const uint64_t inc0 = block_scan(tiles, wsum);
    const uint64_t inc1 = block_scan(mchunks, wsum);
    if (r < a.count) {
        a.local_end[2 * r] = inc0;
        a.local_end[2 * r + 1] = inc1;
    }
    if (threadIdx.x == kChunk - 1) {
        a.chunk_total[2 * blockIdx.x] = inc0;
        a.chunk_total[2 * blockIdx.x + 1] = inc1;
    }
}

__global__ __launch_bounds__(kChunk) void batch_scan_kernel(BatchArgs a)
{
    __shared__ uint64_t wsum[kChunk / 64];
    __shared__ uint64_t carry[2];
    if (threadIdx.x < 2) carry[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < a.nchunks; c0 += kChunk) {
        const uint32_t c = c0 + threadIdx.x;
        for (int j = 0; j < 2; ++j) {
            const uint64_t v = c < a.nchunks ? a.chunk_total[2 * c + j] : 0;
            const uint64_t inc = block_scan(v, wsum) + carry[j];
            if (c < a.nchunks) a.chunk_end[2 * c + j] = inc;
            __syncthreads();
            if (threadIdx.x == kChunk - 1) carry[j] = inc;
            __syncthreads();
        }
    }
    if (threadIdx.x < 2) a.total[threadIdx.x] = carry[threadIdx.x];
}

__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), (int)l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_scan(uint64_t v)
{
    const uint32_t lane = threadIdx.x & 63u;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t t = __shfl_up(v, off);
        if (lane >= (uint32_t)off) v += t;
    }
    return v;
}

// Most chunks whose prefix a wave keeps in registers (one per lane).
constexpr uint32_t kWaveChunks = 64;

// The chunk-level prefix of count j (0: Philox tiles, 1: MRG chunks) as one
// wave sees it.  Up to 64 chunks the wave scans the chunk totals itself
// (lane c holds chunk c: one round of loads, and no scan kernel); beyond
// that the scan kernel's prefixes are read from memory.
struct ChunkPrefix {
    uint64_t inc = 0;     // in registers: prefix through chunk (lane)
    uint64_t excl = 0;    // in registers: prefix before chunk (lane)
    uint64_t total = 0;   // wave-uniform batch total
    bool regs = false;
};

__device__ __forceinline__ ChunkPrefix chunk_prefix(const BatchArgs &a, int j)
{
    ChunkPrefix p;
    p.regs = a.nchunks <= kWaveChunks;
    if (p.regs) {
        const uint32_t lane = threadIdx.x & 63u;
        const uint64_t v = lane < a.nchunks ? a.chunk_total[2 * lane + j] : 0;
        p.inc = wave_scan(v);
        p.excl = p.inc - v;
        p.total = readlane64(p.inc, 63);
    } else {
        p.total = uniform64(a.total[j]);
    }
    return p;
}

// Prefix before chunk c (wave-uniform).
__device__ __forceinline__ uint64_t chunk_base(const BatchArgs &a, int j, const ChunkPrefix &p,
                                               uint32_t c)
{
    if (p.regs) return readlane64(p.excl, c);
    return uniform64(a.chunk_end[2 * c + j] - a.chunk_total[2 * c + j]);
}

// First index i in [lo, hi) with v(i) > T, for v non-decreasing and
// v(hi - 1) > T: a 64-ary search.  Every lane probes one of 64 evenly spaced
// positions at once and a ballot keeps the bracket, so each round shrinks
// the range 64-fold (about 3 dependent loads for 10^4 requests instead of
// 14).  Called by whole waves; wave-uniform result.
template <typename V>
__device__ __forceinline__ uint32_t search64(uint32_t lo, uint32_t hi, uint64_t T, V v)
{
    const uint32_t lane = threadIdx.x & 63u;
    while (hi - lo > 1u) {
        const uint32_t n = hi - lo;
        const uint32_t step = (n + 63u) / 64u;
        const uint32_t p = lo + lane * step;
        const bool above = p >= hi || v(p) > T;
        const uint64_t mask = __builtin_amdgcn_ballot_w64(above);
        const uint32_t f = mask ? (uint32_t)__builtin_ctzll(mask) : 64u;
        const uint32_t nlo = f == 0u ? lo : lo + (f - 1u) * step + 1u;
        const uint32_t nhi = f == 64u ? hi : min(hi, lo + f * step + 1u);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// The chunk holding unit T (T below the batch total): the first chunk
// whose prefix end exceeds T.  Called by whole waves.
__device__ uint32_t find_chunk(const BatchArgs &a, int j, const ChunkPrefix &p, uint64_t T)
{
    if (p.regs) {
        // lanes past the last chunk hold the total, which exceeds T
        const uint64_t m = __builtin_amdgcn_ballot_w64(p.inc > T);
        return uniform((uint32_t)__builtin_ctzll(m));
    }
    return uniform(search64(0u, a.nchunks, T,
                            [&](uint32_t i) { return a.chunk_end[2 * i + j]; }));
}

// The request of chunk c (prefix `base` before it) holding unit T.
__device__ __forceinline__ uint32_t find_in_chunk(const BatchArgs &a, int j, uint32_t c,
                                                  uint64_t base, uint64_t T)
{
    const uint32_t lo = c * kChunk;
    const uint32_t hi = min(a.count, lo + kChunk);
    return uniform(search64(lo, hi, T,
                            [&](uint32_t i) { return base + a.local_end[2 * i + j]; }));
}

// Wave start table, filled during planning: for wave w of the Philox
// grid, the request holding its first tile w * ceil(T / W) (count when the
// wave has no tiles).  One thread per wave, each with its own
// lower-bound searches (over the chunk prefix, then over the chunk's
// requests); generating waves then start with one load instead of a search.
__global__ __launch_bounds__(256) void batch_start_kernel(BatchArgs a)
{
    const uint32_t w = blockIdx.x * 256u + threadIdx.x;
    const ChunkPrefix p = chunk_prefix(a, 0);   // whole waves
    const uint64_t per = (p.total + a.waves - 1) / a.waves;
    const uint64_t T = (uint64_t)w * per;
    // first chunk whose prefix end exceeds T
    uint32_t c = 0;
    uint64_t base = 0;
    if (p.regs) {
        // the chunk ends sit in lane c: a fixed-length search so that every
        // lane takes part in each cross-lane read
        uint32_t n = a.nchunks;
        for (int it = 0; it < 7; ++it) {
            const uint32_t half = n / 2u;
            const uint32_t mid = c + half;
            const uint64_t v = __shfl(p.inc, (int)min(mid, 63u));
            if (n > 0u && v <= T) {
                c = mid + 1u;
                n -= half + 1u;
            } else {
                n = half;
            }
        }
        base = __shfl(p.excl, (int)min(c, 63u));
    } else {
        uint32_t n = a.nchunks;
        while (n > 0u) {
            const uint32_t half = n / 2u;
            if (a.chunk_end[2 * (c + half)] <= T) {
                c += half + 1u;
                n -= half + 1u;
            } else {
                n = half;
            }
        }
        if (c < a.nchunks) base = a.chunk_end[2 * c] - a.chunk_total[2 * c];
    }
    if (w >= a.waves) return;
    uint32_t r = a.count;
    if (T < p.total) {
        r = c * kChunk;
        uint32_t n = min(a.count - r, kChunk);
        while (n > 0u) {
            const uint32_t half = n / 2u;
            if (base + a.local_end[2 * (r + half)] <= T) {
                r += half + 1u;
                n -= half + 1u;
            } else {
                n = half;
            }
        }
    }
    a.wave_start[w] = r;
}

// Slots [lo, hi) of request d in steps of 64 from s0 (see walk_slots_from).
// The range (or mean / sd) step is chosen per segment, which is uniform
// per request, so the loop holds no per-sample select.
template <int KIND, int RANGED>
__device__ __forceinline__ void run_phase(const BatchDesc &d, uint32_t s0, uint32_t lo,
                                          uint32_t hi, uint32_t lane)
{
    switch (d.phase) {
    case 0: walk_slots_from<KIND, 0, RANGED>(d.run, s0, lo, hi, lane); break;
    case 1: walk_slots_from<KIND, 1, RANGED>(d.run, s0, lo, hi, lane); break;
    case 2: walk_slots_from<KIND, 2, RANGED>(d.run, s0, lo, hi, lane); break;
    default: walk_slots_from<KIND, 3, RANGED>(d.run, s0, lo, hi, lane); break;
    }
}

template <int KIND>
__device__ __forceinline__ void run_kind(const BatchDesc &d, uint32_t s0, uint32_t lo,
                                         uint32_t hi, uint32_t lane)
{
    if (has_range_step(KIND) && d.run.ep.ranged)
        run_phase<KIND, 1>(d, s0, lo, hi, lane);
    else
        run_phase<KIND, 0>(d, s0, lo, hi, lane);
}

// WIDE: the batch holds Philox Gaussian FP64 or inverse-CDF Gaussian
// requests.  Their transforms need many more registers, so batches without
// them run a kernel that does not contain them (and keeps its occupancy).
// BM: the batch holds Gaussian requests (either method, FP32 or FP64),
// whose log and rotation tables the kernel stages in LDS; batches without
// them run a kernel that neither stages the tables nor holds their LDS.
// Forced inline: called as a function (the compiler's choice for the wide
// instance), every segment stored the descriptor to scratch for the callee.
template <bool WIDE, bool BM>
__device__ __forceinline__ void run_segment(const BatchDesc &d, uint32_t s0, uint32_t lo,
                                            uint32_t hi, uint32_t lane)
{
    switch (d.kind) {
    case kBits: run_kind<kBits>(d, s0, lo, hi, lane); break;
    case kU32F: run_kind<kU32F>(d, s0, lo, hi, lane); break;
    case kU64F: run_kind<kU64F>(d, s0, lo, hi, lane); break;
    case kGauss:
        if constexpr (BM) run_kind<kGauss>(d, s0, lo, hi, lane);
        break;
    case kI32: run_kind<kI32>(d, s0, lo, hi, lane); break;
    default:
        if constexpr (WIDE) {
            switch (d.kind) {
            case kGauss64:
                if constexpr (BM) run_kind<kGauss64>(d, s0, lo, hi, lane);
                break;
            case kIcdf:
                if constexpr (BM) run_kind<kIcdf>(d, s0, lo, hi, lane);
                break;
            default:
                if constexpr (BM) run_kind<kIcdf64>(d, s0, lo, hi, lane);
                break;
            }
        }
        break;
    }
}

// The descriptor of a (wave-uniform) request, copied into registers so that
// the slot stores cannot force it to be re-read.
__device__ __forceinline__ BatchDesc load_desc(const BatchDesc *p)
{
    BatchDesc d;
    const uint32_t *src = (const uint32_t *)p;
    uint32_t *dst = (uint32_t *)&d;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BatchDesc) / 4); ++i) dst[i] = uniform(src[i]);
    return d;
}

// Groups of the wide kernel hold at most 256 threads, which lets it use up
// to 512 registers per lane instead of spilling past 128.
constexpr uint32_t kWideBlock = 256;

template <bool WIDE, bool BM>
__global__ __launch_bounds__(WIDE ? kWideBlock : 1024) void batch_main_kernel(BatchArgs a)
{
    if constexpr (BM) bm_stage();
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // the chunk prefix and this wave's first request (from the start
    // table) in one round of loads
    const ChunkPrefix p = chunk_prefix(a, 0);
    uint32_t r = wave < a.waves ? uniform(a.wave_start[wave]) : a.count;
    const uint64_t per = (p.total + a.waves - 1) / a.waves;
    uint64_t t = wave * per;
    const uint64_t t1 = min(t + per, p.total);
    if (t >= t1 || r >= a.count) return;
    uint32_t c = r / kChunk;
    uint64_t base = chunk_base(a, 0, p, c);
    while (t < t1 && r < a.count) {
        if (r / kChunk != c) {
            c = r / kChunk;
            base = chunk_base(a, 0, p, c);
        }
        // the descriptor and the prefix end in one round of loads
        const BatchDesc d = load_desc(&a.desc[r]);
        const uint64_t end = base + uniform64(a.local_end[2 * r]);
        const uint64_t start = end - ((uint64_t)d.slot0 + d.nunits + 63) / 64;
        if (end > t) {
            // tiles are 64 slots of a grid shifted by slot0, so that a step's
            // 1 KiB of stores falls on one 1 KiB block of memory
            const uint64_t seg = min(t1, end);
            const uint32_t v0 = (uint32_t)((t - start) * 64);
            const uint32_t v1 = (uint32_t)((seg - start) * 64);
            const uint32_t lo = v0 > d.slot0 ? v0 - d.slot0 : 0u;
            const uint32_t hi = min(v1 - d.slot0, d.nunits);
            run_segment<WIDE, BM>(d, v0 - d.slot0, lo, hi, lane);
            t = seg;
        }
        ++r;
    }
}

// One chunk of an MRG request: 256 threads x kBatchMrgPasses passes of L.
// As in the plain kernel, the thread ranges start h0 elements into the
// output (its first 128-byte boundary; 0 for a paired kind with odd h0),
// and chunk 0 writes the h0 head elements from the request's start state.
template <int KIND>
__device__ void mrg_chunk(const BatchDesc &d, uint64_t k, const uint32_t *c_tab,
                          const uint32_t *u_tab, const uint32_t *pow2, char *lds,
                          uint32_t *wg_state)
{
    using S = MrgShape<KIND>;
    constexpr uint32_t q = kBatchMrgPasses * S::L;
    const uint32_t t = threadIdx.x;
    uint32_t h0 = (uint32_t)((0u - (uint32_t)(uintptr_t)d.run.out_base) & 127u) / S::ESZ;
    if (paired(KIND) && (h0 & 1u)) h0 = 0;
    if (t < 64) {
        uint32_t v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = d.mst[i];
        for (int dg = 0; dg < kCDigits; ++dg) {
            const uint32_t digit = (uint32_t)(k >> (6 * dg)) & 63u;
            if (digit) apply_mat(c_tab + (dg * 64 + digit) * kMatWords, v);
        }
        for (int b = 0; b < 5; ++b)
            if ((h0 >> b) & 1u) apply_mat(pow2 + b * kMatWords, v);
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i) wg_state[i] = v[i];
        }
    }
    __syncthreads();
    uint32_t v[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = wg_state[i];
    if (t) apply_mat(u_tab + t * kMatWords, v);
    MrgState s = mrg_state(v);
    const uint64_t e_wg = k * kMrgThreads * q;
    const uint64_t n_rest = d.run.n > h0 ? d.run.n - h0 : 0;
    char *rng_out = d.run.out_base + (uint64_t)h0 * S::ESZ;
    char *row = mrg_row<KIND>(lds, t);
    const uint32_t h = mrg_head<KIND>(rng_out);
    bool pending = false;   // the previous pass left its rows' last h elements
    uint64_t e_last = e_wg;
    for (uint32_t pass = 0; pass < kBatchMrgPasses; ++pass) {
        const uint64_t e0 = e_wg + (uint64_t)pass * S::L;
        if (e0 >= n_rest) break;   // uniform per group
        if (pending) mrg_carry_tail<KIND>(row, h);
        mrg_fill_row<KIND>(s, row, d.run.ep);
        __syncthreads();
        pending = mrg_store_pass<KIND>(lds, e0, q, n_rest, rng_out, d.run.ep.nt, pending);
        __syncthreads();
        e_last = e0;
    }
    if (pending) mrg_store_tail<KIND>(row, e_last + (uint64_t)t * q, h, rng_out);
    if (k == 0 && t == 0 && h0 != 0) {
        uint32_t v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = d.mst[i];
        MrgState hs = mrg_state(v);
        mrg_fill_row<KIND, true>(hs, row, d.run.ep);
        const uint32_t m = d.run.n < h0 ? (uint32_t)d.run.n : h0;
        for (uint32_t e = 0; e < m; ++e) put_elem<S::ESZ>(d.run.out_base, e, row + e * S::ESZ);
    }
    // the next chunk's wave 0 rewrites wg_state, and the head's row is this
    // thread's own: both follow the loop's last barrier
    __syncthreads();
}

// WIDE: the batch holds MRG inverse-CDF requests, whose transforms need
// about twice the registers of the others (halving the resident groups).
// BM: as for the Philox kernel (here the tables' 6 KiB of LDS would cost a
// resident group per CU).
template <bool WIDE, bool BM>
__global__ __launch_bounds__(kMrgThreads) void batch_mrg_kernel(BatchArgs a)
{
    // LDS rows are 144 bytes for every kind (32 x 4 or 16 x 8, plus 16)
    __shared__ __attribute__((aligned(16))) char lds[kMrgThreads * MrgShape<kU32F>::ROW];
    __shared__ uint32_t wg_state[6];
    static_assert(MrgShape<kU64F>::ROW == MrgShape<kU32F>::ROW, "row size");
    if constexpr (BM) bm_stage();
    const ChunkPrefix p = chunk_prefix(a, 1);
    const uint64_t per = (p.total + a.mgroups - 1) / a.mgroups;
    uint64_t c = (uint64_t)blockIdx.x * per;
    const uint64_t c1 = min(c + per, p.total);
    if (c >= c1) return;
    uint32_t rc = find_chunk(a, 1, p, c);
    uint64_t base = chunk_base(a, 1, p, rc);
    uint32_t r = find_in_chunk(a, 1, rc, base, c);
    while (c < c1 && r < a.count) {
        if (r / kChunk != rc) {
            rc = r / kChunk;
            base = chunk_base(a, 1, p, rc);
        }
        const BatchDesc d = load_desc(&a.desc[r]);
        const uint64_t end = base + uniform64(a.local_end[2 * r + 1]);
        const uint64_t start = end - d.mchunks;
        if (end > c) {
            const uint64_t seg = min(c1, end);
            for (uint64_t k = c - start; k < seg - start; ++k) {
                switch (d.kind) {
                case kBits: mrg_chunk<kBits>(d, k, a.c_tab4, a.u_tab4, a.pow2, lds, wg_state); break;
                case kU32F: mrg_chunk<kU32F>(d, k, a.c_tab4, a.u_tab4, a.pow2, lds, wg_state); break;
                case kU64F: mrg_chunk<kU64F>(d, k, a.c_tab8, a.u_tab8, a.pow2, lds, wg_state); break;
                case kGauss:
                    if constexpr (BM) mrg_chunk<kGauss>(d, k, a.c_tab4, a.u_tab4, a.pow2, lds, wg_state);
                    break;
                case kGauss64:
                    if constexpr (BM) mrg_chunk<kGauss64>(d, k, a.c_tab8, a.u_tab8, a.pow2, lds, wg_state);
                    break;
                case kI32: mrg_chunk<kI32>(d, k, a.c_tab4, a.u_tab4, a.pow2, lds, wg_state); break;
                default:
                    if constexpr (WIDE) {
                        if (d.kind == kIcdf) {
                            if constexpr (BM)
                                mrg_chunk<kIcdf>(d, k, a.c_tab4, a.u_tab4, a.pow2, lds, wg_state);
                        } else if constexpr (BM) {
                            mrg_chunk<kIcdf64>(d, k, a.c_tab8, a.u_tab8, a.pow2, lds, wg_state);
                        }
                    }
                    break;
                }
            }
            c = seg;
        }
        ++r;
    }
}

}  // namespace

hipError_t launch_batch_plan(const BatchArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(batch_plan_kernel, dim3(a.nchunks), dim3(kChunk), 0, s, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (a.nchunks > kWaveChunks) {
        hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(kChunk), 0, s, a);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (a.philox) {
        hipLaunchKernelGGL(batch_start_kernel, dim3((a.waves + 255u) / 256u), dim3(256), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

hipError_t launch_batch_generate(const BatchArgs &a, hipStream_t s)
{
    hipError_t err = hipSuccess;
    if (a.philox) {
        if (a.wide) {
            // same waves in groups of at most kWideBlock threads; waves past
            // a.waves find no tiles and return
            const uint32_t blk = a.block < kWideBlock ? a.block : kWideBlock;
            const uint32_t wpb = blk / 64u;
            const uint32_t groups = (a.waves + wpb - 1u) / wpb;
            if (a.bm)
                hipLaunchKernelGGL((batch_main_kernel<true, true>), dim3(groups), dim3(blk), 0, s,
                                   a);
            else
                hipLaunchKernelGGL((batch_main_kernel<true, false>), dim3(groups), dim3(blk), 0,
                                   s, a);
        } else if (a.bm) {
            hipLaunchKernelGGL((batch_main_kernel<false, true>), dim3(a.groups), dim3(a.block), 0,
                               s, a);
        } else {
            hipLaunchKernelGGL((batch_main_kernel<false, false>), dim3(a.groups), dim3(a.block),
                               0, s, a);
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (a.mrg) {
        const dim3 grid(a.mgroups), block(kMrgThreads);
        if (a.mrg_wide && a.bm)
            hipLaunchKernelGGL((batch_mrg_kernel<true, true>), grid, block, 0, s, a);
        else if (a.mrg_wide)
            hipLaunchKernelGGL((batch_mrg_kernel<true, false>), grid, block, 0, s, a);
        else if (a.bm)
            hipLaunchKernelGGL((batch_mrg_kernel<false, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((batch_mrg_kernel<false, false>), grid, block, 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

}  // namespace mirng
