/*
 * mirng -- bulk random-number generation on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library (libmirng.so).  Plain C types only: device buffers
 * are passed as raw device pointers and streams as `void *` holding a
 * hipStream_t (NULL selects the null stream).  No C++ exception, abort or
 * longjmp crosses this boundary; every entry point returns a mirng_status.
 *
 * The operations follow the problem statement of Pascuzzi & Goli,
 * arXiv:2109.01329:
 *   - the native host-API flow "create a generator of a type -> set seed and
 *     offset -> allocate device memory -> generate -> destroy" (Sec. 4.2);
 *   - oneMKL-style generate calls taking a distribution object with a range
 *     (a, b) or (mean, standard deviation) (Sec. 4.1, Sec. 4.3 listings);
 *   - the range transform r * (b - a) + a, which the paper runs as a second
 *     kernel after vendor generation (Sec. 4.3) and which is fused here
 *     into the generation kernel's epilogue;
 *   - pointer-based (USM-style) memory: the caller owns device memory and
 *     orders work with streams, as the paper's USM API does (Sec. 4.1).
 * The engines are the ones the paper names (Philox4x32x10 and an MRG-based
 * generator, Sec. 4.1 and Sec. 7), defined by Salmon et al. (SC'11) and
 * L'Ecuyer (Oper. Res. 1999); substreams follow L'Ecuyer et al. (Oper.
 * Res. 2002).
 *
 * Conventions (fixed by this library where the paper is silent):
 *   Philox position p counts 32-bit engine words from the seed state and is
 *     a 130-bit integer; word p is word (p mod 4) of the Philox4x32-10
 *     output for the 128-bit counter floor(p / 4); key = (lo32(seed),
 *     hi32(seed)).
 *   MRG32k3a position counts recurrence steps; state words are
 *     (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]); the seed maps
 *     to x1 = (lo32(seed) mod m1, 1, 1), x2 = (hi32(seed) mod m2, 1, 1);
 *     output n is y = x1[n] - x2[n] (+ m1 when x1[n] <= x2[n]), in [1, m1].
 *   Outputs: bits = the engine word (Philox) or y (MRG); uniform FP32 =
 *     (w >> 8) * 2^-24; uniform FP64 = 53 bits of two Philox words (first
 *     word low) * 2^-53, or y / (m1 + 1) for MRG; Gaussian FP32 = Box-Muller
 *     on word pairs (u1 = ((w_a >> 8) + 1) 2^-24, u2 = (w_b >> 8) 2^-24,
 *     z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = ... sin(2 pi u2)).
 *   Gaussian FP64 = Box-Muller in FP64 on FP64 uniform pairs: Philox
 *     u1 = (v_a + 1) 2^-53, u2 = v_b 2^-53 with v_a, v_b the 53-bit values
 *     of words (4j, 4j+1) and (4j+2, 4j+3) (first word low); MRG u1, u2 =
 *     y_a / (m1 + 1), y_b / (m1 + 1) of outputs 2j, 2j+1; results within a
 *     few ulp of the exact transform.
 *   Uniform int32 on [a, b) = a + floor(w (b - a) / 2^32), exact, with w
 *     the engine word (Philox) or y (MRG).
 *   Inverse-CDF Gaussians (the oneMKL "icdf" method, Sec. 4.1 of the
 *     paper): z = Phi^-1(u) evaluated in FP64 with u strictly inside
 *     (0, 1): FP32 kind u = ((w >> 8) + 1/2) 2^-24 from one word (or y);
 *     FP64 kind, Philox u = (floor(v / 2) + 1/2) 2^-52 with v the 53-bit
 *     value of two words as for uniform FP64, MRG u = y / (m1 + 1).  The
 *     FP32 kind rounds z to FP32.  Results lie within a few ulp of the
 *     exact quantile.
 *   Range: uniform r = fma(u, RN(b - a), RN(a)) in the output precision;
 *     Gaussian r = fma(z, RN32(stddev), RN32(mean)); Gaussian FP64
 *     r = fma(z, stddev, mean) (both methods).
 *   Consumption per call: n words, except uniform FP64 and inverse-CDF
 *     Gaussian FP64 on Philox (2n), Gaussian FP32 (2 * ceil(n / 2); for odd
 *     n the last z1 is dropped) and Gaussian FP64 (4 * ceil(n / 2) Philox
 *     words or 2 * ceil(n / 2) MRG steps).
 */
#ifndef MIRNG_H
#define MIRNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIRNG_ABI_VERSION 2

typedef struct mirng_engine_s *mirng_engine;

typedef enum {
    MIRNG_PHILOX4X32_10 = 1,
    MIRNG_MRG32K3A = 2
} mirng_engine_type;

typedef enum {
    MIRNG_BITS_U32 = 1,      /* uint32 out, engine words                     */
    MIRNG_UNIFORM_F32 = 2,   /* float out, [a, b); default (0, 1)            */
    MIRNG_UNIFORM_F64 = 3,   /* double out, [a, b); default (0, 1)           */
    MIRNG_GAUSSIAN_F32 = 4,  /* float out, mean p0, stddev p1; default (0,1) */
    MIRNG_GAUSSIAN_F64 = 5,  /* double out, mean p0, stddev p1; default (0,1) */
    MIRNG_UNIFORM_I32 = 6,   /* int32 out, [a, b), integers a = p0, b = p1   */
    MIRNG_GAUSSIAN_ICDF_F32 = 7,  /* float out, inverse CDF; mean p0, sd p1   */
    MIRNG_GAUSSIAN_ICDF_F64 = 8   /* double out, inverse CDF; mean p0, sd p1  */
} mirng_dist_kind;

/* A distribution: kind plus two parameters.  Uniform: p0 = a, p1 = b with
 * a < b, both finite.  Uniform int32: a and b integers with
 * -2^31 <= a < b <= 2^31.  Gaussian (either method): p0 = mean (finite),
 * p1 = stddev (finite, > 0).  Bits: parameters ignored. */
typedef struct {
    int32_t kind;       /* a mirng_dist_kind */
    int32_t reserved;   /* must be 0 */
    double p0;
    double p1;
} mirng_distribution;

typedef enum {
    MIRNG_OK = 0,
    MIRNG_E_INVALID_ARG = 1,   /* bad pointer, alignment, parameter or size */
    MIRNG_E_UNSUPPORTED = 2,   /* unknown engine type or distribution kind  */
    MIRNG_E_ALLOC = 3,         /* library-internal allocation failed        */
    MIRNG_E_LAUNCH = 4,        /* a kernel launch or async copy failed      */
    MIRNG_E_DEVICE = 5,        /* no usable gfx950 device / runtime error   */
    MIRNG_E_CAPACITY = 6       /* request can never fit a configured cap    */
} mirng_status;

/* Engine state, for checkpoint / resume.
 * Philox: words[0], words[1] = key (k0, k1); words[2..5] = 0;
 *         pos = 130-bit word position, little-endian 64-bit limbs, pos[2] < 4.
 * MRG32k3a: words = (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1]),
 *         x1 words < m1 = 2^32 - 209, x2 words < m2 = 2^32 - 22853, neither
 *         component all zero; pos = steps since the seed state mod 2^192
 *         (informational: it does not define the stream). */
typedef struct {
    int32_t engine_type;
    uint32_t words[6];
    uint32_t reserved;
    uint64_t pos[3];
} mirng_state;

/* One independent request of a batch: the same result as
 * mirng_engine_create(engine_type, seed, offset) followed by
 * mirng_generate(dist, n, out) on a fresh engine. */
typedef struct {
    int32_t engine_type;
    int32_t reserved;
    mirng_distribution dist;
    uint64_t seed;
    uint64_t offset;   /* words (Philox) or steps (MRG) from the seed state */
    uint64_t n;        /* outputs */
    void *out;         /* device pointer, aligned to the output element */
} mirng_request;

/* ------------------------------------------------------------ device set-up */

/* Set up the current device for the library: check that it is a gfx950 GPU
 * and copy the library's resident MRG32k3a jump tables (about 310 KB, a
 * file-scope device array) to it with a host-synchronous copy.  Optional:
 * the first call of any entry point that uses a device does the same, once
 * per device; calling this first keeps that one-time copy out of later
 * calls, which then never synchronise the host or allocate device memory
 * for the tables.  Not a gfx950 device -> DEVICE; copy failure -> DEVICE
 * (retried on the next call). */
mirng_status mirng_device_init(void);

/* ---------------------------------------------------------------- engines */

/* Create an engine of `type` at position `offset` (engine words for Philox,
 * recurrence steps for MRG32k3a) from the seed state of `seed`.  The library
 * owns the engine; release it with mirng_engine_destroy.  Host-only: no
 * device call.  Errors: out == NULL -> INVALID_ARG; unknown type ->
 * UNSUPPORTED; allocation -> ALLOC (then *out is untouched). */
mirng_status mirng_engine_create(int32_t type, uint64_t seed, uint64_t offset,
                                 mirng_engine *out);

/* Destroy an engine.  NULL is accepted and ignored.  Work already enqueued
 * from this engine is unaffected (it holds no device resources). */
mirng_status mirng_engine_destroy(mirng_engine e);

/* Advance the engine by n words (Philox, modulo 2^130) or n steps
 * (MRG32k3a) without generating.  Host-only.  e == NULL -> INVALID_ARG. */
mirng_status mirng_skip_ahead(mirng_engine e, uint64_t n);

/* Same with a multi-word count n = sum(limbs[i] * 2^(64 i)), i < nlimbs,
 * nlimbs <= 3 (counts up to 2^192 - 1; e.g. 2^76 for a substream or 2^127
 * for a stream).  nlimbs > 3, or limbs == NULL with nlimbs > 0 ->
 * INVALID_ARG and the engine is unchanged. */
mirng_status mirng_skip_ahead_multi(mirng_engine e, const uint64_t *limbs,
                                    size_t nlimbs);

/* Copy the engine state out (host memory).  NULL arguments -> INVALID_ARG. */
mirng_status mirng_engine_get_state(mirng_engine e, mirng_state *s);

/* Replace the engine state.  The state's engine_type must equal the
 * engine's; Philox pos[2] must be < 4; MRG words must be in range and
 * neither component all zero.  Otherwise INVALID_ARG, engine unchanged. */
mirng_status mirng_engine_set_state(mirng_engine e, const mirng_state *s);

/* ---------------------------------------------------------------- generate */

/* Write n outputs of distribution d, drawn from the engine's current
 * position onward, to the device buffer `out` (caller-owned; element type
 * per d->kind; must be aligned to the element size), asynchronously on
 * `stream` (a hipStream_t, NULL = null stream).  The engine advances at
 * enqueue by the words the call consumes, so generate(n1); generate(n2)
 * gives the same values as one generate(n1 + n2) (for Gaussians when n1 is
 * even: an odd n1 drops the second value of its last pair).  No host
 * synchronisation.
 * n == 0 -> OK, nothing enqueued, engine unchanged.
 * Errors (engine unchanged): e, d NULL, or out NULL with n > 0, or
 * misaligned out, or bad parameters (uniform a >= b or non-finite;
 * Gaussian stddev <= 0 or non-finite; reserved != 0) -> INVALID_ARG;
 * unknown kind -> UNSUPPORTED; no usable device -> DEVICE.
 * A failed kernel launch returns LAUNCH; the engine has then already been
 * advanced, as the work was accepted for enqueue.  The first call on a
 * device that has not been set up does the one-time set-up of
 * mirng_device_init (a host-synchronous copy); no other host
 * synchronisation or allocation happens here. */
mirng_status mirng_generate(mirng_engine e, const mirng_distribution *d,
                            uint64_t n, void *out, void *stream);

/* MRG32k3a substreams: for s in [first, first + count), write n_each
 * outputs of d from the state 2^76 * s steps past the engine's current
 * state into out[(s - first) * n_each ...], contiguous per substream.
 * One launch.  The engine itself is not advanced.  first + count must not
 * exceed 2^30 (else INVALID_ARG).  Philox engines -> UNSUPPORTED; other
 * errors as mirng_generate. */
mirng_status mirng_generate_substreams(mirng_engine e,
                                       const mirng_distribution *d,
                                       uint64_t first, uint64_t count,
                                       uint64_t n_each, void *out,
                                       void *stream);

/* MRG32k3a streams: as mirng_generate_substreams with streams 2^127 steps
 * apart (L'Ecuyer et al., Oper. Res. 2002: streams of 2^51 substreams of
 * 2^76 steps).  Stream s starts 2^127 * s steps past the engine's current
 * state; combine with mirng_skip_ahead_multi (2^76 * j) on a copy of the
 * engine to reach substream j of a stream.  Same arguments, limits and
 * errors. */
mirng_status mirng_generate_streams(mirng_engine e,
                                    const mirng_distribution *d,
                                    uint64_t first, uint64_t count,
                                    uint64_t n_each, void *out,
                                    void *stream);

/* --------------------------------------------------------------- batching */

/* Batched generation: thousands of independent requests of uneven sizes in
 * one persistent launch -- the inter-event batching that the paper leaves
 * for future work for its calorimeter application, whose events each draw
 * three uniforms per hit (Sec. 5.2, Sec. 7).  A batcher owns a ring of
 * pinned host staging slots and device tables, reused across calls.
 * Requests are validated on the device, per request: a request that fails
 * validation writes nothing and gets a non-OK status (see
 * mirng_batcher_statuses); the others are unaffected.  Both engine types
 * may be mixed in one batch. */

typedef struct mirng_batcher_s *mirng_batcher;

/* Launch shape of the batched kernel (the autotuner's search space); only
 * speed depends on it. */
typedef struct {
    int32_t block;          /* threads per workgroup: 64, 128, 256, 512, 1024 */
    int32_t waves_per_cu;   /* waves of work per CU, 1..4096 */
    int32_t nontemporal;    /* 0: plain stores, 1: streaming (nt) stores */
    int32_t reserved;       /* must be 0 */
} mirng_batch_config;

/* Create a batcher (host-only; device memory is allocated at first use).
 * out == NULL -> INVALID_ARG; allocation -> ALLOC. */
mirng_status mirng_batcher_create(mirng_batcher *out);

/* Destroy a batcher after waiting for its outstanding work.  NULL is
 * accepted and ignored. */
mirng_status mirng_batcher_destroy(mirng_batcher b);

/* Pinned host array for the next batch of `count` requests, to be filled
 * in place and passed to mirng_generate_batch (which then copies nothing on
 * the host).  Waits until the ring slot it hands out is no longer in use by
 * the device.  NULL arguments -> INVALID_ARG; allocation -> ALLOC. */
mirng_status mirng_batcher_stage(mirng_batcher b, size_t count, mirng_request **reqs);

/* Enqueue `count` requests as one batch on `stream`: one host-to-device
 * copy of the request table, a planning kernel (validation, per-request
 * descriptors and MRG32k3a start states, tile prefixes) and two persistent
 * generation kernels (Philox4x32-10 requests, MRG32k3a requests).  Each
 * valid request's output equals that of a fresh engine created with its
 * (type, seed, offset) followed by one mirng_generate call; it does not
 * depend on the other requests, their order or the launch shape.  reqs may
 * be the array of the last mirng_batcher_stage call, or any host array
 * (copied into a staging slot).  count == 0 -> OK; b or reqs NULL ->
 * INVALID_ARG; count >= 2^31 -> INVALID_ARG; device or launch errors ->
 * DEVICE or LAUNCH.  Asynchronous: no host synchronisation. */
mirng_status mirng_generate_batch(mirng_batcher b, const mirng_request *reqs, size_t count,
                                  void *stream);

/* Per-request status of the most recent batch (mirng_status values); waits
 * (host-blocking) until that batch has completed.  count must not exceed
 * that batch's count -> else INVALID_ARG; no batch yet and count > 0 ->
 * INVALID_ARG. */
mirng_status mirng_batcher_statuses(mirng_batcher b, int32_t *statuses, size_t count);

/* Copy out / install the batched kernel's launch shape.  Out-of-range
 * fields -> INVALID_ARG, shape kept. */
mirng_status mirng_batcher_config_get(mirng_batcher b, mirng_batch_config *c);
mirng_status mirng_batcher_config_set(mirng_batcher b, const mirng_batch_config *c);

/* ------------------------------------------------ allocation-free batches */

/* Limits of mirng_generate_batch_noalloc: requests per call, waves of its
 * Philox generation grid, and the size of its fixed device scratch array. */
#define MIRNG_NOALLOC_MAX_REQUESTS 16384
#define MIRNG_NOALLOC_MAX_WAVES 65536
#define MIRNG_NOALLOC_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the batched
 * generation of mirng_generate_batch without a batcher.  Same request
 * semantics and the same planning and generation kernels, so each valid
 * request's output is identical to mirng_generate_batch's; only the
 * launch order differs (see below).
 *   reqs: host array of `count` requests, copied by one hipMemcpyAsync on
 *     `stream` into the library's scratch array.  With pinned host memory
 *     the copy is asynchronous and the array must stay unchanged until the
 *     copy has run on the stream; with pageable memory the runtime may
 *     block the host until the copy is done.
 *   statuses: caller-owned device buffer of `count` int32 (4-byte
 *     aligned), receiving each request's mirng_status from the planning
 *     kernel on `stream`.
 *   cfg: launch shape of the generation kernels (NULL: the shape a new
 *     batcher starts with); the Philox grid is capped at
 *     MIRNG_NOALLOC_MAX_WAVES waves.
 * The batch's device tables (the request table, per-request plans, prefix
 * and wave tables) live in one fixed library-owned array of
 * MIRNG_NOALLOC_SCRATCH_BYTES per GPU, in device memory that the library
 * holds from the device's set-up (mirng_device_init, or the first call of
 * any entry point on that device) until the process ends; nothing in the
 * array needs clearing between calls (planning writes every table before
 * the generation kernels read it).  This call allocates no device or host
 * memory, creates no stream or event and makes no host synchronisation of
 * its own (after the device's one-time set-up).  All work runs in order on
 * `stream`: the copy, planning, then the Philox and MRG32k3a generation
 * kernels one after the other.
 * Concurrency: every call on one GPU uses that GPU's one array, which keeps
 * the last call's contents.  Calls on the same stream are ordered and safe;
 * calls that overlap on one GPU (different streams, or different host
 * threads without ordering) race and may produce wrong outputs.
 * Errors: count == 0 -> OK (nothing enqueued); reqs or statuses NULL, or
 * statuses misaligned, or a bad cfg -> INVALID_ARG; count >
 * MIRNG_NOALLOC_MAX_REQUESTS -> CAPACITY (nothing enqueued); device ->
 * DEVICE; a failed copy or launch -> LAUNCH.  Invalid requests get their
 * status in `statuses` and write nothing. */
mirng_status mirng_generate_batch_noalloc(const mirng_request *reqs, size_t count,
                                          int32_t *statuses,
                                          const mirng_batch_config *cfg, void *stream);

/* ------------------------------------------------------ launch configuration */

/* Launch shape of the Philox kernels: the search space of the autotuner.
 * It changes only speed: every output is the same under every valid shape.
 * walk 0: each wave owns a contiguous run of 16-byte outputs and the grid
 *   holds CUs * waves_per_cu waves of work (any kind, any position).
 * walk 1: a persistent grid of CUs * waves_per_cu resident waves walks the
 *   output grid-stride, blocks_per_lane Philox blocks per lane per step;
 *   used where outputs do not straddle Philox blocks (bits and uniform FP32
 *   at any position, FP64 and Gaussian at even positions), walk 0 elsewhere.
 * walk 2: each wave writes blocks_per_lane independent chunks of 64
 *   16-byte outputs (63 when the position is not a multiple of 4 on the
 *   16-byte grid; the last lane then only supplies words to its neighbour);
 *   the grid size follows from n (any kind, any position).
 * walk 3: each wave writes blocks_per_lane chunks of 64 16-byte outputs at
 *   any position; a workgroup of G waves covers blocks_per_lane * G
 *   consecutive chunks, wave w taking chunks w, G + w, ...; the last lane
 *   of a chunk takes the words it lacks from the next chunk through LDS and
 *   the group's last wave evaluates the one block past the group; the grid
 *   size follows from n (any kind, any position; waves_per_cu unused).
 * Process-wide; set it while no generate call is being enqueued. */
typedef struct {
    int32_t walk;             /* 0 contiguous runs, 1 grid-stride, 2 chunks, 3 group chunks */
    int32_t block;            /* threads per workgroup: 64, 128, 256, 512, 1024 */
    int32_t waves_per_cu;     /* 1..4096 (walk 1: waves in the grid; walks 2, 3: unused) */
    int32_t blocks_per_lane;  /* walk 1: blocks per lane per step; walks 2, 3:
                                 chunks per wave; 1, 2 or 4 (ignored by walk 0)    */
    int32_t nontemporal;      /* 0: plain stores, 1: streaming (nt) stores       */
    int32_t reserved;         /* must be 0 */
} mirng_philox_config;

/* Copy the process-wide shape out.  c == NULL -> INVALID_ARG. */
mirng_status mirng_philox_config_get(mirng_philox_config *c);

/* Install the process-wide shape and drop every kind's own shape (so every
 * kind then uses this one).  c == NULL or any field out of range ->
 * INVALID_ARG and nothing changes.  Host-only. */
mirng_status mirng_philox_config_set(const mirng_philox_config *c);

/* Phase of a Philox launch: the engine word position of the launch's first
 * 16-byte output slot, modulo 4.  It follows from the position and the
 * output address: (position - head * words per element) mod 4, where head
 * is the number of elements between the previous 16-byte boundary and
 * `out` (0 for two-element Gaussian pairs that would straddle that grid).
 * Phase 0 needs no exchange of words between lanes; the other phases do, so
 * the fastest launch shape can differ between them.  Returns the phase of
 * a launch of `kind` at word position `position` (only its value mod 4
 * matters) into `out`; 0 for an unknown kind.  Host-only. */
uint32_t mirng_philox_phase(int32_t kind, uint64_t position, const void *out);

/* The shape that Philox generate calls of distribution `kind` use at phase
 * `phase` (0..3): the kind's own shape at that phase (installed by
 * mirng_philox_config_set_kind or by the autotuner), else the process-wide
 * one.  c == NULL or phase out of range -> INVALID_ARG; kind not a MIRNG_*
 * distribution -> UNSUPPORTED. */
mirng_status mirng_philox_config_get_kind(int32_t kind, int32_t phase, mirng_philox_config *c);

/* Give distribution `kind` its own shape at phase `phase` (0..3), or at all
 * four phases (phase = -1); c == NULL drops it (the kind then follows the
 * process-wide shape there).  Bad kind -> UNSUPPORTED; phase out of range
 * or a field out of range -> INVALID_ARG and nothing changes.  Same
 * threading rule as the process-wide shape.  Host-only. */
mirng_status mirng_philox_config_set_kind(int32_t kind, int32_t phase,
                                          const mirng_philox_config *c);

/* ---------------------------------------------------------------- serving */

/* A serving loop over the batched launch: requests arrive one at a time
 * from any host thread and are answered asynchronously (continuous
 * batching).  The paper measures time-to-solution of single calls and
 * notes that many small calls are dominated by per-call overheads (Sec. 7);
 * a server amortises them by launching whatever has arrived as one batch
 * whenever one of its S streams is free.
 *
 * Admission: requests are admitted in arrival order while the output bytes
 * of admitted, unfinished requests stay within capacity_bytes; a request
 * larger than the capacity on its own is refused at submission
 * (MIRNG_E_CAPACITY).  A batch holds at most max_batch requests.  Each
 * request is validated by the batched kernel, as in mirng_generate_batch,
 * and its final status is that request's status.  The caller owns the
 * output memory and must keep it valid until the request completes.
 * Tickets (about 64 bytes of host memory each) are kept for the server's
 * lifetime, so that any ticket can be polled and the statistics cover
 * every request.  Each stream's batch completes (and frees its stream and
 * its admitted bytes) as soon as it is done, independently of the others.
 *
 * Resident engines: a server holds a table of engine states in device
 * memory (max_engines entries, 56 bytes each), following the paper's
 * native flow "create a generator -> set seed and offset -> generate"
 * (Sec. 4.2) with the generator kept on the device.  A request submitted
 * with mirng_server_submit_engine continues its engine where the requests
 * admitted before it on that engine stopped: its start position is fixed
 * at admission, in arrival order (any 192-bit count of words or steps past
 * the table entry), and the planning kernel derives its start state on the
 * device from the resident entry.  So a sequence of requests served on one
 * engine gives the same values as the same sequence of mirng_generate
 * calls on one engine, whatever the batching, and positions are not
 * limited to 64-bit offsets (MRG32k3a substreams and streams, Philox
 * positions up to 2^130).  Requests on resident engines are validated at
 * submission, so their consumption is final when they are accepted (a
 * request whose batch then fails to launch has still consumed its words,
 * as with mirng_generate).  Engines live as long as the server. */

typedef struct mirng_server_s *mirng_server;

typedef struct {
    int32_t streams;            /* S: batches in flight at once, 1..8 */
    int32_t max_engines;        /* resident engine table entries, 0 .. 2^24; 0 selects 65536 */
    uint64_t capacity_bytes;    /* in-flight output bytes, >= 1 */
    uint64_t max_batch;         /* requests per batch, 1 .. 2^24 */
} mirng_server_config;

typedef struct {
    uint64_t submitted;         /* accepted by mirng_server_submit */
    uint64_t refused;           /* refused at submission (capacity) */
    uint64_t completed;         /* finished, any status */
    uint64_t failed;            /* finished with a non-OK status */
    uint64_t batches;           /* batches launched */
    uint64_t samples;           /* outputs of completed OK requests */
    uint64_t bytes;             /* output bytes of completed OK requests */
    uint64_t max_inflight_bytes;/* high-water mark of admitted, unfinished bytes */
    double latency_p50_ms;      /* submission to completion, completed requests */
    double latency_p99_ms;
    double latency_max_ms;
    double span_s;              /* first submission to last completion */
} mirng_server_stats;

/* Start a server on the current device (threads and streams of its own;
 * streams at the default priority).  NULL arguments or out-of-range
 * fields -> INVALID_ARG; device -> DEVICE; allocation -> ALLOC. */
mirng_status mirng_server_create(const mirng_server_config *cfg, mirng_server *out);

/* Finish every accepted request, then stop the server.  NULL is accepted. */
mirng_status mirng_server_destroy(mirng_server s);

/* Queue one request (copied).  *ticket names it in later calls.  Never
 * blocks on the device.  Request larger than the capacity -> CAPACITY (no
 * ticket); NULL arguments -> INVALID_ARG. */
mirng_status mirng_server_submit(mirng_server s, const mirng_request *req, uint64_t *ticket);

/* Create a resident engine of `type` at position `offset` from the seed
 * state of `seed` (as mirng_engine_create) in the next free entry of the
 * server's device table; *engine names it.  The entry is written with a
 * host-synchronous copy before the call returns.  Table full -> CAPACITY;
 * unknown type -> UNSUPPORTED; NULL arguments -> INVALID_ARG; copy failure
 * -> DEVICE. */
mirng_status mirng_server_engine_create(mirng_server s, int32_t type, uint64_t seed,
                                        uint64_t offset, uint32_t *engine);

/* Queue n outputs of distribution d into `out` (device memory, element
 * aligned, kept valid until the request completes) on resident engine
 * `engine`, continuing it: the request starts where the requests admitted
 * on this engine before it (and its skips) end, and the engine advances by
 * the words (Philox) or steps (MRG32k3a) the request consumes, as
 * mirng_generate on an engine does.  Validation at submission, engine
 * unchanged on error: unknown engine, NULL d or ticket, bad parameters,
 * NULL or misaligned out with n > 0 -> INVALID_ARG; unknown kind ->
 * UNSUPPORTED; n >= 2^32, or the output alone larger than the capacity ->
 * CAPACITY. */
mirng_status mirng_server_submit_engine(mirng_server s, uint32_t engine,
                                        const mirng_distribution *d, uint64_t n, void *out,
                                        uint64_t *ticket);

/* Advance resident engine `engine` by n = sum limbs[i] 2^(64 i) words or
 * steps (nlimbs <= 3), in arrival order with its requests: requests
 * submitted after this call start past the skip.  The count is kept modulo
 * 2^192 (Philox positions modulo 2^130).  Unknown engine, nlimbs > 3 or
 * limbs NULL with nlimbs > 0 -> INVALID_ARG. */
mirng_status mirng_server_engine_skip_ahead(mirng_server s, uint32_t engine,
                                            const uint64_t *limbs, size_t nlimbs);

/* The state of resident engine `engine` after every request and skip
 * submitted on it so far (in the mirng_state layout; for MRG32k3a, pos
 * counts steps since the seed state).  Host-only: the table entry plus the
 * admitted consumption.  Unknown engine or NULL out -> INVALID_ARG. */
mirng_status mirng_server_engine_get_state(mirng_server s, uint32_t engine, mirng_state *out);

/* Replace resident engine `engine`'s state (checkpoint / resume): waits
 * until every accepted request has completed, then rewrites the table
 * entry (host-synchronous) and restarts the engine's count there.  No
 * request may be submitted on this engine while the call runs.  The
 * state's type must equal the engine's and be valid as for
 * mirng_engine_set_state, else INVALID_ARG and nothing changes. */
mirng_status mirng_server_engine_set_state(mirng_server s, uint32_t engine,
                                           const mirng_state *st);

/* Non-blocking: *done = 1 and *status = the request's status once it has
 * completed, else *done = 0.  Unknown ticket -> INVALID_ARG. */
mirng_status mirng_server_poll(mirng_server s, uint64_t ticket, int32_t *done, int32_t *status);

/* Block until the request has completed; *status as for poll and, if
 * latency_ms is not NULL, its submission-to-completion time. */
mirng_status mirng_server_wait(mirng_server s, uint64_t ticket, int32_t *status,
                               double *latency_ms);

/* Block until every accepted request has completed. */
mirng_status mirng_server_drain(mirng_server s);

/* Counters and latency percentiles since creation (waits for nothing). */
mirng_status mirng_server_stats_get(mirng_server s, mirng_server_stats *out);

/* -------------------------------------------------------------- autotuning */

/* The autotuner times every candidate launch shape on the caller's own
 * workload and installs the fastest; only speed depends on the shape.  It
 * runs the workload repeatedly on `stream` (so `out` / the requests' outputs
 * are overwritten), first for about prewarm_ms milliseconds to bring the
 * clocks to their loaded state, then `rounds` rounds over the candidates,
 * each timing `reps` back-to-back launches with HIP events; a candidate's
 * score is its median round.  It synchronises the stream (host-blocking).
 * The paper notes that the block size chosen for a kernel matters (256 vs
 * 1024 threads, Sec. 7) and that per-architecture tuning is future work
 * (Sec. 8).  Results: the chosen shape and its time per launch in
 * milliseconds; either pointer may be NULL.  mirng_autotune_philox times
 * n outputs of `kind` into `out` from an engine at word position `offset`
 * (every launch restarts there) and installs the shape as the shape of
 * `kind` at the phase that position and `out` give (mirng_philox_phase;
 * other kinds and phases keep theirs);
 * mirng_autotune_batch installs it on the batcher.  Errors: bad arguments
 * -> INVALID_ARG; device or launch failures -> DEVICE / LAUNCH (the
 * previous shape is then kept). */
mirng_status mirng_autotune_philox(int32_t kind, uint64_t offset, uint64_t n, void *out,
                                   void *stream, int32_t prewarm_ms, int32_t rounds,
                                   int32_t reps, mirng_philox_config *best, float *best_ms);

/* The Philox launch shapes mirng_autotune_philox times, in its order: the
 * first min(max, total) are copied to out (out may be NULL); returns the
 * total.  Host-only. */
int32_t mirng_philox_candidates(mirng_philox_config *out, int32_t max);

mirng_status mirng_autotune_batch(mirng_batcher b, const mirng_request *reqs, size_t count,
                                  void *stream, int32_t prewarm_ms, int32_t rounds,
                                  int32_t reps, mirng_batch_config *best, float *best_ms);

/* ------------------------------------------------------------------ misc */

/* Static description of a status code (never NULL). */
const char *mirng_status_string(mirng_status s);

/* Library ABI version (MIRNG_ABI_VERSION of the build). */
int32_t mirng_abi_version(void);

/* Words (Philox) or steps (MRG32k3a) that n outputs of kind consume; 0 for
 * an unknown kind.  Host-only. */
uint64_t mirng_words_consumed(int32_t engine_type, int32_t kind, uint64_t n);

#ifdef __cplusplus
}
#endif

#endif /* MIRNG_H */
