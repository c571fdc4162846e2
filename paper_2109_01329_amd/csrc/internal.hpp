// Library-internal declarations shared by the host code and the kernel
// translation units of libmirng.so.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "jobs.hpp"
#include "mirng.h"

namespace mirng {

// ------------------------------------------------------------ constants
// Philox4x32-10 (Salmon et al., SC'11): multipliers and Weyl key bumps.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// MRG32k3a (L'Ecuyer 1999): moduli and multipliers.
constexpr uint64_t kM1 = 4294967087ull;   // 2^32 - 209
constexpr uint64_t kM2 = 4294944443ull;   // 2^32 - 22853
constexpr uint64_t kA12 = 1403580ull;     // x1[n] uses  a12 x1[n-2]
constexpr uint64_t kA13 = 810728ull;      //           - a13 x1[n-3]
constexpr uint64_t kA21 = 527612ull;      // x2[n] uses  a21 x2[n-1]
constexpr uint64_t kA23 = 1370589ull;     //           - a23 x2[n-3]

// Devices the library keeps per-device state for (device ordinals below it).
constexpr int kMaxDevices = 64;

// ------------------------------------------------------------ host math
// 130-bit Philox word position, little-endian 64-bit limbs, l[2] < 4.
struct Pos130 {
    uint64_t l[3];
};

Pos130 pos_add(Pos130 p, const uint64_t *limbs, size_t nlimbs);
Pos130 pos_add_u64(Pos130 p, uint64_t n);
Pos130 pos_sub_u64(Pos130 p, uint64_t n);

// 3x3 matrix modulo m, row-major.
struct Mat3 {
    uint32_t a[9];
};

Mat3 mat_identity();
Mat3 mat_mul(const Mat3 &x, const Mat3 &y, uint64_t m);
void mat_vec(const Mat3 &x, const uint32_t v[3], uint64_t m, uint32_t out[3]);
Mat3 mat_pow_u64(const Mat3 &x, uint64_t n, uint64_t m);
// Companion matrices of the two components acting on (x[n-3], x[n-2], x[n-1]).
const Mat3 &mrg_a1();
const Mat3 &mrg_a2();
// Jump table A^(2^k), k < 192, for component c (0 or 1).
const Mat3 &mrg_pow2(int comp, int k);
// state <- A^n state, n = sum limbs[i] 2^(64 i).
void mrg_jump(uint32_t st[6], const uint64_t *limbs, size_t nlimbs);
void mrg_seed_state(uint64_t seed, uint32_t st[6]);

uint64_t words_consumed(int engine_type, int kind, uint64_t n);

// ------------------------------------------------------------ launches
enum Kind : int32_t {
    kBits = 1, kU32F = 2, kU64F = 3, kGauss = 4, kGauss64 = 5,
    kI32 = 6, kIcdf = 7, kIcdf64 = 8
};

// Bytes of one output and engine words (Philox) per output.
constexpr int elem_bytes(int kind)
{
    return (kind == kU64F || kind == kGauss64 || kind == kIcdf64) ? 8 : 4;
}
constexpr int philox_words_per_elem(int kind) { return elem_bytes(kind) == 8 ? 2 : 1; }
// Kinds whose outputs come in pairs from one Box-Muller transform.
constexpr bool paired(int kind) { return kind == kGauss || kind == kGauss64; }
// Kinds whose transforms read the log and rotation tables that kernels
// stage in LDS (bm_stage in transforms.hpp).
constexpr bool uses_lds_tables(int kind)
{
    return kind == kGauss || kind == kGauss64 || kind == kIcdf || kind == kIcdf64;
}
// Kinds with a range (or mean / sd) step that the defaults make a no-op.
constexpr bool has_range_step(int kind) { return kind != kBits && kind != kI32; }

// Output epilogue parameters shared by the generation kernels.
struct Epilogue {
    float a32, d32;         // uniform F32: fma(u, d, a); Gaussian: fma(z, sd, mean)
    double a64, d64;        // uniform F64: fma(u, d, a); Gaussian F64: fma(z, sd, mean)
    int32_t ranged;         // 0 when the parameters are the defaults
    int32_t nt;             // streaming stores
    int32_t ia;             // uniform int32: a
    uint32_t irm1;          // uniform int32: b - a - 1
};

// The parameter rules of each kind (the ABI's): MIRNG_OK,
// MIRNG_E_INVALID_ARG or MIRNG_E_UNSUPPORTED.  Host and device.
__host__ __device__ inline int32_t check_params(int kind, double p0, double p1)
{
    const bool fin = __builtin_isfinite(p0) && __builtin_isfinite(p1);
    switch (kind) {
    case kBits: return MIRNG_OK;
    case kU32F:
    case kU64F: return (fin && p0 < p1) ? MIRNG_OK : MIRNG_E_INVALID_ARG;
    case kGauss:
    case kGauss64:
    case kIcdf:
    case kIcdf64: return (fin && p1 > 0.0) ? MIRNG_OK : MIRNG_E_INVALID_ARG;
    case kI32:
        return (fin && p0 == __builtin_floor(p0) && p1 == __builtin_floor(p1) &&
                p0 >= -2147483648.0 && p1 <= 2147483648.0 && p0 < p1)
                   ? MIRNG_OK
                   : MIRNG_E_INVALID_ARG;
    default: return MIRNG_E_UNSUPPORTED;
    }
}

// The epilogue of a valid (kind, p0, p1).  Host and device.
__host__ __device__ inline Epilogue epilogue_of(int kind, double p0, double p1, int nt)
{
    Epilogue ep{};
    ep.ranged = (!has_range_step(kind) || (p0 == 0.0 && p1 == 1.0)) ? 0 : 1;
    ep.nt = nt;
    switch (kind) {
    case kU64F:
        ep.a64 = p0;
        ep.d64 = p1 - p0;
        break;
    case kGauss64:
    case kIcdf64:
        ep.a64 = p0;
        ep.d64 = p1;
        break;
    case kGauss:
    case kIcdf:
        ep.a32 = (float)p0;
        ep.d32 = (float)p1;
        break;
    case kI32:
        ep.ia = (int32_t)(int64_t)p0;
        ep.irm1 = (uint32_t)((int64_t)p1 - (int64_t)p0 - 1);
        break;
    default:
        ep.a32 = (float)p0;
        ep.d32 = (float)(p1 - p0);
        break;
    }
    return ep;
}

// Fast Philox launch: block j (counter base + j) carries words that are
// whole output elements j * epb - head .. j * epb - head + epb - 1 (epb = 4,
// or 2 for FP64); it is written with one 16-byte store at its element
// address.  Valid whenever output elements do not straddle blocks: bits and
// uniform FP32 at any position, FP64 and Gaussian at even positions.
struct PhiloxBlocks {
    uint32_t k0, k1;
    uint32_t base[4];       // 128-bit counter of block 0
    uint32_t head;          // elements of block 0 that precede output 0
    uint32_t nblocks;
    uint32_t full_lo;       // blocks [full_lo, full_lo + full_count) are complete
    uint32_t full_count;
    uint64_t n;             // outputs in this launch
    char *out;              // output element 0
    Epilogue ep;
    int32_t kind;
    uint32_t bpl;           // blocks per lane per iteration: 1, 2 or 4
    uint32_t block;         // threads per workgroup
    uint32_t groups;        // workgroups (persistent grid)
};

// A run of 16-byte output slots of one Philox request.  Slot s receives
// engine words q + 4 s .. q + 4 s + 3 with q = 4 * base + phase; element j
// of slot s is output index s * epv + j - head (epv = 4, or 2 for FP64);
// only indices in [0, n) are written, slots [full_lo, full_lo + full_count)
// whole.  out_base (slot 0) is 16-byte aligned, except for Gaussian outputs
// whose word pairs would straddle the 16-byte grid (output 4 mod 8 bytes at
// an odd position): there slots start at the output itself, head = 0, and
// the 16-byte stores are only 4-byte aligned (the path is ALU-bound, so
// their cost does not show).
struct SlotRun {
    uint32_t k0, k1;
    uint32_t base[4];       // 128-bit block index of q
    uint32_t head;
    uint32_t full_lo;
    uint32_t full_count;
    uint32_t pad;
    uint64_t n;
    char *out_base;
    Epilogue ep;
};

// Contiguous-walk Philox launch (every kind and position): each wave owns
// slots_per_wave consecutive slots of the run.
struct PhiloxFill {
    SlotRun run;
    uint32_t phase;         // q mod 4
    uint32_t nslots;
    uint32_t slots_per_wave;
    int32_t kind;
    uint32_t block;         // threads per workgroup
    uint32_t iters;         // 0: contiguous walk; 1, 2, 4: chunked walk, chunks per wave
    uint32_t group_walk;    // 1: iters aligned 64-slot chunks per wave, heads shared in LDS
};

// One request of a batch, as planned on the device.  Philox requests are
// runs of 16-byte slots cut into tiles of 64 slots (one wave each); MRG32k3a
// requests are cut into chunks of 256 threads x kBatchMrgSteps steps (one
// workgroup each).
struct BatchDesc {
    SlotRun run;            // Philox slots; for MRG only n, out_base and ep are used
    uint32_t kind;
    uint32_t phase;         // Philox: q mod 4
    uint32_t nunits;        // Philox: 16-byte slots (0 for MRG)
    uint32_t engine;        // mirng_engine_type
    uint32_t mst[6];        // MRG: state after `offset` steps from the seed state
    uint32_t mchunks;       // MRG: chunks (0 for Philox)
    uint32_t slot0;         // Philox: slot 0's place in its 1 KiB block (tile grid offset)
};

// Steps per MRG thread in a batch chunk: two passes of L (L = 32 outputs,
// or 16 for FP64).
constexpr uint32_t kBatchMrgPasses = 2;

// Device tables of one batch.  Philox tiles and MRG chunks are numbered by
// two inclusive prefixes (entries 2i and 2i + 1 of the prefix arrays), kept
// per chunk of 1024 requests plus a prefix over chunks.
struct BatchArgs {
    const mirng_request *reqs;
    const EngineRef *refs;          // per request, or nullptr: every request has (seed, offset)
    const mirng_state *engines;     // device engine table the references name
    uint32_t count;
    uint32_t nchunks;
    BatchDesc *desc;
    uint64_t *local_end;    // [2 count] inclusive prefixes inside the request's chunk
    uint64_t *chunk_total;  // [2 nchunks] per chunk
    uint64_t *chunk_end;    // [2 nchunks] inclusive prefixes over chunks
    uint64_t *total;        // [2] Philox tiles, MRG chunks of the batch
    uint32_t waves;         // waves of the Philox generation grid
    uint32_t *wave_start;   // [waves] first request of each Philox wave
    uint32_t mgroups;       // workgroups of the MRG generation grid
    int32_t *status;        // per request
    int32_t nt;             // streaming stores
    uint32_t block;         // Philox generation kernel: threads per workgroup
    uint32_t groups;        // Philox generation kernel: workgroups
    int32_t wide;           // some Philox request is Gaussian FP64 (host scan)
    int32_t philox;         // some request names Philox4x32-10 (host scan)
    int32_t mrg;            // some request names MRG32k3a (host scan)
    int32_t mrg_wide;       // some MRG32k3a request is an inverse-CDF Gaussian
    int32_t bm;             // some request's transform reads the LDS tables (uses_lds_tables)
    const uint32_t *pow2;   // MRG A^(2^k), k < 64: [k][comp][9]
    const uint32_t *c_tab4, *u_tab4;   // MRG chunk / thread jumps, 4-byte kinds
    const uint32_t *c_tab8, *u_tab8;   // MRG chunk / thread jumps, FP64
};

// Entries A^(2^k), k < kPow2Entries, of the resident MRG jump tables
// (enough for any 192-bit step count).
constexpr int kPow2Entries = 192;

// Resident MRG jump tables for batches on device `dev`.
struct MrgBatchTables {
    const uint32_t *pow2;   // A^(2^k), k < kPow2Entries: [k][comp][9]
    const uint32_t *c_tab4, *u_tab4, *c_tab8, *u_tab8;
};
hipError_t mrg_batch_tables(int dev, MrgBatchTables &t);

// Per-device set-up, once per device with that device current (called by
// ensure_device): the resident MRG jump tables.
hipError_t mrg_tables_init(int dev);
// Per-device set-up of the allocation-free batch: looks up the device
// address of its fixed scratch array on `dev` (the current device).
hipError_t noalloc_scratch_init(int dev);

// Launch shape and grids of a batch from one pass over its requests (host):
// fills a.waves, a.mgroups, a.block, a.groups, a.nt and the flags of which
// generation kernels have work.  max_waves caps the Philox grid (0: none).
void batch_grids(const mirng_batch_config &cfg, const mirng_request *reqs, size_t count,
                 uint64_t max_waves, BatchArgs &a);
// Waves of the Philox generation grid for launch shape c (whole groups).
size_t grid_waves(const mirng_batch_config &c);
// The batched launch shape a new batcher starts with.
mirng_batch_config batch_default_config();

// Planning (validation, per-request plans, prefix sums) of a batch, then its
// generation kernels; the second may run on another stream once the first
// has completed.
hipError_t launch_batch_plan(const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_generate(const BatchArgs &a, hipStream_t s);
// Allocates every staging slot of `b` for `count` requests on the current
// device (so that later batches of up to `count` requests allocate nothing).
hipError_t batcher_reserve(mirng_batcher b, size_t count);
// mirng_generate_batch with per-request engine references (refs may be
// nullptr): a request whose reference names a resident engine starts from
// entry engines[ref.slot] of a device engine table advanced by ref.skip.
mirng_status generate_batch_refs(mirng_batcher b, const mirng_request *reqs,
                                 const EngineRef *refs, size_t count,
                                 const mirng_state *engines, hipStream_t s);

hipError_t launch_philox_blocks(const PhiloxBlocks &a, hipStream_t s);
hipError_t launch_philox_fill(const PhiloxFill &a, hipStream_t s);

// Launch shape of the Philox fill kernel (process-wide, set through the
// ABI or by the autotuner).
mirng_philox_config &philox_config();   // the process-wide shape
bool philox_config_valid(const mirng_philox_config &c);
bool philox_kind_ok(int kind);
// The phase of a Philox launch of `kind` at word position pos (low limb)
// into out: the position of its first 16-byte slot modulo 4.
uint32_t philox_phase(int kind, uint64_t pos_lo, uintptr_t out);
// The shape generate calls of `kind` at `phase` use: its own, else the
// process-wide one.
mirng_philox_config philox_config_for(int kind, uint32_t phase);
// Install (c != nullptr) or drop (c == nullptr) a kind's own shape at one
// phase (0..3) or at all four (-1); kind valid.
void philox_config_set_kind(int kind, int phase, const mirng_philox_config *c);
// Whether `kind` has its own shape at `phase` (copied to *c if so and c !=
// nullptr).
bool philox_config_kind_set(int kind, int phase, mirng_philox_config *c);

int device_cu_count();
hipError_t ensure_device(int *dev);

}  // namespace mirng
