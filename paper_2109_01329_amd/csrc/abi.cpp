// C-ABI entry points of libmirng.so: argument validation, engine state,
// the plain generate planner and its launches.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.hpp"

struct mirng_engine_s {
    int32_t type;
    // Philox
    uint32_t key[2];
    mirng::Pos130 pos;
    // MRG32k3a
    uint32_t st[6];
    uint64_t steps[3];   // informational position, mod 2^192
};

namespace mirng {

mirng_philox_config &philox_config()
{
    // measured on MI355X at n = 2^28 (launch-shape sweeps in the design
    // notes): group chunks, 256-thread groups, two aligned 1 KiB chunks per
    // wave, ordinary stores; ahead of the contiguous walk at every phase
    static mirng_philox_config c = {3, 256, 1, 2, 0, 0};
    return c;
}

namespace {
// A kind's own launch shape at a phase, if one was installed (per kind or by
// the autotuner); otherwise the kind follows the process-wide shape.  The
// phase is the word position of a launch's first 16-byte slot modulo 4:
// the walks differ there (phase 0 needs no word exchange between lanes),
// and so does the fastest shape.
struct KindShape {
    bool set = false;
    mirng_philox_config c{};
};
KindShape g_kind_shape[kIcdf64 + 1][4];
}  // namespace

bool philox_kind_ok(int kind) { return kind >= kBits && kind <= kIcdf64; }

uint32_t philox_phase(int kind, uint64_t pos_lo, uintptr_t out)
{
    const uintptr_t esz = (uintptr_t)elem_bytes(kind);
    const bool at_out = paired(kind) && (((out & 15u) / esz) & 1u);
    const uint64_t head = at_out ? 0u : (uint64_t)((out & 15u) / esz);
    return (uint32_t)((pos_lo - head * (uint64_t)philox_words_per_elem(kind)) & 3u);
}

mirng_philox_config philox_config_for(int kind, uint32_t phase)
{
    if (philox_kind_ok(kind) && g_kind_shape[kind][phase & 3u].set)
        return g_kind_shape[kind][phase & 3u].c;
    return philox_config();
}

void philox_config_set_kind(int kind, int phase, const mirng_philox_config *c)
{
    for (int ph = 0; ph < 4; ++ph) {
        if (phase >= 0 && ph != phase) continue;
        g_kind_shape[kind][ph].set = c != nullptr;
        if (c) g_kind_shape[kind][ph].c = *c;
    }
}

bool philox_config_kind_set(int kind, int phase, mirng_philox_config *c)
{
    const KindShape &k = g_kind_shape[kind][phase & 3];
    if (k.set && c) *c = k.c;
    return k.set;
}

bool philox_config_valid(const mirng_philox_config &c)
{
    const bool block_ok = c.block == 64 || c.block == 128 || c.block == 256 ||
                          c.block == 512 || c.block == 1024;
    const int wmax = 4096;
    return c.walk >= 0 && c.walk <= 3 && block_ok && c.waves_per_cu >= 1 &&
           c.waves_per_cu <= wmax &&
           (c.blocks_per_lane == 1 || c.blocks_per_lane == 2 || c.blocks_per_lane == 4) &&
           (c.nontemporal == 0 || c.nontemporal == 1) && c.reserved == 0;
}

namespace {

std::mutex g_dev_mu;
int g_dev_checked[kMaxDevices];   // 0 unknown, 1 ok (set up), -1 unusable
int g_dev_cus[kMaxDevices];

}  // namespace

hipError_t ensure_device(int *dev_out)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev_checked[dev] == 0) {
        hipDeviceProp_t prop;
        err = hipGetDeviceProperties(&prop, dev);
        if (err != hipSuccess) return err;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            g_dev_checked[dev] = -1;
        } else {
            // one-time set-up of this device (host-synchronous copies)
            err = mrg_tables_init(dev);
            if (err == hipSuccess) err = noalloc_scratch_init(dev);
            if (err != hipSuccess) return err;   // retried on the next call
            g_dev_checked[dev] = 1;
        }
        g_dev_cus[dev] = prop.multiProcessorCount;
    }
    if (g_dev_checked[dev] < 0) return hipErrorInvalidDeviceFunction;
    if (dev_out) *dev_out = dev;
    return hipSuccess;
}

int device_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return g_dev_cus[dev] > 0 ? g_dev_cus[dev] : 256;
}

namespace {

bool finite(double x) { return std::isfinite(x); }

// Validates a distribution; returns MIRNG_OK or the error status.
mirng_status check_dist(const mirng_distribution *d)
{
    if (!d) return MIRNG_E_INVALID_ARG;
    if (d->reserved != 0) return MIRNG_E_INVALID_ARG;
    return (mirng_status)check_params(d->kind, d->p0, d->p1);
}

size_t elem_size(int kind) { return (size_t)elem_bytes(kind); }

// Largest number of outputs one Philox fill launch takes (slot indices
// stay below 2^31).
constexpr uint64_t kMaxPerLaunch = 1ull << 32;

Epilogue make_epilogue(const mirng_distribution *d, int nt)
{
    return epilogue_of(d->kind, d->p0, d->p1, nt);
}

// Words p .. of the engine into n outputs at out: the contiguous-walk
// kernel, or the grid-stride kernel when it is selected and outputs do not
// straddle Philox blocks.
hipError_t philox_plain(const uint32_t key[2], Pos130 p, const mirng_distribution *d,
                        uint64_t n, char *out, hipStream_t s)
{
    const int kind = d->kind;
    const size_t esz = elem_size(kind);
    const uint32_t wpe = (uint32_t)philox_words_per_elem(kind);
    const uint64_t cus = (uint64_t)device_cu_count();
    while (n > 0) {
        const mirng_philox_config tu = philox_config_for(kind, philox_phase(kind, p.l[0],
                                                                            (uintptr_t)out));
        const Epilogue ep = make_epilogue(d, tu.nontemporal);
        const uint64_t chunk = n < kMaxPerLaunch ? n : kMaxPerLaunch;
        const uint64_t b_lo = (p.l[0] >> 2) | (p.l[1] << 62);   // floor(p / 4), 128 bits
        const uint64_t b_hi = (p.l[1] >> 2) | (p.l[2] << 62);
        // one word per output (and no pairs): any position; two words per
        // output or per pair: even positions; FP64 Gaussian pairs (four
        // words): never
        const bool one_word = wpe == 1 && !paired(kind);
        const bool whole = tu.walk == 1 && kind != kGauss64 &&
                           (one_word || (p.l[0] & 1u) == 0);
        const uintptr_t addr = (uintptr_t)out;
        hipError_t err;
        if (whole) {
            PhiloxBlocks a{};
            a.k0 = key[0];
            a.k1 = key[1];
            a.base[0] = (uint32_t)b_lo;
            a.base[1] = (uint32_t)(b_lo >> 32);
            a.base[2] = (uint32_t)b_hi;
            a.base[3] = (uint32_t)(b_hi >> 32);
            const uint32_t epb = 4u / wpe;
            a.head = (uint32_t)(p.l[0] & 3u) / wpe;
            const uint64_t nblocks = (a.head + chunk + epb - 1) / epb;
            a.nblocks = (uint32_t)nblocks;
            const uint64_t lo = a.head ? 1 : 0;
            const uint64_t hi = (a.head + chunk) / epb;   // blocks below hi end inside n
            a.full_lo = (uint32_t)lo;
            a.full_count = (uint32_t)(hi > lo ? hi - lo : 0);
            a.n = chunk;
            a.out = out;
            a.ep = ep;
            a.kind = kind;
            a.bpl = (uint32_t)tu.blocks_per_lane;
            a.block = (uint32_t)tu.block;
            const uint64_t wpb = (uint64_t)tu.block / 64;
            const uint64_t per = 64ull * a.bpl;
            const uint64_t steps = (nblocks + per - 1) / per;
            const uint64_t want = (cus * tu.waves_per_cu + wpb - 1) / wpb;
            const uint64_t need = (steps + wpb - 1) / wpb;
            a.groups = (uint32_t)(want < need ? want : need);
            err = launch_philox_blocks(a, s);
        } else {
            const uint32_t epv = (uint32_t)(16 / esz);
            // Gaussian pairs that would straddle the 16-byte grid: slots
            // (two pairs of FP32, or one pair of FP64) start at the output
            // itself (16-byte stores at 4- or 8-byte alignment)
            const bool at_out = paired(kind) && (((addr & 15u) / esz) & 1u);
            const uint32_t head = at_out ? 0u : (uint32_t)((addr & 15u) / esz);
            PhiloxFill a{};
            SlotRun &r = a.run;
            r.k0 = key[0];
            r.k1 = key[1];
            const Pos130 q = pos_sub_u64(p, (uint64_t)head * wpe);
            const uint64_t q_lo = (q.l[0] >> 2) | (q.l[1] << 62);
            const uint64_t q_hi = (q.l[1] >> 2) | (q.l[2] << 62);
            r.base[0] = (uint32_t)q_lo;
            r.base[1] = (uint32_t)(q_lo >> 32);
            r.base[2] = (uint32_t)q_hi;
            r.base[3] = (uint32_t)(q_hi >> 32);
            a.phase = (uint32_t)(q.l[0] & 3u);
            r.head = head;
            r.n = chunk;
            const uint64_t nslots = (head + chunk + epv - 1) / epv;
            a.nslots = (uint32_t)nslots;
            if (tu.walk == 3) {
                a.group_walk = 1;
                a.iters = (uint32_t)tu.blocks_per_lane;
                a.slots_per_wave = 64u * a.iters;
            } else if (tu.walk == 2) {
                a.iters = (uint32_t)tu.blocks_per_lane;
                a.slots_per_wave = a.iters * (a.phase ? 63u : 64u);
            } else {
                const uint64_t waves_target =
                    cus * (uint64_t)(tu.walk == 0 ? tu.waves_per_cu : 256);
                const uint64_t iters = (nslots + 64 * waves_target - 1) / (64 * waves_target);
                a.slots_per_wave = (uint32_t)((iters ? iters : 1) * 64);
                a.iters = 0;
            }
            const uint64_t lo = head ? 1 : 0;
            const uint64_t hi = (head + chunk) / epv;   // slots below hi end inside n
            r.full_lo = (uint32_t)lo;
            r.full_count = (uint32_t)(hi > lo ? hi - lo : 0);
            r.out_base = at_out ? out : out - (addr & 15u);
            r.ep = ep;
            a.kind = kind;
            a.block = (uint32_t)(tu.walk == 1 ? 1024 : tu.block);
            err = launch_philox_fill(a, s);
        }
        if (err != hipSuccess) return err;
        p = pos_add_u64(p, words_consumed(MIRNG_PHILOX4X32_10, kind, chunk));
        out += chunk * esz;
        n -= chunk;
    }
    return hipSuccess;
}

void steps_add(uint64_t steps[3], const uint64_t *limbs, size_t nlimbs)
{
    uint64_t carry = 0;
    for (int i = 0; i < 3; ++i) {
        const uint64_t add = (size_t)i < nlimbs ? limbs[i] : 0;
        const uint64_t s1 = steps[i] + add;
        const uint64_t c1 = s1 < add ? 1 : 0;
        const uint64_t s2 = s1 + carry;
        const uint64_t c2 = s2 < carry ? 1 : 0;
        steps[i] = s2;
        carry = c1 | c2;
    }
}

}  // namespace
}  // namespace mirng

using namespace mirng;

// Declared in the MRG translation unit.
namespace mirng {
hipError_t mrg_plain(const uint32_t st[6], const mirng_distribution *d, uint64_t n,
                     char *out, hipStream_t s);
// spacing_log2: 76 (substreams) or 127 (streams), L'Ecuyer et al. 2002.
hipError_t mrg_substreams(const uint32_t st[6], const mirng_distribution *d,
                          uint64_t first, uint64_t count, uint64_t n_each, char *out,
                          hipStream_t s, int spacing_log2);
}  // namespace mirng

extern "C" {

int32_t mirng_abi_version(void) { return MIRNG_ABI_VERSION; }

mirng_status mirng_device_init(void)
{
    return ensure_device(nullptr) == hipSuccess ? MIRNG_OK : MIRNG_E_DEVICE;
}

mirng_status mirng_philox_config_get(mirng_philox_config *c)
{
    if (!c) return MIRNG_E_INVALID_ARG;
    *c = philox_config();
    return MIRNG_OK;
}

mirng_status mirng_philox_config_set(const mirng_philox_config *c)
{
    if (!c || !philox_config_valid(*c)) return MIRNG_E_INVALID_ARG;
    philox_config() = *c;
    for (int k = kBits; k <= kIcdf64; ++k) philox_config_set_kind(k, -1, nullptr);
    return MIRNG_OK;
}

mirng_status mirng_philox_config_get_kind(int32_t kind, int32_t phase, mirng_philox_config *c)
{
    if (!c || phase < 0 || phase > 3) return MIRNG_E_INVALID_ARG;
    if (!philox_kind_ok(kind)) return MIRNG_E_UNSUPPORTED;
    *c = philox_config_for(kind, (uint32_t)phase);
    return MIRNG_OK;
}

mirng_status mirng_philox_config_set_kind(int32_t kind, int32_t phase,
                                          const mirng_philox_config *c)
{
    if (!philox_kind_ok(kind)) return MIRNG_E_UNSUPPORTED;
    if (phase < -1 || phase > 3 || (c && !philox_config_valid(*c))) return MIRNG_E_INVALID_ARG;
    philox_config_set_kind(kind, phase, c);
    return MIRNG_OK;
}

uint32_t mirng_philox_phase(int32_t kind, uint64_t position, const void *out)
{
    return philox_kind_ok(kind) ? philox_phase(kind, position, (uintptr_t)out) : 0u;
}

const char *mirng_status_string(mirng_status s)
{
    switch (s) {
    case MIRNG_OK: return "ok";
    case MIRNG_E_INVALID_ARG: return "invalid argument";
    case MIRNG_E_UNSUPPORTED: return "unsupported engine type or distribution";
    case MIRNG_E_ALLOC: return "allocation failed";
    case MIRNG_E_LAUNCH: return "kernel launch failed";
    case MIRNG_E_DEVICE: return "no usable gfx950 device";
    case MIRNG_E_CAPACITY: return "request exceeds capacity";
    default: return "unknown status";
    }
}

uint64_t mirng_words_consumed(int32_t engine_type, int32_t kind, uint64_t n)
{
    return words_consumed(engine_type, kind, n);
}

mirng_status mirng_engine_create(int32_t type, uint64_t seed, uint64_t offset,
                                 mirng_engine *out)
{
    if (!out) return MIRNG_E_INVALID_ARG;
    if (type != MIRNG_PHILOX4X32_10 && type != MIRNG_MRG32K3A) return MIRNG_E_UNSUPPORTED;
    mirng_engine e = new (std::nothrow) mirng_engine_s();
    if (!e) return MIRNG_E_ALLOC;
    e->type = type;
    if (type == MIRNG_PHILOX4X32_10) {
        e->key[0] = (uint32_t)seed;
        e->key[1] = (uint32_t)(seed >> 32);
        e->pos = Pos130{{offset, 0, 0}};
    } else {
        mrg_seed_state(seed, e->st);
        mrg_jump(e->st, &offset, 1);
        e->steps[0] = offset;
    }
    *out = e;
    return MIRNG_OK;
}

mirng_status mirng_engine_destroy(mirng_engine e)
{
    delete e;
    return MIRNG_OK;
}

mirng_status mirng_skip_ahead_multi(mirng_engine e, const uint64_t *limbs, size_t nlimbs)
{
    if (!e || nlimbs > 3 || (nlimbs > 0 && !limbs)) return MIRNG_E_INVALID_ARG;
    if (e->type == MIRNG_PHILOX4X32_10) {
        e->pos = pos_add(e->pos, limbs, nlimbs);
    } else {
        mrg_jump(e->st, limbs, nlimbs);
        steps_add(e->steps, limbs, nlimbs);
    }
    return MIRNG_OK;
}

mirng_status mirng_skip_ahead(mirng_engine e, uint64_t n)
{
    return mirng_skip_ahead_multi(e, &n, 1);
}

mirng_status mirng_engine_get_state(mirng_engine e, mirng_state *s)
{
    if (!e || !s) return MIRNG_E_INVALID_ARG;
    std::memset(s, 0, sizeof *s);
    s->engine_type = e->type;
    if (e->type == MIRNG_PHILOX4X32_10) {
        s->words[0] = e->key[0];
        s->words[1] = e->key[1];
        for (int i = 0; i < 3; ++i) s->pos[i] = e->pos.l[i];
    } else {
        for (int i = 0; i < 6; ++i) s->words[i] = e->st[i];
        for (int i = 0; i < 3; ++i) s->pos[i] = e->steps[i];
    }
    return MIRNG_OK;
}

mirng_status mirng_engine_set_state(mirng_engine e, const mirng_state *s)
{
    if (!e || !s || s->engine_type != e->type) return MIRNG_E_INVALID_ARG;
    if (e->type == MIRNG_PHILOX4X32_10) {
        if (s->pos[2] > 3) return MIRNG_E_INVALID_ARG;
        for (int i = 2; i < 6; ++i)
            if (s->words[i] != 0) return MIRNG_E_INVALID_ARG;
        e->key[0] = s->words[0];
        e->key[1] = s->words[1];
        for (int i = 0; i < 3; ++i) e->pos.l[i] = s->pos[i];
    } else {
        for (int i = 0; i < 3; ++i)
            if (s->words[i] >= kM1 || s->words[3 + i] >= kM2) return MIRNG_E_INVALID_ARG;
        if (!(s->words[0] | s->words[1] | s->words[2])) return MIRNG_E_INVALID_ARG;
        if (!(s->words[3] | s->words[4] | s->words[5])) return MIRNG_E_INVALID_ARG;
        for (int i = 0; i < 6; ++i) e->st[i] = s->words[i];
        for (int i = 0; i < 3; ++i) e->steps[i] = s->pos[i];
    }
    return MIRNG_OK;
}

mirng_status mirng_generate(mirng_engine e, const mirng_distribution *d, uint64_t n,
                            void *out, void *stream)
{
    if (!e || !d) return MIRNG_E_INVALID_ARG;
    const mirng_status ds = check_dist(d);
    if (ds != MIRNG_OK) return ds;
    if (n == 0) return MIRNG_OK;
    if (!out) return MIRNG_E_INVALID_ARG;
    if (((uintptr_t)out) % elem_size(d->kind) != 0) return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t consumed = words_consumed(e->type, d->kind, n);
    hipError_t err;
    if (e->type == MIRNG_PHILOX4X32_10) {
        const Pos130 p = e->pos;
        e->pos = pos_add_u64(e->pos, consumed);
        err = philox_plain(e->key, p, d, n, (char *)out, s);
    } else {
        uint32_t st[6];
        std::memcpy(st, e->st, sizeof st);
        mrg_jump(e->st, &consumed, 1);
        steps_add(e->steps, &consumed, 1);
        err = mrg_plain(st, d, n, (char *)out, s);
    }
    return err == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

namespace {

mirng_status spaced(mirng_engine e, const mirng_distribution *d, uint64_t first,
                    uint64_t count, uint64_t n_each, void *out, void *stream, int log2)
{
    if (!e || !d) return MIRNG_E_INVALID_ARG;
    if (e->type != MIRNG_MRG32K3A) return MIRNG_E_UNSUPPORTED;
    const mirng_status ds = check_dist(d);
    if (ds != MIRNG_OK) return ds;
    if (count == 0 || n_each == 0) return MIRNG_OK;
    if (!out) return MIRNG_E_INVALID_ARG;
    if (((uintptr_t)out) % elem_size(d->kind) != 0) return MIRNG_E_INVALID_ARG;
    if (first >= (1ull << 30) || count > (1ull << 30) || first + count > (1ull << 30))
        return MIRNG_E_INVALID_ARG;
    if (ensure_device(nullptr) != hipSuccess) return MIRNG_E_DEVICE;
    hipError_t err = mrg_substreams(e->st, d, first, count, n_each, (char *)out,
                                    (hipStream_t)stream, log2);
    return err == hipSuccess ? MIRNG_OK : MIRNG_E_LAUNCH;
}

}  // namespace

mirng_status mirng_generate_substreams(mirng_engine e, const mirng_distribution *d,
                                       uint64_t first, uint64_t count, uint64_t n_each,
                                       void *out, void *stream)
{
    return spaced(e, d, first, count, n_each, out, stream, 76);
}

mirng_status mirng_generate_streams(mirng_engine e, const mirng_distribution *d,
                                    uint64_t first, uint64_t count, uint64_t n_each,
                                    void *out, void *stream)
{
    return spaced(e, d, first, count, n_each, out, stream, 127);
}

}  // extern "C"
