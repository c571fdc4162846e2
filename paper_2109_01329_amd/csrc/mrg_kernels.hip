// MRG32k3a bulk generation for gfx950 (L'Ecuyer, Oper. Res. 1999), with
// substreams 2^76 steps apart (L'Ecuyer et al., Oper. Res. 2002).  The
// paper serves an MRG-based generator through its oneMKL interface
// (arXiv:2109.01329, Sec. 4.1) but does not define it.
//
// Work layout.  A workgroup of 256 threads owns 256 * q consecutive steps of
// one substream; thread t owns the q steps starting at t * q.  The group's
// start state is A^(c 256 q) A^(s 2^76) S, formed from resident tables of
// base-64 digit powers (at most 4 + 5 matrix-vector products, done by one
// wave); thread t then applies A^(t q) from a resident table and runs q
// sequential steps, L at a time through LDS (the shared pass code).
// Short substreams (each within one group) whose outputs start on 128-byte
// lines are instead laid out four to a group, 64 threads each, so that no
// thread idles and each per-thread jump serves four times as many steps;
// the group's four start states are formed side by side by the lanes of
// one wave (pick_spg).
//
// Line-aligned ranges.  The thread ranges start h0 elements into the
// output, h0 = the elements before its first 128-byte boundary (a cache
// line), so that every pass writes whole lines and no two threads share
// one: the group state is advanced by A^h0 (from the A^(2^k) table), and
// group 0 of a substream writes the h0 head elements at the end, from the
// substream's start state.  Gaussian pairs must not straddle a range
// start, so a paired kind with odd h0 keeps h0 = 0 (its passes then carry
// their last elements to the next pass, see mrg_store_pass).
#include <vector>

#include "internal.hpp"
#include "mrg.hpp"

namespace mirng {

struct MrgLaunch {
    uint32_t st[6];
    uint32_t q;               // steps per thread (multiple of L)
    uint32_t chunks_per_sub;  // workgroups per substream
    uint32_t use_sub;         // 0: plain generate (substream 0 only)
    uint32_t spg;             // substreams per workgroup: 1 or 4
    uint64_t n_each;          // outputs per substream
    uint64_t nsub;            // substreams in the launch
    uint64_t s_first;         // first substream index
    const uint32_t *u_tab;    // A^(t q): [t][comp][9]
    const uint32_t *c_tab;    // A^(k 64^d 256 q): [d][k][comp][9]
    const uint32_t *s_tab;    // A^(k 64^d 2^76): [d][k][comp][9]
    const uint32_t *p_tab;    // A^(2^k): [k][comp][9]
    char *out;
    Epilogue ep;
};

constexpr int kThreads = kMrgThreads;
constexpr int kSDigits = 5;   // substream index < 64^5 = 2^30

namespace {

template <int KIND>
__global__ __launch_bounds__(kThreads) void mrg_kernel(MrgLaunch a)
{
    using S = MrgShape<KIND>;
    __shared__ __attribute__((aligned(16))) char lds[kThreads * S::ROW];
    __shared__ uint32_t wg_state[4][6];
    __shared__ uint32_t wg_head[6];
    if constexpr (uses_lds_tables(KIND)) bm_stage();

    const uint32_t t = threadIdx.x;
    const uint32_t g = blockIdx.x;
    // spg = 4 (substream launches only): the group holds substreams
    // sub .. sub + 3, each one whole range of 64 threads whose outputs
    // start on a 128-byte line, so that the group's rows are contiguous as
    // in a single substream.  Thread t serves substream sub + j from step
    // tq q of it.
    const uint32_t spg = a.spg;
    const uint32_t tps_log2 = spg == 4 ? 6u : 8u;
    const uint32_t j = t >> tps_log2;
    const uint32_t tq = t & ((1u << tps_log2) - 1u);
    const uint64_t sub = spg == 1 ? g / a.chunks_per_sub : (uint64_t)g * spg;
    const uint32_t c = spg == 1 ? (uint32_t)(g - sub * a.chunks_per_sub) : 0u;
    const uint64_t nsub_here = spg == 1 ? 1 : (a.nsub - sub < spg ? a.nsub - sub : spg);
    char *sub_out = a.out + sub * a.n_each * S::ESZ;
    // elements before the substream's first 128-byte boundary (0 when spg = 4)
    uint32_t h0 = (uint32_t)((0u - (uint32_t)(uintptr_t)sub_out) & 127u) / S::ESZ;
    if (paired(KIND) && (h0 & 1u)) h0 = 0;

    if (t < 64) {
        uint32_t v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = a.st[i];
        if (a.use_sub) {
            // lane l forms the state of substream sub + l mod spg
            const uint64_t s = a.s_first + sub + (t & (spg - 1u));
            for (int d = 0; d < kSDigits; ++d) {
                const uint32_t k = (uint32_t)(s >> (6 * d)) & 63u;
                if (k) apply_mat(a.s_tab + (d * 64 + k) * kMatWords, v);
            }
        }
        if (c == 0 && t == 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i) wg_head[i] = v[i];
        }
        for (int d = 0; d < kCDigits; ++d) {
            const uint32_t k = (c >> (6 * d)) & 63u;
            if (k) apply_mat(a.c_tab + (d * 64 + k) * kMatWords, v);
        }
        for (int b = 0; b < 5; ++b)
            if ((h0 >> b) & 1u) apply_mat(a.p_tab + b * kMatWords, v);
        if (t < spg) {
#pragma unroll
            for (int i = 0; i < 6; ++i) wg_state[t][i] = v[i];
        }
    }
    __syncthreads();

    uint32_t v[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = wg_state[j][i];
    if (tq) apply_mat(a.u_tab + tq * kMatWords, v);
    MrgState s = mrg_state(v);

    // the ranges' element 0 is element h0 of the substream
    const uint64_t e_wg = (uint64_t)c * kThreads * a.q;
    const uint64_t n_range = nsub_here * a.n_each;
    const uint64_t n_rest = n_range > h0 ? n_range - h0 : 0;
    char *rng_out = sub_out + (uint64_t)h0 * S::ESZ;
    char *row = mrg_row<KIND>(lds, t);
    const uint32_t h = mrg_head<KIND>(rng_out);
    const uint32_t passes = a.q / S::L;

    bool pending = false;   // the previous pass left its rows' last h elements
    uint64_t e_last = e_wg;
    for (uint32_t pass = 0; pass < passes; ++pass) {
        const uint64_t e0 = e_wg + (uint64_t)pass * S::L;
        if (e0 >= n_rest) break;   // uniform per group
        if (pending) mrg_carry_tail<KIND>(row, h);
        mrg_fill_row<KIND>(s, row, a.ep);
        __syncthreads();
        pending = mrg_store_pass<KIND>(lds, e0, a.q, n_rest, rng_out, a.ep.nt, pending);
        __syncthreads();
        e_last = e0;
    }
    if (pending) mrg_store_tail<KIND>(row, e_last + (uint64_t)t * a.q, h, rng_out);
    if (c == 0 && t == 0 && h0 != 0) {
        // the head: one row of L outputs from the substream's start state
        // (h0 < L), of which the first min(h0, n) are the output's
        uint32_t v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = wg_head[i];
        MrgState hs = mrg_state(v);
        mrg_fill_row<KIND, true>(hs, row, a.ep);
        const uint32_t m = a.n_each < h0 ? (uint32_t)a.n_each : h0;
        for (uint32_t k = 0; k < m; ++k) put_elem<S::ESZ>(sub_out, k, row + k * S::ESZ);
    }
}

// ---------------------------------------------------------------- tables

// Every jump table the MRG32k3a kernels read, in one resident array per
// GPU (a file-scope device array, so that no generate call allocates):
//   per steps-per-thread value q = 16 << i, i < kNumQ: A^(t q) for t < 256
//     (the thread table), then A^(k 64^d 256 q) for d < 4, k < 64 (chunk
//     digits);
//   A^(k 64^d 2^76) and A^(k 64^d 2^127), d < 5, k < 64 (substream and
//     stream digits);
//   A^(2^k), k < 192 (jumps by any 192-bit count).
// Each entry is one matrix per component (18 words).  The host builds the
// array once per process; the library's per-device set-up copies it to
// each GPU (about 310 KB).  The jump tables stay in global memory rather
// than LDS: a thread reads its own A^(t q) once per launch (18 words) and
// the digit tables are read by one wave per group, so staging them in LDS
// would copy far more than any group reads.
constexpr int kNumQ = 7;                                       // q = 16 .. 1024
constexpr size_t kUWords = (size_t)kThreads * kMatWords;       // thread table
constexpr size_t kCWords = (size_t)kCDigits * 64 * kMatWords;  // chunk digits
constexpr size_t kSWords = (size_t)kSDigits * 64 * kMatWords;  // spacing digits
constexpr size_t kQWords = kUWords + kCWords;
constexpr size_t kOffS76 = kNumQ * kQWords;
constexpr size_t kOffS127 = kOffS76 + kSWords;
constexpr size_t kOffPow2 = kOffS127 + kSWords;
constexpr size_t kTabWords = kOffPow2 + (size_t)kPow2Entries * kMatWords;

__device__ __align__(256) uint32_t g_mrg_tables[kTabWords];

void put_mat(std::vector<uint32_t> &dst, size_t idx, const Mat3 &m1, const Mat3 &m2)
{
    for (int i = 0; i < 9; ++i) {
        dst[idx * kMatWords + i] = m1.a[i];
        dst[idx * kMatWords + 9 + i] = m2.a[i];
    }
}

// Powers k * base for k < 64, written at [row][k] from entry `at`.
void digit_row(std::vector<uint32_t> &dst, size_t at, size_t row, const Mat3 &b1,
               const Mat3 &b2)
{
    Mat3 p1 = mat_identity(), p2 = mat_identity();
    for (int k = 0; k < 64; ++k) {
        put_mat(dst, at + row * 64 + k, p1, p2);
        p1 = mat_mul(p1, b1, kM1);
        p2 = mat_mul(p2, b2, kM2);
    }
}

std::vector<uint32_t> build_tables()
{
    std::vector<uint32_t> h(kTabWords);
    for (int i = 0; i < kNumQ; ++i) {
        const int lg = 4 + i;                   // q = 2^lg
        const size_t at = (size_t)i * kQWords / kMatWords;
        const Mat3 &aq1 = mrg_pow2(0, lg), &aq2 = mrg_pow2(1, lg);
        Mat3 p1 = mat_identity(), p2 = mat_identity();
        for (int t = 0; t < kThreads; ++t) {
            put_mat(h, at + t, p1, p2);
            p1 = mat_mul(p1, aq1, kM1);
            p2 = mat_mul(p2, aq2, kM2);
        }
        // chunk digit d: base A^(64^d * 256 * q) = A^(2^(6d + 8 + lg))
        for (int d = 0; d < kCDigits; ++d) {
            const int e = 6 * d + 8 + lg;
            digit_row(h, at + kThreads, d, mrg_pow2(0, e), mrg_pow2(1, e));
        }
    }
    for (int d = 0; d < kSDigits; ++d) {
        digit_row(h, kOffS76 / kMatWords, d, mrg_pow2(0, 76 + 6 * d), mrg_pow2(1, 76 + 6 * d));
        digit_row(h, kOffS127 / kMatWords, d, mrg_pow2(0, 127 + 6 * d),
                  mrg_pow2(1, 127 + 6 * d));
    }
    for (int k = 0; k < kPow2Entries; ++k)
        put_mat(h, kOffPow2 / kMatWords + k, mrg_pow2(0, k), mrg_pow2(1, k));
    return h;
}

const std::vector<uint32_t> &host_tables()
{
    static const std::vector<uint32_t> h = build_tables();
    return h;
}

const uint32_t *g_tab_dev[kMaxDevices];   // device address of g_mrg_tables, per GPU

// Device address of the tables on `dev` (set up by mrg_tables_init).
const uint32_t *tables_of(int dev)
{
    return (dev >= 0 && dev < kMaxDevices) ? g_tab_dev[dev] : nullptr;
}

// The thread and chunk tables of steps-per-thread q (a power of two in
// [16, 1024]) on `dev`.
hipError_t tables_for(int dev, uint32_t q, const uint32_t *&u, const uint32_t *&c)
{
    const uint32_t *base = tables_of(dev);
    int i = 0;
    while (i < kNumQ && (16u << i) != q) ++i;
    if (!base || i == kNumQ) return hipErrorInvalidValue;
    u = base + (size_t)i * kQWords;
    c = u + kUWords;
    return hipSuccess;
}

// Steps per thread: a power of two in [L, 1024] (L = outputs per pass: 32,
// or 16 for FP64) chosen so that a launch has about 2048 workgroups (8 per
// CU) for 4-byte outputs, 16384 for uniform FP64 and 4096 for the FP64
// Gaussians, when the size allows, without leaving half a group idle.  A
// pass writes one 128-byte row per thread, rows q elements apart: uniform
// FP64 outputs, at twice the bytes per step, ran 1.5 times faster with the
// rows 512 bytes apart (q = 64 at 2^28 outputs) than 4 KiB apart (q = 512),
// while 4-byte outputs ran fastest at q = 512, where the per-thread and
// per-group jumps cost least.  The VALU-bound FP64 Gaussians gain more from
// fewer jumps than they lose on the row spacing: q = 256 ran 0.565 against
// 0.606 ms (Box-Muller) and 0.830 against 0.868 ms (inverse CDF) per 2^28
// outputs, q = 128 in between; the 4-byte Gaussians ran slower at q = 1024.
uint32_t pick_q(int kind, uint64_t n_each, uint64_t nsub)
{
    const bool wide = elem_bytes(kind) == 8;
    const uint64_t groups = !wide ? 2048 : (kind == kGauss64 || kind == kIcdf64) ? 4096 : 16384;
    uint32_t q = wide ? 16 : 32;   // L outputs per pass
    while (q < 1024 && (uint64_t)kThreads * q * groups < n_each * nsub &&
           (uint64_t)kThreads * q * 2 <= n_each)
        q <<= 1;
    return q;
}

// Substreams per workgroup for a substream launch whose substreams each
// fit one workgroup of q1 steps per thread (n_each <= 256 q1): 4 when each
// substream is exactly one range of 64 threads of q steps (q a power of two
// in [L, 1024]) whose outputs start on a 128-byte line, else 1.  No thread
// then idles, the per-thread jump A^(t q) serves four times more outputs,
// and one wave forms the four substreams' start states side by side (one
// per lane).  Where one substream already fills its group exactly, four
// are taken only up to the q that measured fastest for plain launches (64
// for FP64 outputs, 512 for 4-byte ones): 65536 x 4096 FP64 ran in 0.37
// instead of 0.54 ms at q = 64, but 16384 x 16384 in 0.40 instead of 0.38
// ms at q = 256.
uint32_t pick_spg(int kind, uint64_t n_each, const char *out, uint32_t q1, uint32_t &q)
{
    const uint32_t esz = (uint32_t)elem_bytes(kind);
    const uint32_t L = 128 / esz;
    if (((uintptr_t)out & 127u) != 0 || (n_each * esz) % 128 != 0 ||
        n_each > (uint64_t)kThreads * q1 || n_each % 64 != 0)
        return 1;
    const uint64_t qq = n_each / 64;
    if (qq < L || qq > 1024 || (qq & (qq - 1)) != 0) return 1;
    if (n_each == (uint64_t)kThreads * q1 && qq > (esz == 8 ? 64u : 512u)) return 1;
    q = (uint32_t)qq;
    return 4;
}

hipError_t launch(const MrgLaunch &a, int kind, uint64_t groups, hipStream_t s)
{
    const dim3 grid((uint32_t)groups), block(kThreads);
    switch (kind) {
    case kBits: hipLaunchKernelGGL(mrg_kernel<kBits>, grid, block, 0, s, a); break;
    case kU32F: hipLaunchKernelGGL(mrg_kernel<kU32F>, grid, block, 0, s, a); break;
    case kU64F: hipLaunchKernelGGL(mrg_kernel<kU64F>, grid, block, 0, s, a); break;
    case kGauss: hipLaunchKernelGGL(mrg_kernel<kGauss>, grid, block, 0, s, a); break;
    case kGauss64: hipLaunchKernelGGL(mrg_kernel<kGauss64>, grid, block, 0, s, a); break;
    case kI32: hipLaunchKernelGGL(mrg_kernel<kI32>, grid, block, 0, s, a); break;
    case kIcdf: hipLaunchKernelGGL(mrg_kernel<kIcdf>, grid, block, 0, s, a); break;
    case kIcdf64: hipLaunchKernelGGL(mrg_kernel<kIcdf64>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Streaming stores for 4-byte outputs; ordinary stores for FP64 outputs,
// which measured faster with them (0.52 against 0.56 ms per 2^28 uniform
// FP64 outputs at q = 512).
void fill_params(MrgLaunch &a, const mirng_distribution *d)
{
    a.ep = epilogue_of(d->kind, d->p0, d->p1, elem_bytes(d->kind) == 8 ? 0 : 1);
}

hipError_t run(const uint32_t st[6], const mirng_distribution *d, uint64_t s_first,
               uint64_t nsub, int spacing_log2, uint64_t n_each, char *out, hipStream_t s)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    const bool use_sub = spacing_log2 > 0;
    uint32_t q = pick_q(d->kind, n_each, nsub);
    const uint32_t spg = use_sub ? pick_spg(d->kind, n_each, out, q, q) : 1u;
    const uint32_t *utab = nullptr, *ctab = nullptr;
    err = tables_for(dev, q, utab, ctab);
    if (err != hipSuccess) return err;
    const uint32_t *stab = nullptr;
    if (use_sub) stab = tables_of(dev) + (spacing_log2 == 76 ? kOffS76 : kOffS127);
    MrgLaunch a{};
    for (int i = 0; i < 6; ++i) a.st[i] = st[i];
    a.q = q;
    const uint64_t per_group = (uint64_t)kThreads * q;
    const uint64_t chunks = (n_each + per_group - 1) / per_group;
    a.chunks_per_sub = (uint32_t)chunks;
    a.use_sub = use_sub ? 1 : 0;
    a.spg = spg;
    a.n_each = n_each;
    a.nsub = nsub;
    a.s_first = s_first;
    a.u_tab = utab;
    a.c_tab = ctab;
    a.s_tab = stab;
    a.p_tab = tables_of(dev) + kOffPow2;
    a.out = out;
    fill_params(a, d);
    // one launch per at most 2^31 groups
    const uint64_t groups = spg == 1 ? chunks * nsub : (nsub + spg - 1) / spg;
    if (groups >= (1ull << 31) || chunks >= (1ull << (6 * kCDigits)))
        return hipErrorInvalidValue;
    return launch(a, d->kind, groups, s);
}

}  // namespace

hipError_t mrg_tables_init(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    const std::vector<uint32_t> &h = host_tables();
    void *p = nullptr;
    hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(g_mrg_tables));
    if (err != hipSuccess) return err;
    err = hipMemcpy(p, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (err != hipSuccess) return err;
    g_tab_dev[dev] = (const uint32_t *)p;
    return hipSuccess;
}

hipError_t mrg_batch_tables(int dev, MrgBatchTables &t)
{
    const uint32_t *base = tables_of(dev);
    if (!base) return hipErrorNotInitialized;
    t.pow2 = base + kOffPow2;
    hipError_t err = tables_for(dev, 32 * kBatchMrgPasses, t.u_tab4, t.c_tab4);
    if (err == hipSuccess) err = tables_for(dev, 16 * kBatchMrgPasses, t.u_tab8, t.c_tab8);
    return err;
}

hipError_t mrg_plain(const uint32_t st[6], const mirng_distribution *d, uint64_t n,
                     char *out, hipStream_t s)
{
    return run(st, d, 0, 1, 0, n, out, s);
}

hipError_t mrg_substreams(const uint32_t st[6], const mirng_distribution *d,
                          uint64_t first, uint64_t count, uint64_t n_each, char *out,
                          hipStream_t s, int spacing_log2)
{
    if (first + count > (1ull << (6 * kSDigits))) return hipErrorInvalidValue;
    if (spacing_log2 != 76 && spacing_log2 != 127) return hipErrorInvalidValue;
    return run(st, d, first, count, spacing_log2, n_each, out, s);
}

}  // namespace mirng
