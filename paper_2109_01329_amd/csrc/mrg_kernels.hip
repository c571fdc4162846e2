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
// sequential steps.  Each pass of L steps goes through LDS (rows padded by
// 16 bytes so 8 consecutive lanes hit distinct banks) and is written back
// as 128-byte segments, one per thread, with 16-byte stores.
//
// The recurrence runs in FP64: all products are below 2^53 and exact, the
// quotient by m is estimated by a multiply with 1/m biased by -2^-30 so that
// the floor is never too large, and one conditional subtraction finishes
// the reduction.  The results are the exact integers of the definition.
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "transforms.hpp"

namespace mirng {

struct MrgLaunch {
    uint32_t st[6];
    uint32_t q;               // steps per thread (multiple of L)
    uint32_t chunks_per_sub;  // workgroups per substream
    uint32_t use_sub;         // 0: plain generate (substream 0 only)
    uint32_t vec_ok;          // output base is 16-byte aligned
    uint64_t n_each;          // outputs per substream
    uint64_t s_first;         // first substream index
    const uint32_t *u_tab;    // A^(t q): [t][comp][9]
    const uint32_t *c_tab;    // A^(k 64^d 256 q): [d][k][comp][9]
    const uint32_t *s_tab;    // A^(k 64^d 2^76): [d][k][comp][9]
    char *out;
    int32_t ranged;
    float a32, d32;
    double a64, d64;
};

constexpr int kThreads = 256;
constexpr int kCDigits = 4;   // chunk index < 64^4 = 2^24
constexpr int kSDigits = 5;   // substream index < 64^5 = 2^30
constexpr int kMatWords = 18; // two 3x3 matrices

namespace {

// x mod m1 for any 64-bit x (2^32 = 209 mod m1).
__device__ __forceinline__ uint32_t red_m1(uint64_t x)
{
    x = (x >> 32) * 209u + (x & 0xFFFFFFFFull);
    x = (x >> 32) * 209u + (x & 0xFFFFFFFFull);
    return (uint32_t)(x >= kM1 ? x - kM1 : x);
}

// x mod m2 for any 64-bit x (2^32 = 22853 mod m2).
__device__ __forceinline__ uint32_t red_m2(uint64_t x)
{
    x = (x >> 32) * 22853u + (x & 0xFFFFFFFFull);
    x = (x >> 32) * 22853u + (x & 0xFFFFFFFFull);
    return (uint32_t)(x >= kM2 ? x - kM2 : x);
}

// v <- M v for both components; M points at 18 words (comp 0 then comp 1).
__device__ __forceinline__ void apply_mat(const uint32_t *M, uint32_t v[6])
{
    uint32_t r[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint64_t a = red_m1((uint64_t)M[3 * i] * v[0]) +
                           (uint64_t)red_m1((uint64_t)M[3 * i + 1] * v[1]) +
                           red_m1((uint64_t)M[3 * i + 2] * v[2]);
        r[i] = red_m1(a);
        const uint64_t b = red_m2((uint64_t)M[9 + 3 * i] * v[3]) +
                           (uint64_t)red_m2((uint64_t)M[9 + 3 * i + 1] * v[4]) +
                           red_m2((uint64_t)M[9 + 3 * i + 2] * v[5]);
        r[3 + i] = red_m2(b);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = r[i];
}

constexpr double kM1d = 4294967087.0;
constexpr double kM2d = 4294944443.0;
constexpr double kInvM1 = 1.0 / 4294967087.0;
constexpr double kInvM2 = 1.0 / 4294944443.0;
constexpr double kNorm = 1.0 / 4294967088.0;   // 1 / (m1 + 1), rounded once

struct MrgState {
    double a0, a1, a2;   // x1[n-3], x1[n-2], x1[n-1]
    double b0, b1, b2;   // x2[n-3], x2[n-2], x2[n-1]
};

// One step; returns the combined output y in [1, m1] as an exact double.
__device__ __forceinline__ double mrg_step(MrgState &s)
{
    double p1 = __builtin_fma(1403580.0, s.a1, -810728.0 * s.a0);
    const double k1 = __builtin_floor(__builtin_fma(p1, kInvM1, -0x1p-30));
    p1 = __builtin_fma(-k1, kM1d, p1);
    p1 = (p1 >= kM1d) ? p1 - kM1d : p1;
    double p2 = __builtin_fma(527612.0, s.b2, -1370589.0 * s.b0);
    const double k2 = __builtin_floor(__builtin_fma(p2, kInvM2, -0x1p-30));
    p2 = __builtin_fma(-k2, kM2d, p2);
    p2 = (p2 >= kM2d) ? p2 - kM2d : p2;
    s.a0 = s.a1; s.a1 = s.a2; s.a2 = p1;
    s.b0 = s.b1; s.b1 = s.b2; s.b2 = p2;
    const double y = p1 - p2;
    return (p1 <= p2) ? y + kM1d : y;
}

__device__ __forceinline__ float y_to_u01f(double y)
{
    return (float)(__builtin_floor(y * 0x1p-8) * 0x1p-24);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void mrg_kernel(MrgLaunch a)
{
    constexpr int ESZ = KIND == kU64F ? 8 : 4;
    constexpr int L = 128 / ESZ;           // outputs per thread per pass
    constexpr int ROW = L * ESZ + 16;      // padded LDS row, bytes
    constexpr int VPR = L * ESZ / 16;      // 16-byte vectors per row
    constexpr int EPV = 16 / ESZ;          // elements per vector
    __shared__ __attribute__((aligned(16))) char lds[kThreads * ROW];
    __shared__ uint32_t wg_state[6];

    const uint32_t t = threadIdx.x;
    const uint32_t g = blockIdx.x;
    const uint32_t sub = g / a.chunks_per_sub;
    const uint32_t c = g - sub * a.chunks_per_sub;

    if (t < 64) {
        uint32_t v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) v[i] = a.st[i];
        if (a.use_sub) {
            const uint64_t s = a.s_first + sub;
            for (int d = 0; d < kSDigits; ++d) {
                const uint32_t k = (uint32_t)(s >> (6 * d)) & 63u;
                if (k) apply_mat(a.s_tab + (d * 64 + k) * kMatWords, v);
            }
        }
        for (int d = 0; d < kCDigits; ++d) {
            const uint32_t k = (c >> (6 * d)) & 63u;
            if (k) apply_mat(a.c_tab + (d * 64 + k) * kMatWords, v);
        }
        if (t == 0) {
#pragma unroll
            for (int i = 0; i < 6; ++i) wg_state[i] = v[i];
        }
    }
    __syncthreads();

    uint32_t v[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = wg_state[i];
    if (t) apply_mat(a.u_tab + t * kMatWords, v);
    MrgState s{(double)v[0], (double)v[1], (double)v[2],
               (double)v[3], (double)v[4], (double)v[5]};

    const uint64_t e_wg = (uint64_t)c * kThreads * a.q;
    char *sub_out = a.out + (uint64_t)sub * a.n_each * ESZ;
    char *row = lds + t * ROW;
    const uint32_t passes = a.q / L;

    for (uint32_t pass = 0; pass < passes; ++pass) {
        if (e_wg + (uint64_t)pass * L >= a.n_each) break;   // uniform per group
        // generate L outputs into this thread's LDS row
#pragma unroll
        for (int l = 0; l < L; l += EPV) {
            u32x4 pk;
            if constexpr (KIND == kBits) {
                pk.x = (uint32_t)mrg_step(s); pk.y = (uint32_t)mrg_step(s);
                pk.z = (uint32_t)mrg_step(s); pk.w = (uint32_t)mrg_step(s);
            } else if constexpr (KIND == kU32F) {
                f32x4 f;
                f.x = y_to_u01f(mrg_step(s)); f.y = y_to_u01f(mrg_step(s));
                f.z = y_to_u01f(mrg_step(s)); f.w = y_to_u01f(mrg_step(s));
                if (a.ranged) {
                    f.x = __builtin_fmaf(f.x, a.d32, a.a32);
                    f.y = __builtin_fmaf(f.y, a.d32, a.a32);
                    f.z = __builtin_fmaf(f.z, a.d32, a.a32);
                    f.w = __builtin_fmaf(f.w, a.d32, a.a32);
                }
                pk = __builtin_bit_cast(u32x4, f);
            } else if constexpr (KIND == kU64F) {
                f64x2 d;
                d.x = mrg_step(s) * kNorm;
                d.y = mrg_step(s) * kNorm;
                if (a.ranged) {
                    d.x = __builtin_fma(d.x, a.d64, a.a64);
                    d.y = __builtin_fma(d.y, a.d64, a.a64);
                }
                pk = __builtin_bit_cast(u32x4, d);
            } else {
                const uint32_t w0 = (uint32_t)mrg_step(s);
                const uint32_t w1 = (uint32_t)mrg_step(s);
                const uint32_t w2 = (uint32_t)mrg_step(s);
                const uint32_t w3 = (uint32_t)mrg_step(s);
                f32x4 f;
                f.xy = box_muller(w0, w1);
                f.zw = box_muller(w2, w3);
                if (a.ranged) {
                    f.x = __builtin_fmaf(f.x, a.d32, a.a32);
                    f.y = __builtin_fmaf(f.y, a.d32, a.a32);
                    f.z = __builtin_fmaf(f.z, a.d32, a.a32);
                    f.w = __builtin_fmaf(f.w, a.d32, a.a32);
                }
                pk = __builtin_bit_cast(u32x4, f);
            }
            *(u32x4 *)(row + (l / EPV) * 16) = pk;
        }
        __syncthreads();
        // write the group's 256 segments of L outputs back to memory
        for (uint32_t vi = t; vi < (uint32_t)(kThreads * VPR); vi += kThreads) {
            const uint32_t seg = vi / VPR;
            const uint32_t ch = vi - seg * VPR;
            const uint64_t e = e_wg + (uint64_t)seg * a.q + (uint64_t)pass * L +
                               (uint64_t)ch * EPV;
            const u32x4 val = *(const u32x4 *)(lds + seg * ROW + ch * 16);
            char *dst = sub_out + e * ESZ;
            if (a.vec_ok && e + EPV <= a.n_each) {
                __builtin_nontemporal_store(val, (u32x4 *)dst);
            } else {
#pragma unroll
                for (int j = 0; j < EPV; ++j) {
                    if (e + j < a.n_each) {
                        if constexpr (ESZ == 4) {
                            ((uint32_t *)dst)[j] = val[j];
                        } else {
                            ((uint64_t *)dst)[j] =
                                ((uint64_t)val[2 * j + 1] << 32) | val[2 * j];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tables

void put_mat(std::vector<uint32_t> &dst, size_t idx, const Mat3 &m1, const Mat3 &m2)
{
    for (int i = 0; i < 9; ++i) {
        dst[idx * kMatWords + i] = m1.a[i];
        dst[idx * kMatWords + 9 + i] = m2.a[i];
    }
}

// Powers k * base for k < 64, written at [row][k].
void digit_row(std::vector<uint32_t> &dst, size_t row, const Mat3 &b1, const Mat3 &b2)
{
    Mat3 p1 = mat_identity(), p2 = mat_identity();
    for (int k = 0; k < 64; ++k) {
        put_mat(dst, row * 64 + k, p1, p2);
        p1 = mat_mul(p1, b1, kM1);
        p2 = mat_mul(p2, b2, kM2);
    }
}

// A^n for n = 2^e * m with small m, through the power-of-two table.
void pow_shifted(uint64_t mult, int shift, Mat3 &r1, Mat3 &r2)
{
    r1 = mat_identity();
    r2 = mat_identity();
    for (int b = 0; mult; ++b, mult >>= 1) {
        if (mult & 1) {
            r1 = mat_mul(r1, mrg_pow2(0, b + shift), kM1);
            r2 = mat_mul(r2, mrg_pow2(1, b + shift), kM2);
        }
    }
}

struct DeviceTables {
    uint32_t *u = nullptr;   // per q
    uint32_t *c = nullptr;   // per q
};

std::mutex g_tab_mu;
std::map<std::pair<int, uint32_t>, DeviceTables> g_q_tables;
std::map<int, uint32_t *> g_sub_tables;

hipError_t upload(const std::vector<uint32_t> &h, uint32_t **d)
{
    hipError_t err = hipMalloc((void **)d, h.size() * sizeof(uint32_t));
    if (err != hipSuccess) return err;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
}

hipError_t tables_for(int dev, uint32_t q, DeviceTables &out)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_q_tables.find({dev, q});
    if (it != g_q_tables.end()) {
        out = it->second;
        return hipSuccess;
    }
    // q is a power of two: A^q from the 2^k table
    int lg = 0;
    while ((1u << lg) < q) ++lg;
    const Mat3 &aq1 = mrg_pow2(0, lg), &aq2 = mrg_pow2(1, lg);
    std::vector<uint32_t> u((size_t)kThreads * kMatWords);
    Mat3 p1 = mat_identity(), p2 = mat_identity();
    for (int t = 0; t < kThreads; ++t) {
        put_mat(u, t, p1, p2);
        p1 = mat_mul(p1, aq1, kM1);
        p2 = mat_mul(p2, aq2, kM2);
    }
    std::vector<uint32_t> c((size_t)kCDigits * 64 * kMatWords);
    for (int d = 0; d < kCDigits; ++d) {
        // base = A^(64^d * 256 * q) = A^(2^(6d + 8 + lg))
        const int e = 6 * d + 8 + lg;
        digit_row(c, d, mrg_pow2(0, e), mrg_pow2(1, e));
    }
    DeviceTables t;
    hipError_t err = upload(u, &t.u);
    if (err == hipSuccess) err = upload(c, &t.c);
    if (err != hipSuccess) return err;
    g_q_tables[{dev, q}] = t;
    out = t;
    return hipSuccess;
}

hipError_t substream_table(int dev, uint32_t **out)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_sub_tables.find(dev);
    if (it != g_sub_tables.end()) {
        *out = it->second;
        return hipSuccess;
    }
    std::vector<uint32_t> s((size_t)kSDigits * 64 * kMatWords);
    for (int d = 0; d < kSDigits; ++d) {
        const int e = 76 + 6 * d;   // 64^d * 2^76
        digit_row(s, d, mrg_pow2(0, e), mrg_pow2(1, e));
    }
    uint32_t *ptr = nullptr;
    hipError_t err = upload(s, &ptr);
    if (err != hipSuccess) return err;
    g_sub_tables[dev] = ptr;
    *out = ptr;
    return hipSuccess;
}

// Steps per thread: a power of two in [L, 1024] (L = outputs per pass: 32,
// or 16 for FP64) chosen so that a launch has about 2048 workgroups (8 per
// CU) when the size allows, without leaving half a group idle.
uint32_t pick_q(int kind, uint64_t n_each, uint64_t nsub)
{
    uint32_t q = kind == kU64F ? 16 : 32;
    while (q < 1024 && (uint64_t)kThreads * q * 2048 < n_each * nsub &&
           (uint64_t)kThreads * q * 2 <= n_each)
        q <<= 1;
    return q;
}

hipError_t launch(const MrgLaunch &a, int kind, uint64_t groups, hipStream_t s)
{
    const dim3 grid((uint32_t)groups), block(kThreads);
    switch (kind) {
    case kBits: hipLaunchKernelGGL(mrg_kernel<kBits>, grid, block, 0, s, a); break;
    case kU32F: hipLaunchKernelGGL(mrg_kernel<kU32F>, grid, block, 0, s, a); break;
    case kU64F: hipLaunchKernelGGL(mrg_kernel<kU64F>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(mrg_kernel<kGauss>, grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

void fill_params(MrgLaunch &a, const mirng_distribution *d)
{
    a.ranged = (d->kind == kBits || (d->p0 == 0.0 && d->p1 == 1.0)) ? 0 : 1;
    if (d->kind == kU64F) {
        a.a64 = d->p0;
        a.d64 = d->p1 - d->p0;
    } else if (d->kind == kGauss) {
        a.a32 = (float)d->p0;
        a.d32 = (float)d->p1;
    } else {
        a.a32 = (float)d->p0;
        a.d32 = (float)(d->p1 - d->p0);
    }
}

hipError_t run(const uint32_t st[6], const mirng_distribution *d, uint64_t s_first,
               uint64_t nsub, bool use_sub, uint64_t n_each, char *out, hipStream_t s)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    const uint32_t q = pick_q(d->kind, n_each, nsub);
    DeviceTables tb;
    err = tables_for(dev, q, tb);
    if (err != hipSuccess) return err;
    uint32_t *stab = nullptr;
    if (use_sub) {
        err = substream_table(dev, &stab);
        if (err != hipSuccess) return err;
    }
    MrgLaunch a{};
    for (int i = 0; i < 6; ++i) a.st[i] = st[i];
    a.q = q;
    const uint64_t per_group = (uint64_t)kThreads * q;
    const uint64_t chunks = (n_each + per_group - 1) / per_group;
    a.chunks_per_sub = (uint32_t)chunks;
    a.use_sub = use_sub ? 1 : 0;
    // 16-byte stores need every substream's start on the 16-byte grid
    const uint64_t esz = d->kind == kU64F ? 8 : 4;
    a.vec_ok = ((uintptr_t)out & 15u) == 0 && (!use_sub || (n_each * esz) % 16 == 0) ? 1 : 0;
    a.n_each = n_each;
    a.s_first = s_first;
    a.u_tab = tb.u;
    a.c_tab = tb.c;
    a.s_tab = stab;
    a.out = out;
    fill_params(a, d);
    // one launch per at most 2^31 groups
    const uint64_t groups = chunks * nsub;
    if (groups >= (1ull << 31) || chunks >= (1ull << (6 * kCDigits)))
        return hipErrorInvalidValue;
    return launch(a, d->kind, groups, s);
}

}  // namespace

hipError_t mrg_plain(const uint32_t st[6], const mirng_distribution *d, uint64_t n,
                     char *out, hipStream_t s)
{
    return run(st, d, 0, 1, false, n, out, s);
}

hipError_t mrg_substreams(const uint32_t st[6], const mirng_distribution *d,
                          uint64_t first, uint64_t count, uint64_t n_each, char *out,
                          hipStream_t s)
{
    if (first + count > (1ull << (6 * kSDigits))) return hipErrorInvalidValue;
    return run(st, d, first, count, true, n_each, out, s);
}

}  // namespace mirng
