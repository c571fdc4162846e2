// Host-side engine arithmetic: Philox word positions (130-bit) and
// MRG32k3a jumps by 3x3 matrix powers modulo m (L'Ecuyer 1999; substream
// spacing 2^76 of L'Ecuyer et al. 2002).
#include <mutex>

#include "internal.hpp"

namespace mirng {

// ---------------------------------------------------------------- Philox

Pos130 pos_add(Pos130 p, const uint64_t *limbs, size_t nlimbs)
{
    uint64_t carry = 0;
    for (int i = 0; i < 3; ++i) {
        const uint64_t add = (size_t)i < nlimbs ? limbs[i] : 0;
        const uint64_t s1 = p.l[i] + add;
        const uint64_t c1 = s1 < add ? 1 : 0;
        const uint64_t s2 = s1 + carry;
        const uint64_t c2 = s2 < carry ? 1 : 0;
        p.l[i] = s2;
        carry = c1 | c2;
    }
    p.l[2] &= 3u;   // modulo 2^130
    return p;
}

Pos130 pos_add_u64(Pos130 p, uint64_t n)
{
    return pos_add(p, &n, 1);
}

Pos130 pos_sub_u64(Pos130 p, uint64_t n)
{
    // p - n mod 2^130 == p + (2^130 - n)
    const uint64_t neg[3] = {~n + 1, n ? ~0ull : 0ull, n ? 3ull : 0ull};
    return pos_add(p, neg, 3);
}

// ---------------------------------------------------------------- MRG32k3a

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (a * b) % m;   // a, b < 2^32: the product fits in 64 bits
}

Mat3 mat_identity()
{
    Mat3 r{};
    r.a[0] = r.a[4] = r.a[8] = 1;
    return r;
}

Mat3 mat_mul(const Mat3 &x, const Mat3 &y, uint64_t m)
{
    Mat3 r{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            uint64_t s = 0;
            for (int k = 0; k < 3; ++k) s += mulmod(x.a[3 * i + k], y.a[3 * k + j], m);
            r.a[3 * i + j] = (uint32_t)(s % m);
        }
    return r;
}

void mat_vec(const Mat3 &x, const uint32_t v[3], uint64_t m, uint32_t out[3])
{
    uint32_t r[3];
    for (int i = 0; i < 3; ++i) {
        uint64_t s = 0;
        for (int k = 0; k < 3; ++k) s += mulmod(x.a[3 * i + k], v[k], m);
        r[i] = (uint32_t)(s % m);
    }
    out[0] = r[0]; out[1] = r[1]; out[2] = r[2];
}

Mat3 mat_pow_u64(const Mat3 &x, uint64_t n, uint64_t m)
{
    Mat3 r = mat_identity(), b = x;
    while (n) {
        if (n & 1) r = mat_mul(r, b, m);
        b = mat_mul(b, b, m);
        n >>= 1;
    }
    return r;
}

const Mat3 &mrg_a1()
{
    static const Mat3 a = {{0, 1, 0, 0, 0, 1, (uint32_t)(kM1 - kA13), (uint32_t)kA12, 0}};
    return a;
}

const Mat3 &mrg_a2()
{
    static const Mat3 a = {{0, 1, 0, 0, 0, 1, (uint32_t)(kM2 - kA23), 0, (uint32_t)kA21}};
    return a;
}

namespace {
struct Pow2Table {
    Mat3 t[2][192];
    Pow2Table()
    {
        t[0][0] = mrg_a1();
        t[1][0] = mrg_a2();
        for (int k = 1; k < 192; ++k) {
            t[0][k] = mat_mul(t[0][k - 1], t[0][k - 1], kM1);
            t[1][k] = mat_mul(t[1][k - 1], t[1][k - 1], kM2);
        }
    }
};
const Pow2Table &pow2_table()
{
    static const Pow2Table table;   // thread-safe static initialisation
    return table;
}
}  // namespace

const Mat3 &mrg_pow2(int comp, int k)
{
    return pow2_table().t[comp][k];
}

void mrg_jump(uint32_t st[6], const uint64_t *limbs, size_t nlimbs)
{
    const Pow2Table &tb = pow2_table();
    for (size_t i = 0; i < nlimbs && i < 3; ++i) {
        uint64_t w = limbs[i];
        for (int b = 0; w; ++b, w >>= 1) {
            if (!(w & 1)) continue;
            const int k = (int)i * 64 + b;
            mat_vec(tb.t[0][k], st, kM1, st);
            mat_vec(tb.t[1][k], st + 3, kM2, st + 3);
        }
    }
}

void mrg_seed_state(uint64_t seed, uint32_t st[6])
{
    st[0] = (uint32_t)((seed & 0xFFFFFFFFull) % kM1);
    st[1] = 1;
    st[2] = 1;
    st[3] = (uint32_t)((seed >> 32) % kM2);
    st[4] = 1;
    st[5] = 1;
}

uint64_t words_consumed(int engine_type, int kind, uint64_t n)
{
    switch (kind) {
    case kBits:
    case kU32F:
    case kI32:
    case kIcdf: return n;
    case kU64F:
    case kIcdf64: return engine_type == MIRNG_PHILOX4X32_10 ? 2 * n : n;
    case kGauss: return 2 * ((n + 1) / 2);
    case kGauss64: return (engine_type == MIRNG_PHILOX4X32_10 ? 4 : 2) * ((n + 1) / 2);
    default: return 0;
    }
}

}  // namespace mirng
