/*
 * CPU oracle for the mirng hot path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load, call or execute anything in this directory.  The GPU library never
 * links it and shares no code, header, table or constant with it.
 *
 * What it computes: the plain, sequential definition of every value the GPU
 * path produces, in definition order, scalar code, no blocking or fusion.
 *
 * Sources.  The paper (Pascuzzi & Goli, arXiv:2109.01329) names the two
 * engine families it serves -- Philox- and MRG-based generators (Sec. 4.1)
 * and Philox4x32x10 for its measurements (Sec. 7) -- and the oneMKL-style
 * distributions with a range (a, b) or (mean, stddev) (Sec. 4.1), plus the
 * range transform r * (b - a) + a applied after generation (Sec. 4.3,
 * transform listing).  It does not define the engines; those come from:
 *   [S11] Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 *         1, 2, 3", SC'11 (the Philox-4xW bijection, R = 10 rounds).
 *   [L99] L'Ecuyer, "Good parameters and implementations for combined
 *         multiple recursive random number generators", Oper. Res. 47(1),
 *         1999 (MRG32k3a: moduli, multipliers, combination, output scale).
 *   [L02] L'Ecuyer, Simard, Chen, Kelton, Oper. Res. 50(6), 2002
 *         (substreams 2^76 steps apart).
 *   [BM58] Box & Muller, Ann. Math. Stat. 29, 1958.
 * Where the paper is silent the project's readings are used; each is named
 * at its use (R-numbers) and listed in the design notes.
 *
 * Parity status per function is stated at each definition ("pinned by").
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC (no FMA
 * contraction, so every rounding below is the one written).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------
 * Philox-4xW, [S11].
 *
 * One round maps counter (x0,x1,x2,x3) with round key (k0,k1) to
 *   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0)),
 * where hi/lo are the upper/lower W bits of the 2W-bit product.  Between
 * rounds the key is bumped by the Weyl constants (W0, W1).  Ten rounds; the
 * output is the final counter in order.
 *
 * The round body is written once as a macro and instantiated for W = 32
 * (the engine) and W = 64.  The W = 64 instance exists so that the shared
 * round structure can be pinned against numpy's Philox4x64-10, which is an
 * independent implementation of the same bijection (tests/).
 * ---------------------------------------------------------------------- */

/* Multipliers of [S11] for Philox-4x32 and Philox-4x64. */
#define PHILOX_M4x32_0 0xD2511F53u
#define PHILOX_M4x32_1 0xCD9E8D57u
#define PHILOX_M4x64_0 0xD2E7470EE14C6C93ull
#define PHILOX_M4x64_1 0xCA5A826395121157ull
/* Weyl key increments of [S11]: leading bits of the fractional parts of
 * the golden ratio and of sqrt(3) - 1 (closed forms pinned in tests/). */
#define PHILOX_W32_0 0x9E3779B9u
#define PHILOX_W32_1 0xBB67AE85u
#define PHILOX_W64_0 0x9E3779B97F4A7C15ull
#define PHILOX_W64_1 0xBB67AE8584CAA73Bull

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    u128 p = (u128)a * (u128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define PHILOX4_BIJECTION(NAME, T, MULHILO, M0, M1, W0, W1)                  \
    void NAME(const T ctr[4], const T key[2], int rounds, T out[4])          \
    {                                                                        \
        T x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];                \
        T k0 = key[0], k1 = key[1];                                          \
        for (int r = 0; r < rounds; ++r) {                                   \
            if (r > 0) { k0 = (T)(k0 + (W0)); k1 = (T)(k1 + (W1)); }         \
            T hi0, lo0, hi1, lo1;                                            \
            MULHILO((M0), x0, &hi0, &lo0);                                   \
            MULHILO((M1), x2, &hi1, &lo1);                                   \
            T y0 = hi1 ^ x1 ^ k0;                                            \
            T y1 = lo1;                                                      \
            T y2 = hi0 ^ x3 ^ k1;                                            \
            T y3 = lo0;                                                      \
            x0 = y0; x1 = y1; x2 = y2; x3 = y3;                              \
        }                                                                    \
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;                  \
    }

/* Philox4x32 with an explicit round count (10 for the engine); pinned by:
 * shared round structure vs numpy Philox4x64-10, Weyl constants vs closed
 * form; multipliers from [S11] only (see the design notes). */
PHILOX4_BIJECTION(orc_philox4x32, uint32_t, mulhilo32,
                  PHILOX_M4x32_0, PHILOX_M4x32_1, PHILOX_W32_0, PHILOX_W32_1)
/* Philox4x64 instance: exists only to pin the shared round structure. */
PHILOX4_BIJECTION(orc_philox4x64, uint64_t, mulhilo64,
                  PHILOX_M4x64_0, PHILOX_M4x64_1, PHILOX_W64_0, PHILOX_W64_1)

void orc_philox_constants(uint64_t out[8])
{
    out[0] = PHILOX_M4x32_0; out[1] = PHILOX_M4x32_1;
    out[2] = PHILOX_W32_0;   out[3] = PHILOX_W32_1;
    out[4] = PHILOX_M4x64_0; out[5] = PHILOX_M4x64_1;
    out[6] = PHILOX_W64_0;   out[7] = PHILOX_W64_1;
}

/* Word stream of the Philox engine (readings R2-R5).
 * Engine key (k0, k1) = (lo32(seed), hi32(seed)).  Word position p is a
 * 130-bit integer given as three little-endian 64-bit limbs (pos[2] < 4).
 * Word p is word (p mod 4) of the output of the 128-bit counter floor(p/4)
 * written as four little-endian 32-bit words.  out[i] = word (p + i) mod
 * 2^130.  Pinned by: position arithmetic vs Python big integers (tests/). */
void orc_philox_words(uint32_t k0, uint32_t k1, const uint64_t pos[3],
                      uint64_t n, uint32_t *out)
{
    uint64_t lo = pos[0], mid = pos[1], top = pos[2] & 3u;
    uint32_t key[2] = {k0, k1};
    uint32_t blk[4];
    int have = 0;
    for (uint64_t i = 0; i < n; ++i) {
        unsigned lane = (unsigned)(lo & 3u);
        if (!have || lane == 0) {
            /* counter = floor(p / 4) over the 130-bit position */
            uint32_t ctr[4];
            uint64_t c_lo = (lo >> 2) | (mid << 62);
            uint64_t c_hi = (mid >> 2) | (top << 62);
            ctr[0] = (uint32_t)c_lo; ctr[1] = (uint32_t)(c_lo >> 32);
            ctr[2] = (uint32_t)c_hi; ctr[3] = (uint32_t)(c_hi >> 32);
            orc_philox4x32(ctr, key, 10, blk);
            have = 1;
        }
        out[i] = blk[lane];
        /* p += 1 modulo 2^130 */
        lo += 1;
        if (lo == 0) {
            mid += 1;
            if (mid == 0) top = (top + 1) & 3u;
        }
    }
}

/* ------------------------------------------------------------------------
 * MRG32k3a, [L99].
 * Component 1: x1[n] = (1403580 x1[n-2] - 810728 x1[n-3]) mod m1.
 * Component 2: x2[n] = (527612 x2[n-1] - 1370589 x2[n-3]) mod m2.
 * State words are (x[n-3], x[n-2], x[n-1]) for each component.
 * Combined integer output y[n] = x1[n] - x2[n] if x1[n] > x2[n], else
 * x1[n] - x2[n] + m1, so y is in [1, m1] (reading R9: step, then output).
 * ---------------------------------------------------------------------- */
#define MRG_M1 4294967087ull
#define MRG_M2 4294944443ull
#define MRG_A12 1403580ull
#define MRG_A13 810728ull
#define MRG_A21 527612ull
#define MRG_A23 1370589ull

void orc_mrg_constants(uint64_t out[6])
{
    out[0] = MRG_M1; out[1] = MRG_M2;
    out[2] = MRG_A12; out[3] = MRG_A13; out[4] = MRG_A21; out[5] = MRG_A23;
}

/* Seeding (reading R8): x1 = (lo32(seed) mod m1, 1, 1),
 * x2 = (hi32(seed) mod m2, 1, 1) as (x[-3], x[-2], x[-1]). */
void orc_mrg_seed(uint64_t seed, uint64_t st[6])
{
    st[0] = (seed & 0xFFFFFFFFull) % MRG_M1; st[1] = 1; st[2] = 1;
    st[3] = (seed >> 32) % MRG_M2;          st[4] = 1; st[5] = 1;
}

/* One step of the recurrence; returns the combined output y in [1, m1].
 * Pinned by: primitivity of both characteristic polynomials (full period
 * m^3 - 1 of [L99]) and brute force against the jump (tests/). */
uint32_t orc_mrg_step(uint64_t st[6])
{
    int64_t p1 = (int64_t)(MRG_A12 * st[1]) - (int64_t)(MRG_A13 * st[0]);
    p1 %= (int64_t)MRG_M1;
    if (p1 < 0) p1 += (int64_t)MRG_M1;
    int64_t p2 = (int64_t)(MRG_A21 * st[5]) - (int64_t)(MRG_A23 * st[3]);
    p2 %= (int64_t)MRG_M2;
    if (p2 < 0) p2 += (int64_t)MRG_M2;
    st[0] = st[1]; st[1] = st[2]; st[2] = (uint64_t)p1;
    st[3] = st[4]; st[4] = st[5]; st[5] = (uint64_t)p2;
    int64_t y = p1 - p2;
    if (p1 <= p2) y += (int64_t)MRG_M1;
    return (uint32_t)y;
}

void orc_mrg_words(uint64_t st[6], uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = orc_mrg_step(st);
}

/* Jump ahead by n steps with the polynomial method: for a recurrence with
 * characteristic polynomial P, t^n = c0 + c1 t + c2 t^2 (mod P, m) gives
 * x[k+n] = c0 x[k] + c1 x[k+1] + c2 x[k+2].  This is a different algorithm
 * from the matrix powers the GPU library uses.  n is a 192-bit integer in
 * three little-endian 64-bit limbs.  P1(t) = t^3 - 1403580 t + 810728,
 * P2(t) = t^3 - 527612 t^2 + 1370589. */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((u128)a * (u128)b) % m);
}

/* r = a * b mod (t^3 - (e2 t^2 + e1 t + e0)), coefficients mod m.
 * The reduction rule is t^3 = e2 t^2 + e1 t + e0. */
static void polymulmod(const uint64_t a[3], const uint64_t b[3],
                       const uint64_t e[3], uint64_t m, uint64_t r[3])
{
    uint64_t prod[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            prod[i + j] = (prod[i + j] + mulmod(a[i], b[j], m)) % m;
    /* fold degree 4 then degree 3 */
    for (int d = 4; d >= 3; --d) {
        uint64_t c = prod[d];
        prod[d] = 0;
        for (int k = 0; k < 3; ++k)
            prod[d - 3 + k] = (prod[d - 3 + k] + mulmod(c, e[k], m)) % m;
    }
    r[0] = prod[0]; r[1] = prod[1]; r[2] = prod[2];
}

static void poly_tpow(const uint64_t n[3], const uint64_t e[3], uint64_t m,
                      uint64_t r[3])
{
    uint64_t acc[3] = {1, 0, 0};
    int top = 191;
    while (top >= 0 && !((n[top / 64] >> (top % 64)) & 1u)) --top;
    for (int bit = top; bit >= 0; --bit) {
        uint64_t sq[3];
        polymulmod(acc, acc, e, m, sq);
        memcpy(acc, sq, sizeof acc);
        if ((n[bit / 64] >> (bit % 64)) & 1u) {
            const uint64_t t[3] = {0, 1, 0};
            polymulmod(acc, t, e, m, sq);
            memcpy(acc, sq, sizeof acc);
        }
    }
    memcpy(r, acc, sizeof acc);
}

static void jump_component(uint64_t s[3], const uint64_t n[3],
                           const uint64_t e[3], uint64_t m)
{
    uint64_t c[3], c1[3], c2[3];
    const uint64_t t[3] = {0, 1, 0};
    poly_tpow(n, e, m, c);
    polymulmod(c, t, e, m, c1);
    polymulmod(c1, t, e, m, c2);
    uint64_t out[3];
    const uint64_t *rows[3] = {c, c1, c2};
    for (int j = 0; j < 3; ++j) {
        uint64_t v = 0;
        for (int i = 0; i < 3; ++i)
            v = (v + mulmod(rows[j][i], s[i], m)) % m;
        out[j] = v;
    }
    memcpy(s, out, sizeof out);
}

/* Pinned by: brute-force stepping, group-order and primitivity identities,
 * agreement with plain 3x3 matrix powers over Python integers (tests/). */
void orc_mrg_skip(uint64_t st[6], const uint64_t n[3])
{
    /* t^3 = 0 t^2 + 1403580 t - 810728 (mod m1) */
    const uint64_t e1[3] = {MRG_M1 - MRG_A13, MRG_A12, 0};
    /* t^3 = 527612 t^2 + 0 t - 1370589 (mod m2) */
    const uint64_t e2[3] = {MRG_M2 - MRG_A23, 0, MRG_A21};
    jump_component(st, n, e1, MRG_M1);
    jump_component(st + 3, n, e2, MRG_M2);
}

/* ------------------------------------------------------------------------
 * Distributions (readings R10-R16).  Kinds match the library's numbering:
 * 1 = raw 32-bit words, 2 = uniform FP32, 3 = uniform FP64,
 * 4 = Gaussian (returned here as the FP64 transform; the library's FP32
 * result must be within 2 ulp of it), 5 = Gaussian FP64 (R21),
 * 6 = uniform int32 on [a, b) (R23), 7 = Gaussian FP32 by the inverse
 * normal CDF, 8 = Gaussian FP64 by the inverse normal CDF (R24; both
 * returned as the FP64 transform).
 * ---------------------------------------------------------------------- */

/* R10: u = (w >> 8) * 2^-24, exact, in [0, 1 - 2^-24]. */
float orc_u01_f32(uint32_t w)
{
    return (float)(w >> 8) * 0x1p-24f;
}

/* R11, Philox: 53 bits from two words, first word is the low half. */
double orc_u01_f64_words(uint32_t w_lo, uint32_t w_hi)
{
    uint64_t v = ((uint64_t)w_hi << 32) | (uint64_t)w_lo;
    return (double)(v >> 11) * 0x1p-53;
}

/* R11, MRG: u = y * norm, norm the nearest double to 1 / (m1 + 1), one
 * IEEE multiply ([L99] output scale). */
double orc_u01_f64_mrg(uint32_t y)
{
    const double norm = 1.0 / (double)(MRG_M1 + 1);
    return (double)y * norm;
}

/* Range transform of the paper (Sec. 4.3): r = u (b - a) + a, read as one
 * fused multiply-add in the output precision with (b - a) rounded once to
 * that precision (R12). */
float orc_range_f32(float u, double a, double b)
{
    float d = (float)(b - a);
    return fmaf(u, d, (float)a);
}

double orc_range_f64(double u, double a, double b)
{
    return fma(u, b - a, a);
}

/* sin(pi x) and cos(pi x) for x in [0, 2) by exact reduction (R16):
 * j = nearest integer to 2x, t = x - j/2 in [-1/4, 1/4] (exact), then
 * rotate by j quarter turns. */
static void sincospi_exact(double x, double *s, double *c)
{
    double j = nearbyint(2.0 * x);
    double t = x - 0.5 * j;
    double st = sin(M_PI * t), ct = cos(M_PI * t);
    int q = ((int)j) & 3;
    switch (q) {
    case 0: *s = st;  *c = ct;  break;
    case 1: *s = ct;  *c = -st; break;
    case 2: *s = -st; *c = -ct; break;
    default: *s = -ct; *c = st; break;
    }
}

/* Box-Muller ([BM58]) on a word pair (R13): u1 = ((w_a >> 8) + 1) 2^-24 in
 * (0, 1], u2 = (w_b >> 8) 2^-24 in [0, 1), r = sqrt(-2 ln u1),
 * z0 = r cos(2 pi u2), z1 = r sin(2 pi u2), all in FP64.
 * Pinned by: mpmath at 50 digits, special cases, moments (tests/). */
void orc_box_muller(uint32_t w_a, uint32_t w_b, double *z0, double *z1)
{
    double u1 = (double)((w_a >> 8) + 1u) * 0x1p-24;
    double u2 = (double)(w_b >> 8) * 0x1p-24;
    double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi_exact(2.0 * u2, &s, &c);
    *z0 = r * c;
    *z1 = r * s;
}

/* Gaussian FP64 (R21): Box-Muller ([BM58]) on a pair of FP64 uniforms,
 * u1 in (0, 1] and u2 in [0, 1), evaluated with libm in FP64:
 * r = sqrt(-2 ln u1), z0 = r cos(2 pi u2), z1 = r sin(2 pi u2).
 * Pinned by: mpmath at 50 digits, special cases, moments (tests/). */
void orc_box_muller64(double u1, double u2, double *z0, double *z1)
{
    double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi_exact(2.0 * u2, &s, &c);
    *z0 = r * c;
    *z1 = r * s;
}

/* The FP64 uniform pair of a Gaussian FP64 output pair (R21).  Philox: four
 * words; u1 = (v_a + 1) 2^-53 with v_a the 53 bits of (w0, w1) (first word
 * low, as for uniform FP64), u2 = v_b 2^-53 from (w2, w3).  MRG: two
 * outputs y_a, y_b; u1 = y_a / (m1 + 1), u2 = y_b / (m1 + 1), each one
 * multiply by the rounded scale (as for uniform FP64). */
void orc_gauss64_uniforms(int mrg, const uint32_t *w, double *u1, double *u2)
{
    if (mrg) {
        *u1 = orc_u01_f64_mrg(w[0]);
        *u2 = orc_u01_f64_mrg(w[1]);
    } else {
        *u1 = orc_u01_f64_words(w[0], w[1]) + 0x1p-53;
        *u2 = orc_u01_f64_words(w[2], w[3]);
    }
}

/* R23: uniform integer on [a, b), -2^31 <= a < b <= 2^31: the word read as
 * the fraction w / 2^32, scaled by r = b - a and floored, all in exact
 * integer arithmetic: a + floor(w r / 2^32).
 * Pinned by: exhaustive counts over all 2^32 words for small r (each value
 * gets floor or ceil of 2^32 / r words), brute force over small words,
 * the extremes of the range (tests/). */
int32_t orc_uniform_i32(uint32_t w, double a, double b)
{
    const int64_t ia = (int64_t)a, ib = (int64_t)b;
    const uint64_t r = (uint64_t)(ib - ia);                 /* 1 .. 2^32 */
    const uint64_t k = (uint64_t)(((u128)w * r) >> 32);     /* 0 .. r - 1 */
    return (int32_t)(ia + (int64_t)k);
}

/* Standard normal quantile z = Phi^{-1}(u), u in (0, 1), by its definition:
 * the z with Phi(z) = u (R24).  With q = min(u, 1 - u) (1 - u is exact for
 * u >= 1/2) and t = |z| >= 0:
 *   q > 1/4:  erf(t / sqrt 2) = 1 - 2q   (exact right-hand side);
 *   q <= 1/4: erfc(t / sqrt 2) = 2q      (exact right-hand side),
 * so each side is a monotone function of t evaluated where libm is
 * accurate.  t is found by bisection over the bit patterns of non-negative
 * doubles (ordered like the doubles themselves) down to two neighbours,
 * keeping the one whose function value is closer; z = -t for u < 1/2.
 * Pinned by: mpmath's erfinv at 50 digits, the symmetry
 * Phi^{-1}(1 - u) = -Phi^{-1}(u), known quantiles, scipy's ndtri (tests/). */
static double quantile_side(double t, int center)
{
    const double x = t * M_SQRT1_2;
    return center ? erf(x) : erfc(x);
}

double orc_normal_quantile(double u)
{
    if (u == 0.5) return 0.0;
    const double q = u < 0.5 ? u : 1.0 - u;
    const int center = q > 0.25;
    const double target = center ? 1.0 - 2.0 * q : 2.0 * q;
    /* erf rises with t, erfc falls; search [0, 40] (erfc(40 / sqrt 2) is 0) */
    uint64_t lo, hi;
    double d = 0.0;
    memcpy(&lo, &d, 8);
    d = 40.0;
    memcpy(&hi, &d, 8);
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        double t;
        memcpy(&t, &mid, 8);
        const double f = quantile_side(t, center);
        const int below = center ? (f < target) : (f > target);
        if (below) lo = mid;
        else hi = mid;
    }
    double tl, th;
    memcpy(&tl, &lo, 8);
    memcpy(&th, &hi, 8);
    const double el = fabs(quantile_side(tl, center) - target);
    const double eh = fabs(quantile_side(th, center) - target);
    const double t = el <= eh ? tl : th;
    return u < 0.5 ? -t : t;
}

/* The uniform behind an inverse-CDF Gaussian (R24), strictly inside (0, 1):
 * FP32 kind: u = ((w >> 8) + 1/2) 2^-24 from one word (Philox word or MRG
 * output).  FP64 kind, Philox: with v the 53 bits of (w0, w1) as for
 * uniform FP64, u = (floor(v / 2) + 1/2) 2^-52 (53 significant bits,
 * exact); MRG: u = y / (m1 + 1) as for uniform FP64, which is never 0 or
 * 1. */
double orc_icdf_uniform(int kind, int mrg, const uint32_t *w)
{
    if (kind == 7) return ((double)(w[0] >> 8) + 0.5) * 0x1p-24;
    if (mrg) return orc_u01_f64_mrg(w[0]);
    const uint64_t v = (((uint64_t)w[1] << 32) | (uint64_t)w[0]) >> 11;
    return ((double)(v >> 1) + 0.5) * 0x1p-52;
}

/* Apply a distribution to a word stream (kind numbering above).  For the
 * Philox engine U-F64 takes two words per output; for MRG one (R11).
 * Gaussian pairs use words (2j, 2j+1); odd n discards the last z1 (R14).
 * Output arrays: kind 1 -> uint32, 2 -> float, 3 -> double, 4 -> double
 * (z * stddev + mean in FP64), 5 -> double, 6 -> int32, 7 and 8 -> double
 * (z * stddev + mean in FP64). */
void orc_apply(int kind, int mrg, const uint32_t *w, uint64_t n,
               double p0, double p1, void *out)
{
    uint64_t i;
    switch (kind) {
    case 1:
        memcpy(out, w, n * sizeof(uint32_t));
        break;
    case 2: {
        float *o = (float *)out;
        for (i = 0; i < n; ++i) o[i] = orc_range_f32(orc_u01_f32(w[i]), p0, p1);
        break;
    }
    case 3: {
        double *o = (double *)out;
        for (i = 0; i < n; ++i) {
            double u = mrg ? orc_u01_f64_mrg(w[i])
                           : orc_u01_f64_words(w[2 * i], w[2 * i + 1]);
            o[i] = orc_range_f64(u, p0, p1);
        }
        break;
    }
    case 4: {
        double *o = (double *)out;
        for (i = 0; i < n; i += 2) {
            double z0, z1;
            orc_box_muller(w[i], w[i + 1], &z0, &z1);
            o[i] = z0 * p1 + p0;
            if (i + 1 < n) o[i + 1] = z1 * p1 + p0;
        }
        break;
    }
    case 5: {
        /* pair j uses words 4j .. 4j + 3 (Philox) or outputs 2j, 2j + 1 (MRG) */
        double *o = (double *)out;
        for (i = 0; i < n; i += 2) {
            double u1, u2, z0, z1;
            orc_gauss64_uniforms(mrg, w + (mrg ? i : 2 * i), &u1, &u2);
            orc_box_muller64(u1, u2, &z0, &z1);
            o[i] = z0 * p1 + p0;
            if (i + 1 < n) o[i + 1] = z1 * p1 + p0;
        }
        break;
    }
    case 6: {
        int32_t *o = (int32_t *)out;
        for (i = 0; i < n; ++i) o[i] = orc_uniform_i32(w[i], p0, p1);
        break;
    }
    case 7:
    case 8: {
        /* FP64 on Philox: words 2i, 2i + 1; otherwise word i */
        double *o = (double *)out;
        const int step = (kind == 8 && !mrg) ? 2 : 1;
        for (i = 0; i < n; ++i) {
            const double z = orc_normal_quantile(orc_icdf_uniform(kind, mrg, w + step * i));
            o[i] = z * p1 + p0;
        }
        break;
    }
    default:
        break;
    }
}

/* Number of engine words (Philox) or steps (MRG) that n outputs consume
 * (R14, R21, R24): U-F64 and inverse-CDF Gaussian FP64 on Philox take 2
 * per output, Gaussian FP32 2 per started pair, Gaussian FP64 4 (Philox)
 * or 2 (MRG) per started pair, everything else 1. */
uint64_t orc_words_consumed(int kind, int mrg, uint64_t n)
{
    if (kind == 3 || kind == 8) return mrg ? n : 2 * n;
    if (kind == 4) return 2 * ((n + 1) / 2);
    if (kind == 5) return (mrg ? 2 : 4) * ((n + 1) / 2);
    return n;
}

/* Full plain generate, the definition written out: words at the engine's
 * position, then the distribution.  `scratch` must hold
 * orc_words_consumed(kind, 0, n) words.  Philox: position pos[3] (130-bit);
 * the caller advances it. */
void orc_philox_generate(uint64_t seed, const uint64_t pos[3], int kind,
                         double p0, double p1, uint64_t n,
                         uint32_t *scratch, void *out)
{
    uint64_t nw = orc_words_consumed(kind, 0, n);
    orc_philox_words((uint32_t)seed, (uint32_t)(seed >> 32), pos, nw, scratch);
    orc_apply(kind, 0, scratch, n, p0, p1, out);
}

/* MRG: the state st is advanced in place by the consumed steps. */
void orc_mrg_generate(uint64_t st[6], int kind, double p0, double p1,
                      uint64_t n, uint32_t *scratch, void *out)
{
    uint64_t nw = orc_words_consumed(kind, 1, n);
    orc_mrg_words(st, nw, scratch);
    orc_apply(kind, 1, scratch, n, p0, p1, out);
}

/* The two factors of the Box-Muller transform on their own, over arrays of
 * words, for exhaustive component checks (all 2^24 inputs of each):
 * r[i] = sqrt(-2 ln u1(w[i])), s[i] = sin(2 pi u2(w[i])),
 * c[i] = cos(2 pi u2(w[i])). */
void orc_box_muller_factors(const uint32_t *w, uint64_t n, double *r,
                            double *s, double *c)
{
    for (uint64_t i = 0; i < n; ++i) {
        double u1 = (double)((w[i] >> 8) + 1u) * 0x1p-24;
        double u2 = (double)(w[i] >> 8) * 0x1p-24;
        if (r) r[i] = sqrt(-2.0 * log(u1));
        if (s && c) sincospi_exact(2.0 * u2, &s[i], &c[i]);
    }
}
