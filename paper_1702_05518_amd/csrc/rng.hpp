// rng.hpp -- device random numbers of the sampler.
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): a counter-based generator, so every draw is a pure
// function of (key, counter) and needs no state in memory.  Key = the chain's
// 64-bit seed; counter = (site or attempt, sweep, instance, tag).
//
// Normals: Box & Muller (1958), cosine branch.  Gamma: Marsaglia & Tsang
// (2000), "A simple method for generating gamma variables", without the
// squeeze test (the squeeze accepts a subset of the full test, so leaving it
// out changes no decision).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmrf {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Ten Philox rounds.  Each round multiplies two counter words by the Philox
// multipliers, mixes the high halves with the other two words and the key,
// and advances the key by the Weyl increments.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kIncA = 0x9E3779B9u, kIncB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t a_hi = (uint32_t)(pa >> 32), a_lo = (uint32_t)pa;
        const uint32_t b_hi = (uint32_t)(pb >> 32), b_lo = (uint32_t)pb;
        c0 = b_hi ^ c1 ^ k0;
        c1 = b_lo;
        c2 = a_hi ^ c3 ^ k1;
        c3 = a_lo;
        k0 += kIncA;
        k1 += kIncB;
    }
    return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 draw_words(uint64_t seed, uint32_t c0, uint32_t c1,
                                             uint32_t c2, uint32_t c3)
{
    return philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// (0,1) uniform from the top 52 bits of a word pair: (m + 1/2) 2^-52, exact
// in FP64, never 0 or 1.
__device__ __forceinline__ double open_uniform_f64(uint32_t hi, uint32_t lo)
{
    const uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}

// Natural logarithm of an open uniform u in (0, 1) (u >= 2^-53), from the
// reduction u = m 2^k with m in [sqrt(1/2), sqrt(2)) and
//     log u = k log 2 + 2 atanh(s),   s = (m - 1) / (m + 1),   |s| < 0.1716,
// where 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ...) is the Taylor series of
// atanh, summed here to the s^20/21 term (the rest is below 3e-17 relative).
// m - 1 is exact and log 2 is split into a head with trailing zero bits
// (k times it is exact) and a tail, so the result is within a few ulps of
// the correctly rounded logarithm.  About 35 instructions against ~100 for
// the general double-double library log, which dominates the Polya-Gamma
// sampler and the FP64 Box-Muller draw otherwise.
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // log 2 to 43 bits
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // log 2 - kLn2Hi
__host__ __device__ inline double log_open_unit(double u)
{
    int k;
    double m = frexp(u, &k);                // u = m 2^k, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m += m;
        --k;
    }
    const double f = m - 1.0;               // exact (m within a factor 2 of 1)
    const double s = f / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double two_s = s + s;
    const double kd = (double)k;
    // k log2_hi + (2 s + (k log2_lo + 2 s s^2 p)), small terms first
    return fma(kd, kLn2Hi, two_s + fma(kd, kLn2Lo, two_s * s2 * p));
}

// cos(2 pi u) for u in [0, 1]: folded by the symmetries of the cosine,
// cos(2 pi u) = cos(2 pi (1 - u)) into v in [0, 1/2] and
// cos(2 pi v) = -cos(2 pi (1/2 - v)) into v in [0, 1/4] (both subtractions
// exact), then the Taylor series of cos(w), w = 2 pi v <= pi/2, summed to the
// w^22 / 22! term (the rest is below 2e-17).  Within a few 1e-16 of the exact
// value in absolute terms, which is what the Box-Muller product needs.
constexpr double kTwoPi = 6.283185307179586476925;
__host__ __device__ inline double cos_2pi_unit(double u)
{
    double v = u > 0.5 ? 1.0 - u : u;
    const bool neg = v > 0.25;
    if (neg)
        v = 0.5 - v;
    const double w = kTwoPi * v;
    const double w2 = w * w;
    // sum_{n=0..11} (-1)^n w^(2n) / (2n)!, Horner in w^2
    double p = 1.0 / 1124000727777607680000.0;                  // 1 / 22!
    p = fma(p, w2, -1.0 / 2432902008176640000.0);                // 1 / 20!
    p = fma(p, w2, 1.0 / 6402373705728000.0);                    // 1 / 18!
    p = fma(p, w2, -1.0 / 20922789888000.0);                     // 1 / 16!
    p = fma(p, w2, 1.0 / 87178291200.0);                         // 1 / 14!
    p = fma(p, w2, -1.0 / 479001600.0);                          // 1 / 12!
    p = fma(p, w2, 1.0 / 3628800.0);                             // 1 / 10!
    p = fma(p, w2, -1.0 / 40320.0);                              // 1 / 8!
    p = fma(p, w2, 1.0 / 720.0);                                 // 1 / 6!
    p = fma(p, w2, -1.0 / 24.0);                                 // 1 / 4!
    p = fma(p, w2, 0.5);                                         // the w^2 / 2! term
    p = fma(-p, w2, 1.0);
    return neg ? -p : p;
}

// sin(2 pi u) for u in [0, 1] as cos(2 pi (u - 1/4)), the argument moved
// back into [0, 1] by one period below u = 1/4.  For multiples of 2^-53 (the
// open uniforms) both shifts are exact: u - 1/4 lies in [0, 3/4] and u + 3/4
// in [3/4, 1), and every multiple of 2^-53 there is a double, so the error is
// cos_2pi_unit's.
__host__ __device__ inline double sin_2pi_unit(double u)
{
    return cos_2pi_unit(u < 0.25 ? u + 0.75 : u - 0.25);
}

// FP64 standard normal of one Philox block.  log u1 and cos(2 pi u2) come
// from log_open_unit and cos_2pi_unit: the library values up to a few ulps
// (no double-double logarithm, no general range reduction), with much
// lighter instruction sequences.
__device__ __forceinline__ double normal_f64(const Words4 &w)
{
    const double u1 = open_uniform_f64(w.w0, w.w1);
    const double u2 = open_uniform_f64(w.w2, w.w3);
    return sqrt(-2.0 * log_open_unit(u1)) * cos_2pi_unit(u2);
}

// FP32 standard normal of the same block: the same two uniforms carried to
// FP32 precision (u1 keeps its relative precision down to 2^-56 so the tail
// tracks the FP64 draw), then Box-Muller on the hardware transcendental
// units: log2, square root, and the cosine whose argument is in revolutions,
// so cos(2 pi u2) is a single instruction.
__device__ __forceinline__ float normal_f32(const Words4 &w)
{
    const float u1 = fmaf((float)w.w0, 0x1p-32f, fmaf((float)(w.w1 >> 8), 0x1p-56f, 0x1p-57f));
    const float u2 = (float)w.w2 * 0x1p-32f;
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;   // -2 ln 2
    return __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1)) *
           __builtin_amdgcn_cosf(u2);
}

// Both Box-Muller normals of one block (the paired contract: the cosine
// branch for the lower-ranked site of a pair, the sine branch for its
// partner); one logarithm and one square root serve the two.
__device__ __forceinline__ void normal_pair_f64(const Words4 &w, double &zc, double &zs)
{
    const double u1 = open_uniform_f64(w.w0, w.w1);
    const double u2 = open_uniform_f64(w.w2, w.w3);
    const double r = sqrt(-2.0 * log_open_unit(u1));
    zc = r * cos_2pi_unit(u2);
    zs = r * sin_2pi_unit(u2);
}

__device__ __forceinline__ void normal_pair_f32(const Words4 &w, float &zc, float &zs)
{
    const float u1 = fmaf((float)w.w0, 0x1p-32f, fmaf((float)(w.w1 >> 8), 0x1p-56f, 0x1p-57f));
    const float u2 = (float)w.w2 * 0x1p-32f;
    constexpr float kMinus2Ln2 = -1.38629436111989061883f;   // -2 ln 2
    const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1));
    zc = r * __builtin_amdgcn_cosf(u2);
    zs = r * __builtin_amdgcn_sinf(u2);
}

template <typename Real> __device__ __forceinline__ Real site_normal(const Words4 &w);
template <> __device__ __forceinline__ double site_normal<double>(const Words4 &w)
{
    return normal_f64(w);
}
template <> __device__ __forceinline__ float site_normal<float>(const Words4 &w)
{
    return normal_f32(w);
}

template <typename Real>
__device__ __forceinline__ void site_normal_pair(const Words4 &w, Real &zc, Real &zs);
template <>
__device__ __forceinline__ void site_normal_pair<double>(const Words4 &w, double &zc, double &zs)
{
    normal_pair_f64(w, zc, zs);
}
template <>
__device__ __forceinline__ void site_normal_pair<float>(const Words4 &w, float &zc, float &zs)
{
    normal_pair_f32(w, zc, zs);
}

constexpr int kGammaMaxAttempts = 64;

// Marsaglia-Tsang constants of a shape >= 1: d = shape - 1/3, c = 1/sqrt(9 d)
// (the shapes depend only on n and the priors, so they are computed once per
// chain on the host, with the same operations).
struct GammaShape {
    double d, c;
};

// Gamma(shape, rate) for the hyperparameter draw after sweep `sweep`.
// Attempt k takes its normal from counter (2k, sweep, instance, tag) and its
// uniform from counter (2k + 1, ...).  Returns false when every attempt was
// rejected (the caller flags a numeric error).
__device__ inline bool gamma_draw(GammaShape g, double rate, uint64_t seed, uint32_t sweep,
                                  uint32_t instance, uint32_t tag, double *out)
{
    const double d = g.d, c = g.c;
    for (int k = 0; k < kGammaMaxAttempts; ++k) {
        const double z = normal_f64(draw_words(seed, (uint32_t)(2 * k), sweep, instance, tag));
        const double cz = c * z;
        if (cz <= -1.0)
            continue;
        const double L = 3.0 * log1p(cz);        // log of v = (1 + c z)^3
        const double v = exp(L);
        const Words4 wu = draw_words(seed, (uint32_t)(2 * k + 1), sweep, instance, tag);
        const double u = open_uniform_f64(wu.w0, wu.w1);
        // accept iff log u < z^2/2 + d - d v + d log v, with 1 - v + log v
        // evaluated as L - expm1(L) to avoid cancellation at large d
        if (log(u) < 0.5 * z * z + d * (L - expm1(L))) {
            *out = d * v / rate;
            return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Polya-Gamma variates (Polson, Scott & Windle 2013, Sec. 4, after Devroye
// 2009).  PG(1, c) = J*(1, |c|/2) / 4; J*(1, z) is drawn by rejection from
// an envelope of two pieces split at t = 0.64 -- a truncated exponential on
// (t, inf) and a truncated inverse Gaussian on (0, t) -- with the
// alternating-series test of the J*(1) density.  PG(m, c) for an integer m is
// the sum of m independent PG(1, c) terms.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793;
constexpr double kPgT = 0.64;
constexpr float kLn2f = 0.693147180559945309f;
constexpr float kLog2ef = 1.442695040888963407f;
constexpr float kPi2f = 9.869604401089358619f;      // pi^2
constexpr unsigned kPgMaxUniforms = 2048;   // uniforms available to one PG(1, c) draw
constexpr int kPgMaxTerms = 200;            // series terms per acceptance test

// Uniform stream of term j of one site's PG draw: uniform u is half (u & 1) of
// the Philox block at counter (site, sweep, instance, 2^31 | j << 10 | u >> 1).
struct PgStream {
    uint64_t seed;
    uint32_t site, sweep, instance, j;
    uint32_t used;
    bool exhausted;
    Words4 blk{};               // the block of the last even-numbered uniform

    // Uniform `used`: an even one computes its block and keeps it for the
    // odd one that follows (one Philox evaluation per two uniforms).
    __device__ double next()
    {
        const uint32_t u = used;
        if (u >= kPgMaxUniforms) {
            exhausted = true;
            return 0.5;
        }
        used = u + 1;
        if (u & 1u)
            return open_uniform_f64(blk.w2, blk.w3);
        blk = draw_words(seed, site, sweep, instance, 0x80000000u | (j << 10) | (u >> 1));
        return open_uniform_f64(blk.w0, blk.w1);
    }
    __device__ double normal()
    {
        const double u1 = next();
        const double u2 = next();
        return sqrt(-2.0 * log_open_unit(u1)) * cos_2pi_unit(u2);
    }
};

__device__ inline double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

// Terms of the alternating series of the J*(1) density at x, in order.
// Term n is pi (n + 1/2) c E^((2n+1)^2) with, right of t (x > t), c = 1 and
// E = exp(-pi^2 x / 8), and left of t, c = (2 / (pi x))^(3/2) and
// E = exp(-1 / (2 x)).  The powers come from one exp by the recurrence
// E^((2n+1)^2) = E^((2n-1)^2) * E^(8n), so each term after the first costs
// two multiplications; the values equal the per-term exponentials up to a
// few ulps.
struct PgSeries {
    double c, e, e8, ratio, power;
    int n;

    __device__ explicit PgSeries(double x)
    {
        if (x > kPgT) {
            c = 1.0;
            e = exp(-0.125 * kPi * kPi * x);
        } else {
            const double r = 2.0 / (kPi * x);
            c = r * sqrt(r);
            e = exp(-0.5 / x);
        }
        const double e2 = e * e, e4 = e2 * e2;
        e8 = e4 * e4;
        ratio = 1.0;
        power = e;
        n = 0;
    }
    // the current term, then advance to the next one
    __device__ double next()
    {
        const double v = kPi * ((double)n + 0.5) * c * power;
        ratio *= e8;                 // E^(8 (n + 1))
        power *= ratio;              // E^((2n + 3)^2)
        ++n;
        return v;
    }
};

// IG(1/z, 1) restricted to (0, t).  z < 1/t: the z = 0 law on (0, t) from a
// normal tail beyond 1/sqrt(t) (1/X = (1 + t E1)^2 / t, E1^2 <= 2 E2 / t),
// kept with probability exp(-z^2 X / 2).  Otherwise: Michael, Schucany &
// Haas's transformation, repeated until X < t.
__device__ inline double pg_left(double z, PgStream &s)
{
    const double t = kPgT;
    if (z < 1.0 / t) {
        for (;;) {
            double u1, e1 = -1.0;
            for (;;) {
                u1 = s.next();
                const double u2 = s.next();
                // The test e1^2 > 2 e2 / t first from single-precision
                // logarithms (hardware log2): their error is below 1e-6 (1 + e)
                // for every e, so a difference beyond 1e-3 (1 + both sides)
                // decides it as the double-precision test would; only closer
                // calls take the double logarithms.  The same decisions, so
                // the same draws, with far fewer double logarithms.
                const float a1 = -kLn2f * __builtin_amdgcn_logf((float)u1);
                const float a2 = -kLn2f * __builtin_amdgcn_logf((float)u2);
                const float lhs = a1 * a1, rhs = 2.0f * a2 / (float)t;
                const float guard = 1e-3f * (1.0f + lhs + rhs);
                bool reject;
                if (lhs - rhs > guard) {
                    reject = true;
                } else if (rhs - lhs > guard) {
                    reject = false;
                } else {
                    e1 = -log_open_unit(u1);
                    reject = e1 * e1 > 2.0 * -log_open_unit(u2) / t;
                }
                if (!reject || s.exhausted)
                    break;
                e1 = -1.0;
            }
            if (e1 < 0.0)
                e1 = -log_open_unit(u1);
            const double x = t / ((1.0 + t * e1) * (1.0 + t * e1));
            // u <= exp(w), w = -z^2 x / 2 in (-0.79, 0]: first against the
            // single-precision exponential (relative error below 1e-6), the
            // double one only within 1e-4 of it
            const double u = s.next();
            const double w = -0.5 * z * z * x;
            const double ef = (double)__builtin_amdgcn_exp2f((float)w * kLog2ef);
            bool keep;
            if (u < ef * (1.0 - 1e-4))
                keep = true;
            else if (u > ef * (1.0 + 1e-4))
                keep = false;
            else
                keep = u <= exp(w);
            if (keep || s.exhausted)
                return x;
        }
    }
    const double mu = 1.0 / z;
    for (;;) {
        const double nrm = s.normal();
        const double y = nrm * nrm;
        const double my = mu * y;
        double x = mu + 0.5 * mu * my - 0.5 * mu * sqrt(4.0 * my + my * my);
        if (s.next() > mu / (mu + x))
            x = mu * mu / x;
        if (x < t || s.exhausted)
            return x;
    }
}

// Envelope of PG(1, c) for one tilt: z = |c| / 2, rate K of the right piece
// and the probability p / (p + q) of drawing from it.
struct PgEnvelope {
    double z, K, right;
};

__device__ inline PgEnvelope pg_envelope(double c)
{
    const double t = kPgT;
    PgEnvelope e;
    e.z = 0.5 * fabs(c);
    e.K = kPi * kPi / 8.0 + 0.5 * e.z * e.z;
    const double p = kPi / (2.0 * e.K) * exp(-e.K * t);
    double q;
    if (e.z == 0.0) {
        q = 2.0 * erfc(1.0 / sqrt(2.0 * t));
    } else {
        const double a = std_normal_cdf((t * e.z - 1.0) / sqrt(t));
        const double b = e.z < 700.0 ? exp(e.z) * std_normal_cdf(-(t * e.z + 1.0) / sqrt(t)) : 0.0;
        q = 2.0 * (exp(-e.z) * a + b);
    }
    e.right = p / (p + q);
    return e;
}

// PG(1, c) from the stream of term j; false when the stream ran out.
__device__ inline bool pg1_draw(const PgEnvelope &e, uint64_t seed, uint32_t site, uint32_t sweep,
                                uint32_t instance, uint32_t j, double *out)
{
    PgStream s{seed, site, sweep, instance, j, 0u, false, Words4{}};
    for (;;) {
        double x;
        if (s.next() < e.right)
            x = kPgT - log_open_unit(s.next()) / e.K;
        else
            x = pg_left(e.z, s);
        const double u = s.next();
        if (s.exhausted)
            return false;
        // The first test of the series, Y = u a0 <= a0 - a1, is u <= 1 - 3 E^8
        // (a1 / a0 = 3 E^8 for both forms of the terms), with 3 E^8 below
        // 0.006 here.  From the single-precision exponential (error below
        // 1e-8 absolute at these values) a u more than 1e-5 below it is
        // accepted as the double-precision series would; otherwise the
        // series runs as written.
        {
            const float xf = (float)x;
            const float w = x > kPgT ? -kPi2f * xf : -4.0f * __builtin_amdgcn_rcpf(xf);
            const float q = 3.0f * __builtin_amdgcn_exp2f(w * kLog2ef);
            if (u < 1.0 - (double)q - 1e-5) {
                *out = 0.25 * x;
                return true;
            }
        }
        PgSeries terms(x);
        double S = terms.next();
        const double Y = u * S;
        for (int n = 1; n <= kPgMaxTerms; ++n) {
            if (n & 1) {
                S -= terms.next();
                if (Y <= S) {
                    *out = 0.25 * x;
                    return true;
                }
            } else {
                S += terms.next();
                if (Y > S)
                    break;
            }
        }
    }
}

} // namespace gmrf
