/*
 * gmrf_oracle.c -- CPU oracle for the chromatic Gibbs sampler of a Gaussian
 * Markov random field with a CAR prior (Brown, McMahan & Self, "Sampling
 * Strategies for Fast Updating of Gaussian Markov Random Fields", 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * Everything is FP64, scalar loops in original site order, IEEE
 * round-to-nearest, built without fast-math and without FP contraction.
 *
 * What it computes (paper references are to sections / equations /
 * algorithms of the paper):
 *   - Gaussian full conditional of the field given y and the precisions
 *     (Sec. 2.2: x | y ~ N(Qp^{-1} b, Qp^{-1}), Qp = A'S^{-1}A + Q,
 *     b = A'S^{-1}y + Q mu), specialised to A = I, S = I/lam, mu = 0 and the
 *     CAR precision Q = tau (D - rho W) (Sec. 3.1 IAR model, rho = 1; Sec. 3.2
 *     proper CAR).  Per site (Sec. 3.1 local characteristics, written with
 *     precisions tau = 1/tau^2 and lam = 1/sigma^2):
 *         Qii = tau * D_ii + lam,
 *         m_i = (lam * y_i + tau * rho * sum_{j~i} x_j) / Qii,
 *         x_i ~ N(m_i, 1/Qii).
 *   - The chromatic Gibbs step (Sec. 2.3, Algorithm 1): colors in ascending
 *     order; every site of a color is drawn from its conditional given the
 *     other colors (lower colors already at their new values).
 *   - The conjugate hyperparameter draws (Sec. 3.1 full conditionals of
 *     sigma^2 and tau^2, recast as Gamma laws of the precisions, rate form):
 *         tau | x ~ Gamma(a_tau + r/2, b_tau + x'(D - rho W)x / 2),
 *         lam | x ~ Gamma(a_lam + n/2, b_lam + ||y - x||^2 / 2),
 *     r = n - (#connected components) for the intrinsic prior, n otherwise.
 *   - Running posterior mean / variance accumulators (Sec. 3.1 posterior
 *     mean images).
 *   - Optionally the intercept of the Sec. 3.1 image model, y = 1 b0 + x + e
 *     with a flat prior on b0: the site mean uses y_i - b0, the iteration
 *     draws b0 | x, lam ~ N(mean(y - x), 1 / (n lam)) before lam and tau
 *     (the paper's order b0, sigma^2, tau^2, field), lam's sum of squares is
 *     ||y - 1 b0 - x||^2 with the new b0, and the accumulators collect the
 *     image b0 + x (the quantity the paper reports).
 *   - Optionally the binomial model of Sec. 3.2: Y_i ~ Bin(m_i, pi_i) with
 *     logit(pi_i) = b0 + x_i, made conditionally Gaussian by the Polya-Gamma
 *     augmentation the paper cites (Polson, Scott & Windle 2013): with
 *     kappa_i = Y_i - m_i / 2 and psi_i ~ PG(m_i, b0 + x_i),
 *         Qii = tau * D_ii + psi_i,
 *         m_i = (kappa_i - psi_i * b0 + tau * rho * sum_{j~i} x_j) / Qii,
 *     b0 | x, psi ~ N(sum(kappa - psi x) / P, 1 / P), P = sum psi + 1/v0
 *     (prior b0 ~ N(0, v0), v0 = 0 meaning flat), and tau as above.  The
 *     supplement that details the paper's sampler is not available; the
 *     reading here draws psi_i right before x_i in the site's color pass,
 *     which equals drawing all of psi first because psi_i depends on its
 *     own site only.
 *   - The greedy coloring of the paper's supplementary greedy algorithm
 *     (peel maximal independent sets, always taking the smallest remaining
 *     site).
 *
 * Random numbers (the paper uses R's generator; this is the reading both
 * sides share): Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by
 * the 64-bit seed, counter (c0, c1, c2, c3) = (site or attempt, sweep,
 * instance, tag); Box & Muller (1958) cosine branch for normals; Marsaglia &
 * Tsang (2000) for Gamma variates.
 *
 * Random-number contract version 2 (selectable per chain; version 1 above is
 * the default): the sites of each color, taken in ascending original id, are
 * paired by their rank in the color, ranks (2m, 2m + 1).  Both sites of a
 * pair take their site normal from the one Philox block keyed by the id of
 * the lower-ranked site: that site the cosine branch (so its value is the
 * version-1 normal of its own id), its partner the sine branch of the same
 * two uniforms.  A color's last site, when its count is odd, is unpaired and
 * takes the cosine branch of its own block.  Box-Muller's two branches are
 * independent standard normals, so the sweep's noise keeps its law; only
 * which counter feeds which site changes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11: multipliers and Weyl key increments) */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_MUL0 0xD2511F53u
#define ORC_PHILOX_MUL1 0xCD9E8D57u
#define ORC_PHILOX_KEYINC0 0x9E3779B9u
#define ORC_PHILOX_KEYINC1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)ORC_PHILOX_MUL0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_MUL1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += ORC_PHILOX_KEYINC0;   /* key schedule: Weyl sequence */
        k1 += ORC_PHILOX_KEYINC1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void orc_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t w[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = c0; ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, w);
}

/* Uniform on (0,1) from two 32-bit words: the top 52 bits m give
 * (m + 1/2) * 2^-52, which is exact in FP64 and never 0 or 1. */
double orc_uniform52(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}

#define ORC_TWO_PI 6.283185307179586

/* Standard normal: Box-Muller, cosine branch, from one Philox block. */
double orc_normal(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t w[4];
    double u1, u2;
    orc_words(seed, c0, c1, c2, c3, w);
    u1 = orc_uniform52(w[0], w[1]);
    u2 = orc_uniform52(w[2], w[3]);
    return sqrt(-2.0 * log(u1)) * cos(ORC_TWO_PI * u2);
}

/* Version-2 site normal: the Box-Muller pair of the Philox block at counter
 * (key, c1, c2, c3), its cosine branch (branch 0) or sine branch (branch 1). */
double orc_normal_pair(uint64_t seed, uint32_t key, uint32_t branch, uint32_t c1, uint32_t c2,
                       uint32_t c3)
{
    uint32_t w[4];
    double u1, u2, r;
    orc_words(seed, key, c1, c2, c3, w);
    u1 = orc_uniform52(w[0], w[1]);
    u2 = orc_uniform52(w[2], w[3]);
    r = sqrt(-2.0 * log(u1));
    return branch ? r * sin(ORC_TWO_PI * u2) : r * cos(ORC_TWO_PI * u2);
}

/* The version-2 pairing of a colored graph: key[i] is the id of the
 * lower-ranked site of i's pair within its color (i itself when i is
 * unpaired or ranked first), branch[i] 1 for the higher-ranked site, else 0.
 * One pass in ascending id keeps, per color, the site still waiting for a
 * partner.  Returns 0, or 1 on a color outside 0 .. k-1. */
int32_t orc_rng_pairs(int64_t n, const int32_t *color, int32_t k, int32_t *key, uint8_t *branch)
{
    int64_t i;
    int64_t *waiting = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    int32_t c;
    for (c = 0; c < k; ++c)
        waiting[c] = -1;
    for (i = 0; i < n; ++i) {
        c = color[i];
        if (c < 0 || c >= k) {
            free(waiting);
            return 1;
        }
        if (waiting[c] < 0) {
            key[i] = (int32_t)i;
            branch[i] = 0;
            waiting[c] = i;
        } else {
            key[i] = (int32_t)waiting[c];
            branch[i] = 1;
            waiting[c] = -1;
        }
    }
    free(waiting);
    return 0;
}

/* Gamma(shape, rate) by Marsaglia & Tsang (2000), shape >= 1, no squeeze.
 * Attempt k uses the normal of counter (2k, sweep, instance, tag) and the
 * uniform (first 52-bit uniform of the block) of counter (2k+1, ...).
 * Returns the number of attempts used (>= 1), or -1 when max_attempts were
 * all rejected, or -2 for an invalid shape / rate. */
int orc_gamma(double shape, double rate, uint64_t seed, uint32_t sweep, uint32_t instance,
              uint32_t tag, int max_attempts, double *out)
{
    double d, c;
    int k;
    if (!(shape >= 1.0) || !(rate > 0.0) || !isfinite(shape) || !isfinite(rate))
        return -2;
    d = shape - 1.0 / 3.0;
    c = 1.0 / sqrt(9.0 * d);
    for (k = 0; k < max_attempts; ++k) {
        uint32_t w[4];
        double z = orc_normal(seed, (uint32_t)(2 * k), sweep, instance, tag);
        double cz = c * z;
        double L, v, u, lhs, rhs;
        if (cz <= -1.0)
            continue;
        L = 3.0 * log1p(cz);          /* log v, v = (1 + c z)^3 */
        v = exp(L);
        orc_words(seed, (uint32_t)(2 * k + 1), sweep, instance, tag, w);
        u = orc_uniform52(w[0], w[1]);
        lhs = log(u);
        rhs = 0.5 * z * z + d * (L - expm1(L));   /* z^2/2 + d - d v + d log v */
        if (lhs < rhs) {
            *out = d * v / rate;
            return k + 1;
        }
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Graph utilities                                                            */
/* ------------------------------------------------------------------------ */

/* Greedy k-coloring (supplementary greedy algorithm): color j collects a
 * maximal independent set of the still-uncolored sites by repeatedly taking
 * the smallest remaining candidate and striking it and its neighbours from
 * the candidate set.  Colors are 0-based in discovery order.  Returns k. */
int32_t orc_greedy_coloring(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            int32_t *color)
{
    int64_t remaining = n, i, e;
    int32_t j = 0;
    int32_t *struck = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (i = 0; i < n; ++i) {
        color[i] = -1;
        struck[i] = -1;
    }
    while (remaining > 0) {
        /* candidates of color j: uncolored sites not struck during color j;
         * scanning in ascending order takes min of the candidate set */
        for (i = 0; i < n; ++i) {
            if (color[i] != -1 || struck[i] == j)
                continue;
            color[i] = j;
            --remaining;
            for (e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                struck[col[e]] = j;
        }
        ++j;
    }
    free(struck);
    return j;
}

/* Number of connected components (breadth-first search). */
int64_t orc_components(int64_t n, const int64_t *row_ptr, const int32_t *col)
{
    int64_t comps = 0, s, head, tail, e;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    unsigned char *seen = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    for (s = 0; s < n; ++s) {
        if (seen[s])
            continue;
        ++comps;
        head = tail = 0;
        queue[tail++] = s;
        seen[s] = 1;
        while (head < tail) {
            int64_t v = queue[head++];
            for (e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int64_t u = col[e];
                if (!seen[u]) {
                    seen[u] = 1;
                    queue[tail++] = u;
                }
            }
        }
    }
    free(queue);
    free(seen);
    return comps;
}

/* ------------------------------------------------------------------------ */
/* Polya-Gamma variates (Polson, Scott & Windle 2013, JASA 108, Sec. 4,      */
/* after Devroye 2009): PG(1, c) = J*(1, |c|/2) / 4, J* drawn by rejection    */
/* from a two-piece envelope (truncated exponential right of t, truncated     */
/* inverse Gaussian left of t) with the alternating-series acceptance test.   */
/* PG(b, c) for integer b is the sum of b independent PG(1, c).               */
/* ------------------------------------------------------------------------ */
#define ORC_PI 3.141592653589793
#define ORC_PG_T 0.64                 /* Devroye's switch point t */
#define ORC_PG_MAX_UNIFORMS 2048      /* uniforms available to one PG(1, c) draw */
#define ORC_PG_MAX_TERMS 200          /* series terms per acceptance test */

/* The uniform stream of one PG(1, c) draw: uniform number u (0-based) is
 * half (u & 1) of the Philox block at counter
 * (site, sweep, instance, 0x80000000 | j << 10 | u >> 1), j the index of the
 * PG(1, c) term inside PG(m_i, c) (j < 2^21). */
typedef struct {
    uint64_t seed;
    uint32_t site, sweep, instance, j;
    uint32_t used;
    int exhausted;
} orc_ustream;

static double orc_ustream_next(orc_ustream *s)
{
    uint32_t w[4];
    uint32_t u = s->used;
    if (u >= ORC_PG_MAX_UNIFORMS) {
        s->exhausted = 1;
        return 0.5;
    }
    s->used = u + 1;
    orc_words(s->seed, s->site, s->sweep, s->instance, 0x80000000u | (s->j << 10) | (u >> 1), w);
    return (u & 1u) ? orc_uniform52(w[2], w[3]) : orc_uniform52(w[0], w[1]);
}

/* Standard normal from the next two uniforms of the stream (Box-Muller). */
static double orc_ustream_normal(orc_ustream *s)
{
    double u1 = orc_ustream_next(s);
    double u2 = orc_ustream_next(s);
    return sqrt(-2.0 * log(u1)) * cos(ORC_TWO_PI * u2);
}

static double orc_std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* n-th term of the alternating series of the J*(1) density, in the form used
 * left (x <= t) and right (x > t) of the switch point. */
static double orc_pg_term(int n, double x)
{
    double h = (double)n + 0.5;
    if (x > ORC_PG_T)
        return ORC_PI * h * exp(-0.5 * h * h * ORC_PI * ORC_PI * x);
    {
        double r = 2.0 / (ORC_PI * x);
        return ORC_PI * h * r * sqrt(r) * exp(-2.0 * h * h / x);
    }
}

/* Inverse Gaussian IG(mu = 1/z, 1) truncated to (0, t).  For mu > t (z < 1/t,
 * z = 0 included): the z = 0 law truncated to (0, t) through 1/X =
 * (1 + t E1)^2 / t with E1^2 <= 2 E2 / t (normal-tail rejection), then
 * accepted with probability exp(-z^2 X / 2).  For mu <= t: the
 * Michael-Schucany-Haas transformation, repeated until X < t. */
static double orc_pg_left(double z, orc_ustream *s)
{
    const double t = ORC_PG_T;
    if (z < 1.0 / t) {
        for (;;) {
            double e1, e2, x;
            do {
                e1 = -log(orc_ustream_next(s));
                e2 = -log(orc_ustream_next(s));
            } while (e1 * e1 > 2.0 * e2 / t && !s->exhausted);
            x = t / ((1.0 + t * e1) * (1.0 + t * e1));
            if (orc_ustream_next(s) <= exp(-0.5 * z * z * x) || s->exhausted)
                return x;
        }
    } else {
        const double mu = 1.0 / z;
        for (;;) {
            double nrm = orc_ustream_normal(s);
            double y = nrm * nrm;
            double my = mu * y;
            double x = mu + 0.5 * mu * my - 0.5 * mu * sqrt(4.0 * my + my * my);
            if (orc_ustream_next(s) > mu / (mu + x))
                x = mu * mu / x;
            if (x < t || s->exhausted)
                return x;
        }
    }
}

/* PG(1, c) from the stream of term j.  Returns 0 and *out, or -1 when the
 * stream ran out (probability far below 1e-100). */
int orc_pg1(double c, uint64_t seed, uint32_t site, uint32_t sweep, uint32_t instance, uint32_t j,
            double *out)
{
    const double t = ORC_PG_T;
    const double z = 0.5 * fabs(c);
    const double K = ORC_PI * ORC_PI / 8.0 + 0.5 * z * z;
    double p, q;
    orc_ustream s;
    s.seed = seed;
    s.site = site;
    s.sweep = sweep;
    s.instance = instance;
    s.j = j;
    s.used = 0;
    s.exhausted = 0;
    /* masses of the two envelope pieces */
    p = ORC_PI / (2.0 * K) * exp(-K * t);
    if (z == 0.0) {
        q = 2.0 * erfc(1.0 / sqrt(2.0 * t));
    } else {
        double a = orc_std_normal_cdf((t * z - 1.0) / sqrt(t));
        double b = z < 700.0 ? exp(z) * orc_std_normal_cdf(-(t * z + 1.0) / sqrt(t)) : 0.0;
        q = 2.0 * (exp(-z) * a + b);
    }
    for (;;) {
        double x, S, Y;
        int n;
        if (orc_ustream_next(&s) < p / (p + q))
            x = t - log(orc_ustream_next(&s)) / K;
        else
            x = orc_pg_left(z, &s);
        S = orc_pg_term(0, x);
        Y = orc_ustream_next(&s) * S;
        if (s.exhausted)
            return -1;
        for (n = 1; n <= ORC_PG_MAX_TERMS; ++n) {
            if (n & 1) {
                S -= orc_pg_term(n, x);
                if (Y <= S) {
                    *out = 0.25 * x;
                    return 0;
                }
            } else {
                S += orc_pg_term(n, x);
                if (Y > S)
                    break;
            }
        }
    }
}

/* PG(b, c) for an integer b >= 0: the sum of PG(1, c) terms j = 0 .. b-1 in
 * order (PG(0, c) = 0). */
int orc_pg(int32_t b, double c, uint64_t seed, uint32_t site, uint32_t sweep, uint32_t instance,
           double *out)
{
    double sum = 0.0, v;
    int32_t j;
    for (j = 0; j < b; ++j) {
        if (orc_pg1(c, seed, site, sweep, instance, (uint32_t)j, &v))
            return -1;
        sum += v;
    }
    *out = sum;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampler                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int64_t *row_ptr;   /* n + 1 */
    const int32_t *col;       /* neighbours of each site, ascending */
    const int32_t *color;     /* proper coloring, 0 .. k-1 */
    int32_t k;
    double rho;               /* 1 = intrinsic (IAR) prior */
    const double *y;          /* observations, original order */
    double a_tau, b_tau, a_lam, b_lam;
    int64_t rank;             /* r in the tau shape a_tau + r/2 */
    int64_t burn_in;          /* sweeps with index < burn_in are not accumulated */
    uint64_t seed;
    uint32_t instance;
    int32_t intercept;        /* 1: the model has an intercept b0 */
    int32_t likelihood;       /* 0 Gaussian (y = b0 + x + e), 1 binomial logit */
    const int32_t *trials;    /* binomial: m_i (y holds the successes Y_i) */
    double beta0_var;         /* binomial: prior variance v0 of b0 (0 = flat) */
    int32_t rng_version;      /* 1 (or 0): one block per site; 2: paired sites */
    const int32_t *pair_key;  /* version 2: orc_rng_pairs of the coloring */
    const uint8_t *pair_branch;
} orc_problem;

#define ORC_BINOMIAL 1

typedef struct {
    double *x;                /* current field, original order */
    double *s1, *s2;          /* running sums of x and x^2 */
    double tau, lam;          /* prior precision, noise precision */
    int64_t sweep;            /* number of completed sweeps */
    int64_t n_acc;            /* number of accumulated sweeps */
    double q, sse;            /* x'(D - rho W)x and ||y - b0 - x||^2 after the last sweep */
    int32_t status;           /* 0 ok, 1 Gamma attempt cap hit or non-finite draw */
    double beta0;             /* intercept (stays 0 without the intercept) */
    double *psi;              /* binomial: the psi_i of the last sweep (n) */
    double rsum;              /* binomial: sum_i (kappa_i - psi_i x_i) after the last sweep */
} orc_chain;

#define ORC_WITH_HYPER 1u
#define ORC_ZERO_NOISE 2u
#define ORC_GAMMA_MAX_ATTEMPTS 64

/* Pairwise (recursive halving) sum, a fixed summation tree. */
static double orc_pairwise(const double *v, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        int64_t i;
        for (i = 0; i < n; ++i)
            s += v[i];
        return s;
    }
    return orc_pairwise(v, n / 2) + orc_pairwise(v + n / 2, n - n / 2);
}

/* q = x'(D - rho W)x written edge-wise as
 *   (1 - rho) sum_i D_ii x_i^2 + rho sum_{i<j, i~j} (x_i - x_j)^2,
 * and sse = sum_i (y_i - b0 - x_i)^2; each as a pairwise sum of per-site
 * terms. */
static void orc_quadratic_terms_b0(const orc_problem *p, const double *x, double b0, double *q,
                                   double *sse);

void orc_quadratic_terms(const orc_problem *p, const double *x, double *q, double *sse)
{
    orc_quadratic_terms_b0(p, x, 0.0, q, sse);
}

static void orc_quadratic_terms_b0(const orc_problem *p, const double *x, double b0, double *q,
                                   double *sse)
{
    int64_t n = p->n, i, e;
    double *tq = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *ts = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (i = 0; i < n; ++i) {
        double deg = (double)(p->row_ptr[i + 1] - p->row_ptr[i]);
        double edge = 0.0, r;
        for (e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
            int64_t j = p->col[e];
            if (j > i) {
                double d = x[i] - x[j];
                edge += d * d;
            }
        }
        tq[i] = (1.0 - p->rho) * deg * x[i] * x[i] + p->rho * edge;
        r = p->y[i] - b0 - x[i];
        ts[i] = r * r;
    }
    *q = orc_pairwise(tq, n);
    *sse = orc_pairwise(ts, n);
    free(tq);
    free(ts);
}

/* Draw tau then lam from the reductions of the last completed sweep, using
 * sweep index (sweep - 1) in the Philox counter. */
int orc_hyper(const orc_problem *p, orc_chain *s)
{
    uint32_t t = (uint32_t)(s->sweep - 1);
    double tau, lam;
    int a1, a2;
    if (p->likelihood == ORC_BINOMIAL) {
        /* b0 | x, psi ~ N(sum(kappa - psi x) / P, 1/P) (the sse slot holds
         * sum psi after a binomial sweep), then tau */
        if (p->intercept) {
            double P = s->sse + (p->beta0_var > 0.0 ? 1.0 / p->beta0_var : 0.0);
            double z = orc_normal(p->seed, 0u, t, p->instance, 3u);
            s->beta0 = s->rsum / P + z / sqrt(P);
        }
        a1 = orc_gamma(p->a_tau + 0.5 * (double)p->rank, p->b_tau + 0.5 * s->q, p->seed, t,
                       p->instance, 1u, ORC_GAMMA_MAX_ATTEMPTS, &tau);
        if (a1 < 0 || !isfinite(tau) || !isfinite(s->beta0)) {
            s->status = 1;
            return 1;
        }
        s->tau = tau;
        return 0;
    }
    if (p->intercept) {
        /* b0 | x, lam ~ N(mean(y - x), 1 / (n lam)), then lam's sum of squares
         * with the new b0 (the x of the last sweep is unchanged) */
        int64_t i, n = p->n;
        double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double mean, z, qq;
        for (i = 0; i < n; ++i)
            d[i] = p->y[i] - s->x[i];
        mean = orc_pairwise(d, n) / (double)n;
        free(d);
        z = orc_normal(p->seed, 0u, t, p->instance, 3u);
        s->beta0 = mean + z / sqrt((double)n * s->lam);
        orc_quadratic_terms_b0(p, s->x, s->beta0, &qq, &s->sse);
    }
    a1 = orc_gamma(p->a_tau + 0.5 * (double)p->rank, p->b_tau + 0.5 * s->q, p->seed, t,
                       p->instance, 1u, ORC_GAMMA_MAX_ATTEMPTS, &tau);
    a2 = orc_gamma(p->a_lam + 0.5 * (double)p->n, p->b_lam + 0.5 * s->sse, p->seed, t,
                       p->instance, 2u, ORC_GAMMA_MAX_ATTEMPTS, &lam);
    if (a1 < 0 || a2 < 0 || !isfinite(tau) || !isfinite(lam)) {
        s->status = 1;
        return 1;
    }
    s->tau = tau;
    s->lam = lam;
    return 0;
}

/* One site of Algorithm 1: conditional mean and precision, then the draw. */
static void orc_update_site(const orc_problem *p, orc_chain *s, int64_t i, uint32_t t,
                            uint32_t flags)
{
    double sum = 0.0, deg, Qii, m, z;
    int64_t e;
    for (e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e)
        sum += s->x[p->col[e]];
    deg = (double)(p->row_ptr[i + 1] - p->row_ptr[i]);
    if (p->likelihood == ORC_BINOMIAL) {
        /* psi_i | x_i, b0 ~ PG(m_i, b0 + x_i), with this site's old x_i */
        double psi = 0.0, kappa = p->y[i] - 0.5 * (double)p->trials[i];
        if (orc_pg(p->trials[i], s->beta0 + s->x[i], p->seed, (uint32_t)i, t, p->instance, &psi))
            s->status = 1;
        s->psi[i] = psi;
        Qii = s->tau * deg + psi;
        m = (kappa - psi * s->beta0 + s->tau * p->rho * sum) / Qii;
    } else {
        Qii = s->tau * deg + s->lam;
        m = (s->lam * (p->y[i] - s->beta0) + s->tau * p->rho * sum) / Qii;
    }
    if (flags & ORC_ZERO_NOISE)
        z = 0.0;
    else if (p->rng_version == 2)
        z = orc_normal_pair(p->seed, (uint32_t)p->pair_key[i], p->pair_branch[i], t, p->instance,
                            0u);
    else
        z = orc_normal(p->seed, (uint32_t)i, t, p->instance, 0u);
    s->x[i] = m + z / sqrt(Qii);
}

/* Run nsweeps sweeps.  visit (optional, length n) lists the sites in the
 * order they are visited inside each color; NULL means ascending id.  The
 * result does not depend on it because a color's sites never read one
 * another.  nthreads > 1 spreads the sites of one color over threads. */
int orc_sweeps(const orc_problem *p, orc_chain *s, int64_t nsweeps, uint32_t flags,
               const int64_t *visit, int32_t nthreads)
{
    int64_t it, n = p->n;
    if (p->rng_version == 2 && n > 0 && (!p->pair_key || !p->pair_branch))
        return 1;
#ifdef _OPENMP
    if (nthreads < 1)
        nthreads = 1;
#else
    (void)nthreads;
#endif
    for (it = 0; it < nsweeps; ++it) {
        uint32_t t = (uint32_t)s->sweep;
        int32_t c;
        int64_t i;
        for (c = 0; c < p->k; ++c) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
            for (i = 0; i < n; ++i) {
                int64_t site = visit ? visit[i] : i;
                if (p->color[site] == c)
                    orc_update_site(p, s, site, t, flags);
            }
        }
        if (s->status)
            return 1;
        orc_quadratic_terms_b0(p, s->x, s->beta0, &s->q, &s->sse);
        if (p->likelihood == ORC_BINOMIAL) {
            /* the b0 conditional's sums: sum psi (in the sse slot) and
             * sum (kappa - psi x) */
            double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
            s->sse = orc_pairwise(s->psi, n);
            for (i = 0; i < n; ++i)
                d[i] = (p->y[i] - 0.5 * (double)p->trials[i]) - s->psi[i] * s->x[i];
            s->rsum = orc_pairwise(d, n);
            free(d);
        }
        if ((int64_t)t >= p->burn_in) {
            for (i = 0; i < n; ++i) {
                double phi = s->x[i] + s->beta0;   /* the image b0 + x (x without b0) */
                s->s1[i] += phi;
                s->s2[i] += phi * phi;
            }
            s->n_acc += 1;
        }
        s->sweep += 1;
        if (flags & ORC_WITH_HYPER) {
            if (orc_hyper(p, s))
                return 1;
        }
    }
    return 0;
}

/* Posterior mean S1/N and unbiased variance (S2 - S1^2/N)/(N-1). */
void orc_stats(const orc_chain *s, int64_t n, double *mean, double *var)
{
    int64_t i;
    double N = (double)s->n_acc;
    for (i = 0; i < n; ++i) {
        mean[i] = s->s1[i] / N;
        var[i] = (s->s2[i] - s->s1[i] * s->s1[i] / N) / (N - 1.0);
    }
}
