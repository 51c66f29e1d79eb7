// gmrf.hip -- HIP kernels and C ABI of libgmrf (gfx950).
//
// Hot path (Sec. 2.3, Algorithm 1, with the full conditionals of Sec. 3.1 /
// 3.2 and the conjugate precision draws of Sec. 3.1):
//
//   * Lattice graphs (4- and 8-neighbour stencils, parity colorings): ONE
//     kernel per sweep.  Each workgroup owns a TH x TW tile of the lattice,
//     stages the tile plus the halo its phases read (k rings, k the number
//     of colors; for 8 neighbours one ring fewer before the tile) in LDS,
//     and runs the k color phases in LDS.  Phase j updates the sites of color
//     j on the tile grown by k-1-j rings, so the values that later phases read
//     at the tile border are recomputed locally instead of being exchanged:
//     the random numbers are keyed by (site, sweep), so a recomputed halo site
//     is bitwise the value its owning tile computes.  The lattice state is
//     ping-ponged between two buffers (sweep t reads buffer t&1 and writes the
//     other), so tiles never see a neighbour's new values through memory.
//   * General graphs (CSR): one kernel per color over a contiguous color slab
//     of a color-permuted CSR; sites of one color never read each other, so
//     the slab is updated in place.
//   * Every sweep kernel fuses the reductions q = x'(D - rho W)x (each edge
//     counted once, by its higher-colored endpoint, after both ends are final)
//     and sse = ||y - x||^2 in FP64, and the posterior accumulators.  Blocks
//     leave FP64 partials; the end of a sweep sums them in fixed slot order
//     and draws tau and lam on the device, so a sweep has no host round trip.
//     A lattice sweep kernel begins by ending the previous sweep of its call:
//     every block sums that sweep's partials and draws the same tau and lam
//     while its tile loads are in flight (one block records them), so a
//     lattice sweep is ONE launch; a one-block commit kernel ends the last
//     sweep of each call.  General graphs end every sweep with that kernel.
//     The rate-free parts of the draws (the Marsaglia-Tsang variate at rate
//     1, the beta0 normal) depend only on the sweep index: a small kernel
//     draws them up to kUnitBatch sweeps ahead, so no sweep kernel carries
//     the Gamma sampler's registers.
//   * The sweep index t lives in device memory, so a captured HIP graph of
//     sweeps can be replayed.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_set>
#include <type_traits>
#include <utility>
#include <vector>

#include "gmrf.h"
#include "internal.hpp"
#include "rng.hpp"

namespace gmrf {

const char *error_cstr();

// ---------------------------------------------------------------------------
// device-side chain state
// ---------------------------------------------------------------------------
struct DevState {
    double tau, lam;            // current precisions
    double q, sse;              // reductions of the last completed sweep (sse at beta0)
    unsigned long long sweep;   // completed sweeps
    long long n_acc;            // accumulated sweeps
    unsigned int status;        // bit 0: Gamma draw failed / non-finite; bit 1: no unit variates
    unsigned int pad;
    double beta0;               // intercept (0 without one)
    double rsum;                // sum_i (y_i - beta0 - x_i) of the last completed sweep
    double *trace;              // NULL, or (tau, lam, beta0) per completed sweep
    long long trace_cap;        // rows of trace
    unsigned long long unit_base;   // sweep index of the first row of the unit-variate ring
    // Within one call of lattice sweeps: (tau, lam, beta0) that relative sweep
    // j >= 1 of the call runs with, at hs[j & 1] (relative sweep 0 runs with
    // the committed tau, lam, beta0 above).  The commit at the end of the call
    // moves the last draws into the committed fields.
    double hs[2][3];
};

constexpr unsigned kStatusGamma = 1u;
constexpr unsigned kStatusUnits = 2u;

// The random parts of the draws after sweep t, which do not depend on the
// sweep's reductions: the beta0 normal (tag-3 normal at counter (0, t)) and,
// in lane 0 for tau (tag 1) and lane 1 for lam (tag 2), the Marsaglia-Tsang
// variate d v of the conditional's shape at rate 1.  Its accept / reject
// decisions involve only the shape, and the draw at rate b is (d v) / b, the
// division gamma_draw ends with, so drawing the unit variate early changes
// no bit of the result.
struct UnitDraws {
    double z, g;
    bool ok;
};

// Sweeps of a call between two unit-variate launches, and the rows of the
// ring (one more: a lattice call's sweep at the start of a group ends the
// previous group's last sweep).
constexpr int kUnitBatch = 128;
constexpr int kUnitRows = kUnitBatch + 1;

struct SweepArgs {
    DevState *st;
    double *partials;           // three doubles (q, sse, rsum) per block slot
    double *s1, *s2;            // posterior accumulators (layout of x)
    GammaShape g_tau, g_lam;    // Marsaglia-Tsang constants of a_tau + r/2, a_lam + n/2
    double b_tau, b_lam;
    double rho;
    long long burn_in;
    unsigned long long seed;
    unsigned int instance;
    int with_hyper;
    int total_slots;            // blocks per sweep (all color passes)
    int intercept;              // 1: draw beta0 before tau / lam
    int likelihood;             // 0 Gaussian, 1 binomial logit (Polya-Gamma)
    int dry;                    // timing runs: write no chain state, trace or accumulators
    double b0_prec;             // binomial: prior precision of beta0 (0 = flat)
    double n_sites;
    UnitDraws *units;           // ring of 2 kUnitRows unit variates (sweep - unit_base, lane)
    int slot_stride;            // lattice: doubles between the two partial buffers / kPartials
    int deferred;               // 1: lattice sweeps end in the next sweep kernel of the call
};

constexpr int kPartials = 3;

constexpr int kThreads = 256;   // CSR passes and stats kernels

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Barrier that orders LDS only: global loads issued before it stay in flight
// (a plain __syncthreads() would also wait for every outstanding global load).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block sum of three values in a fixed tree; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *red)
{
    constexpr int W = NT / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid] = a;
        red[W + wid] = b;
        red[2 * W + wid] = c;
    }
    lds_barrier();
    if (threadIdx.x == 0) {
        a = red[0];
        b = red[W];
        c = red[2 * W];
        for (int w = 1; w < W; ++w) {
            a += red[w];
            b += red[W + w];
            c += red[2 * W + w];
        }
    }
}

// The FP64 sums a sweep block contributes: q = x'(D - rho W)x terms, and the
// residuals r_i = y_i - beta0 - x_i as sse = sum r_i^2 and rsum = sum r_i.
// For the binomial model the last two slots hold sum psi_i and
// sum (kappa_i - psi_i x_i), the sums of the beta0 conditional.
struct Red {
    double q = 0.0, sse = 0.0, rsum = 0.0;
};

// A sweep block's partials, summed later in slot order (P: the sweep's
// partial buffer).
template <int NT>
__device__ __forceinline__ void write_partials(double *P, Red r, int slot)
{
    __shared__ double red[kPartials * (NT / 64)];
    block_sum3<NT>(r.q, r.sse, r.rsum, red);
    if (threadIdx.x == 0) {
        P[kPartials * slot] = r.q;
        P[kPartials * slot + 1] = r.sse;
        P[kPartials * slot + 2] = r.rsum;
    }
}

// Values of the chain state that the end-of-sweep draws read.
struct HyperIn {
    double tau, lam, beta0;
};

__device__ __forceinline__ UnitDraws unit_draws(const SweepArgs &a, unsigned t, int lane)
{
    UnitDraws u{0.0, 0.0, false};
    if (a.with_hyper && a.intercept)
        u.z = normal_f64(draw_words(a.seed, 0u, t, a.instance, 3u));
    if (a.with_hyper && lane < (a.likelihood ? 1 : 2))    // no noise precision if binomial
        u.ok = gamma_draw(lane == 0 ? a.g_tau : a.g_lam, 1.0, a.seed, t, a.instance,
                          (unsigned)(lane + 1), &u.g);
    return u;
}

// The draws after sweep t (Sec. 3.1 conjugate conditionals, precisions in
// rate form), in lanes 0 and 1 of one wavefront, from the lane's unit
// variates `u`; `r` holds the reductions of sweep t, `in` the state the
// sweep ran with.  With an intercept, first
//     beta0 ~ N(mean(y - x), 1 / (n lam))      (flat prior on beta0)
// and sse and rsum move to the new beta0:  with d = beta0' - beta0,
//     sum (r_i - d)^2 = sse - 2 d rsum + n d^2,   sum (r_i - d) = rsum - n d.
// Then tau (lane 0) and lam (lane 1).  Lane 0 stores the reductions; the
// trace row t, if any, gets (tau, lam, beta0) after the draws.  With commit
// the draws also become the chain's committed tau, lam and beta0 (without
// it, inside a call of lattice sweeps, the caller keeps them).
__device__ __forceinline__ HyperIn end_of_sweep_draws(const SweepArgs &a, unsigned t, Red r,
                                                      const HyperIn &in, int lane,
                                                      const UnitDraws &u, bool commit = true)
{
    double b0 = in.beta0;
    if (a.with_hyper && a.intercept) {
        if (a.likelihood) {
            // binomial (Sec. 3.2 augmented model): beta0 | x, psi ~
            // N(sum(kappa - psi x) / P, 1 / P), P = sum psi + prior precision
            const double P = r.sse + a.b0_prec;
            b0 = r.rsum / P + u.z / sqrt(P);
        } else {
            const double mean = in.beta0 + r.rsum / a.n_sites;
            b0 = mean + u.z / sqrt(a.n_sites * in.lam);
            const double d = b0 - in.beta0;
            r.sse = r.sse - 2.0 * d * r.rsum + a.n_sites * d * d;
            r.rsum = r.rsum - a.n_sites * d;
        }
    }
    double v = lane == 0 ? in.tau : in.lam;
    if (a.with_hyper && lane < (a.likelihood ? 1 : 2)) {
        const double rate = lane == 0 ? a.b_tau + 0.5 * r.q : a.b_lam + 0.5 * r.sse;
        const double draw = u.ok ? u.g / rate : 0.0;
        if (u.ok && isfinite(draw) && draw > 0.0 && isfinite(b0)) {
            v = draw;
            if (!a.dry && commit) {
                if (lane == 0)
                    a.st->tau = v;
                else
                    a.st->lam = v;
            }
        } else if (!a.dry) {
            atomicOr(&a.st->status, kStatusGamma);
        }
    }
    const double other = __shfl(v, 1, 64);   // lam after the draw, from lane 1
    if (lane == 0 && !a.dry) {
        a.st->q = r.q;
        a.st->sse = r.sse;
        a.st->rsum = r.rsum;
        if (commit)
            a.st->beta0 = b0;
        double *const tr = a.st->trace;   // read at run time: batches and graphs see changes
        if (tr && (long long)t < a.st->trace_cap) {
            tr[3 * (size_t)t] = v;
            tr[3 * (size_t)t + 1] = other;
            tr[3 * (size_t)t + 2] = b0;
        }
    }
    return HyperIn{v, other, b0};    // valid in lane 0
}

// The same with the unit variates drawn in place.
__device__ __forceinline__ HyperIn end_of_sweep_draws(const SweepArgs &a, unsigned t, Red r,
                                                      const HyperIn &in, int lane)
{
    return end_of_sweep_draws(a, t, r, in, lane, unit_draws(a, t, lane));
}

// The persistent kernels draw the unit variates of kUnitBatch sweeps at a
// time, one thread per (sweep, lane), ahead of the sweeps: they depend only on
// the sweep index, so no sweep then waits for a Gamma draw.
// Unit variates of sweeps t .. t + cnt - 1 (cnt <= kUnitBatch) into
// ub[sweep - t][lane]; the caller synchronises before reading them.
template <int NT>
__device__ __forceinline__ void unit_draw_batch(const SweepArgs &a, unsigned t, int cnt,
                                                UnitDraws (*ub)[2])
{
    static_assert(NT >= 2 * kUnitBatch, "one thread per sweep and lane");
    const int i = (int)threadIdx.x;
    if (i < 2 * cnt)
        ub[i >> 1][i & 1] = unit_draws(a, t + (unsigned)(i >> 1), i & 1);
}

// The unit-variate ring.  Before a group of at most kUnitBatch sweeps a
// small kernel draws the unit variates of the sweeps the group ends, one
// thread per (sweep, lane), so that the end of a sweep only divides by the
// rates.  Its rows start at sweep st->sweep + first (the committed sweep
// count plus the sweeps of the call not yet committed); for a lattice call
// the rows of a later group start one sweep before it, whose end the
// group's first sweep kernel computes.
__device__ __forceinline__ void unit_ring_fill(const SweepArgs &a, int first, int cnt)
{
    const unsigned t = (unsigned)(a.st->sweep + (unsigned long long)first);
    for (int i = (int)threadIdx.x; i < 2 * cnt; i += (int)blockDim.x)
        a.units[i] = unit_draws(a, t + (unsigned)(i >> 1), i & 1);
    if (threadIdx.x == 0)
        a.st->unit_base = (unsigned long long)t;
}

// Rows (first, count) of the ring for the group of the call's sweeps g ..
// g + n - 1 (host and device).
__host__ __device__ inline void unit_rows(int deferred, int g, int n, int *first, int *cnt)
{
    const int back = deferred && g > 0 ? 1 : 0;   // the previous group's last sweep
    *first = deferred ? g - back : 0;             // general graphs commit every sweep
    *cnt = n + back;
}

constexpr int kUnitThreads = 256;

__global__ __launch_bounds__(kUnitThreads) void unit_draw_kernel(SweepArgs a, int g, int n)
{
    int first, cnt;
    unit_rows(a.deferred, g, n, &first, &cnt);
    unit_ring_fill(a, first, cnt);
}

// Batched form: block b fills the ring of chain b.
__global__ __launch_bounds__(kUnitThreads) void unit_draw_batch_kernel(const SweepArgs *args,
                                                                        int g, int n)
{
    SweepArgs a = args[blockIdx.x];
    a.with_hyper = 1;
    int first, cnt;
    unit_rows(a.deferred, g, n, &first, &cnt);
    unit_ring_fill(a, first, cnt);
}

// Partial buffer of relative sweep rel of a call (lattice chains alternate
// two buffers, so a sweep kernel can read its predecessor's partials while
// its blocks write their own).
__device__ __forceinline__ double *partials_of(const SweepArgs &a, int rel)
{
    return a.partials + (size_t)kPartials * (size_t)a.slot_stride * (size_t)(rel & 1);
}

// The state relative sweep rel of a call runs with: the committed values
// for rel 0, else the ones the sweep before it drew.
__device__ __forceinline__ HyperIn inputs_of(const SweepArgs &a, int rel)
{
    if (rel == 0)
        return HyperIn{a.st->tau, a.st->lam, a.st->beta0};
    const double *h = a.st->hs[rel & 1];
    return HyperIn{h[0], h[1], h[2]};
}

// End of sweep t, run by a whole block (NT >= kFinishThreads threads): sum
// its partials P in slot order (thread i < kFinishThreads takes slots i,
// i + kFinishThreads, ..., then a fixed tree), and draw beta0 / tau / lam
// from the ring's unit variates (end_of_sweep_draws, which also stores q /
// sse and the trace row unless a.dry).  Returns the draws in every thread.
// The two halves (fold_partials, then a barrier, then fold_draws) may be run
// apart, with other work between them.
constexpr int kFinishThreads = 256;

struct FoldLds {
    double red[kPartials * (kFinishThreads / 64)];
    double hyp[3];
};

// Per-wave sums of the partials into L.red (U: slots per thread in flight).
template <int U>
__device__ __forceinline__ void fold_partials(const SweepArgs &a, const double *P, FoldLds &L)
{
    constexpr int W = kFinishThreads / 64;
    const int lane = (int)threadIdx.x & 63, wid = (int)threadIdx.x >> 6;
    if (wid < W) {
        Red r;
        for (int i0 = threadIdx.x; i0 < a.total_slots; i0 += U * kFinishThreads) {
            double v[kPartials * U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * kFinishThreads;
#pragma unroll
                for (int w = 0; w < kPartials; ++w)
                    v[kPartials * u + w] = P[kPartials * min(i, a.total_slots - 1) + w];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * kFinishThreads < a.total_slots) {
                    r.q += v[kPartials * u];
                    r.sse += v[kPartials * u + 1];
                    r.rsum += v[kPartials * u + 2];
                }
        }
        r.q = wave_sum(r.q);
        r.sse = wave_sum(r.sse);
        r.rsum = wave_sum(r.rsum);
        if (lane == 0) {
            L.red[wid] = r.q;
            L.red[W + wid] = r.sse;
            L.red[2 * W + wid] = r.rsum;
        }
    }
}

// The wave sums in order, and the draws (after a barrier that follows
// fold_partials); ends with a barrier.
__device__ __forceinline__ HyperIn fold_draws(const SweepArgs &a, unsigned t, const HyperIn &in,
                                              bool commit, FoldLds &L)
{
    constexpr int W = kFinishThreads / 64;
    const int lane = (int)threadIdx.x & 63, wid = (int)threadIdx.x >> 6;
    if (wid == 0) {
        Red r;
        r.q = L.red[0];
        r.sse = L.red[W];
        r.rsum = L.red[2 * W];
        for (int w = 1; w < W; ++w) {
            r.q += L.red[w];
            r.sse += L.red[W + w];
            r.rsum += L.red[2 * W + w];
        }
        UnitDraws u{0.0, 0.0, false};
        if (a.with_hyper && lane < 2) {
            const unsigned long long row = (unsigned long long)t - a.st->unit_base;
            if (row < (unsigned long long)kUnitRows)
                u = a.units[2 * row + lane];
            else if (!a.dry)
                atomicOr(&a.st->status, kStatusUnits);
        }
        const HyperIn out = end_of_sweep_draws(a, t, r, in, lane, u, commit);
        if (lane == 0) {
            L.hyp[0] = out.tau;
            L.hyp[1] = out.lam;
            L.hyp[2] = out.beta0;
        }
    }
    lds_barrier();
    return HyperIn{L.hyp[0], L.hyp[1], L.hyp[2]};
}

template <int NT>
__device__ __forceinline__ HyperIn end_sweep_block(const SweepArgs &a, const double *P, unsigned t,
                                                   const HyperIn &in, bool commit)
{
    static_assert(NT >= kFinishThreads && NT % 64 == 0, "the finish needs kFinishThreads threads");
    __shared__ FoldLds L;
    fold_partials<4>(a, P, L);
    lds_barrier();
    return fold_draws(a, t, in, commit, L);
}

// Commit the end of a call: end its relative sweep rel (the last of the
// call's count sweeps) and make the draws the chain's state, count the
// call's accumulated sweeps and advance the sweep count.  General graphs
// commit every sweep (rel 0, count 1).
__device__ __forceinline__ void commit_block(const SweepArgs &a, int rel, int count)
{
    const unsigned long long t0 = a.st->sweep;
    const unsigned t = (unsigned)(t0 + (unsigned long long)rel);
    const HyperIn in = inputs_of(a, rel);
    end_sweep_block<kFinishThreads>(a, partials_of(a, rel), t, in, true);
    if (threadIdx.x == 0 && !a.dry) {
        const long long lo = (long long)t0 > a.burn_in ? (long long)t0 : a.burn_in;
        const long long acc = (long long)t0 + count - lo;
        if (acc > 0)
            a.st->n_acc += acc;
        a.st->sweep = t0 + (unsigned long long)count;
    }
}

__global__ __launch_bounds__(kFinishThreads) void commit_kernel(SweepArgs a, int rel, int count)
{
    commit_block(a, rel, count);
}

// Batched form: block b commits chain b of the table; with_hyper: this call's
// GMRF_WITH_HYPER (the tables are built once).
__global__ __launch_bounds__(kFinishThreads) void commit_batch_kernel(const SweepArgs *args, int rel,
                                                                       int count, int with_hyper)
{
    SweepArgs a = args[blockIdx.x];
    a.with_hyper = with_hyper;
    commit_block(a, rel, count);
}

// ---------------------------------------------------------------------------
// the site update shared by every sweep kernel
// ---------------------------------------------------------------------------
// Conditional precision Qii = tau D_ii + lam (Sec. 3.1 local characteristics
// in precision form) and its scales 1/Qii and Qii^-1/2.  Every kernel computes
// them with this one instruction sequence, so a site recomputed in a tile
// halo is bitwise the value its owner computes.
template <typename Real>
__device__ __forceinline__ void site_scales(Real tau, Real lam, int deg, Real &inv_q, Real &isd)
{
    const Real Q = fma(tau, (Real)deg, lam);
    if constexpr (sizeof(Real) == 8) {
        inv_q = 1.0 / Q;
        isd = 1.0 / sqrt(Q);
    } else {
        inv_q = 1.0f / Q;
        isd = __builtin_amdgcn_rsqf(Q);
    }
}

// x_i = m_i + z / sqrt(Qii), m_i = (lam y_i + tau rho s_i) / Qii.
template <typename Real>
__device__ __forceinline__ Real site_draw(Real yv, Real s, Real z, Real lam, Real tau_rho,
                                          Real inv_q, Real isd)
{
    const Real m = fma(tau_rho, s, lam * yv) * inv_q;
    return fma(z, isd, m);
}

// ---------------------------------------------------------------------------
// lattice: fused all-colors sweep
// ---------------------------------------------------------------------------
template <typename Real> struct LatArgs {
    Real *x0, *x1;              // ping-pong state buffers, row-major
    const Real *y;
    int rows, cols;
    int tiles_c;                // tiles per lattice row
};

// Color of a lattice site under the parity coloring of the stencil.
template <int ST> __host__ __device__ constexpr int parity_color(int pr, int pc)
{
    return ST == 4 ? ((pr + pc) & 1) : (2 * (pr & 1) + (pc & 1));
}

// Does the neighbour at offset (dr, dc) of a color-J site have a lower color?
// (J's parities: 8-neighbour: row parity J>>1, column parity J&1;
// 4-neighbour: r + c parity J, represented as row parity 0, column parity J.)
template <int ST, int J> __host__ __device__ constexpr bool lower_nb(int dr, int dc)
{
    return ST == 4 ? (parity_color<4>(0, J + dr + dc) < J)
                   : (parity_color<8>((J >> 1) + dr, (J & 1) + dc) < J);
}

template <typename Real> struct SiteCtx {
    Real tau, lam, tau_rho;
    Real beta0_r;               // intercept in the state precision
    double beta0;
    Real inv_q_full, isd_full;  // 1/Qii and Qii^-1/2 of a site with all k neighbours
    const Real *qtab;           // LDS: 1/Qii for degree 0 .. ST, then Qii^-1/2 (qtab_fill)
    double one_minus_rho, rho;
    unsigned t;
    unsigned long long seed;
    unsigned instance;
};

// Tile geometry of the fused lattice kernel: TH x TW interior sites, NT
// threads, the halo (see below); the accumulator read-modify-write of the
// interior is issued CH sites per thread at a time.
template <int ST_, int TH_, int TW_, int NT_, int CH_> struct LatCfg {
    static constexpr int ST = ST_, TH = TH_, TW = TW_, NT = NT_, CH = CH_;
    static constexpr int K = ST == 4 ? 2 : 4;
    // Halo rings.  With the tile at an even (r0, c0), phase J computes the
    // color-J sites of the tile grown by K - 1 - J rings and reads one ring
    // further.  8 neighbours: phase 0's sites (even rows and columns) reach
    // ring 2 before the tile and ring 3 after it (rows r0 - 2 and
    // r0 + TH + 2, likewise for columns), so the phases read 3 rings before
    // and 4 after; 4 neighbours: 2 and 2.  H (rings before, the LDS offset of
    // the tile) and HH (rings after):
    static constexpr int H = ST == 8 ? K - 1 : K;
    static constexpr int HH = K;
    static constexpr int LH = TH + H + HH, LW = TW + H + HH;
    static_assert(TH % 2 == 0 && TW % 2 == 0, "tile sides must be even");
    static_assert(NT % 64 == 0, "whole wavefronts");
};

// 1/Qii and Qii^-1/2 for every degree 0 .. ST into the LDS table (threads
// 0 .. ST), with site_scales, so a lookup is bitwise the per-site value.  The
// caller synchronises before the table is read.
template <typename Real, int ST>
__device__ __forceinline__ void qtab_fill(Real *qtab, Real tau, Real lam)
{
    const int d = (int)threadIdx.x;
    if (d <= ST)
        site_scales<Real>(tau, lam, d, qtab[d], qtab[ST + 1 + d]);
}

// One site of Algorithm 1 on the LDS tile: neighbour sum in ascending
// original-id order, conditional mean and precision, the draw with the
// site's standard normal z; for interior sites also the q / sse terms.
// Cells of the tile outside the lattice hold 0 (lattice_load), so the
// neighbour sum adds every stencil cell: a missing neighbour adds 0, which
// leaves each partial sum of the in-lattice neighbours unchanged.
// INTERIOR: the tile and its halo lie inside the lattice, so every site has
// all its neighbours (compile-time flags).
template <typename Real, typename Cfg, int J, bool INTERIOR, bool B0>
__device__ __forceinline__ void lattice_site(Real *xs, Real yv, Real z, int r, int c, int r0,
                                             int c0, int rows, int cols, const SiteCtx<Real> &sc,
                                             Red &rd)
{
    constexpr int ST = Cfg::ST, H = Cfg::H, LW = Cfg::LW;
    Real *p = xs + (r - r0 + H) * LW + (c - c0 + H);
    const bool up = INTERIOR || r > 0, dn = INTERIOR || r + 1 < rows;
    const bool lf = INTERIOR || c > 0, rt = INTERIOR || c + 1 < cols;
    Real s = (Real)0;
    if (ST == 8) s += p[-LW - 1];
    s += p[-LW];
    if (ST == 8) s += p[-LW + 1];
    s += p[-1];
    s += p[1];
    if (ST == 8) s += p[LW - 1];
    s += p[LW];
    if (ST == 8) s += p[LW + 1];

    Real inv_q, isd;
    if constexpr (INTERIOR) {
        inv_q = sc.inv_q_full;
        isd = sc.isd_full;
    } else {
        const int nr = 1 + (int)up + (int)dn, nc = 1 + (int)lf + (int)rt;
        const int deg = ST == 8 ? nr * nc - 1 : nr + nc - 2;
        inv_q = sc.qtab[deg];
        isd = sc.qtab[ST + 1 + deg];
    }
    const Real yeff = B0 ? yv - sc.beta0_r : yv;
    const Real xn = site_draw<Real>(yeff, s, z, sc.lam, sc.tau_rho, inv_q, isd);
    *p = xn;

    if (r >= r0 && r < r0 + Cfg::TH && c >= c0 && c < c0 + Cfg::TW) {
        const double xd = (double)xn;
        double edge = 0.0;
#define GMRF_EDGE(cond, dr, dc, off)                                                  \
    if (lower_nb<ST, J>(dr, dc) && (cond)) {                                          \
        const double d = xd - (double)p[off];                                         \
        edge += d * d;                                                                \
    }
        if (ST == 8) GMRF_EDGE(up && lf, -1, -1, -LW - 1)
        GMRF_EDGE(up, -1, 0, -LW)
        if (ST == 8) GMRF_EDGE(up && rt, -1, 1, -LW + 1)
        GMRF_EDGE(lf, 0, -1, -1)
        GMRF_EDGE(rt, 0, 1, 1)
        if (ST == 8) GMRF_EDGE(dn && lf, 1, -1, LW - 1)
        GMRF_EDGE(dn, 1, 0, LW)
        if (ST == 8) GMRF_EDGE(dn && rt, 1, 1, LW + 1)
#undef GMRF_EDGE
        int deg = ST;
        if constexpr (!INTERIOR) {
            const int nr = 1 + (int)up + (int)dn, nc = 1 + (int)lf + (int)rt;
            deg = ST == 8 ? nr * nc - 1 : nr + nc - 2;
        }
        rd.q += sc.one_minus_rho * (double)deg * xd * xd + sc.rho * edge;
        if constexpr (B0) {
            const double rr = (double)yv - sc.beta0 - xd;
            rd.sse += rr * rr;
            rd.rsum += rr;
        } else {
            const double rr = (double)yv - xd;
            rd.sse += rr * rr;
        }
    }
}

// Quotient and remainder of idx by d (0 <= idx < 2^24, d >= 1) through an FP32
// reciprocal with a one-step correction.
__device__ __forceinline__ int div_small(int idx, int d, float rcp, int &rem)
{
    int qt = (int)((float)idx * rcp);
    qt -= (qt * d > idx);
    qt += ((qt + 1) * d <= idx);
    rem = idx - qt * d;
    return qt;
}

// The color-J sites of the tile grown by E = k-1-J rings: rows ra .. rb - 1
// and columns ca .. cb - 1 (8 neighbours: ra and ca moved to the parities of
// J), nR rows of at most nC sites each.  Unit idx = R nC + C of a phase is
// the site (ra + R, ca + ((r + ca + J) & 1) + 2 C) for 4 neighbours and
// (ra + 2 R, ca + 2 C) for 8.
struct PhaseGeom {
    int ra, rb, ca, cb, nR, nC;
};

template <typename Cfg, int J>
__device__ __forceinline__ PhaseGeom phase_geom(int r0, int c0, int rows, int cols)
{
    constexpr int E = Cfg::K - 1 - J;
    PhaseGeom g;
    g.ra = max(r0 - E, 0);
    g.rb = min(r0 + Cfg::TH + E, rows);
    g.ca = max(c0 - E, 0);
    g.cb = min(c0 + Cfg::TW + E, cols);
    if constexpr (Cfg::ST == 8) {
        g.ra += ((g.ra & 1) != (J >> 1));
        g.ca += ((g.ca & 1) != (J & 1));
        g.nR = g.rb > g.ra ? (g.rb - g.ra + 1) >> 1 : 0;
    } else {
        g.nR = g.rb > g.ra ? g.rb - g.ra : 0;
    }
    g.nC = g.cb > g.ca ? (g.cb - g.ca + 1) >> 1 : 0;
    return g;
}

// Most units of a phase of the grown tile (phase 0 grows the most).
template <typename Cfg> constexpr int phase_units(int J)
{
    return Cfg::ST == 8 ? (Cfg::TH / 2 + Cfg::K - 1 - J) * (Cfg::TW / 2 + Cfg::K - 1 - J)
                        : (Cfg::TH + 2 * (Cfg::K - 1 - J)) *
                              ((Cfg::TW + 2 * (Cfg::K - 1 - J) + 1) / 2);
}

// Phase J: every color-J site of the grown tile.  The iteration count per
// thread has a compile-time bound, so the y loads of all of a thread's sites
// are issued before the first site is computed; mid() runs between the
// loads and the sites (work that hides their latency).  zin: the sites'
// normals, drawn ahead by lattice_normals at the units' indices (paired
// random-number contract), or NULL to draw each site's own block here.
template <typename Real, typename Cfg, int J, bool INTERIOR, bool B0, typename Mid>
__device__ __forceinline__ void lattice_phase(Real *xs, const Real *__restrict__ y, int r0,
                                              int c0, int rows, int cols, const SiteCtx<Real> &sc,
                                              Red &rd, const Real *zin, Mid &&mid)
{
    constexpr int NT = Cfg::NT;
    constexpr int NI = (phase_units<Cfg>(J) + NT - 1) / NT;
    const PhaseGeom g = phase_geom<Cfg, J>(r0, c0, rows, cols);
    const int total = g.nR * g.nC;
    const float rcp = 1.0f / (float)max(g.nC, 1);
    int rr[NI], cc[NI];
    Real yv[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        int C;
        const int R = div_small(idx, max(g.nC, 1), rcp, C);
        int r, c;
        if constexpr (Cfg::ST == 8) {
            r = g.ra + 2 * R;
            c = g.ca + 2 * C;
        } else {
            r = g.ra + R;
            c = g.ca + ((r + g.ca + J) & 1) + 2 * C;
        }
        const bool ok = idx < total && c < g.cb;
        rr[k] = ok ? r : -1;
        cc[k] = c;
        // clamped address: always inside the lattice, used only when ok
        const int rc = min(max(r, 0), rows - 1), ccl = min(max(c, 0), cols - 1);
        yv[k] = y[(size_t)rc * cols + ccl];
    }
    mid();
#pragma unroll
    for (int k = 0; k < NI; ++k)
        if (rr[k] >= 0) {
            Real z;
            if (zin) {
                z = zin[(int)threadIdx.x + k * NT];
            } else {
                const unsigned site = (unsigned)rr[k] * (unsigned)cols + (unsigned)cc[k];
                z = site_normal<Real>(draw_words(sc.seed, site, sc.t, sc.instance, 0u));
            }
            lattice_site<Real, Cfg, J, INTERIOR, B0>(xs, yv[k], z, rr[k], cc[k], r0, c0, rows,
                                                     cols, sc, rd);
        }
}

// The normals of phase J's sites under the paired random-number contract,
// into zb at the phase's unit indices.  The sites of a color, ranked by
// original id, share one Philox block per rank pair (2m, 2m + 1): the
// cosine branch for the first, the sine branch for the second.  With the
// lattice width a multiple of 4 every row holds an even number of sites of
// each of its colors, so the pairs are (r, c) and (r, c + 2) with bit 1 of c
// clear, keyed by the id of (r, c).  A thread takes pair slots here (one
// block and one Box-Muller radius for two sites) and the site updates take
// one site per thread, so the update reads the tile with the stride of the
// unpaired phase; a slot cut by the edge of the grown tile stores the one
// normal inside.
template <typename Real, typename Cfg, int J>
__device__ __forceinline__ void lattice_normals(Real *zb, int r0, int c0, int rows, int cols,
                                                const SiteCtx<Real> &sc)
{
    constexpr int E = Cfg::K - 1 - J;
    constexpr int NT = Cfg::NT;
    static_assert(Cfg::TW % 4 == 0, "pair slots need tile columns at multiples of 4");
    // rows of the grown tile that hold color-J sites, and pair slots per row
    // (c0 is a multiple of 4, so columns c0 - E .. c0 + TW + E - 1 meet at
    // most TW / 4 + 2 slots)
    constexpr int MR = Cfg::ST == 8 ? Cfg::TH / 2 + E : Cfg::TH + 2 * E;
    constexpr int MP = Cfg::TW / 4 + 2;
    constexpr int NI = (MR * MP + NT - 1) / NT;
    const PhaseGeom g = phase_geom<Cfg, J>(r0, c0, rows, cols);
    const int pa = g.ca >> 2;
    int nP;
    if constexpr (Cfg::ST == 8) {
        const int cl = g.cb - 1 - (((g.cb - 1) & 1) != (J & 1));   // last column of parity J & 1
        nP = cl >= g.ca ? (cl >> 2) - pa + 1 : 0;
    } else {
        nP = g.cb > g.ca ? ((g.cb - 1) >> 2) - pa + 1 : 0;
    }
    const int total = g.nR * nP;
    const float rcp = 1.0f / (float)max(nP, 1);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx < total) {
            int P;
            const int R = div_small(idx, max(nP, 1), rcp, P);
            const int r = Cfg::ST == 8 ? g.ra + 2 * R : g.ra + R;
            const int off = Cfg::ST == 8 ? (J & 1) : ((r + J) & 1);
            const int c = 4 * (pa + P) + off;
            const bool in1 = c >= g.ca && c < g.cb, in2 = c + 2 >= g.ca && c + 2 < g.cb;
            if (in1 || in2) {
                const unsigned key = (unsigned)r * (unsigned)cols + (unsigned)c;
                Real zc, zs;
                site_normal_pair<Real>(draw_words(sc.seed, key, sc.t, sc.instance, 0u), zc, zs);
                Real *const zrow = zb + R * g.nC;
                if (in1)
                    zrow[(c - g.ca) >> 1] = zc;
                if (in2)
                    zrow[(c + 2 - g.ca) >> 1] = zs;
            }
        }
    }
}

// The k color phases of one tile, separated by LDS barriers.  V2: the chain
// draws by the paired contract; zb then holds two buffers of
// phase_units<Cfg>(0) normals, and the caller has drawn phase 0's into the
// first and synchronised.  Each phase draws the next phase's normals into
// the other buffer between its y loads and its site updates; the barrier
// that ends the phase publishes them.
template <typename Real, typename Cfg, bool INTERIOR, bool B0, bool V2>
__device__ __forceinline__ void lattice_phases(Real *xs, const Real *__restrict__ y, int r0,
                                               int c0, int rows, int cols, const SiteCtx<Real> &sc,
                                               Red &rd, Real *zb)
{
    constexpr int ZN = phase_units<Cfg>(0);
    auto none = [] {};
    if constexpr (V2) {
        lattice_phase<Real, Cfg, 0, INTERIOR, B0>(
            xs, y, r0, c0, rows, cols, sc, rd, zb,
            [&] { lattice_normals<Real, Cfg, 1>(zb + ZN, r0, c0, rows, cols, sc); });
        lds_barrier();
        if constexpr (Cfg::K == 4) {
            lattice_phase<Real, Cfg, 1, INTERIOR, B0>(
                xs, y, r0, c0, rows, cols, sc, rd, zb + ZN,
                [&] { lattice_normals<Real, Cfg, 2>(zb, r0, c0, rows, cols, sc); });
            lds_barrier();
            lattice_phase<Real, Cfg, 2, INTERIOR, B0>(
                xs, y, r0, c0, rows, cols, sc, rd, zb,
                [&] { lattice_normals<Real, Cfg, 3>(zb + ZN, r0, c0, rows, cols, sc); });
            lds_barrier();
            lattice_phase<Real, Cfg, 3, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd,
                                                      zb + ZN, none);
            lds_barrier();
        } else {
            lattice_phase<Real, Cfg, 1, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd,
                                                      zb + ZN, none);
            lds_barrier();
        }
    } else {
        const Real *const nz = nullptr;
        lattice_phase<Real, Cfg, 0, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd, nz, none);
        lds_barrier();
        lattice_phase<Real, Cfg, 1, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd, nz, none);
        lds_barrier();
        if constexpr (Cfg::K == 4) {
            lattice_phase<Real, Cfg, 2, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd, nz,
                                                      none);
            lds_barrier();
            lattice_phase<Real, Cfg, 3, INTERIOR, B0>(xs, y, r0, c0, rows, cols, sc, rd, nz,
                                                      none);
            lds_barrier();
        }
    }
}

// LDS normals of a V2 tile: two phase buffers (one element otherwise).
template <typename Cfg, bool V2> constexpr int zbuf_len()
{
    return V2 ? 2 * phase_units<Cfg>(0) : 1;
}

// XCD-aware tile order: the hardware hands block b to XCD b mod 8, so give
// each XCD a contiguous run of tiles (rows of the lattice) to keep the halo
// re-reads of neighbouring tiles inside one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int per = nb >> 3, rem = nb & 7, x = b & 7;
    return x * per + min(x, rem) + (b >> 3);
}

// Stage the tile whose top-left interior site is (r0, c0), with its halo,
// into LDS, in two steps so that other work can run while the loads are in
// flight: lattice_load issues every load of the thread (cells outside the
// lattice become 0, their loads using an address clamped into the lattice,
// which the site update relies on), lattice_store writes them to LDS.
template <typename Cfg> constexpr int tile_loads()
{
    return (Cfg::LH * Cfg::LW + Cfg::NT - 1) / Cfg::NT;
}

template <typename Real, typename Cfg>
__device__ __forceinline__ void lattice_load(Real (&v)[tile_loads<Cfg>()],
                                             const Real *__restrict__ src, int r0, int c0,
                                             int rows, int cols)
{
    constexpr int H = Cfg::H, LW = Cfg::LW, NT = Cfg::NT;
#pragma unroll
    for (int k = 0; k < tile_loads<Cfg>(); ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        const int lr = idx / LW, lc = idx - (idx / LW) * LW;
        const int r = r0 - H + lr, c = c0 - H + lc;
        const int rc = min(max(r, 0), rows - 1), cc = min(max(c, 0), cols - 1);
        v[k] = src[(size_t)rc * cols + cc];
        if (r != rc || c != cc)
            v[k] = (Real)0;
    }
}

template <typename Real, typename Cfg>
__device__ __forceinline__ void lattice_store(Real *xs, const Real (&v)[tile_loads<Cfg>()])
{
    constexpr int NL = tile_loads<Cfg>(), NT = Cfg::NT;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (k < NL - 1 || idx < Cfg::LH * Cfg::LW)
            xs[idx] = v[k];
    }
}

// Tiles of a lattice take one of two compiled paths, an interior one (tile
// and halo inside the lattice: compile-time neighbour flags and scales) and
// the general one, or the general one alone.  The second halves the
// kernel's code, which on this target decides more than the per-site
// arithmetic once the code outgrows the instruction cache.
#ifndef GMRF_LAT_SPLIT
#define GMRF_LAT_SPLIT 1
#endif

// B0: the chain has an intercept (compile time, so that chains without one
// run code with no trace of it).  rel: the sweep's index within its call
// (sweep t = committed count + rel).  fold: the sweep before it in the call
// has not been ended: every block ends it first (sums its partials and draws
// tau, lam, beta0, identically in every block; the tile loads wait, since
// holding them across the draws would cost the kernel its occupancy), and
// the block of tile 0 records the draws for the next sweep kernel and the
// commit.  Without fold the sweep runs with the committed
// state (the first sweep of a call, and timing runs).  V2: the chain draws
// its site normals by the paired contract (lattice_normals).
template <typename Real, typename Cfg, bool B0, bool V2>
__device__ __forceinline__ void lattice_sweep_block(const LatArgs<Real> &la, const SweepArgs &a,
                                                    const int tile, const int rel, const int fold)
{
    constexpr int H = Cfg::H, LH = Cfg::LH, LW = Cfg::LW, NT = Cfg::NT;
    constexpr int TH = Cfg::TH, TW = Cfg::TW;
    constexpr int NPT = (TH * TW + NT - 1) / NT;       // interior sites per thread
    constexpr int CH = Cfg::CH < NPT ? Cfg::CH : NPT;  // accumulator batch
    __shared__ Real xs[LH * LW];
    __shared__ Real qtab[2 * (Cfg::ST + 1)];
    __shared__ Real zb[zbuf_len<Cfg, V2>()];

    const unsigned t = (unsigned)(a.st->sweep + (unsigned long long)rel);
    const Real *src = (t & 1u) ? la.x1 : la.x0;
    Real *dst = (t & 1u) ? la.x0 : la.x1;
    const int rows = la.rows, cols = la.cols;
    const int tr = tile / la.tiles_c, tc = tile - tr * la.tiles_c;
    const int r0 = tr * TH, c0 = tc * TW;
    const bool acc = (long long)t >= a.burn_in;

    HyperIn hin;
    if (fold) {
        SweepArgs fa = a;
        fa.dry = a.dry || tile != 0;      // one block stores the reductions and the trace
        hin = end_sweep_block<NT>(fa, partials_of(a, rel - 1), t - 1u, inputs_of(a, rel - 1),
                                  false);
        if (!fa.dry && threadIdx.x == 0) {
            double *const h = a.st->hs[rel & 1];
            h[0] = hin.tau;
            h[1] = hin.lam;
            h[2] = hin.beta0;
        }
    } else {
        hin = inputs_of(a, 0);
    }
    Real v[tile_loads<Cfg>()];
    lattice_load<Real, Cfg>(v, src, r0, c0, rows, cols);

    SiteCtx<Real> sc;
    sc.tau = (Real)hin.tau;
    sc.lam = (Real)hin.lam;
    sc.tau_rho = (Real)(hin.tau * a.rho);
    site_scales<Real>(sc.tau, sc.lam, Cfg::ST, sc.inv_q_full, sc.isd_full);
    sc.beta0 = B0 ? hin.beta0 : 0.0;
    sc.beta0_r = (Real)sc.beta0;
    sc.one_minus_rho = 1.0 - a.rho;
    sc.rho = a.rho;
    sc.t = t;
    sc.seed = a.seed;
    sc.instance = a.instance;
    sc.qtab = qtab;
    // phase 0's paired normals while the tile loads are in flight
    if constexpr (V2)
        lattice_normals<Real, Cfg, 0>(zb, r0, c0, rows, cols, sc);

    lattice_store<Real, Cfg>(xs, v);
    qtab_fill<Real, Cfg::ST>(qtab, sc.tau, sc.lam);
    lds_barrier();

    Red rd;
#if GMRF_LAT_SPLIT
    const bool interior = r0 >= H && c0 >= H && r0 + TH + Cfg::HH <= rows &&
                          c0 + TW + Cfg::HH <= cols;
    if (interior)
        lattice_phases<Real, Cfg, true, B0, V2>(xs, la.y, r0, c0, rows, cols, sc, rd, zb);
    else
#endif
        lattice_phases<Real, Cfg, false, B0, V2>(xs, la.y, r0, c0, rows, cols, sc, rd, zb);

    // Write the interior back and update the accumulators, CH sites per
    // thread per batch so their loads are in flight together.
#pragma unroll
    for (int k0 = 0; k0 < NPT; k0 += CH) {
        double o1[CH], o2[CH];
        size_t g[CH];
        bool ok[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int idx = (int)threadIdx.x + (k0 + j) * NT;
            const int r = r0 + idx / TW, c = c0 + idx % TW;
            ok[j] = (k0 + j < NPT) && idx < TH * TW && r < rows && c < cols;
            g[j] = (size_t)min(r, rows - 1) * cols + min(c, cols - 1);
            o1[j] = 0.0;
            o2[j] = 0.0;
            if (acc) {
                o1[j] = a.s1[g[j]];
                o2[j] = a.s2[g[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            if (ok[j]) {
                const int idx = (int)threadIdx.x + (k0 + j) * NT;
                const Real v = xs[(idx / TW + H) * LW + idx % TW + H];
                dst[g[j]] = v;
                if (acc) {
                    // the accumulated image is beta0 + x (x alone without an intercept)
                    const double dv = B0 ? (double)v + sc.beta0 : (double)v;
                    a.s1[g[j]] = o1[j] + dv;
                    a.s2[g[j]] = o2[j] + dv * dv;
                }
            }
        }
    }
    write_partials<NT>(partials_of(a, rel), rd, tile);
}

template <typename Real, typename Cfg, bool B0, bool V2>
__global__ __launch_bounds__(Cfg::NT) void lattice_sweep_kernel(LatArgs<Real> la, SweepArgs a,
                                                                int rel, int fold)
{
    lattice_sweep_block<Real, Cfg, B0, V2>(la, a, xcd_tile((int)blockIdx.x, (int)gridDim.x), rel,
                                           fold);
}

// A lattice that fits one tile, many sweeps in one launch (one block): the
// field stays in LDS (after a sweep every site of the tile is final, so the
// next sweep needs no reload), this thread's accumulators stay in registers,
// and the end-of-sweep reductions and draws run in the block itself.  Every
// operation is the one the tile kernel and the end of its sweep perform for a
// single-tile lattice, in the same order, so the results are bitwise those of
// tile shape 0.  With a.dry set (timing) it writes only the state buffer that
// the sweep after the last one would overwrite.
template <typename Real, typename Cfg, bool B0, bool V2>
__global__ __launch_bounds__(Cfg::NT) void lattice_persistent_kernel(LatArgs<Real> la, SweepArgs a,
                                                                     int nsweeps)
{
    constexpr int H = Cfg::H, LH = Cfg::LH, LW = Cfg::LW, NT = Cfg::NT;
    constexpr int TH = Cfg::TH, TW = Cfg::TW;
    constexpr int NPT = (TH * TW + NT - 1) / NT;
    __shared__ Real xs[LH * LW];
    __shared__ Real qtab[2 * (Cfg::ST + 1)];
    __shared__ double red[kPartials * (NT / 64)];
    __shared__ double hyp[3];
    __shared__ UnitDraws ub[kUnitBatch][2];
    __shared__ Real zb[zbuf_len<Cfg, V2>()];
    const int rows = la.rows, cols = la.cols;
    const int lane = (int)threadIdx.x & 63;
    unsigned t = (unsigned)a.st->sweep;
    long long nacc = a.st->n_acc;
    double tau = a.st->tau, lam = a.st->lam, b0 = B0 ? a.st->beta0 : 0.0;
    {
        Real v[tile_loads<Cfg>()];
        lattice_load<Real, Cfg>(v, (t & 1u) ? la.x1 : la.x0, 0, 0, rows, cols);
        lattice_store<Real, Cfg>(xs, v);
    }
    double s1r[NPT], s2r[NPT];
    int gi[NPT];
    bool own[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        const int r = idx / TW, c = idx % TW;
        own[k] = idx < TH * TW && r < rows && c < cols;
        gi[k] = min(r, rows - 1) * cols + min(c, cols - 1);
        s1r[k] = a.s1[gi[k]];
        s2r[k] = a.s2[gi[k]];
    }
    bool accumulated = false;
    lds_barrier();
    for (int s = 0; s < nsweeps; ++s) {
        if (s % kUnitBatch == 0) {
            unit_draw_batch<NT>(a, t, min(kUnitBatch, nsweeps - s), ub);
            lds_barrier();
        }
        SiteCtx<Real> sc;
        sc.tau = (Real)tau;
        sc.lam = (Real)lam;
        sc.tau_rho = (Real)(tau * a.rho);
        site_scales<Real>(sc.tau, sc.lam, Cfg::ST, sc.inv_q_full, sc.isd_full);
        sc.beta0 = b0;
        sc.beta0_r = (Real)sc.beta0;
        sc.one_minus_rho = 1.0 - a.rho;
        sc.rho = a.rho;
        sc.t = t;
        sc.seed = a.seed;
        sc.instance = a.instance;
        sc.qtab = qtab;
        qtab_fill<Real, Cfg::ST>(qtab, sc.tau, sc.lam);
        if constexpr (V2)
            lattice_normals<Real, Cfg, 0>(zb, 0, 0, rows, cols, sc);
        lds_barrier();
        Red rd;
        lattice_phases<Real, Cfg, false, B0, V2>(xs, la.y, 0, 0, rows, cols, sc, rd, zb);
        if ((long long)t >= a.burn_in) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (own[k]) {
                    const int idx = (int)threadIdx.x + k * NT;
                    const Real v = xs[(idx / TW + H) * LW + idx % TW + H];
                    const double dv = B0 ? (double)v + sc.beta0 : (double)v;
                    s1r[k] = s1r[k] + dv;
                    s2r[k] = s2r[k] + dv * dv;
                }
            }
            ++nacc;
            accumulated = true;
        }
        block_sum3<NT>(rd.q, rd.sse, rd.rsum, red);
        if (threadIdx.x < 64) {
            // the end-of-sweep sum over one partial slot: x + 0 + ... = x
            rd.q = __shfl(rd.q, 0, 64);
            rd.sse = __shfl(rd.sse, 0, 64);
            rd.rsum = __shfl(rd.rsum, 0, 64);
            const HyperIn out = end_of_sweep_draws(a, t, rd, HyperIn{tau, lam, b0}, lane,
                                                   ub[s % kUnitBatch][lane < 2 ? lane : 0]);
            if (lane == 0) {
                hyp[0] = out.tau;
                hyp[1] = out.lam;
                hyp[2] = out.beta0;
            }
        }
        lds_barrier();
        tau = hyp[0];
        lam = hyp[1];
        b0 = hyp[2];
        ++t;
    }
    // the state after the last sweep: x in buffer t mod 2, the accumulators,
    // the counters (the draws already stored tau, lam, beta0 and reductions)
    Real *dst = (t & 1u) ? la.x1 : la.x0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (own[k]) {
            const int idx = (int)threadIdx.x + k * NT;
            dst[gi[k]] = xs[(idx / TW + H) * LW + idx % TW + H];
            if (accumulated && !a.dry) {
                a.s1[gi[k]] = s1r[k];
                a.s2[gi[k]] = s2r[k];
            }
        }
    }
    if (threadIdx.x == 0 && !a.dry) {
        a.st->n_acc = nacc;
        a.st->sweep = (unsigned long long)t;
    }
}

// Batched lattice sweep: the tile table lists the tiles of every lattice
// chain of the batch, chain by chain; each chain's partial slots are its own
// tile indices, as in a standalone sweep.
template <typename Real> struct LatJob {
    LatArgs<Real> la;
    SweepArgs a;
};
struct LatTile {
    int job, tile;
};

// with_hyper: this call's GMRF_WITH_HYPER (the job tables are built once);
// rel, fold: as for lattice_sweep_block, the same for every chain.
template <typename Real, typename Cfg, bool B0>
__global__ __launch_bounds__(Cfg::NT) void lattice_batch_kernel(const LatJob<Real> *jobs,
                                                                const LatTile *tiles,
                                                                int with_hyper, int rel, int fold)
{
    const LatTile tl = tiles[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const LatJob<Real> &j = jobs[tl.job];
    SweepArgs a = j.a;
    a.with_hyper = with_hyper;
    lattice_sweep_block<Real, Cfg, B0, false>(j.la, a, tl.tile, rel, fold);
}

// ---------------------------------------------------------------------------
// general graphs: one color slab per launch
// ---------------------------------------------------------------------------
template <typename Real> struct CsrArgs {
    const int *row_ptr;         // permuted CSR (slab positions)
    const int *col;
    const int *orig;            // slab position -> original id (random-number key)
    Real *x;
    const Real *y;              // y (Gaussian) or kappa = Y - m/2 (binomial)
    const int *trials;          // binomial: m_i (slab order); NULL otherwise
    const int *chunk_off;       // binomial: first term chunk of each slab position (n + 1)
    const int *chunk_site;      // binomial: slab position of each chunk
    double *chunk_sum;          // binomial: run sums of the PG(1, .) terms (see below)
    PgEnvelope *env;            // binomial: each site's PG envelope for the current sweep
    double *psi;                // binomial: each site's psi for the current sweep
};

// One site per thread.  The first NB neighbours are gathered in one batch
// (all column indices, then all values) and stay in registers for the q
// terms.  With WIDE, longer rows continue in batches of NB, so a row costs
// two dependent loads per batch rather than per neighbour; otherwise one
// entry at a time.  The summation order is the row order, i.e. ascending
// original neighbour id, in every variant.  Wide batches suit launches bound
// by load latency (one chain's color pass: most Delaunay rows, up to 12
// entries, in one round); the batched launch is bound by load throughput and
// pays for the clamped repeats of short rows, so it gathers 8 and continues
// entry by entry.
constexpr int kCsrBatch = 12;          // per-chain kernels
constexpr int kCsrBatchShared = 8;     // the batched color pass

// Row entries eb .. eb + NB - 1, each clamped to the row's last entry e1 - 1:
// their column indices and the neighbour values.
template <int NB, typename Real>
__device__ __forceinline__ void csr_gather(const int *col, const Real *x, int eb, int e1,
                                           int (&j)[NB], Real (&v)[NB])
{
#pragma unroll
    for (int k = 0; k < NB; ++k)
        j[k] = col[min(eb + k, e1 - 1)];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        v[k] = x[j[k]];
}

// Scalars of the chain state that a color pass reads.
struct CsrScalars {
    double tau, lam, beta0;
    unsigned t;
    bool acc;                   // this sweep adds to the posterior accumulators
};

__device__ __forceinline__ CsrScalars csr_scalars(const SweepArgs &a, bool b0)
{
    CsrScalars v;
    v.tau = a.st->tau;
    v.lam = a.st->lam;
    v.beta0 = b0 ? a.st->beta0 : 0.0;
    v.t = (unsigned)a.st->sweep;
    v.acc = (long long)v.t >= a.burn_in;
    return v;
}

// Site p (slab position) of the color slab starting at lo: the update of
// Algorithm 1 with the field read from and written to x (the global state,
// or its copy in LDS), the accumulators, and this site's q / sse / rsum
// terms added to rd.  Gaussian (Sec. 3.1): Qii = tau D_ii + lam,
// m = (lam (y_i - beta0) + tau rho s_i) / Qii.  Binomial (BIN, Sec. 3.2 with
// psi_p drawn beforehand): Qii = tau D_ii + psi_p,
// m = (kappa_p - psi_p beta0 + tau rho s_i) / Qii, and the sse / rsum slots
// take psi_p and kappa_p - psi_p x_p.
template <typename Real, bool B0, bool BIN, int NB = kCsrBatch, bool WIDE = true>
__device__ __forceinline__ void csr_site(const CsrArgs<Real> &ca, const SweepArgs &a, Real *x,
                                         const int p, const int lo, const CsrScalars &v, Red &rd)
{
    const Real tau = (Real)v.tau, tau_rho = (Real)(v.tau * a.rho);
    const int e0 = ca.row_ptr[p], e1 = ca.row_ptr[p + 1];
    const int deg = e1 - e0;
    const Real yv = ca.y[p];
    const double psi = BIN ? ca.psi[p] : 0.0;
    const unsigned id = (unsigned)ca.orig[p];
    double o1 = 0.0, o2 = 0.0;
    if (v.acc) {
        o1 = a.s1[p];
        o2 = a.s2[p];
    }
    int cj[NB];
    Real nb[NB];
    csr_gather<NB>(ca.col, x, e0, max(e1, 1), cj, nb);   // clamped; entry k used only if k < deg
    Real s = (Real)0;
#pragma unroll
    for (int k = 0; k < NB; ++k)
        if (k < deg)
            s += nb[k];
    if constexpr (WIDE) {
        for (int eb = e0 + NB; eb < e1; eb += NB) {
            int tj[NB];
            Real tv[NB];
            csr_gather<NB>(ca.col, x, eb, e1, tj, tv);
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (eb + k < e1)
                    s += tv[k];
        }
    } else {
        for (int e = e0 + NB; e < e1; ++e)
            s += x[ca.col[e]];
    }
    const Real z = site_normal<Real>(draw_words(a.seed, id, v.t, a.instance, 0u));
    Real xn;
    if constexpr (BIN) {
        const Real Q = fma(tau, (Real)deg, (Real)psi);
        Real inv_q, isd;
        if constexpr (sizeof(Real) == 8) {
            inv_q = 1.0 / Q;
            isd = 1.0 / sqrt(Q);
        } else {
            inv_q = 1.0f / Q;
            isd = __builtin_amdgcn_rsqf(Q);
        }
        const Real beff = (Real)((double)yv - psi * v.beta0);
        xn = fma(z, isd, fma(tau_rho, s, beff) * inv_q);
    } else {
        const Real lam = (Real)v.lam;
        Real inv_q, isd;
        site_scales<Real>(tau, lam, deg, inv_q, isd);
        const Real yeff = B0 ? yv - (Real)v.beta0 : yv;
        xn = site_draw<Real>(yeff, s, z, lam, tau_rho, inv_q, isd);
    }
    x[p] = xn;
    const double xd = (double)xn;
    double edge = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k)
        if (k < deg && cj[k] < lo) {   // lower color: already final this sweep
            const double d = xd - (double)nb[k];
            edge += d * d;
        }
    if constexpr (WIDE) {
        for (int eb = e0 + NB; eb < e1; eb += NB) {
            int tj[NB];
            Real tv[NB];
            csr_gather<NB>(ca.col, x, eb, e1, tj, tv);
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (eb + k < e1 && tj[k] < lo) {
                    const double d = xd - (double)tv[k];
                    edge += d * d;
                }
        }
    } else {
        for (int e = e0 + NB; e < e1; ++e) {
            const int j = ca.col[e];
            if (j < lo) {
                const double d = xd - (double)x[j];
                edge += d * d;
            }
        }
    }
    rd.q += (1.0 - a.rho) * (double)deg * xd * xd + a.rho * edge;
    if constexpr (BIN) {
        rd.sse += psi;
        rd.rsum += (double)yv - psi * xd;
    } else {
        const double rr = B0 ? (double)yv - v.beta0 - xd : (double)yv - xd;
        rd.sse += rr * rr;
        if (B0)
            rd.rsum += rr;
    }
    if (v.acc) {
        // accumulated image beta0 + x (the linear predictor for the binomial model)
        const double phi = B0 ? xd + v.beta0 : xd;
        a.s1[p] = o1 + phi;
        a.s2[p] = o2 + phi * phi;
    }
}

// Sites p0 + threadIdx.x of the color slab [lo, lo + cnt); partial slot
// `slot`.
template <typename Real, bool B0, bool BIN, int NB = kCsrBatch, bool WIDE = true>
__device__ __forceinline__ void csr_pass_block(const CsrArgs<Real> &ca, const SweepArgs &a,
                                               const int lo, const int cnt, const int p0,
                                               const int slot)
{
    const CsrScalars v = csr_scalars(a, B0);
    const int p = p0 + (int)threadIdx.x;
    Red rd;
    if (p < lo + cnt)
        csr_site<Real, B0, BIN, NB, WIDE>(ca, a, ca.x, p, lo, v, rd);
    write_partials<kThreads>(a.partials, rd, slot);
}

// Block b takes chunk xcd_tile(b) of the slab (kThreads sites each), so each
// XCD sweeps a contiguous eighth of the slab; the breadth-first slab order
// keeps that eighth's neighbours in nearby stretches of the other slabs,
// inside the XCD's own L2.  A chunk's partial slot is slot_base + chunk.
template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void csr_pass_kernel(CsrArgs<Real> ca, SweepArgs a, int lo,
                                                            int cnt, int slot_base)
{
    const int chunk = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    csr_pass_block<Real, B0, false>(ca, a, lo, cnt, lo + chunk * kThreads, slot_base + chunk);
}

// Batched color pass: one entry per block over the color-c slabs of every
// general-graph chain of the batch.
template <typename Real> struct CsrJob {
    CsrArgs<Real> ca;
    SweepArgs a;
};
struct CsrBlock {
    int job, lo, cnt, p0, slot;
};

template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void csr_batch_kernel(const CsrJob<Real> *jobs,
                                                             const CsrBlock *blocks,
                                                             int with_hyper)
{
    const CsrBlock bk = blocks[xcd_tile((int)blockIdx.x, (int)gridDim.x)];   // chains per XCD
    const CsrJob<Real> &j = jobs[bk.job];
    SweepArgs a = j.a;
    a.with_hyper = with_hyper;
    csr_pass_block<Real, B0, false, kCsrBatchShared, false>(j.ca, a, bk.lo, bk.cnt, bk.p0,
                                                         bk.slot);
}

// ---------------------------------------------------------------------------
// general graphs, one launch per sweep: chunks with recomputed closures
// ---------------------------------------------------------------------------
// The general-graph counterpart of the fused lattice sweep.  Block b takes
// chunk b (graph_host.cpp, build_chunks).  It stages in LDS the values from
// before the sweep of the chunk's staged sites (R_b, then H_b), and y, the
// original id and the local neighbour list of every R_b site, with every
// load issued up front.  Then for each color c in order it computes every
// R_b site of color c from its neighbours in LDS -- lower-colored ones
// already hold their new values (they are in R_b and were computed in an
// earlier color), higher-colored ones still the old ones -- exactly the
// update the color passes make, with the same random numbers (keyed by
// site) and the same summation order (ascending original neighbour id), so a
// recomputed site is bitwise its owner's value; the color phases touch only
// LDS.  Last, the sites the chunk owns (one consecutive run of slab
// positions per color) add their q / sse terms (each edge once, at its
// higher-colored endpoint, whose lower-colored neighbours are the staged
// slots below its color's first slot), update the accumulators and are
// written back, their loads batched.  The state is ping-ponged between two
// buffers (sweep t reads buffer t & 1), so no block sees another's new values
// through memory.
template <typename Real> struct FusedArgs {
    const int *ch_loc, *ch_row, *ch_adj, *ch_meta;   // per-chunk bases and metadata
    const int *loc_site;                             // slab position of each staged site
    const unsigned short *loc_row, *loc_adj;         // local adjacency of the R sites
    const unsigned *loc_id;                          // original id of each staged site
    Real *x0, *x1;                                   // ping-pong state, slab order
    const Real *y;                                   // y (slab order)
    int k;                                           // colors
};

constexpr int kFusedGather = 8;                      // neighbour indices read per batch
constexpr int kQtabDeg = 64;                         // degrees with tabulated scales
constexpr int kFusedCH = 4;                          // sites per thread per batch
constexpr int kFoldUnroll = 8;                       // partial slots per thread in flight

__host__ __device__ constexpr size_t lds_align16(size_t b) { return (b + 15) / 16 * 16; }

// Neighbour sum of a staged site in row order (local neighbours e0 .. e1 - 1),
// continuing the running sum sum.
template <typename Real>
__device__ __forceinline__ Real fused_nbr_sum(const Real *xs, const unsigned short *adj, int e0,
                                              int e1, Real sum)
{
    for (int eb = e0; eb < e1; eb += kFusedGather) {
        int l[kFusedGather];
#pragma unroll
        for (int q = 0; q < kFusedGather; ++q)
            l[q] = adj[min(eb + q, e1 - 1)];
#pragma unroll
        for (int q = 0; q < kFusedGather; ++q)
            if (eb + q < e1)
                sum += xs[l[q]];
    }
    return sum;
}

// Chunk b of a chain (rel, fold: as for the lattice sweep kernel).  Order of
// work, so that independent loads are in flight together: the chunk's local
// rows and neighbours go to LDS by direct global-to-LDS copies; the slab
// positions of the first kFusedCH * kThreads staged sites load beside the
// previous sweep's partials (first half of the fold); their values and y
// (gathers) go to LDS; the normal variates of the R sites (keyed by
// original id and sweep only) go to LDS; the fold's draws; the color phases
// run in LDS, each owned site's q / sse terms, accumulators and write-back
// taken as it is drawn.
template <typename Real, bool B0>
__device__ __forceinline__ void csr_fused_block(const FusedArgs<Real> &fa, const SweepArgs &a,
                                                const int b, const int rel, const int fold)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    __shared__ Real qtab[2 * kQtabDeg];
    __shared__ int sm[3 * kFusedMaxColors + 1];
    __shared__ FoldLds fl;

    const unsigned t = (unsigned)(a.st->sweep + (unsigned long long)rel);
    const Real *src = (t & 1u) ? fa.x1 : fa.x0;
    Real *dst = (t & 1u) ? fa.x0 : fa.x1;
    const int k = fa.k;
    const int *meta = fa.ch_meta + (size_t)b * (3 * k + 1);
    const int loc0 = fa.ch_loc[b], nloc = fa.ch_loc[b + 1] - loc0;
    const int nr = meta[k];
    const int row0 = fa.ch_row[b], adj0 = fa.ch_adj[b], nadj = fa.ch_adj[b + 1] - adj0;
    const int *site = fa.loc_site + loc0;
    const unsigned *sid = fa.loc_id + loc0;
    // the chunk's own LDS image (chunk_lds_bytes of its counts; the launch
    // reserves the graph's largest): staged values, y and variates of R, R's
    // local rows (padded to whole 16-byte vectors) and neighbours
    Real *xs = reinterpret_cast<Real *>(fused_lds);
    size_t off = lds_align16(sizeof(Real) * (size_t)nloc);
    Real *ys = reinterpret_cast<Real *>(fused_lds + off);
    off += lds_align16(sizeof(Real) * (size_t)nr);
    Real *zs = reinterpret_cast<Real *>(fused_lds + off);
    off += lds_align16(sizeof(Real) * (size_t)nr);
    unsigned short *lrow = reinterpret_cast<unsigned short *>(fused_lds + off);
    off += lds_align16(sizeof(unsigned short) * (size_t)(nr + 1));
    unsigned short *ladj = reinterpret_cast<unsigned short *>(fused_lds + off);
    for (int i = (int)threadIdx.x; i < 3 * k + 1; i += kThreads)
        sm[i] = meta[i];

    // rows and neighbours: each chunk's start is on a 16-byte boundary and
    // both are padded to whole 16-byte vectors; lane L of a wave copies
    // vector i to the wave's LDS base + 16 L
    {
        const int nrow4 = (nr + 1 + 7) / 8, nadj4 = nadj / 8;
        const uint4 *grow = reinterpret_cast<const uint4 *>(fa.loc_row + row0);
        const uint4 *gadj = reinterpret_cast<const uint4 *>(fa.loc_adj + adj0);
        uint4 *srow = reinterpret_cast<uint4 *>(lrow);
        uint4 *sadj = reinterpret_cast<uint4 *>(ladj);
        const int lane = (int)threadIdx.x & 63;
        for (int i = (int)threadIdx.x; i - lane < nrow4; i += kThreads)
            if (i < nrow4)
                __builtin_amdgcn_global_load_lds(grow + i, srow + (i - lane), 16, 0, 0);
        for (int i = (int)threadIdx.x; i - lane < nadj4; i += kThreads)
            if (i < nadj4)
                __builtin_amdgcn_global_load_lds(gadj + i, sadj + (i - lane), 16, 0, 0);
    }

    // staging, kFusedCH sites per thread at a time; the first batch's slab
    // positions load beside the fold's partials
    auto stage = [&](const int base, const bool first) {
        int p[kFusedCH];
        unsigned id[kFusedCH];
#pragma unroll
        for (int j = 0; j < kFusedCH; ++j) {
            const int s = min(base + (int)threadIdx.x + j * kThreads, nloc - 1);
            p[j] = site[s];
            if constexpr (sizeof(Real) == 4)
                id[j] = sid[s];
        }
        if (first && fold)
            fold_partials<kFoldUnroll>(a, partials_of(a, rel - 1), fl);
        Real xv[kFusedCH], yv[kFusedCH];
#pragma unroll
        for (int j = 0; j < kFusedCH; ++j) {
            xv[j] = src[p[j]];
            yv[j] = fa.y[p[j]];
        }
        if constexpr (sizeof(Real) == 4) {
            // FP32: the batch's variates while its gathers are in flight (the
            // FP64 draw needs more registers than this point has spare)
#pragma unroll
            for (int j = 0; j < kFusedCH; ++j) {
                const int s = base + (int)threadIdx.x + j * kThreads;
                if (s < nr)
                    zs[s] = site_normal<Real>(draw_words(a.seed, id[j], t, a.instance, 0u));
            }
        }
#pragma unroll
        for (int j = 0; j < kFusedCH; ++j) {
            const int s = base + (int)threadIdx.x + j * kThreads;
            if (s < nloc)
                xs[s] = xv[j];
            if (s < nr)
                ys[s] = yv[j];
        }
    };
    stage(0, true);
    for (int base = kFusedCH * kThreads; base < nloc; base += kFusedCH * kThreads)
        stage(base, false);
    // the variates of the R sites (FP64)
    if constexpr (sizeof(Real) == 8)
        for (int s = (int)threadIdx.x; s < nr; s += kThreads)
            zs[s] = site_normal<Real>(draw_words(a.seed, sid[s], t, a.instance, 0u));
    // every wave's direct copies have landed (a full barrier waits for them)
    __syncthreads();
    HyperIn hin;
    if (fold) {      // end the previous sweep of the call (as the lattice kernel does)
        SweepArgs ea = a;
        ea.dry = a.dry || b != 0;
        hin = fold_draws(ea, t - 1u, inputs_of(a, rel - 1), false, fl);
        if (!ea.dry && threadIdx.x == 0) {
            double *const h = a.st->hs[rel & 1];
            h[0] = hin.tau;
            h[1] = hin.lam;
            h[2] = hin.beta0;
        }
    } else {
        hin = inputs_of(a, 0);
    }
    const Real tau = (Real)hin.tau, lam = (Real)hin.lam, tau_rho = (Real)(hin.tau * a.rho);
    const double beta0 = B0 ? hin.beta0 : 0.0;
    const bool acc = (long long)t >= a.burn_in;
    if (threadIdx.x < kQtabDeg)
        site_scales<Real>(tau, lam, (int)threadIdx.x, qtab[threadIdx.x],
                          qtab[kQtabDeg + threadIdx.x]);
    lds_barrier();

    // the color phases, in LDS.  The owned sites of color c are the first
    // owned[c] R sites of its run, at consecutive slab positions from
    // ostart[c]: a thread that draws one also adds its q / sse terms (its
    // lower-color neighbours hold this sweep's values), adds it to its
    // accumulators and writes it back.  The accumulators take atomic adds
    // whose results are not read back, so no phase waits on global memory;
    // each accumulator takes one add per sweep, so each sum is the plain
    // sum, bit for bit.
    Red rd;
    for (int c = 0; c < k; ++c) {
        const int lo = sm[c], hi = sm[c + 1], own = sm[k + 1 + c], ost = sm[2 * k + 1 + c];
        for (int s = lo + (int)threadIdx.x; s < hi; s += kThreads) {
            const int e0 = lrow[s], e1 = lrow[s + 1], deg = e1 - e0;
            // the first kFusedGather neighbours stay in registers for the
            // q term; the rest (rare) are read again
            int l[kFusedGather];
            Real v[kFusedGather];
#pragma unroll
            for (int q = 0; q < kFusedGather; ++q)
                l[q] = ladj[min(e0 + q, e1 - 1)];
#pragma unroll
            for (int q = 0; q < kFusedGather; ++q)
                v[q] = xs[l[q]];
            Real sum = (Real)0;
#pragma unroll
            for (int q = 0; q < kFusedGather; ++q)
                if (q < deg)
                    sum += v[q];
            if (deg > kFusedGather)
                sum = fused_nbr_sum<Real>(xs, ladj, e0 + kFusedGather, e1, sum);
            Real inv_q, isd;
            if (deg < kQtabDeg) {
                inv_q = qtab[deg];
                isd = qtab[kQtabDeg + deg];
            } else {
                site_scales<Real>(tau, lam, deg, inv_q, isd);
            }
            const Real yv = ys[s];
            const Real yeff = B0 ? yv - (Real)beta0 : yv;
            const Real xn = site_draw<Real>(yeff, sum, zs[s], lam, tau_rho, inv_q, isd);
            xs[s] = xn;
            const int o = s - lo;
            if (o < own) {
                const int pos = ost + o;
                const double xd = (double)xn;
                double edge = 0.0;              // lower colors: this sweep's values
#pragma unroll
                for (int q = 0; q < kFusedGather; ++q)
                    if (q < deg && l[q] < lo) {
                        const double d = xd - (double)v[q];
                        edge += d * d;
                    }
                for (int e = e0 + kFusedGather; e < e1; ++e) {
                    const int le = ladj[e];
                    if (le < lo) {
                        const double d = xd - (double)xs[le];
                        edge += d * d;
                    }
                }
                rd.q += (1.0 - a.rho) * (double)deg * xd * xd + a.rho * edge;
                const double rr = B0 ? (double)yv - beta0 - xd : (double)yv - xd;
                rd.sse += rr * rr;
                if (B0)
                    rd.rsum += rr;
                if (acc) {
                    const double phi = B0 ? xd + beta0 : xd;
                    unsafeAtomicAdd(a.s1 + pos, phi);
                    unsafeAtomicAdd(a.s2 + pos, phi * phi);
                }
                dst[pos] = xn;
            }
        }
        lds_barrier();
    }
    write_partials<kThreads>(partials_of(a, rel), rd, b);
}

// Block b takes chunk xcd_tile(b): each XCD sweeps a contiguous run of
// chunks, which the locality order makes a compact region.
template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void csr_fused_kernel(FusedArgs<Real> fa, SweepArgs a,
                                                             int rel, int fold)
{
    csr_fused_block<Real, B0>(fa, a, xcd_tile((int)blockIdx.x, (int)gridDim.x), rel, fold);
}

// Batched form: one entry per block over the chunks of every chunked
// general-graph chain of a batch (chain by chain, so each XCD takes a run of
// chains); with_hyper, rel and fold as for lattice_batch_kernel.
template <typename Real> struct FusedJob {
    FusedArgs<Real> fa;
    SweepArgs a;
};
struct FusedBlock {
    int job, chunk;
};

template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void csr_fused_batch_kernel(const FusedJob<Real> *jobs,
                                                                   const FusedBlock *blocks,
                                                                   int with_hyper, int rel,
                                                                   int fold)
{
    const FusedBlock bk = blocks[xcd_tile((int)blockIdx.x, (int)gridDim.x)];
    const FusedJob<Real> &j = jobs[bk.job];
    SweepArgs a = j.a;
    a.with_hyper = with_hyper;
    csr_fused_block<Real, B0>(j.fa, a, bk.chunk, rel, fold);
}

// ---------------------------------------------------------------------------
// general graphs whose field fits in LDS: one block, the field in LDS
// ---------------------------------------------------------------------------
// The field of a small general graph (n values within kCsrLdsBytes) stays in
// LDS for the whole launch, and one block does what the k color-pass
// launches and the commit kernel do, in the same order of operations: each
// color's slab is cut into the same groups of kThreads sites as the pass
// kernels' blocks (each wavefront takes 64 consecutive sites of a group,
// every site in the lane it has there), the groups' FP64 partials land in
// the same slots, and the slots are summed as the commit kernel sums them.
// So the results are bitwise those of the color passes, without their
// k + 1 launches per sweep, whose dispatch latency dominates small graphs.
// A Gaussian chain runs all the sweeps of a call in one launch; a binomial
// chain one sweep per launch, after its Polya-Gamma launches.
constexpr int kCsrPersistThreads = 512;
constexpr int kCsrPersistColors = 32;           // most colors the slab table holds
constexpr int kCsrLdsBytes = 122880;            // LDS for the field (gfx950: 160 KB per CU)
constexpr int kCsrPersistSlots = 160;           // n / kThreads + k slots at most
struct SlabTable {
    int off[kCsrPersistColors + 1];             // first slab position of each color, then n
    int k;
};

template <typename Real, bool B0, bool BIN>
__global__ __launch_bounds__(kCsrPersistThreads) void csr_persistent_kernel(CsrArgs<Real> ca,
                                                                            SweepArgs a,
                                                                            SlabTable sl,
                                                                            int nsweeps)
{
    constexpr int NT = kCsrPersistThreads, GW = kThreads / 64;   // wavefronts per group
    constexpr int GPI = NT / kThreads;                           // groups per iteration
    __shared__ Real xs[kCsrLdsBytes / sizeof(Real)];
    __shared__ double wpart[kCsrPersistSlots * GW * kPartials];   // wavefront sums of a group
    __shared__ double red[kPartials * GW];
    __shared__ double hyp[3];
    __shared__ UnitDraws ub[kUnitBatch][2];
    const int n = sl.off[sl.k];
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    for (int p = (int)threadIdx.x; p < n; p += NT)
        xs[p] = ca.x[p];
    CsrScalars v = csr_scalars(a, B0);
    long long nacc = a.st->n_acc;
    lds_barrier();
    for (int s = 0; s < nsweeps; ++s) {
        if (s % kUnitBatch == 0) {
            unit_draw_batch<NT>(a, v.t, min(kUnitBatch, nsweeps - s), ub);
            lds_barrier();
        }
        int slot0 = 0;
        for (int c = 0; c < sl.k; ++c) {
            const int lo = sl.off[c], hi = sl.off[c + 1];
            const int groups = (hi - lo + kThreads - 1) / kThreads;
            for (int g0 = 0; g0 < groups; g0 += GPI) {
                const int g = g0 + wave / GW, w = wave % GW;
                const int p = lo + g * kThreads + w * 64 + lane;
                Red rd;
                if (g < groups && p < hi)
                    csr_site<Real, B0, BIN>(ca, a, xs, p, lo, v, rd);
                rd.q = wave_sum(rd.q);
                rd.sse = wave_sum(rd.sse);
                rd.rsum = wave_sum(rd.rsum);
                if (lane == 0 && g < groups) {
                    double *const wp = wpart + ((slot0 + g) * GW + w) * kPartials;
                    wp[0] = rd.q;
                    wp[1] = rd.sse;
                    wp[2] = rd.rsum;
                }
            }
            slot0 += groups;
            lds_barrier();
        }
        // the commit kernel's sum: thread i < kThreads adds slots i, i + kThreads,
        // ... (each slot the pass block's sum of its wavefronts, in order), then
        // the fixed tree over the first kThreads threads
        Red r;
        if ((int)threadIdx.x < kThreads) {
            for (int i = (int)threadIdx.x; i < slot0; i += kThreads) {
                const double *const wp = wpart + i * GW * kPartials;
                double q = wp[0], e = wp[1], m = wp[2];
                for (int w = 1; w < GW; ++w) {
                    q += wp[w * kPartials];
                    e += wp[w * kPartials + 1];
                    m += wp[w * kPartials + 2];
                }
                r.q += q;
                r.sse += e;
                r.rsum += m;
            }
        }
        r.q = wave_sum(r.q);
        r.sse = wave_sum(r.sse);
        r.rsum = wave_sum(r.rsum);
        if (lane == 0 && wave < GW) {
            red[wave] = r.q;
            red[GW + wave] = r.sse;
            red[2 * GW + wave] = r.rsum;
        }
        lds_barrier();
        if (threadIdx.x < 64) {
            r.q = red[0];
            r.sse = red[GW];
            r.rsum = red[2 * GW];
            for (int w = 1; w < GW; ++w) {
                r.q += red[w];
                r.sse += red[GW + w];
                r.rsum += red[2 * GW + w];
            }
            const HyperIn out = end_of_sweep_draws(a, v.t, r, HyperIn{v.tau, v.lam, v.beta0},
                                                   lane, ub[s % kUnitBatch][lane < 2 ? lane : 0]);
            if (lane == 0) {
                hyp[0] = out.tau;
                hyp[1] = out.lam;
                hyp[2] = out.beta0;
            }
        }
        if (v.acc)
            ++nacc;
        lds_barrier();
        v.tau = hyp[0];
        v.lam = hyp[1];
        v.beta0 = B0 ? hyp[2] : 0.0;
        ++v.t;
        v.acc = (long long)v.t >= a.burn_in;
    }
    for (int p = (int)threadIdx.x; p < n; p += NT)
        ca.x[p] = xs[p];
    if (threadIdx.x == 0 && !a.dry) {
        a.st->n_acc = nacc;
        a.st->sweep = (unsigned long long)v.t;
    }
}

// ---------------------------------------------------------------------------
// general graphs, binomial logit model (Sec. 3.2 with Polya-Gamma
// augmentation): two launches per color
// ---------------------------------------------------------------------------
// psi_p ~ PG(m_p, beta0 + x_p) is the sum of m_p PG(1, .) terms.  Every
// psi_p of a sweep depends only on beta0 and site p's value at the start of
// the sweep (no color pass changes a site before its own), so all of them
// are drawn before the color passes:
//   * the envelope kernel, one thread per site;
//   * the term kernel: the terms of all sites are cut into chunks of
//     kPgChunk consecutive terms of one site, one thread per chunk over the
//     whole graph (so work is spread evenly whatever the m_p).  Chunk q runs
//     on lane q mod 64 and the chunks of a site are consecutive, so a site's
//     chunks fall into one run of lanes per wavefront; a segmented scan over
//     the lanes leaves each run's sum in its last chunk's slot;
//   * the psi kernel, one wavefront per site: psi_p is the sum of the site's
//     run sums (at most m_p / (64 kPgChunk) + 2 of them), lane l taking runs
//     l, l + 64, ... and a fixed tree joining the lanes.
// Each color pass then runs one thread per site: x_p ~ N(m, 1/Q) with
// Q = tau D_pp + psi_p, m = (kappa_p - psi_p beta0 + tau rho sum_{j~p} x_j) / Q.
constexpr int kPsiSites = kThreads / 64;        // sites per block of the psi kernel
constexpr int kPgChunk = 4;                     // PG(1, .) terms per chunk

// The PG envelope of sites lo .. lo + cnt - 1 (tilt beta0 + x_p), so that
// the term kernel's threads need not each evaluate its erfc and exp.  Run
// over all sites at the start of a sweep: beta0 is fixed during the sweep and
// no color pass changes a site before that site's own pass, so every
// envelope is the one of the site's pass.
template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void pg_env_kernel(CsrArgs<Real> ca, SweepArgs a, int lo,
                                                          int cnt)
{
    const int p = lo + (int)blockIdx.x * kThreads + (int)threadIdx.x;
    if (p >= lo + cnt)
        return;
    const double b0 = B0 ? a.st->beta0 : 0.0;
    ca.env[p] = pg_envelope(b0 + (double)ca.x[p]);
}

// Chunks 0 .. nq - 1; the grid is whole blocks of whole wavefronts, so chunk
// q runs on lane q mod 64.
template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void pg_chunk_kernel(CsrArgs<Real> ca, SweepArgs a, int nq)
{
    const int q = (int)blockIdx.x * kThreads + (int)threadIdx.x;
    const int lane = (int)threadIdx.x & 63;
    const bool valid = q < nq;
    const int p = valid ? ca.chunk_site[q] : -1;
    double sum = 0.0;
    if (valid) {
        const int m = ca.trials[p];
        const int j0 = (q - ca.chunk_off[p]) * kPgChunk;
        const int j1 = min(j0 + kPgChunk, m);
        const unsigned t = (unsigned)a.st->sweep;
        const unsigned id = (unsigned)ca.orig[p];
        const PgEnvelope env = ca.env[p];      // drawn with beta0 by pg_env_kernel<Real, B0>
        bool ok = true;
        for (int j = j0; j < j1; ++j) {
            double v = 0.0;
            ok = pg1_draw(env, a.seed, id, t, a.instance, (unsigned)j, &v) && ok;
            sum += v;
        }
        if (!ok)
            atomicOr(&a.st->status, kStatusGamma);
    }
    // Segmented inclusive scan over the lanes, segments = runs of one site
    // (lanes past nq form a run of their own and store nothing).
    const int prev = __shfl_up(p, 1, 64), next = __shfl_down(p, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || prev != p);
    const unsigned long long upto = heads & ((2ull << lane) - 1ull);   // lanes 0 .. lane
    const int start = 63 - __builtin_clzll(upto);                      // lane 0 is a head
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(sum, off, 64);
        if (lane - off >= start)
            sum += o;
    }
    if (valid && (lane == 63 || next != p))
        ca.chunk_sum[q] = sum;
}

// psi_p of sites lo .. lo + cnt - 1, one wavefront per site.  The run sums
// of site p sit in the last chunk of each run: at the chunks q = 63 mod 64
// inside [c0, c1 - 1) (run r at (c0 | 63) + 64 r) and at c1 - 1 (the last run).
template <typename Real>
__global__ __launch_bounds__(kThreads) void pg_psi_kernel(CsrArgs<Real> ca, int lo, int cnt)
{
    const int lane = (int)threadIdx.x & 63;
    const int p = lo + (int)blockIdx.x * kPsiSites + ((int)threadIdx.x >> 6);
    if (p >= lo + cnt)      // uniform across the wavefront
        return;
    const int c0 = ca.chunk_off[p], c1 = ca.chunk_off[p + 1];
    double part = 0.0;
    if (c1 > c0) {
        const int qa = c0 | 63, ql = c1 - 1;
        const int runs = (qa < ql ? (ql - qa + 63) / 64 : 0) + 1;
        for (int r = lane; r < runs; r += 64)
            part += ca.chunk_sum[r == runs - 1 ? ql : qa + 64 * r];
    }
    const double psi = wave_sum(part);
    if (lane == 0)
        ca.psi[p] = psi;
}

// One color pass of the binomial model, one site per thread (the PG terms
// and psi drawn beforehand).
template <typename Real, bool B0>
__global__ __launch_bounds__(kThreads) void csr_binomial_pass_kernel(CsrArgs<Real> ca, SweepArgs a,
                                                                     int lo, int cnt, int slot_base)
{
    const int chunk = xcd_tile((int)blockIdx.x, (int)gridDim.x);   // as csr_pass_kernel
    csr_pass_block<Real, B0, true>(ca, a, lo, cnt, lo + chunk * kThreads, slot_base + chunk);
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// Redraw after the last completed sweep from its stored reductions (one
// wavefront); bitwise what the end of that sweep draws with hyperparameters
// on.
__global__ void hyper_kernel(SweepArgs a)
{
    const unsigned t = (unsigned)(a.st->sweep - 1ull);
    const HyperIn in{a.st->tau, a.st->lam, a.st->beta0};
    Red r;
    r.q = a.st->q;
    r.sse = a.st->sse;
    r.rsum = a.st->rsum;
    end_of_sweep_draws(a, t, r, in, (int)threadIdx.x);
}

__global__ void set_hyper_kernel(DevState *st, double tau, double lam)
{
    st->tau = tau;
    st->lam = lam;
}

// Set the intercept; for the Gaussian model the stored residual sums move
// with it so that a redraw from them stays consistent with x (the binomial
// sums do not involve beta0).
__global__ void set_intercept_kernel(DevState *st, double beta0, double n, int binomial)
{
    if (!binomial) {
        const double d = beta0 - st->beta0;
        st->sse = st->sse - 2.0 * d * st->rsum + n * d * d;
        st->rsum = st->rsum - n * d;
    }
    st->beta0 = beta0;
}

// Posterior mean S1/N and variance (S2 - S1^2/N)/(N - 1), un-permuted to the
// original site order (orig NULL for a lattice).
__global__ void stats_kernel(const double *s1, const double *s2, const int *orig, long long n,
                             const DevState *st, double *mean, double *var)
{
    const double N = (double)st->n_acc;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        const long long o = orig ? (long long)orig[p] : p;
        mean[o] = s1[p] / N;
        var[o] = (s2[p] - s1[p] * s1[p] / N) / (N - 1.0);
    }
}

// Scratch of gmrf_sweep_static: the two partial buffers (kStaticSlots slots of
// kPartials doubles each) and the unit-variate ring, in place of the ones in
// the chain's workspace.  One copy per device, for the life of the process.
constexpr int kStaticSlots = 8192;
constexpr size_t kStaticPartialBytes = 2 * (size_t)kStaticSlots * kPartials * sizeof(double);
constexpr size_t kScratchBytes = kStaticPartialBytes + 2 * (size_t)kUnitRows * sizeof(UnitDraws);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

} // namespace gmrf

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace gmrf;

struct gmrf_graph {
    HostGraph h;
    int *d_row_ptr = nullptr, *d_col = nullptr, *d_orig = nullptr;
    // chunks of the one-launch sweep (shape 1), when h.chunks_ok
    int *d_ch_loc = nullptr, *d_ch_row = nullptr, *d_ch_adj = nullptr, *d_ch_meta = nullptr;
    int *d_loc_site = nullptr;
    unsigned *d_loc_id = nullptr;
    unsigned short *d_loc_row = nullptr, *d_loc_adj = nullptr;
};

struct gmrf_chain {
    const gmrf_graph *g = nullptr;
    gmrf_precision prec = GMRF_FP64;
    gmrf_model model{};
    uint64_t seed = 0;
    uint32_t instance = 0;
    int64_t rank = 0;
    DevState *d_state = nullptr;
    void *d_x[2] = {nullptr, nullptr};
    void *d_y = nullptr;
    double *d_s1 = nullptr, *d_s2 = nullptr;
    double *d_partials = nullptr;
    double *d_stats = nullptr;
    UnitDraws *d_units = nullptr;     // ring of unit variates drawn ahead of the sweeps
    int slot_stride = 0;              // partial slots reserved per buffer (lattice: two)
    int total_slots = 0;              // partial slots of one sweep (current tile shape)
    int lat_tile = 0;                 // shape: lattice tile (index into kTiles); general
                                      // graph: 0 color passes, kPersistent one block
    bool binomial = false;            // binomial logit likelihood (general graphs only)
    int *d_trials = nullptr;          // binomial: m_i in slab order
    int *d_chunk_off = nullptr;       // binomial: PG term chunk tables (see pg_chunk_kernel)
    int *d_chunk_site = nullptr;
    double *d_chunk_sum = nullptr;
    PgEnvelope *d_env = nullptr;
    double *d_psi = nullptr;
    int n_chunks = 0;                 // binomial: PG term chunks of all sites
    std::vector<int> pass_blocks;     // CSR: blocks per color pass
    uint64_t host_sweeps = 0;         // sweeps enqueued (host view)
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int, unsigned>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
};

struct gmrf_batch {
    std::vector<gmrf_chain *> chains;
    gmrf_precision prec = GMRF_FP64;
    // device job tables (inside the batch workspace)
    // lattice groups w = (stencil 8) + 2 (intercept) + 4 (tile shape); general-
    // graph groups g = intercept.  Each group is its own launch (its kernel is
    // specialised).
    void *lat_jobs[8] = {};
    LatTile *lat_tiles[8] = {};
    int lat_tile_count[8] = {};
    void *csr_jobs[2] = {};
    CsrBlock *csr_blocks[2] = {};
    // chunked general-graph chains (shape 1), by intercept setting g: groups
    // g (ended in the next sweep's launch) and 2 + g (more partial slots than
    // kDeferredMaxSlots: every sweep ends in the per-sweep commit launch)
    void *fused_jobs[4] = {};
    FusedBlock *fused_blocks[4] = {};
    int fused_count[4] = {};
    int fused_lds = 0;
    std::vector<int> csr_color_off[2];            // per color index: first block
    SweepArgs *unit_args = nullptr;               // per chain, for the unit-variate launches
    SweepArgs *csr_commit = nullptr;              // general-graph chains: commit every sweep
    SweepArgs *lat_commit = nullptr;              // one-launch chains (lattices, chunked
                                                  // general graphs): commit at a call's end
    int n_csr = 0, n_lat = 0;
    char *ws = nullptr;                           // the caller's workspace (job tables)
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int, unsigned>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
};

namespace {

// Lattice tile shapes (rows x cols of the tile, threads per block).  Shape 0
// suits large lattices (fewest recomputed halo sites per interior site);
// shape 1 suits small and mid-size ones, where more, smaller blocks shorten
// the per-block chain of dependent phases.  Measured on MI355X, shape 1 is
// 25-40% faster per sweep up to 1024 x 1024 and shape 0 is faster at
// 2048 x 2048.  Shape 2 is shape 0's tile for a lattice that fits in it,
// swept by the persistent one-block kernel (many sweeps per launch).
struct TileShape {
    int th, tw, nt;
};
constexpr TileShape kTiles[GMRF_NUM_TILES] = {{64, 64, 512}, {32, 32, 256}, {64, 64, 512}};
constexpr int kPersistent = 2;
constexpr int kFused = 1;          // general graphs: the chunked one-launch sweep
template <int ST, int K>
using LatticeCfg = LatCfg<ST, kTiles[K].th, kTiles[K].tw, kTiles[K].nt, 4>;
static_assert(GMRF_NUM_TILES == 3, "tile dispatch below covers three shapes");

// Tile configuration (0 or 1) whose kernels sweep a chain of shape k.
int tile_cfg(int k) { return k == kPersistent ? 0 : k; }

// Can shape k sweep this lattice?
bool tile_fits(const HostGraph &h, int k)
{
    return k != kPersistent || (h.rows <= kTiles[0].th && h.cols <= kTiles[0].tw);
}

#define GMRF_HIP(expr)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(GMRF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_lattice(const gmrf_graph *g) { return g->h.stencil != 0; }

// One-launch sweeps: lattices and chunked general graphs sweep in one kernel
// whose blocks can end the previous sweep of the call themselves.  Each block
// then sums every partial slot, so that is done only up to kDeferredMaxSlots
// slots; beyond, each sweep ends in its own one-block commit launch.
constexpr int kDeferredMaxSlots = 2048;
bool one_launch(const gmrf_chain *c) { return is_lattice(c->g) || c->lat_tile == kFused; }

size_t real_size(gmrf_precision p) { return p == GMRF_FP64 ? 8 : 4; }

int lattice_blocks(const HostGraph &h, int k)
{
    const int tr = (h.rows + kTiles[k].th - 1) / kTiles[k].th;
    const int tc = (h.cols + kTiles[k].tw - 1) / kTiles[k].tw;
    return tr * tc;
}

// Default tile shape: the persistent kernel for a lattice that fits one tile;
// else the large tile once it yields enough blocks to cover the chip twice
// (256 CUs), the small one below that.
int default_tile(const HostGraph &h)
{
    if (tile_fits(h, kPersistent))
        return kPersistent;
    return lattice_blocks(h, 0) >= 512 ? 0 : 1;
}

// Partial slots to reserve: the most any tile shape needs.
int max_lattice_blocks(const HostGraph &h)
{
    int m = 0;
    for (int k = 0; k < GMRF_NUM_TILES; ++k)
        if (tile_fits(h, k))
            m = std::max(m, lattice_blocks(h, k));
    return m;
}

// Chain workspace layout; ptrs may be NULL to only compute the size.  A
// binomial chain adds the trials, the term chunk tables, and per-site
// envelopes and psi.
size_t chain_layout(const gmrf_graph *g, gmrf_precision p, char *base, gmrf_chain *c,
                    bool binomial, int64_t n_chunks = 0)
{
    const int64_t n = g->h.n;
    const size_t rs = real_size(p);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return base ? base + at : nullptr;
    };
    int slots = 0, reserve = 0;
    std::vector<int> pass_blocks;
    if (is_lattice(g)) {
        slots = lattice_blocks(g->h, c ? c->lat_tile : 0);
        reserve = max_lattice_blocks(g->h);
    } else {
        for (int32_t col = 0; col < g->h.k; ++col) {
            const int cnt = g->h.slab_offsets[col + 1] - g->h.slab_offsets[col];
            const int nb = (cnt + kThreads - 1) / kThreads;
            pass_blocks.push_back(nb);
            slots += nb;
        }
        reserve = std::max(slots, g->h.chunks_ok ? g->h.nchunks : 0);
        if (c && c->lat_tile == kFused)
            slots = g->h.nchunks;
    }
    char *st = take(sizeof(DevState));
    char *x0 = take(rs * n);
    char *x1 = take(rs * n);
    char *y = take(rs * n);
    char *s1 = take(8 * n);
    char *s2 = take(8 * n);
    // one-launch sweeps alternate two partial buffers (a sweep kernel ends
    // the previous sweep from its buffer while writing its own)
    char *part = take(8 * kPartials * (size_t)std::max(reserve, 1) * 2);
    char *units = take(sizeof(UnitDraws) * 2 * kUnitRows);
    char *stats = take(16 * n);
    char *trials = binomial ? take(4 * n) : nullptr;
    char *chunk_off = binomial ? take(4 * (size_t)(n + 1)) : nullptr;
    char *chunk_site = binomial ? take(4 * (size_t)std::max<int64_t>(n_chunks, 1)) : nullptr;
    char *chunk_sum = binomial ? take(8 * (size_t)std::max<int64_t>(n_chunks, 1)) : nullptr;
    char *env = binomial ? take(sizeof(PgEnvelope) * (size_t)n) : nullptr;
    char *psi = binomial ? take(8 * (size_t)n) : nullptr;
    if (c) {
        c->d_psi = reinterpret_cast<double *>(psi);
        c->d_trials = reinterpret_cast<int *>(trials);
        c->d_chunk_off = reinterpret_cast<int *>(chunk_off);
        c->d_chunk_site = reinterpret_cast<int *>(chunk_site);
        c->d_chunk_sum = reinterpret_cast<double *>(chunk_sum);
        c->d_env = reinterpret_cast<PgEnvelope *>(env);
        c->d_state = reinterpret_cast<DevState *>(st);
        c->d_x[0] = x0;
        c->d_x[1] = x1;
        c->d_y = y;
        c->d_s1 = reinterpret_cast<double *>(s1);
        c->d_s2 = reinterpret_cast<double *>(s2);
        c->d_partials = reinterpret_cast<double *>(part);
        c->d_stats = reinterpret_cast<double *>(stats);
        c->d_units = reinterpret_cast<UnitDraws *>(units);
        c->slot_stride = std::max(reserve, 1);
        c->total_slots = slots;
        c->pass_blocks = pass_blocks;
    }
    return off;
}

// Arguments of a timing run (dry): the draws are computed but not stored,
// and the accumulator updates go to the chain's statistics scratch (2n
// doubles) instead of S1 / S2, with the memory traffic of real ones, so that
// the chain's state and accumulators stay as they are.
SweepArgs dry_args(SweepArgs a, const gmrf_chain *c)
{
    a.dry = 1;
    a.s1 = c->d_stats;
    a.s2 = c->d_stats + c->g->h.n;
    return a;
}

SweepArgs make_args(const gmrf_chain *c, unsigned flags)
{
    SweepArgs a{};
    a.st = c->d_state;
    a.partials = c->d_partials;
    a.s1 = c->d_s1;
    a.s2 = c->d_s2;
    const double shape_tau = c->model.a_tau + 0.5 * (double)c->rank;
    const double shape_lam = c->model.a_lam + 0.5 * (double)c->g->h.n;
    a.g_tau.d = shape_tau - 1.0 / 3.0;
    a.g_tau.c = 1.0 / std::sqrt(9.0 * a.g_tau.d);
    a.g_lam.d = shape_lam - 1.0 / 3.0;
    a.g_lam.c = 1.0 / std::sqrt(9.0 * a.g_lam.d);
    a.b_tau = c->model.b_tau;
    a.b_lam = c->model.b_lam;
    a.rho = c->g->h.rho;
    a.burn_in = (long long)c->model.burn_in;
    a.seed = c->seed;
    a.instance = c->instance;
    a.with_hyper = (flags & GMRF_WITH_HYPER) ? 1 : 0;
    a.total_slots = c->total_slots;
    a.intercept = c->model.intercept ? 1 : 0;
    a.likelihood = c->binomial ? 1 : 0;
    a.b0_prec = c->binomial && c->model.beta0_var > 0.0 ? 1.0 / c->model.beta0_var : 0.0;
    a.n_sites = (double)c->g->h.n;
    a.units = c->d_units;
    a.slot_stride = c->slot_stride;
    a.deferred = one_launch(c) && c->total_slots <= kDeferredMaxSlots ? 1 : 0;
    return a;
}

template <typename Real> LatArgs<Real> lattice_args(const gmrf_chain *c, int shape = -1)
{
    const HostGraph &h = c->g->h;
    if (shape < 0)
        shape = c->lat_tile;
    LatArgs<Real> la;
    la.x0 = static_cast<Real *>(c->d_x[0]);
    la.x1 = static_cast<Real *>(c->d_x[1]);
    la.y = static_cast<const Real *>(c->d_y);
    la.rows = h.rows;
    la.cols = h.cols;
    la.tiles_c = (h.cols + kTiles[shape].tw - 1) / kTiles[shape].tw;
    return la;
}

template <typename Real> CsrArgs<Real> csr_args(const gmrf_chain *c)
{
    CsrArgs<Real> ca;
    ca.row_ptr = c->g->d_row_ptr;
    ca.col = c->g->d_col;
    ca.orig = c->g->d_orig;
    ca.x = static_cast<Real *>(c->d_x[0]);
    ca.y = static_cast<const Real *>(c->d_y);
    ca.trials = c->d_trials;
    ca.chunk_off = c->d_chunk_off;
    ca.chunk_site = c->d_chunk_site;
    ca.chunk_sum = c->d_chunk_sum;
    ca.env = c->d_env;
    ca.psi = c->d_psi;
    return ca;
}

// ev0 / ev1 (optional): events the dispatch itself records at the start and
// the end of the sweep kernel(s), for the profiling entry point.
template <typename Real, int ST, int K>
void launch_lattice_shape(const gmrf_chain *c, const SweepArgs &a, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1, int rel, int fold)
{
    const LatArgs<Real> la = lattice_args<Real>(c);
    using Cfg = LatticeCfg<ST, K>;
    const bool v2 = c->model.rng_version == 2;
    auto kern = c->model.intercept
                    ? (v2 ? lattice_sweep_kernel<Real, Cfg, true, true>
                          : lattice_sweep_kernel<Real, Cfg, true, false>)
                    : (v2 ? lattice_sweep_kernel<Real, Cfg, false, true>
                          : lattice_sweep_kernel<Real, Cfg, false, false>);
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(c->total_slots), dim3(Cfg::NT), 0, s, ev0, ev1, 0, la,
                              a, rel, fold);
    else
        hipLaunchKernelGGL(kern, dim3(c->total_slots), dim3(Cfg::NT), 0, s, la, a, rel, fold);
}

template <typename Real, int ST>
void launch_lattice(const gmrf_chain *c, const SweepArgs &a, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1, int rel, int fold)
{
    if (tile_cfg(c->lat_tile) == 0)
        launch_lattice_shape<Real, ST, 0>(c, a, s, ev0, ev1, rel, fold);
    else
        launch_lattice_shape<Real, ST, 1>(c, a, s, ev0, ev1, rel, fold);
}

// nsweeps sweeps of a shape-2 chain in one launch of the persistent kernel.
template <typename Real, int ST>
void launch_persistent_typed(const gmrf_chain *c, const SweepArgs &a, int nsweeps, hipStream_t s,
                             hipEvent_t ev0, hipEvent_t ev1)
{
    const LatArgs<Real> la = lattice_args<Real>(c);
    using Cfg = LatticeCfg<ST, 0>;
    const bool v2 = c->model.rng_version == 2;
    auto kern = c->model.intercept
                    ? (v2 ? lattice_persistent_kernel<Real, Cfg, true, true>
                          : lattice_persistent_kernel<Real, Cfg, true, false>)
                    : (v2 ? lattice_persistent_kernel<Real, Cfg, false, true>
                          : lattice_persistent_kernel<Real, Cfg, false, false>);
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(1), dim3(Cfg::NT), 0, s, ev0, ev1, 0, la, a, nsweeps);
    else
        hipLaunchKernelGGL(kern, dim3(1), dim3(Cfg::NT), 0, s, la, a, nsweeps);
}

SlabTable slab_table(const HostGraph &h)
{
    SlabTable sl{};
    sl.k = h.k;
    for (int32_t col = 0; col <= h.k; ++col)
        sl.off[col] = (int)h.slab_offsets[col];
    return sl;
}

// nsweeps sweeps (binomial: one, after the Polya-Gamma launches) of a shape-2
// general-graph chain in one launch of the persistent kernel.
template <typename Real>
void launch_csr_persistent(const gmrf_chain *c, const SweepArgs &a, int nsweeps, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1)
{
    const CsrArgs<Real> ca = csr_args<Real>(c);
    const SlabTable sl = slab_table(c->g->h);
    const bool b0 = c->model.intercept;
    auto kern = c->binomial ? (b0 ? csr_persistent_kernel<Real, true, true>
                                  : csr_persistent_kernel<Real, false, true>)
                            : (b0 ? csr_persistent_kernel<Real, true, false>
                                  : csr_persistent_kernel<Real, false, false>);
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(1), dim3(kCsrPersistThreads), 0, s, ev0, ev1, 0, ca, a,
                              sl, nsweeps);
    else
        hipLaunchKernelGGL(kern, dim3(1), dim3(kCsrPersistThreads), 0, s, ca, a, sl, nsweeps);
}

void launch_persistent(const gmrf_chain *c, const SweepArgs &a, int nsweeps, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const bool f64 = c->prec == GMRF_FP64;
    if (!is_lattice(c->g))
        f64 ? launch_csr_persistent<double>(c, a, nsweeps, s, ev0, ev1)
            : launch_csr_persistent<float>(c, a, nsweeps, s, ev0, ev1);
    else if (c->g->h.stencil == 4)
        f64 ? launch_persistent_typed<double, 4>(c, a, nsweeps, s, ev0, ev1)
            : launch_persistent_typed<float, 4>(c, a, nsweeps, s, ev0, ev1);
    else
        f64 ? launch_persistent_typed<double, 8>(c, a, nsweeps, s, ev0, ev1)
            : launch_persistent_typed<float, 8>(c, a, nsweeps, s, ev0, ev1);
}

// Can the persistent one-block kernel sweep this general graph (its field in
// LDS, its colors in the slab table)?
bool csr_persist_fits(const HostGraph &h, gmrf_precision p)
{
    if (h.stencil != 0 || h.k > kCsrPersistColors ||
        h.n * (int64_t)real_size(p) > (int64_t)kCsrLdsBytes)
        return false;
    int64_t slots = 0;
    for (int32_t col = 0; col < h.k; ++col)
        slots += (h.slab_offsets[col + 1] - h.slab_offsets[col] + kThreads - 1) / kThreads;
    return slots <= kCsrPersistSlots;
}

// Can the chunked one-launch sweep take this chain?  (Its graph's chunks fit
// the LDS and index limits; not the binomial model, whose Polya-Gamma draws
// run per site before the color passes.)
bool csr_fused_fits(const HostGraph &h, gmrf_precision p, bool binomial)
{
    return h.stencil == 0 && h.chunks_ok && !binomial &&
           (p == GMRF_FP64 ? h.max_image8 : h.max_image4) <= kFusedLaunchLds;
}

// Default shape of a general-graph chain: the one block while it covers
// every color's slab in at most two rounds of its threads (measured on
// MI355X with Delaunay graphs: one block 15.2 against 24.3 us per sweep at
// 500 sites, 29.4 against 35.4 at 4,000, slower from ~5,000 sites on, where
// its serial rounds outlast the k + 1 launches), else the chunked one-launch
// sweep where it fits, else the color passes.
int csr_default_shape(const HostGraph &h, gmrf_precision p, bool binomial)
{
    // the chunked sweep first: on Delaunay graphs of 300 to 50,000 sites it
    // is as fast as the one-block shape at 300 to 1,000 sites (within 4%)
    // and faster from 2,000 sites on, and faster than the color passes at
    // every size
    if (csr_fused_fits(h, p, binomial))
        return kFused;
    bool small = csr_persist_fits(h, p);
    for (int32_t col = 0; small && col < h.k; ++col)
        if (h.slab_offsets[col + 1] - h.slab_offsets[col] > 2 * kCsrPersistThreads)
            small = false;
    return small ? kPersistent : 0;
}

// Partial slots of one sweep of a general-graph chain in shape k.
int csr_slots(const gmrf_chain *c, int k)
{
    if (k == kFused)
        return c->g->h.nchunks;
    int slots = 0;
    for (int nb : c->pass_blocks)
        slots += nb;
    return slots;
}

// Do all the sweeps of a call run in one launch?  (Shape 2, except for the
// binomial model, whose Polya-Gamma launches come between sweeps.)
bool is_persistent(const gmrf_chain *c) { return c->lat_tile == kPersistent && !c->binomial; }

// Does the chain draw the hyperparameters inside its sweep kernel (no commit
// kernel)?
bool draws_in_sweep(const gmrf_chain *c) { return c->lat_tile == kPersistent; }

// Launch configuration of the small element-wise kernels.
int elementwise_blocks(int64_t n)
{
    return (int)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
}


// Arguments of the chunked one-launch sweep; x0 / x1 are the chain's two
// state buffers (swap: the other way round, for timing runs whose current
// buffer is not the one the sweep parity reads).
template <typename Real> FusedArgs<Real> fused_args(const gmrf_chain *c, bool swap = false)
{
    const gmrf_graph *g = c->g;
    FusedArgs<Real> fa;
    fa.ch_loc = g->d_ch_loc;
    fa.ch_row = g->d_ch_row;
    fa.ch_adj = g->d_ch_adj;
    fa.ch_meta = g->d_ch_meta;
    fa.loc_site = g->d_loc_site;
    fa.loc_row = g->d_loc_row;
    fa.loc_adj = g->d_loc_adj;
    fa.loc_id = g->d_loc_id;
    fa.x0 = static_cast<Real *>(c->d_x[swap ? 1 : 0]);
    fa.x1 = static_cast<Real *>(c->d_x[swap ? 0 : 1]);
    fa.y = static_cast<const Real *>(c->d_y);
    fa.k = g->h.k;
    return fa;
}

// LDS of the chunked sweep for a graph's chunks in precision Real: the
// largest chunk image (each block lays out its own chunk's).
template <typename Real> size_t fused_lds_bytes(const HostGraph &h)
{
    return (size_t)(sizeof(Real) == 8 ? h.max_image8 : h.max_image4);
}

template <typename Real>
void launch_fused(const gmrf_chain *c, const FusedArgs<Real> &fa, const SweepArgs &a,
                  hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int rel, int fold)
{
    const HostGraph &h = c->g->h;
    auto kern = c->model.intercept ? csr_fused_kernel<Real, true> : csr_fused_kernel<Real, false>;
    const size_t lds = fused_lds_bytes<Real>(h);
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(h.nchunks), dim3(kThreads), lds, s, ev0, ev1, 0, fa, a,
                              rel, fold);
    else
        hipLaunchKernelGGL(kern, dim3(h.nchunks), dim3(kThreads), lds, s, fa, a, rel, fold);
}

template <typename Real>
void launch_csr(const gmrf_chain *c, const SweepArgs &a, hipStream_t s, hipEvent_t ev0,
                hipEvent_t ev1, int rel = 0, int fold = 0)
{
    const HostGraph &h = c->g->h;
    if (c->lat_tile == kFused) {
        launch_fused<Real>(c, fused_args<Real>(c), a, s, ev0, ev1, rel, fold);
        return;
    }
    const CsrArgs<Real> ca = csr_args<Real>(c);
    int slot = 0, last = -1;
    for (int32_t col = 0; col < h.k; ++col)
        if (c->pass_blocks[col] > 0)
            last = col;
    // Binomial: the envelopes, the PG terms and psi of every site, one launch
    // each, before the color passes (psi alone when no site has trials).
    if (c->binomial) {
        const int nq = c->n_chunks;
        const int nsite = (int)h.n;
        auto ek = c->model.intercept ? pg_env_kernel<Real, true> : pg_env_kernel<Real, false>;
        auto tk = c->model.intercept ? pg_chunk_kernel<Real, true> : pg_chunk_kernel<Real, false>;
        const int eb = (nsite + kThreads - 1) / kThreads, tb = (nq + kThreads - 1) / kThreads;
        const int pb = (nsite + kPsiSites - 1) / kPsiSites;
        if (nq > 0) {
            if (ev0)
                hipExtLaunchKernelGGL(ek, dim3(eb), dim3(kThreads), 0, s, ev0, nullptr, 0, ca, a,
                                      0, nsite);
            else
                hipLaunchKernelGGL(ek, dim3(eb), dim3(kThreads), 0, s, ca, a, 0, nsite);
            ev0 = nullptr;
        }
        if (nq > 0) {
            if (ev0)
                hipExtLaunchKernelGGL(tk, dim3(tb), dim3(kThreads), 0, s, ev0, nullptr, 0, ca, a,
                                      nq);
            else
                hipLaunchKernelGGL(tk, dim3(tb), dim3(kThreads), 0, s, ca, a, nq);
            ev0 = nullptr;
        }
        if (ev0)
            hipExtLaunchKernelGGL(pg_psi_kernel<Real>, dim3(pb), dim3(kThreads), 0, s, ev0,
                                  nullptr, 0, ca, 0, nsite);
        else
            hipLaunchKernelGGL(pg_psi_kernel<Real>, dim3(pb), dim3(kThreads), 0, s, ca, 0, nsite);
        ev0 = nullptr;
        if (c->lat_tile == kPersistent) {       // the color passes and draws in one block
            launch_csr_persistent<Real>(c, a, 1, s, ev0, ev1);
            return;
        }
    }
    for (int32_t col = 0; col < h.k; ++col) {
        const int nb = c->pass_blocks[col];
        if (nb == 0)
            continue;
        const int lo = h.slab_offsets[col], cnt = h.slab_offsets[col + 1] - lo;
        hipEvent_t e0 = slot == 0 ? ev0 : nullptr, e1 = col == last ? ev1 : nullptr;
        auto kern = c->binomial ? (c->model.intercept ? csr_binomial_pass_kernel<Real, true>
                                                      : csr_binomial_pass_kernel<Real, false>)
                                : (c->model.intercept ? csr_pass_kernel<Real, true>
                                                      : csr_pass_kernel<Real, false>);
        const int threads = kThreads;
        if (e0 || e1)
            hipExtLaunchKernelGGL(kern, dim3(nb), dim3(threads), 0, s, e0, e1, 0, ca, a, lo, cnt,
                                  slot);
        else
            hipLaunchKernelGGL(kern, dim3(nb), dim3(threads), 0, s, ca, a, lo, cnt, slot);
        slot += nb;
    }
}

// The sweep kernels of relative sweep rel of a call (a lattice: one launch,
// which ends the previous sweep of the call unless rel is 0; a general
// graph: the color passes).  A timing run (a.dry) repeats relative sweep 0:
// it never advances the sweep count, so every repetition reads the current
// state buffer and writes only the other one.
void launch_sweep_kernels(const gmrf_chain *c, const SweepArgs &a, hipStream_t s, int rel,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const bool f64 = c->prec == GMRF_FP64;
    if (a.dry || !a.deferred)   // every sweep committed on its own: relative sweep 0
        rel = 0;
    const int fold = rel > 0 ? 1 : 0;
    if (is_lattice(c->g)) {
        if (c->g->h.stencil == 4)
            f64 ? launch_lattice<double, 4>(c, a, s, ev0, ev1, rel, fold)
                : launch_lattice<float, 4>(c, a, s, ev0, ev1, rel, fold);
        else
            f64 ? launch_lattice<double, 8>(c, a, s, ev0, ev1, rel, fold)
                : launch_lattice<float, 8>(c, a, s, ev0, ev1, rel, fold);
    } else {
        f64 ? launch_csr<double>(c, a, s, ev0, ev1, rel, fold)
            : launch_csr<float>(c, a, s, ev0, ev1, rel, fold);
    }
}

void launch_commit(const SweepArgs &a, int rel, int count, hipStream_t s)
{
    hipLaunchKernelGGL(commit_kernel, dim3(1), dim3(kFinishThreads), 0, s, a, rel, count);
}

// Before relative sweep i of a call of nsweeps: the unit-variate launch of
// its group (every kUnitBatch sweeps, when the sweeps draw the
// hyperparameters and the chain's kernels do not draw their own).
void launch_units_ahead(const gmrf_chain *c, const SweepArgs &a, int i, int nsweeps,
                        hipStream_t s)
{
    if (!a.with_hyper || draws_in_sweep(c) || i % kUnitBatch != 0)
        return;
    hipLaunchKernelGGL(unit_draw_kernel, dim3(1), dim3(kUnitThreads), 0, s, a, i,
                       std::min(kUnitBatch, nsweeps - i));
}

// After relative sweep i of a call of nsweeps: its commit where one is due
// (one-launch sweeps -- lattices and chunked general graphs -- after the
// call's last sweep; color passes after every sweep; none where the kernels
// draw themselves, or for timing runs of one-launch sweeps).
void launch_commit_after(const gmrf_chain *c, const SweepArgs &a, int i, int nsweeps,
                         hipStream_t s)
{
    if (draws_in_sweep(c))
        return;
    if (!a.deferred)
        launch_commit(a, 0, 1, s);
    else if (i == nsweeps - 1 && !a.dry)
        launch_commit(a, i, nsweeps, s);
}

// nsweeps sweeps of a chain with per-sweep launches.
void launch_sweeps(const gmrf_chain *c, const SweepArgs &a, int nsweeps, hipStream_t s)
{
    for (int i = 0; i < nsweeps; ++i) {
        launch_units_ahead(c, a, i, nsweeps, s);
        launch_sweep_kernels(c, a, s, i);
        launch_commit_after(c, a, i, nsweeps, s);
    }
}

int read_state(gmrf_chain *c, DevState *out, hipStream_t s)
{
    GMRF_HIP(hipMemcpyAsync(out, c->d_state, sizeof(DevState), hipMemcpyDeviceToHost, s));
    GMRF_HIP(hipStreamSynchronize(s));
    return GMRF_OK;
}

int check_status(const DevState &st)
{
    if (st.status & kStatusGamma)
        return fail(GMRF_E_NUMERIC,
                    "device: a tau/lam Gamma draw hit the attempt cap or was not finite");
    return GMRF_OK;
}

// Current state buffer: lattice chains and chunked general-graph chains
// (shape 1) ping-pong on the sweep parity; the other general-graph shapes
// update buffer 0 in place.
void *current_x(const gmrf_chain *c, uint64_t sweep)
{
    return is_lattice(c->g) || c->lat_tile == kFused ? c->d_x[sweep & 1u] : c->d_x[0];
}

// x in layout order (Real) <-> original-order doubles.
template <typename Real>
void to_layout(const gmrf_chain *c, const double *x, std::vector<char> &buf)
{
    const int64_t n = c->g->h.n;
    buf.resize(sizeof(Real) * n);
    Real *o = reinterpret_cast<Real *>(buf.data());
    for (int64_t p = 0; p < n; ++p)
        o[p] = (Real)x[is_lattice(c->g) ? p : c->g->h.orig_of_slab[p]];
}

template <typename Real>
void from_layout(const gmrf_chain *c, const std::vector<char> &buf, double *x)
{
    const int64_t n = c->g->h.n;
    const Real *o = reinterpret_cast<const Real *>(buf.data());
    for (int64_t p = 0; p < n; ++p)
        x[is_lattice(c->g) ? p : c->g->h.orig_of_slab[p]] = (double)o[p];
}

int upload_real(const gmrf_chain *c, void *dst, const double *x, hipStream_t s)
{
    std::vector<char> buf;
    if (c->prec == GMRF_FP64)
        to_layout<double>(c, x, buf);
    else
        to_layout<float>(c, x, buf);
    GMRF_HIP(hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
    GMRF_HIP(hipStreamSynchronize(s));
    return GMRF_OK;
}

int upload_doubles_layout(const gmrf_chain *c, double *dst, const double *x, hipStream_t s)
{
    const int64_t n = c->g->h.n;
    std::vector<double> buf(n);
    for (int64_t p = 0; p < n; ++p)
        buf[p] = x[is_lattice(c->g) ? p : c->g->h.orig_of_slab[p]];
    GMRF_HIP(hipMemcpyAsync(dst, buf.data(), 8 * n, hipMemcpyHostToDevice, s));
    GMRF_HIP(hipStreamSynchronize(s));
    return GMRF_OK;
}

// Upload m_i in slab order and build the PG term chunk tables: chunk_off[p]
// = first chunk of slab position p (chunks of a color are contiguous because
// its slab is), chunk_site[q] = the slab position chunk q belongs to.
int upload_trials_layout(gmrf_chain *c, const int32_t *trials, hipStream_t s)
{
    const HostGraph &h = c->g->h;
    const int64_t n = h.n;
    std::vector<int32_t> buf(n), off(n + 1, 0), site;
    for (int64_t p = 0; p < n; ++p) {
        buf[p] = trials[h.orig_of_slab[p]];
        off[p + 1] = off[p] + (buf[p] + kPgChunk - 1) / kPgChunk;
    }
    site.resize(std::max<int64_t>(off[n], 1));
    for (int64_t p = 0; p < n; ++p)
        for (int q = off[p]; q < off[p + 1]; ++q)
            site[q] = (int32_t)p;
    c->n_chunks = off[n];
    GMRF_HIP(hipMemcpyAsync(c->d_trials, buf.data(), 4 * n, hipMemcpyHostToDevice, s));
    GMRF_HIP(hipMemcpyAsync(c->d_chunk_off, off.data(), 4 * (n + 1), hipMemcpyHostToDevice, s));
    GMRF_HIP(hipMemcpyAsync(c->d_chunk_site, site.data(), 4 * site.size(), hipMemcpyHostToDevice,
                            s));
    GMRF_HIP(hipStreamSynchronize(s));
    return GMRF_OK;
}

int download_doubles_layout(const gmrf_chain *c, const double *src, double *x, hipStream_t s)
{
    const int64_t n = c->g->h.n;
    std::vector<double> buf(n);
    GMRF_HIP(hipMemcpyAsync(buf.data(), src, 8 * n, hipMemcpyDeviceToHost, s));
    GMRF_HIP(hipStreamSynchronize(s));
    for (int64_t p = 0; p < n; ++p)
        x[is_lattice(c->g) ? p : c->g->h.orig_of_slab[p]] = buf[p];
    return GMRF_OK;
}

bool finite_array(const double *v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i]))
            return false;
    return true;
}

// Host image of a batch's job tables and the offsets of its sections.
struct BatchImage {
    std::vector<char> bytes;
    size_t off_lat_jobs[8] = {}, off_lat_tiles[8] = {};
    size_t off_csr_jobs[2] = {}, off_csr_blocks[2] = {}, off_units = 0;
    size_t off_csr_commit = 0, off_lat_commit = 0;
    size_t off_fused_jobs[4] = {}, off_fused_blocks[4] = {};
    int n_csr = 0, n_lat = 0;
    int lat_tile_count[8] = {};
    int fused_count[4] = {};
    int fused_lds = 0;                            // bytes of LDS of the batched chunked launch
    std::vector<int> csr_color_off[2];
};

template <typename T> size_t append(std::vector<char> &img, const std::vector<T> &v)
{
    const size_t at = align_up(img.size());
    img.resize(at + align_up(sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty())
        std::memcpy(img.data() + at, v.data(), sizeof(T) * v.size());
    return at;
}

// Job tables of a batch.  force >= 0 lays every lattice chain out in tile
// configuration `force` instead of its own shape, and dry makes the lattice
// jobs timing runs (dry_args), for the batch autotuner.
template <typename Real>
void build_batch_image(const std::vector<gmrf_chain *> &cs, BatchImage &im, int force = -1,
                       bool dry = false)
{
    std::vector<LatJob<Real>> ljobs[8];
    std::vector<LatTile> ltiles[8];
    std::vector<CsrJob<Real>> cjobs[2];
    std::vector<std::vector<CsrBlock>> cblocks[2];   // per color index
    std::vector<SweepArgs> units, csr_commit, lat_commit;   // lat_commit: every one-launch chain
    std::vector<FusedJob<Real>> fjobs[4];
    std::vector<FusedBlock> fblocks[4];
    for (const gmrf_chain *c : cs) {
        SweepArgs a = make_args(c, 0u);
        // shared launches end a one-launch chain's sweep in the next, except a
        // chunked chain with more partial slots than every block can sum,
        // which commits every sweep as it does on its own
        const bool own_commit = c->lat_tile == kFused && !is_lattice(c->g) &&
                                c->total_slots > kDeferredMaxSlots;
        if (one_launch(c))
            a.deferred = own_commit ? 0 : 1;
        units.push_back(a);
        const HostGraph &h = c->g->h;
        const int g = c->model.intercept ? 1 : 0;
        if (is_lattice(c->g)) {
            const int cfg = force >= 0 ? force : tile_cfg(c->lat_tile);
            const int w = (h.stencil == 8 ? 1 : 0) + 2 * g + 4 * cfg;
            const int job = (int)ljobs[w].size();
            const int tiles = lattice_blocks(h, cfg);
            SweepArgs la_args = dry ? dry_args(a, c) : a;
            la_args.total_slots = tiles;       // the partial slots of this chain's sweep
            ljobs[w].push_back(LatJob<Real>{lattice_args<Real>(c, cfg), la_args});
            lat_commit.push_back(la_args);
            for (int t = 0; t < tiles; ++t)
                ltiles[w].push_back(LatTile{job, t});
        } else if (c->lat_tile == kFused) {
            const int fg = own_commit ? 2 + g : g;
            const int job = (int)fjobs[fg].size();
            fjobs[fg].push_back(FusedJob<Real>{fused_args<Real>(c), a});
            (own_commit ? csr_commit : lat_commit).push_back(a);
            for (int b = 0; b < h.nchunks; ++b)
                fblocks[fg].push_back(FusedBlock{job, b});
            im.fused_lds = std::max(im.fused_lds, (int)fused_lds_bytes<Real>(h));
        } else {
            const int job = (int)cjobs[g].size();
            cjobs[g].push_back(CsrJob<Real>{csr_args<Real>(c), a});
            csr_commit.push_back(a);
            if ((int)cblocks[g].size() < h.k)
                cblocks[g].resize(h.k);
            int slot = 0;
            for (int32_t col = 0; col < h.k; ++col) {
                const int lo = h.slab_offsets[col], cnt = h.slab_offsets[col + 1] - lo;
                for (int b = 0; b < c->pass_blocks[col]; ++b)
                    cblocks[g][col].push_back(
                        CsrBlock{job, lo, cnt, lo + b * kThreads, slot + b});
                slot += c->pass_blocks[col];
            }
        }
    }
    for (int w = 0; w < 8; ++w) {
        im.off_lat_jobs[w] = append(im.bytes, ljobs[w]);
        im.off_lat_tiles[w] = append(im.bytes, ltiles[w]);
        im.lat_tile_count[w] = (int)ltiles[w].size();
    }
    for (int g = 0; g < 2; ++g) {
        std::vector<CsrBlock> flat;
        im.csr_color_off[g].assign(1, 0);
        for (const auto &v : cblocks[g]) {
            flat.insert(flat.end(), v.begin(), v.end());
            im.csr_color_off[g].push_back((int)flat.size());
        }
        im.off_csr_jobs[g] = append(im.bytes, cjobs[g]);
        im.off_csr_blocks[g] = append(im.bytes, flat);
    }
    for (int fg = 0; fg < 4; ++fg) {
        im.off_fused_jobs[fg] = append(im.bytes, fjobs[fg]);
        im.off_fused_blocks[fg] = append(im.bytes, fblocks[fg]);
        im.fused_count[fg] = (int)fblocks[fg].size();
    }
    im.off_units = append(im.bytes, units);
    im.off_csr_commit = append(im.bytes, csr_commit);
    im.off_lat_commit = append(im.bytes, lat_commit);
    im.n_csr = (int)csr_commit.size();
    im.n_lat = (int)lat_commit.size();
}

int check_batch_chains(gmrf_chain *const *chains, int32_t count, gmrf_precision *prec)
{
    if (!chains || count < 1)
        return fail(GMRF_E_INVALID_ARG, "batch: need at least one chain");
    std::unordered_set<const gmrf_chain *> seen;
    seen.reserve((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const gmrf_chain *c = chains[i];
        if (!c)
            return fail(GMRF_E_INVALID_ARG, "batch: NULL chain at index " + std::to_string(i));
        if (!seen.insert(c).second)
            return fail(GMRF_E_INVALID_ARG, "batch: chain at index " + std::to_string(i) +
                                                " appears twice");
        if (c->prec != chains[0]->prec)
            return fail(GMRF_E_INVALID_ARG, "batch: all chains must have one precision");
        if (c->binomial)
            return fail(GMRF_E_INVALID_ARG, "batch: binomial chains are swept on their own "
                                            "(chain at index " + std::to_string(i) + ")");
        if (c->model.rng_version == 2)
            return fail(GMRF_E_INVALID_ARG, "batch: rng_version 2 chains are swept on their own "
                                            "(chain at index " + std::to_string(i) + ")");
    }
    *prec = chains[0]->prec;
    return GMRF_OK;
}

int build_image(gmrf_chain *const *chains, int32_t count, BatchImage &im, gmrf_precision *prec,
                int force = -1, bool dry = false)
{
    const int rc = check_batch_chains(chains, count, prec);
    if (rc != GMRF_OK)
        return rc;
    const std::vector<gmrf_chain *> cs(chains, chains + count);
    if (*prec == GMRF_FP64)
        build_batch_image<double>(cs, im, force, dry);
    else
        build_batch_image<float>(cs, im, force, dry);
    return GMRF_OK;
}

// Workspace of a batch: the largest of its tables with the chains' own
// shapes and with every lattice chain in either tile configuration (the
// autotuner lays the tables out again in the same workspace).  `own`, if
// given, is the image with the chains' own shapes, already built; without
// lattice chains the three layouts are one.
int batch_bytes(gmrf_chain *const *chains, int32_t count, size_t *bytes,
                const BatchImage *own = nullptr)
{
    size_t most = own ? align_up(own->bytes.size()) : 0;
    bool lattices = false;
    for (int32_t i = 0; chains && i < count && !lattices; ++i)
        lattices = chains[i] && is_lattice(chains[i]->g);
    for (int force = own ? 0 : -1; force <= (lattices ? 1 : -1); ++force) {
        BatchImage im;
        gmrf_precision prec;
        const int rc = build_image(chains, count, im, &prec, force);
        if (rc != GMRF_OK)
            return rc;
        most = std::max(most, align_up(im.bytes.size()));
    }
    *bytes = most;
    return GMRF_OK;
}

// Point the batch at the tables of image im, uploaded into its workspace.
int install_image(gmrf_batch *b, const BatchImage &im, hipStream_t stream)
{
    GMRF_HIP(hipMemcpyAsync(b->ws, im.bytes.data(), im.bytes.size(), hipMemcpyHostToDevice,
                            stream));
    GMRF_HIP(hipStreamSynchronize(stream));
    for (int w = 0; w < 8; ++w) {
        b->lat_jobs[w] = b->ws + im.off_lat_jobs[w];
        b->lat_tiles[w] = reinterpret_cast<LatTile *>(b->ws + im.off_lat_tiles[w]);
        b->lat_tile_count[w] = im.lat_tile_count[w];
    }
    for (int g = 0; g < 2; ++g) {
        b->csr_jobs[g] = b->ws + im.off_csr_jobs[g];
        b->csr_blocks[g] = reinterpret_cast<CsrBlock *>(b->ws + im.off_csr_blocks[g]);
        b->csr_color_off[g] = im.csr_color_off[g];
    }
    for (int fg = 0; fg < 4; ++fg) {
        b->fused_jobs[fg] = b->ws + im.off_fused_jobs[fg];
        b->fused_blocks[fg] = reinterpret_cast<FusedBlock *>(b->ws + im.off_fused_blocks[fg]);
        b->fused_count[fg] = im.fused_count[fg];
    }
    b->unit_args = reinterpret_cast<SweepArgs *>(b->ws + im.off_units);
    b->csr_commit = reinterpret_cast<SweepArgs *>(b->ws + im.off_csr_commit);
    b->lat_commit = reinterpret_cast<SweepArgs *>(b->ws + im.off_lat_commit);
    b->n_csr = im.n_csr;
    b->n_lat = im.n_lat;
    b->fused_lds = im.fused_lds;
    return GMRF_OK;
}

template <typename Real, int ST, bool B0, int K>
void launch_lattice_group(const gmrf_batch *b, int hyper, int rel, int fold, hipStream_t s)
{
    const int w = (ST == 8 ? 1 : 0) + (B0 ? 2 : 0) + 4 * K;
    using Cfg = LatticeCfg<ST, K>;
    if (b->lat_tile_count[w] > 0)
        hipLaunchKernelGGL((lattice_batch_kernel<Real, Cfg, B0>), dim3(b->lat_tile_count[w]),
                           dim3(Cfg::NT), 0, s,
                           static_cast<const LatJob<Real> *>(b->lat_jobs[w]), b->lat_tiles[w],
                           hyper, rel, fold);
}

template <typename Real, bool B0>
void launch_csr_group(const gmrf_batch *b, size_t col, int hyper, hipStream_t s)
{
    const int g = B0 ? 1 : 0;
    if (col + 1 >= b->csr_color_off[g].size())
        return;
    const int nb = b->csr_color_off[g][col + 1] - b->csr_color_off[g][col];
    if (nb > 0)
        hipLaunchKernelGGL((csr_batch_kernel<Real, B0>), dim3(nb), dim3(kThreads), 0, s,
                           static_cast<const CsrJob<Real> *>(b->csr_jobs[g]),
                           b->csr_blocks[g] + b->csr_color_off[g][col], hyper);
}

// rel, fold: as for lattice_sweep_block (relative sweep of the call; end the
// previous one first).
template <typename Real>
void launch_batch_lattice_kernels(const gmrf_batch *b, int hyper, int rel, int fold,
                                  hipStream_t s)
{
    launch_lattice_group<Real, 4, false, 0>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 8, false, 0>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 4, true, 0>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 8, true, 0>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 4, false, 1>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 8, false, 1>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 4, true, 1>(b, hyper, rel, fold, s);
    launch_lattice_group<Real, 8, true, 1>(b, hyper, rel, fold, s);
}

template <typename Real, bool B0>
void launch_fused_group(const gmrf_batch *b, int hyper, int rel, int fold, hipStream_t s)
{
    const int g = B0 ? 1 : 0;
    if (b->fused_count[g] > 0)
        hipLaunchKernelGGL((csr_fused_batch_kernel<Real, B0>), dim3(b->fused_count[g]),
                           dim3(kThreads), (size_t)b->fused_lds, s,
                           static_cast<const FusedJob<Real> *>(b->fused_jobs[g]),
                           b->fused_blocks[g], hyper, rel, fold);
    // the chains whose every sweep ends in the per-sweep commit: each sweep
    // runs from the committed state (relative sweep 0, nothing to end)
    if (b->fused_count[2 + g] > 0)
        hipLaunchKernelGGL((csr_fused_batch_kernel<Real, B0>), dim3(b->fused_count[2 + g]),
                           dim3(kThreads), (size_t)b->fused_lds, s,
                           static_cast<const FusedJob<Real> *>(b->fused_jobs[2 + g]),
                           b->fused_blocks[2 + g], hyper, 0, 0);
}

template <typename Real>
void launch_batch_sweep_kernels(const gmrf_batch *b, int hyper, int rel, int fold, hipStream_t s)
{
    launch_batch_lattice_kernels<Real>(b, hyper, rel, fold, s);
    launch_fused_group<Real, false>(b, hyper, rel, fold, s);
    launch_fused_group<Real, true>(b, hyper, rel, fold, s);
    // color c of every general-graph chain before color c + 1 of any
    const size_t ncol = std::max(b->csr_color_off[0].size(), b->csr_color_off[1].size());
    for (size_t col = 0; col + 1 < ncol; ++col) {
        launch_csr_group<Real, false>(b, col, hyper, s);
        launch_csr_group<Real, true>(b, col, hyper, s);
    }
}

// nsweeps sweeps of every chain of a batch: the shared launches of each
// sweep (the last launch covering a chain ends that chain's sweep), and with
// hyperparameter draws, ahead of every kUnitBatch sweeps, one launch that
// draws the unit variates of every chain.
void launch_batch_sweeps(const gmrf_batch *b, int nsweeps, unsigned flags, hipStream_t s)
{
    const int hyper = (flags & GMRF_WITH_HYPER) ? 1 : 0;
    for (int i = 0; i < nsweeps; ++i) {
        if (hyper && i % kUnitBatch == 0)
            hipLaunchKernelGGL(unit_draw_batch_kernel, dim3((unsigned)b->chains.size()),
                               dim3(kUnitThreads), 0, s, b->unit_args, i,
                               std::min(kUnitBatch, nsweeps - i));
        if (b->prec == GMRF_FP64)
            launch_batch_sweep_kernels<double>(b, hyper, i, i > 0 ? 1 : 0, s);
        else
            launch_batch_sweep_kernels<float>(b, hyper, i, i > 0 ? 1 : 0, s);
        if (b->n_csr > 0)       // general graphs: every sweep ends in its own commit
            hipLaunchKernelGGL(commit_batch_kernel, dim3((unsigned)b->n_csr),
                               dim3(kFinishThreads), 0, s, b->csr_commit, 0, 1, hyper);
    }
    if (b->n_lat > 0 && nsweeps > 0)   // one-launch chains: the call's last sweep
        hipLaunchKernelGGL(commit_batch_kernel, dim3((unsigned)b->n_lat), dim3(kFinishThreads), 0,
                           s, b->lat_commit, nsweeps - 1, nsweeps, hyper);
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current (every device holds its own copy at its
// own address; in host code the array's name is only a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

int scratch_address(unsigned char **out)
{
    int dev = -1;
    GMRF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(GMRF_E_DEVICE, "sweep_static: device index " + std::to_string(dev) +
                                       " beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        GMRF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch[dev];
    return GMRF_OK;
}

// Destroy the cached captured sweeps of a chain.
void drop_graphs(gmrf_chain *c)
{
    for (auto &kv : c->graphs)
        (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t gdef : c->graph_defs)
        (void)hipGraphDestroy(gdef);
    c->graphs.clear();
    c->graph_defs.clear();
}

// The autotuner for a Gaussian chain on a general graph: times `reps`
// whole sweeps of every shape that fits (0 color passes, 1 chunked one
// launch, 2 one block) in dry mode, on a copy of the field in the chain's
// other state buffer where a shape updates the field in place, so the
// chain's state, accumulators and sweep count are unchanged.
template <typename Real>
int csr_autotune(gmrf_chain *c, int32_t reps, hipStream_t stream, double *t, int *win)
{
    const HostGraph &h = c->g->h;
    const int keep = c->lat_tile;
    const int cur = keep == kFused ? (int)(c->host_sweeps & 1u) : 0;   // buffer holding x
    const size_t bytes = real_size(c->prec) * (size_t)h.n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GMRF_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    *win = keep;
    for (int k = 0; k < GMRF_NUM_TILES && he == hipSuccess; ++k) {
        t[k] = 0.0;
        const bool fits = k == 0 || (k == kFused && csr_fused_fits(h, c->prec, false)) ||
                          (k == kPersistent && csr_persist_fits(h, c->prec));
        if (!fits)
            continue;
        c->lat_tile = k;
        c->total_slots = csr_slots(c, k);
        const SweepArgs a = dry_args(make_args(c, GMRF_WITH_HYPER), c);
        CsrArgs<Real> ca = csr_args<Real>(c);
        ca.x = static_cast<Real *>(c->d_x[1 - cur]);          // the in-place shapes' copy
        // the chunked sweep reads buffer (sweep & 1): make that the current one
        const FusedArgs<Real> fa = fused_args<Real>(c, (int)(c->host_sweeps & 1u) != cur);
        auto one = [&](hipStream_t s) {
            if (k == kFused) {
                launch_fused<Real>(c, fa, a, s, nullptr, nullptr, 0, 0);
            } else if (k == kPersistent) {
                const SlabTable sl = slab_table(h);
                auto kern = c->model.intercept ? csr_persistent_kernel<Real, true, false>
                                               : csr_persistent_kernel<Real, false, false>;
                hipLaunchKernelGGL(kern, dim3(1), dim3(kCsrPersistThreads), 0, s, ca, a, sl, 1);
            } else {
                int slot = 0;
                for (int32_t col = 0; col < h.k; ++col) {
                    const int nb = c->pass_blocks[col];
                    if (nb == 0)
                        continue;
                    const int lo = h.slab_offsets[col], cnt = h.slab_offsets[col + 1] - lo;
                    auto kern = c->model.intercept ? csr_pass_kernel<Real, true>
                                                   : csr_pass_kernel<Real, false>;
                    hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), 0, s, ca, a, lo, cnt, slot);
                    slot += nb;
                }
            }
        };
        if (k != kFused)
            he = hipMemcpyAsync(ca.x, c->d_x[cur], bytes, hipMemcpyDeviceToDevice, stream);
        for (int i = 0; i < 2 && he == hipSuccess; ++i)
            one(stream);
        if (he == hipSuccess)
            he = hipEventRecord(e0, stream);
        for (int i = 0; i < reps && he == hipSuccess; ++i)
            one(stream);
        if (he == hipSuccess)
            he = hipEventRecord(e1, stream);
        if (he == hipSuccess)
            he = hipGetLastError();
        if (he == hipSuccess)
            he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess)
            he = hipEventElapsedTime(&ms, e0, e1);
        t[k] = 1e3 * (double)ms / reps;
        if (he == hipSuccess && (k == 0 || t[k] < t[*win]))
            *win = k;
    }
    (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    c->lat_tile = keep;
    c->total_slots = csr_slots(c, keep);
    if (he != hipSuccess)
        return fail(GMRF_E_DEVICE, std::string("chain_autotune: ") + hipGetErrorString(he));
    return GMRF_OK;
}

} // namespace

extern "C" {

const char *gmrf_last_error(void) { return error_cstr(); }

int gmrf_version(void) { return 10000; }

size_t gmrf_graph_footprint(const gmrf_graph_desc *d)
{
    clear_error();
    if (!d) {
        set_error("graph_footprint: NULL description");
        return 0;
    }
    if (d->lat_stencil != 0)
        return 0;
    if (d->n < 1 || !d->row_ptr) {
        set_error("graph_footprint: n >= 1 and row_ptr are required");
        return 0;
    }
    // the chunk tables' size depends on the graph: build its host form
    HostGraph h;
    if (build_host_graph(d, &h) != GMRF_OK)
        return 0;
    return graph_device_bytes(h);
}

int gmrf_graph_create(const gmrf_graph_desc *d, void *d_ws, size_t ws_bytes, hipStream_t stream,
                      gmrf_graph **out)
{
    clear_error();
    if (!out)
        return fail(GMRF_E_INVALID_ARG, "graph_create: out is NULL");
    *out = nullptr;
    gmrf_graph *g = new gmrf_graph();
    int rc = build_host_graph(d, &g->h);
    if (rc != GMRF_OK) {
        delete g;
        return rc;
    }
    if (!is_lattice(g)) {
        const size_t need = graph_device_bytes(g->h);
        if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0) {
            delete g;
            return fail(GMRF_E_WORKSPACE, "graph_create: workspace NULL, misaligned or smaller "
                                          "than gmrf_graph_footprint (" +
                                              std::to_string(need) + " bytes)");
        }
        char *b = static_cast<char *>(d_ws);
        g->d_row_ptr = reinterpret_cast<int *>(b);
        b += align_up(sizeof(int) * (size_t)(g->h.n + 1));
        g->d_col = reinterpret_cast<int *>(b);
        b += align_up(sizeof(int) * (size_t)std::max<int64_t>(g->h.nnz, 1));
        g->d_orig = reinterpret_cast<int *>(b);
        b += align_up(sizeof(int) * (size_t)g->h.n);
        std::vector<std::pair<void *, std::pair<const void *, size_t>>> chunk_up;
        if (g->h.chunks_ok) {
            auto place = [&](auto *&dptr, const auto &vec) {
                using T = typename std::decay_t<decltype(vec)>::value_type;
                dptr = reinterpret_cast<std::remove_reference_t<decltype(dptr)>>(b);
                b += align_up(sizeof(T) * std::max<size_t>(vec.size(), 1));
                if (!vec.empty())
                    chunk_up.push_back({(void *)dptr, {vec.data(), sizeof(T) * vec.size()}});
            };
            place(g->d_ch_loc, g->h.ch_loc);
            place(g->d_ch_row, g->h.ch_row);
            place(g->d_ch_adj, g->h.ch_adj);
            place(g->d_ch_meta, g->h.ch_meta);
            place(g->d_loc_site, g->h.loc_site);
            place(g->d_loc_id, g->h.loc_id);
            place(g->d_loc_row, g->h.loc_row);
            place(g->d_loc_adj, g->h.loc_adj);
        }
        static const int kNoNeighbour = 0;   // the column entry of a graph without edges
        hipError_t e = hipMemcpyAsync(g->d_row_ptr, g->h.row_ptr.data(),
                                      sizeof(int) * (g->h.n + 1), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = g->h.nnz > 0 ? hipMemcpyAsync(g->d_col, g->h.col.data(), sizeof(int) * g->h.nnz,
                                              hipMemcpyHostToDevice, stream)
                             : hipMemcpyAsync(g->d_col, &kNoNeighbour, sizeof(int),
                                              hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->d_orig, g->h.orig_of_slab.data(), sizeof(int) * g->h.n,
                               hipMemcpyHostToDevice, stream);
        for (const auto &u : chunk_up)
            if (e == hipSuccess)
                e = hipMemcpyAsync(u.first, u.second.first, u.second.second,
                                   hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            delete g;
            return fail(GMRF_E_DEVICE, std::string("graph_create: upload: ") + hipGetErrorString(e));
        }
    }
    *out = g;
    return GMRF_OK;
}

int gmrf_graph_destroy(gmrf_graph *g)
{
    delete g;
    return GMRF_OK;
}

int gmrf_graph_info(const gmrf_graph *g, int64_t *n, int32_t *k, int64_t *components,
                    int64_t *nnz)
{
    if (!g)
        return fail(GMRF_E_INVALID_ARG, "graph_info: NULL graph");
    if (n) *n = g->h.n;
    if (k) *k = g->h.k;
    if (components) *components = g->h.components;
    if (nnz) *nnz = g->h.nnz;
    return GMRF_OK;
}

int gmrf_greedy_coloring(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                         int32_t *color_out, int32_t *k_out)
{
    clear_error();
    return greedy_coloring_host(n, row_ptr, col_idx, color_out, k_out);
}

size_t gmrf_chain_footprint(const gmrf_graph *g, gmrf_precision p)
{
    if (!g || (p != GMRF_FP64 && p != GMRF_FP32_ACC64)) {
        set_error("chain_footprint: NULL graph or bad precision");
        return 0;
    }
    return chain_layout(g, p, nullptr, nullptr, false);
}

// Number of PG term chunks of a binomial chain (trials in original order).
// Most PG term chunks of one chain: chunk indices, and the grid of one thread
// per chunk rounded up to whole blocks, stay within int.
constexpr int64_t kMaxChunks = INT32_MAX - kThreads;

static int64_t count_chunks(const gmrf_graph *g, const int32_t *trials)
{
    int64_t nc = 0;
    for (int64_t i = 0; i < g->h.n; ++i)
        nc += (std::max(trials[i], 0) + kPgChunk - 1) / kPgChunk;
    return nc;
}

size_t gmrf_binomial_footprint(const gmrf_graph *g, gmrf_precision p, const int32_t *trials)
{
    clear_error();
    if (!g || (p != GMRF_FP64 && p != GMRF_FP32_ACC64) || is_lattice(g) || !trials) {
        set_error("binomial_footprint: NULL or lattice graph, bad precision or NULL trials");
        return 0;
    }
    const int64_t nc = count_chunks(g, trials);
    if (nc > kMaxChunks) {
        set_error("binomial_footprint: too many trials in total");
        return 0;
    }
    return chain_layout(g, p, nullptr, nullptr, true, nc);
}

// Common body of the two chain constructors.  binomial: y holds the
// successes Y_i and trials the m_i.
static int chain_create_impl(const char *who, const gmrf_graph *g, const gmrf_model *m,
                             const double *y, const int32_t *trials, const double *x0,
                             gmrf_precision p, uint64_t seed, uint32_t instance, void *d_ws,
                             size_t ws_bytes, hipStream_t stream, gmrf_chain **out)
{
    const std::string w = who;
    if (!out)
        return fail(GMRF_E_INVALID_ARG, w + ": out is NULL");
    *out = nullptr;
    const bool binomial = trials != nullptr;
    if (!g || !m || !y)
        return fail(GMRF_E_INVALID_ARG, w + ": graph, model and y are required");
    if (p != GMRF_FP64 && p != GMRF_FP32_ACC64)
        return fail(GMRF_E_INVALID_ARG, w + ": bad precision");
    if (binomial && is_lattice(g))
        return fail(GMRF_E_INVALID_ARG, w + ": the binomial model needs a general (CSR) graph");
    const int64_t n = g->h.n;
    // rank of D - rho W (Sec. 2.1, Sec. 3.2): one null direction per connected
    // component for rho = 1; for rho < 1 the rows of isolated sites are zero
    // and every other row block is nonsingular
    const int64_t rank = g->h.rho == 1.0 ? n - g->h.components : n - g->h.isolated;
    const double shape_tau = m->a_tau + 0.5 * (double)rank, shape_lam = m->a_lam + 0.5 * (double)n;
    if (!(m->b_tau > 0.0) || !(shape_tau >= 1.0) || !std::isfinite(m->a_tau) ||
        !std::isfinite(m->b_tau) ||
        (!binomial && (!(m->b_lam > 0.0) || !(shape_lam >= 1.0) || !std::isfinite(m->a_lam) ||
                       !std::isfinite(m->b_lam))))
        return fail(GMRF_E_INVALID_ARG, w + ": priors need rates > 0 and conditional shapes "
                                            "a_tau + r/2 >= 1 (Gaussian: a_lam + n/2 >= 1)");
    if (!(m->tau0 > 0.0) || !(m->lam0 > 0.0) || !std::isfinite(m->tau0) ||
        !std::isfinite(m->lam0))
        return fail(GMRF_E_INVALID_ARG, w + ": tau0 and lam0 must be finite and > 0");
    if (m->burn_in < 0)
        return fail(GMRF_E_INVALID_ARG, w + ": burn_in must be >= 0");
    if ((m->intercept != 0 && m->intercept != 1) || !std::isfinite(m->beta0) ||
        (m->intercept == 0 && m->beta0 != 0.0))
        return fail(GMRF_E_INVALID_ARG, w + ": intercept must be 0 or 1 and beta0 finite (and 0 "
                                            "without an intercept)");
    if (m->likelihood != (binomial ? GMRF_BINOMIAL : GMRF_GAUSSIAN))
        return fail(GMRF_E_INVALID_ARG, w + ": model likelihood does not match the constructor");
    if (!binomial && m->beta0_var != 0.0)
        return fail(GMRF_E_INVALID_ARG, w + ": beta0_var applies to the binomial model only");
    if (binomial && (!(m->beta0_var >= 0.0) || !std::isfinite(m->beta0_var)))
        return fail(GMRF_E_INVALID_ARG, w + ": beta0_var must be finite and >= 0");
    if (m->rng_version < 0 || m->rng_version > 2)
        return fail(GMRF_E_INVALID_ARG, w + ": rng_version must be 0, 1 or 2");
    if (m->rng_version == 2 && (!is_lattice(g) || g->h.cols % 4 != 0))
        return fail(GMRF_E_INVALID_ARG, w + ": rng_version 2 needs a lattice whose width is a "
                                            "multiple of 4");
    if (!finite_array(y, n) || (x0 && !finite_array(x0, n)))
        return fail(GMRF_E_INVALID_ARG, w + ": y and x0 must be finite");
    std::vector<double> kappa;
    if (binomial) {
        int64_t total = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t mi = trials[i];
            const int32_t sp = g->h.slab_of_orig[i];
            const int64_t deg = g->h.row_ptr[sp + 1] - g->h.row_ptr[sp];
            if (mi < 0 || mi >= (1 << 21) || y[i] < 0.0 || y[i] > (double)mi ||
                y[i] != std::floor(y[i]))
                return fail(GMRF_E_INVALID_ARG, w + ": site " + std::to_string(i) +
                                                    ": need 0 <= Y_i <= m_i < 2^21, Y_i integer");
            if (mi == 0 && deg == 0)
                return fail(GMRF_E_INVALID_ARG, w + ": site " + std::to_string(i) +
                                                    " has no neighbours and no trials");
            total += mi;
        }
        if (m->intercept && m->beta0_var == 0.0 && total == 0)
            return fail(GMRF_E_INVALID_ARG, w + ": a flat beta0 prior needs some trials");
        kappa.resize(n);
        for (int64_t i = 0; i < n; ++i)
            kappa[i] = y[i] - 0.5 * (double)trials[i];
    }
    const int64_t n_chunks = binomial ? count_chunks(g, trials) : 0;
    if (n_chunks > kMaxChunks)
        return fail(GMRF_E_INVALID_ARG, w + ": too many trials in total");
    const size_t need = chain_layout(g, p, nullptr, nullptr, binomial, n_chunks);
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
        return fail(GMRF_E_WORKSPACE, w + ": workspace NULL, misaligned or smaller than the "
                                          "footprint (" + std::to_string(need) + " bytes)");
    gmrf_chain *c = new gmrf_chain();
    c->g = g;
    c->prec = p;
    c->model = *m;
    c->seed = seed;
    c->instance = instance;
    c->rank = rank;
    c->binomial = binomial;
    c->lat_tile = is_lattice(g) ? default_tile(g->h) : csr_default_shape(g->h, p, binomial);
    chain_layout(g, p, static_cast<char *>(d_ws), c, binomial, n_chunks);

    auto cleanup = [&](int rc) {
        delete c;
        return rc;
    };
    DevState st{};
    st.tau = m->tau0;
    st.lam = m->lam0;
    st.beta0 = m->beta0;
    st.unit_base = 1ull << 63;   // the ring holds no sweep's variates yet
    hipError_t e = hipMemcpyAsync(c->d_state, &st, sizeof st, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->d_s1, 0, 8 * n, stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->d_s2, 0, 8 * n, stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->d_partials, 0,
                           8 * kPartials *
                               (size_t)std::max(is_lattice(g) ? max_lattice_blocks(g->h)
                                                              : c->total_slots,
                                                1),
                           stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return cleanup(fail(GMRF_E_DEVICE, w + ": " + hipGetErrorString(e)));
    int rc = upload_real(c, c->d_y, binomial ? kappa.data() : y, stream);
    if (rc == GMRF_OK && binomial)
        rc = upload_trials_layout(c, trials, stream);
    if (rc != GMRF_OK)
        return cleanup(rc);
    std::vector<double> zeros;
    if (!x0) {
        zeros.assign(n, 0.0);
        x0 = zeros.data();
    }
    rc = upload_real(c, c->d_x[0], x0, stream);
    if (rc != GMRF_OK)
        return cleanup(rc);
    *out = c;
    return GMRF_OK;
}

int gmrf_chain_create(const gmrf_graph *g, const gmrf_model *m, const double *y, const double *x0,
                      gmrf_precision p, uint64_t seed, uint32_t instance, void *d_ws,
                      size_t ws_bytes, hipStream_t stream, gmrf_chain **out)
{
    clear_error();
    return chain_create_impl("chain_create", g, m, y, nullptr, x0, p, seed, instance, d_ws,
                             ws_bytes, stream, out);
}

int gmrf_chain_create_binomial(const gmrf_graph *g, const gmrf_model *m, const double *successes,
                               const int32_t *trials, const double *x0, gmrf_precision p,
                               uint64_t seed, uint32_t instance, void *d_ws, size_t ws_bytes,
                               hipStream_t stream, gmrf_chain **out)
{
    clear_error();
    if (!trials) {
        if (out)
            *out = nullptr;
        return fail(GMRF_E_INVALID_ARG, "chain_create_binomial: trials are required");
    }
    return chain_create_impl("chain_create_binomial", g, m, successes, trials, x0, p, seed,
                             instance, d_ws, ws_bytes, stream, out);
}

int gmrf_chain_destroy(gmrf_chain *c)
{
    if (!c)
        return GMRF_OK;
    drop_graphs(c);
    if (c->capture_stream)
        (void)hipStreamDestroy(c->capture_stream);
    delete c;
    return GMRF_OK;
}

int gmrf_sweep(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream)
{
    clear_error();
    if (!c || nsweeps < 0 || (flags & ~(GMRF_WITH_HYPER | GMRF_CAPTURE)))
        return fail(GMRF_E_INVALID_ARG, "sweep: NULL chain, negative count or unknown flag");
    if (nsweeps == 0)
        return GMRF_OK;
    const SweepArgs a = make_args(c, flags);
    if (flags & GMRF_CAPTURE) {
        const auto key = std::make_pair((int)nsweeps, flags & GMRF_WITH_HYPER);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            if (!c->capture_stream)
                GMRF_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            GMRF_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
            if (is_persistent(c))
                launch_persistent(c, a, nsweeps, c->capture_stream);
            else
                launch_sweeps(c, a, nsweeps, c->capture_stream);
            hipGraph_t gdef = nullptr;
            const hipError_t le = hipGetLastError();
            GMRF_HIP(hipStreamEndCapture(c->capture_stream, &gdef));
            if (le != hipSuccess) {
                (void)hipGraphDestroy(gdef);
                return fail(GMRF_E_DEVICE, std::string("sweep: capture: ") + hipGetErrorString(le));
            }
            hipGraphExec_t exec = nullptr;
            GMRF_HIP(hipGraphInstantiate(&exec, gdef, nullptr, nullptr, 0));
            c->graph_defs.push_back(gdef);
            it = c->graphs.emplace(key, exec).first;
        }
        GMRF_HIP(hipGraphLaunch(it->second, stream));
    } else if (is_persistent(c)) {
        launch_persistent(c, a, nsweeps, stream);
        GMRF_HIP(hipGetLastError());
    } else {
        launch_sweeps(c, a, nsweeps, stream);
        GMRF_HIP(hipGetLastError());
    }
    c->host_sweeps += (uint64_t)nsweeps;
    return GMRF_OK;
}

int gmrf_sweep_static(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream)
{
    clear_error();
    if (!c || nsweeps < 0 || (flags & ~GMRF_WITH_HYPER))
        return fail(GMRF_E_INVALID_ARG, "sweep_static: NULL chain, negative count or a flag "
                                        "other than GMRF_WITH_HYPER");
    if (c->binomial)
        return fail(GMRF_E_INVALID_ARG, "sweep_static: binomial chains keep their Polya-Gamma "
                                        "scratch in the chain workspace; use gmrf_sweep");
    if (c->total_slots > kStaticSlots)
        return fail(GMRF_E_INVALID_ARG,
                    "sweep_static: the chain needs " + std::to_string(c->total_slots) +
                        " partial slots per sweep, more than the static scratch's " +
                        std::to_string(kStaticSlots) + " (use gmrf_sweep)");
    if (nsweeps == 0)
        return GMRF_OK;
    unsigned char *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != GMRF_OK)
        return rc;
    SweepArgs a = make_args(c, flags);
    a.partials = reinterpret_cast<double *>(base);
    a.slot_stride = kStaticSlots;
    a.units = reinterpret_cast<UnitDraws *>(base + kStaticPartialBytes);
    if (is_persistent(c))
        launch_persistent(c, a, nsweeps, stream);
    else
        launch_sweeps(c, a, nsweeps, stream);
    GMRF_HIP(hipGetLastError());
    c->host_sweeps += (uint64_t)nsweeps;
    return GMRF_OK;
}

int gmrf_sweep_timed(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream,
                     double *kernel_ms, double *span_ms)
{
    clear_error();
    if (!c || nsweeps < 0 || !kernel_ms || (flags & ~GMRF_WITH_HYPER))
        return fail(GMRF_E_INVALID_ARG, "sweep_timed: NULL chain / output, negative count or "
                                        "unsupported flag");
    *kernel_ms = 0.0;
    if (span_ms)
        *span_ms = 0.0;
    const SweepArgs a = make_args(c, flags);
    // events are created before the first launch, so the span covers only
    // device work: first sweep kernel's start to the end of the last commit
    std::vector<hipEvent_t> ev(2 * (size_t)nsweeps + 1, nullptr);
    int rc = GMRF_OK;
    for (auto &e : ev) {
        const hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) {
            rc = fail(GMRF_E_DEVICE, std::string("sweep_timed: ") + hipGetErrorString(he));
            break;
        }
    }
    if (rc == GMRF_OK && nsweeps > 0 && is_persistent(c)) {
        // one launch carries every sweep (and its draws): its duration is both
        hipError_t he = hipSuccess;
        launch_persistent(c, a, nsweeps, stream, ev[0], ev[1]);
        he = hipGetLastError();
        if (he == hipSuccess)
            he = hipStreamSynchronize(stream);
        float ms = 0.0f;
        if (he == hipSuccess)
            he = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (he != hipSuccess) {
            rc = fail(GMRF_E_DEVICE, std::string("sweep_timed: ") + hipGetErrorString(he));
        } else {
            *kernel_ms = ms;
            if (span_ms)
                *span_ms = ms;
        }
        c->host_sweeps += (uint64_t)nsweeps;
    } else if (rc == GMRF_OK && nsweeps > 0) {
        hipError_t he = hipSuccess;
        for (int i = 0; i < nsweeps && he == hipSuccess; ++i) {
            launch_units_ahead(c, a, i, nsweeps, stream);
            launch_sweep_kernels(c, a, stream, i, ev[2 * i], ev[2 * i + 1]);
            launch_commit_after(c, a, i, nsweeps, stream);
            he = hipGetLastError();
        }
        if (he == hipSuccess)
            he = hipEventRecord(ev[2 * (size_t)nsweeps], stream);
        if (he == hipSuccess)
            he = hipStreamSynchronize(stream);
        double total = 0.0;
        for (int i = 0; i < nsweeps && he == hipSuccess; ++i) {
            float ms = 0.0f;
            he = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            total += ms;
        }
        float span = 0.0f;
        if (he == hipSuccess)
            he = hipEventElapsedTime(&span, ev[0], ev[2 * (size_t)nsweeps]);
        if (he != hipSuccess) {
            rc = fail(GMRF_E_DEVICE, std::string("sweep_timed: ") + hipGetErrorString(he));
        } else {
            *kernel_ms = total;
            if (span_ms)
                *span_ms = span;
        }
        c->host_sweeps += (uint64_t)nsweeps;
    }
    for (auto &e : ev)
        if (e)
            (void)hipEventDestroy(e);
    return rc;
}

int gmrf_hyper_update(gmrf_chain *c, hipStream_t stream)
{
    clear_error();
    if (!c)
        return fail(GMRF_E_INVALID_ARG, "hyper_update: NULL chain");
    if (c->host_sweeps == 0)
        return fail(GMRF_E_INVALID_ARG, "hyper_update: no completed sweep");
    const SweepArgs a = make_args(c, GMRF_WITH_HYPER);
    hipLaunchKernelGGL(hyper_kernel, dim3(1), dim3(64), 0, stream, a);
    GMRF_HIP(hipGetLastError());
    return GMRF_OK;
}

int gmrf_set_hyper(gmrf_chain *c, double tau, double lam, hipStream_t stream)
{
    clear_error();
    if (!c || !(tau > 0.0) || !(lam > 0.0) || !std::isfinite(tau) || !std::isfinite(lam))
        return fail(GMRF_E_INVALID_ARG, "set_hyper: NULL chain or tau / lam not finite and > 0");
    hipLaunchKernelGGL(set_hyper_kernel, dim3(1), dim3(1), 0, stream, c->d_state, tau, lam);
    GMRF_HIP(hipGetLastError());
    return GMRF_OK;
}

int gmrf_posterior_stats(gmrf_chain *c, double *mean, double *var, int64_t *n_acc, uint32_t flags,
                         hipStream_t stream)
{
    clear_error();
    if (!c || !mean || !var || (flags != GMRF_PTR_HOST && flags != GMRF_PTR_DEVICE) ||
        (flags == GMRF_PTR_DEVICE && n_acc))
        return fail(GMRF_E_INVALID_ARG, "posterior_stats: bad arguments");
    const int64_t n = c->g->h.n;
    double *dm = flags == GMRF_PTR_DEVICE ? mean : c->d_stats;
    double *dv = flags == GMRF_PTR_DEVICE ? var : c->d_stats + n;
    const int blocks = elementwise_blocks(n);
    const int *orig = is_lattice(c->g) ? nullptr : c->g->d_orig;
    DevState st;
    if (flags == GMRF_PTR_HOST) {      // the host form checks N first
        int rc = read_state(c, &st, stream);
        if (rc == GMRF_OK)
            rc = check_status(st);
        if (rc != GMRF_OK)
            return rc;
        if (st.n_acc < 2)
            return fail(GMRF_E_INVALID_ARG, "posterior_stats: " + std::to_string(st.n_acc) +
                                                " accumulated sweeps; the variance needs 2");
    }
    hipLaunchKernelGGL(stats_kernel, dim3(blocks), dim3(kThreads), 0, stream, c->d_s1, c->d_s2,
                       orig, (long long)n, c->d_state, dm, dv);
    GMRF_HIP(hipGetLastError());
    if (flags == GMRF_PTR_DEVICE)
        return GMRF_OK;
    GMRF_HIP(hipMemcpyAsync(mean, dm, 8 * n, hipMemcpyDeviceToHost, stream));
    GMRF_HIP(hipMemcpyAsync(var, dv, 8 * n, hipMemcpyDeviceToHost, stream));
    GMRF_HIP(hipStreamSynchronize(stream));
    if (n_acc)
        *n_acc = st.n_acc;
    return check_status(st);
}

int gmrf_get_state(gmrf_chain *c, double *x, double *tau, double *lam, uint64_t *sweep,
                   hipStream_t stream)
{
    clear_error();
    if (!c)
        return fail(GMRF_E_INVALID_ARG, "get_state: NULL chain");
    DevState st;
    int rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    if (x) {
        const int64_t n = c->g->h.n;
        std::vector<char> buf(real_size(c->prec) * n);
        GMRF_HIP(hipMemcpyAsync(buf.data(), current_x(c, st.sweep), buf.size(),
                                hipMemcpyDeviceToHost, stream));
        GMRF_HIP(hipStreamSynchronize(stream));
        if (c->prec == GMRF_FP64)
            from_layout<double>(c, buf, x);
        else
            from_layout<float>(c, buf, x);
    }
    if (tau) *tau = st.tau;
    if (lam) *lam = st.lam;
    if (sweep) *sweep = st.sweep;
    return check_status(st);
}

int gmrf_set_state(gmrf_chain *c, const double *x, double tau, double lam, uint64_t sweep,
                   hipStream_t stream)
{
    clear_error();
    if (!c || !(tau > 0.0) || !(lam > 0.0) || !std::isfinite(tau) || !std::isfinite(lam) ||
        sweep > 0xFFFFFFFFull)
        return fail(GMRF_E_INVALID_ARG, "set_state: NULL chain, bad tau / lam or sweep >= 2^32");
    if (x && !finite_array(x, c->g->h.n))
        return fail(GMRF_E_INVALID_ARG, "set_state: x must be finite");
    DevState st;
    int rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    if (x) {
        rc = upload_real(c, current_x(c, sweep), x, stream);
        if (rc != GMRF_OK)
            return rc;
    } else if (is_lattice(c->g) && ((st.sweep ^ sweep) & 1u)) {
        // keep x: move it to the buffer the new sweep parity reads
        const size_t bytes = real_size(c->prec) * (size_t)c->g->h.n;
        GMRF_HIP(hipMemcpyAsync(current_x(c, sweep), current_x(c, st.sweep), bytes,
                                hipMemcpyDeviceToDevice, stream));
    }
    st.tau = tau;
    st.lam = lam;
    st.sweep = sweep;
    GMRF_HIP(hipMemcpyAsync(c->d_state, &st, sizeof st, hipMemcpyHostToDevice, stream));
    GMRF_HIP(hipStreamSynchronize(stream));
    c->host_sweeps = sweep;
    return GMRF_OK;
}

int gmrf_get_accumulators(gmrf_chain *c, double *s1, double *s2, int64_t *n_acc,
                          hipStream_t stream)
{
    clear_error();
    if (!c || !s1 || !s2)
        return fail(GMRF_E_INVALID_ARG, "get_accumulators: bad arguments");
    int rc = download_doubles_layout(c, c->d_s1, s1, stream);
    if (rc == GMRF_OK)
        rc = download_doubles_layout(c, c->d_s2, s2, stream);
    if (rc != GMRF_OK)
        return rc;
    DevState st;
    rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    if (n_acc)
        *n_acc = st.n_acc;
    return GMRF_OK;
}

int gmrf_set_accumulators(gmrf_chain *c, const double *s1, const double *s2, int64_t n_acc,
                          hipStream_t stream)
{
    clear_error();
    if (!c || !s1 || !s2 || n_acc < 0)
        return fail(GMRF_E_INVALID_ARG, "set_accumulators: bad arguments");
    int rc = upload_doubles_layout(c, c->d_s1, s1, stream);
    if (rc == GMRF_OK)
        rc = upload_doubles_layout(c, c->d_s2, s2, stream);
    if (rc != GMRF_OK)
        return rc;
    DevState st;
    rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    st.n_acc = n_acc;
    GMRF_HIP(hipMemcpyAsync(c->d_state, &st, sizeof st, hipMemcpyHostToDevice, stream));
    GMRF_HIP(hipStreamSynchronize(stream));
    return GMRF_OK;
}

int gmrf_get_intercept(gmrf_chain *c, double *beta0, hipStream_t stream)
{
    clear_error();
    if (!c || !beta0)
        return fail(GMRF_E_INVALID_ARG, "get_intercept: NULL chain or output");
    DevState st;
    int rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    *beta0 = st.beta0;
    return check_status(st);
}

int gmrf_set_intercept(gmrf_chain *c, double beta0, hipStream_t stream)
{
    clear_error();
    if (!c || !std::isfinite(beta0) || !c->model.intercept)
        return fail(GMRF_E_INVALID_ARG, "set_intercept: NULL chain, non-finite beta0 or a chain "
                                        "without an intercept");
    hipLaunchKernelGGL(set_intercept_kernel, dim3(1), dim3(1), 0, stream, c->d_state, beta0,
                       (double)c->g->h.n, c->binomial ? 1 : 0);
    GMRF_HIP(hipGetLastError());
    return GMRF_OK;
}

int gmrf_set_trace(gmrf_chain *c, double *d_trace, int64_t capacity, hipStream_t stream)
{
    clear_error();
    if (!c || capacity < 0 || (capacity > 0 && !d_trace))
        return fail(GMRF_E_INVALID_ARG, "set_trace: NULL chain, negative capacity or NULL buffer");
    DevState st;
    int rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    st.trace = capacity > 0 ? d_trace : nullptr;
    st.trace_cap = capacity > 0 ? (long long)capacity : 0;
    GMRF_HIP(hipMemcpyAsync(c->d_state, &st, sizeof st, hipMemcpyHostToDevice, stream));
    GMRF_HIP(hipStreamSynchronize(stream));
    return GMRF_OK;
}

int gmrf_chain_get_tile(const gmrf_chain *c, int32_t *tile, int32_t *tile_rows, int32_t *tile_cols,
                        int32_t *threads)
{
    clear_error();
    if (!c)
        return fail(GMRF_E_INVALID_ARG, "chain_get_tile: NULL chain");
    if (!is_lattice(c->g)) {
        if (tile) *tile = c->lat_tile;
        if (tile_rows) *tile_rows = 0;
        if (tile_cols) *tile_cols = 0;
        if (threads) *threads = c->lat_tile == kPersistent ? kCsrPersistThreads : kThreads;
        return GMRF_OK;
    }
    const TileShape &t = kTiles[c->lat_tile];
    if (tile) *tile = c->lat_tile;
    if (tile_rows) *tile_rows = t.th;
    if (tile_cols) *tile_cols = t.tw;
    if (threads) *threads = t.nt;
    return GMRF_OK;
}

int gmrf_chain_set_tile(gmrf_chain *c, int32_t tile)
{
    clear_error();
    if (!c || tile < 0 || tile >= GMRF_NUM_TILES)
        return fail(GMRF_E_INVALID_ARG, "chain_set_tile: NULL chain, or tile not in 0 .. "
                                        "GMRF_NUM_TILES - 1");
    if (!is_lattice(c->g)) {
        if ((tile == kFused && !csr_fused_fits(c->g->h, c->prec, c->binomial)) ||
            (tile == kPersistent && !csr_persist_fits(c->g->h, c->prec)))
            return fail(GMRF_E_INVALID_ARG, "chain_set_tile: a general graph takes shape 0; "
                                            "shape 1 when its chunks fit (not for the binomial "
                                            "model); shape 2 when its field fits in LDS (at most "
                                            "122880 bytes of state) and it has at most 32 colors");
        if (tile != c->lat_tile) {
            // shape 1 keeps x in buffer (sweep & 1), the others in buffer 0:
            // move it when the chain has run an odd number of sweeps
            if ((tile == kFused) != (c->lat_tile == kFused) && (c->host_sweeps & 1u)) {
                const size_t bytes = real_size(c->prec) * (size_t)c->g->h.n;
                GMRF_HIP(hipDeviceSynchronize());
                GMRF_HIP(tile == kFused
                             ? hipMemcpy(c->d_x[1], c->d_x[0], bytes, hipMemcpyDeviceToDevice)
                             : hipMemcpy(c->d_x[0], c->d_x[1], bytes, hipMemcpyDeviceToDevice));
            }
            c->lat_tile = tile;
            c->total_slots = csr_slots(c, tile);
            drop_graphs(c);
        }
        return GMRF_OK;
    }
    if (!tile_fits(c->g->h, tile))
        return fail(GMRF_E_INVALID_ARG, "chain_set_tile: shape 2 needs a lattice of at most "
                                        "64 x 64 sites");
    if (tile != c->lat_tile) {
        c->lat_tile = tile;
        c->total_slots = lattice_blocks(c->g->h, tile);
        drop_graphs(c);     // captured sweeps carry the old launch shape
    }
    return GMRF_OK;
}

int gmrf_chain_autotune(gmrf_chain *c, int32_t reps, hipStream_t stream, int32_t *best,
                        double *us_per_sweep)
{
    clear_error();
    if (!c || reps < 1 || reps > 100000 || c->binomial)
        return fail(GMRF_E_INVALID_ARG, "chain_autotune: NULL or binomial chain, or reps not "
                                        "in 1 .. 100000");
    if (!is_lattice(c->g)) {
        double t[GMRF_NUM_TILES] = {};
        int win = c->lat_tile;
        const int rc = c->prec == GMRF_FP64 ? csr_autotune<double>(c, reps, stream, t, &win)
                                            : csr_autotune<float>(c, reps, stream, t, &win);
        if (rc != GMRF_OK)
            return rc;
        if (us_per_sweep)
            for (int k = 0; k < GMRF_NUM_TILES; ++k)
                us_per_sweep[k] = t[k];
        if (best)
            *best = win;
        return gmrf_chain_set_tile(c, win);
    }
    const int keep = c->lat_tile;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GMRF_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    double t[GMRF_NUM_TILES] = {};
    int win = keep;
    for (int k = 0; k < GMRF_NUM_TILES && he == hipSuccess; ++k) {
        t[k] = 0.0;
        if (!tile_fits(c->g->h, k))
            continue;
        c->lat_tile = k;
        c->total_slots = lattice_blocks(c->g->h, k);
        // Whole sweeps (the sweep kernels, or the persistent
        // kernel) in dry mode (dry_args), so the sweep kernels write only the
        // other state buffer, the partial slots and the statistics scratch
        // and the chain is unchanged; the persistent kernel runs an odd
        // number of sweeps so that it too ends in the other state buffer.
        const SweepArgs a = dry_args(make_args(c, GMRF_WITH_HYPER), c);
        const int odd = reps | 1;
        if (k == kPersistent) {
            launch_persistent(c, a, 1, stream);
            he = hipEventRecord(e0, stream);
            if (he == hipSuccess)
                launch_persistent(c, a, odd, stream);
        } else {
            launch_sweeps(c, a, 2, stream);
            he = hipEventRecord(e0, stream);
            if (he == hipSuccess)
                launch_sweeps(c, a, reps, stream);
        }
        if (he == hipSuccess)
            he = hipEventRecord(e1, stream);
        if (he == hipSuccess)
            he = hipGetLastError();
        if (he == hipSuccess)
            he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess)
            he = hipEventElapsedTime(&ms, e0, e1);
        t[k] = 1e3 * (double)ms / (k == kPersistent ? odd : reps);
        if (he == hipSuccess && (k == 0 || t[k] < t[win]))
            win = k;
    }
    (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    c->lat_tile = keep;
    c->total_slots = lattice_blocks(c->g->h, keep);
    if (he != hipSuccess)
        return fail(GMRF_E_DEVICE, std::string("chain_autotune: ") + hipGetErrorString(he));
    if (us_per_sweep)
        for (int k = 0; k < GMRF_NUM_TILES; ++k)
            us_per_sweep[k] = t[k];
    if (best)
        *best = win;
    return gmrf_chain_set_tile(c, win);
}

int gmrf_last_reductions(gmrf_chain *c, double *q, double *sse, hipStream_t stream)
{
    clear_error();
    if (!c)
        return fail(GMRF_E_INVALID_ARG, "last_reductions: NULL chain");
    DevState st;
    int rc = read_state(c, &st, stream);
    if (rc != GMRF_OK)
        return rc;
    if (q) *q = st.q;
    if (sse) *sse = st.sse;
    return GMRF_OK;
}

size_t gmrf_batch_footprint(gmrf_chain *const *chains, int32_t count)
{
    clear_error();
    size_t bytes = 0;
    if (batch_bytes(chains, count, &bytes) != GMRF_OK)
        return 0;
    return bytes;
}

int gmrf_batch_create(gmrf_chain *const *chains, int32_t count, void *d_ws, size_t ws_bytes,
                      hipStream_t stream, gmrf_batch **out)
{
    clear_error();
    if (!out)
        return fail(GMRF_E_INVALID_ARG, "batch_create: out is NULL");
    *out = nullptr;
    BatchImage im;
    gmrf_precision prec;
    int rc = build_image(chains, count, im, &prec);
    if (rc != GMRF_OK)
        return rc;
    size_t need = 0;
    rc = batch_bytes(chains, count, &need, &im);
    if (rc != GMRF_OK)
        return rc;
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0)
        return fail(GMRF_E_WORKSPACE, "batch_create: workspace NULL, misaligned or smaller than "
                                      "gmrf_batch_footprint (" +
                                          std::to_string(need) + " bytes)");
    gmrf_batch *b = new gmrf_batch();
    b->chains.assign(chains, chains + count);
    b->prec = prec;
    b->ws = static_cast<char *>(d_ws);
    rc = install_image(b, im, stream);
    if (rc != GMRF_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return GMRF_OK;
}

int gmrf_batch_autotune(gmrf_batch *b, int32_t reps, hipStream_t stream, int32_t *best,
                        double *us_per_sweep)
{
    clear_error();
    if (!b || reps < 1 || reps > 100000)
        return fail(GMRF_E_INVALID_ARG, "batch_autotune: NULL batch or reps not in 1 .. 100000");
    if (best)
        *best = -1;
    if (us_per_sweep)
        us_per_sweep[0] = us_per_sweep[1] = 0.0;
    std::vector<gmrf_chain *> lat;
    for (gmrf_chain *c : b->chains)
        if (is_lattice(c->g))
            lat.push_back(c);
    if (lat.empty())
        return GMRF_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GMRF_HIP(hipEventCreate(&e0));
    const hipError_t ce = hipEventCreate(&e1);
    if (ce != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GMRF_E_DEVICE, std::string("batch_autotune: ") + hipGetErrorString(ce));
    }
    double us[2] = {0.0, 0.0};
    int rc = GMRF_OK;
    for (int k = 0; k < 2 && rc == GMRF_OK; ++k) {
        BatchImage im;
        gmrf_precision prec;
        rc = build_image(b->chains.data(), (int32_t)b->chains.size(), im, &prec, k, true);
        if (rc == GMRF_OK)
            rc = install_image(b, im, stream);
        if (rc != GMRF_OK)
            break;
        // one untimed pass, then reps timed passes of the lattice tiles
        hipError_t he = hipSuccess;
        for (int r = 0; r <= reps && he == hipSuccess; ++r) {
            if (r == 1)
                he = hipEventRecord(e0, stream);
            if (he == hipSuccess) {
                // dry passes repeat relative sweep 0 (see launch_sweep_kernels)
                b->prec == GMRF_FP64 ? launch_batch_lattice_kernels<double>(b, 1, 0, 0, stream)
                                     : launch_batch_lattice_kernels<float>(b, 1, 0, 0, stream);
                he = hipGetLastError();
            }
        }
        if (he == hipSuccess)
            he = hipEventRecord(e1, stream);
        if (he == hipSuccess)
            he = hipStreamSynchronize(stream);
        float ms = 0.0f;
        if (he == hipSuccess)
            he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess)
            rc = fail(GMRF_E_DEVICE, std::string("batch_autotune: ") + hipGetErrorString(he));
        us[k] = 1e3 * (double)ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == GMRF_OK) {
        const int k = us[1] < us[0] ? 1 : 0;
        for (gmrf_chain *c : lat) {
            if (c->lat_tile != k) {
                c->lat_tile = k;
                c->total_slots = lattice_blocks(c->g->h, k);
                drop_graphs(c);
            }
        }
        if (best)
            *best = k;
        if (us_per_sweep) {
            us_per_sweep[0] = us[0];
            us_per_sweep[1] = us[1];
        }
    }
    // the batch's own tables again (with the chosen shapes), and no stale graphs
    BatchImage im;
    gmrf_precision prec;
    int rc2 = build_image(b->chains.data(), (int32_t)b->chains.size(), im, &prec);
    if (rc2 == GMRF_OK)
        rc2 = install_image(b, im, stream);
    for (auto &kv : b->graphs)
        (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t gdef : b->graph_defs)
        (void)hipGraphDestroy(gdef);
    b->graphs.clear();
    b->graph_defs.clear();
    return rc != GMRF_OK ? rc : rc2;
}

int gmrf_batch_destroy(gmrf_batch *b)
{
    if (!b)
        return GMRF_OK;
    for (auto &kv : b->graphs)
        (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t gdef : b->graph_defs)
        (void)hipGraphDestroy(gdef);
    if (b->capture_stream)
        (void)hipStreamDestroy(b->capture_stream);
    delete b;
    return GMRF_OK;
}

int gmrf_batch_sweep(gmrf_batch *b, int32_t nsweeps, uint32_t flags, hipStream_t stream)
{
    clear_error();
    if (!b || nsweeps < 0 || (flags & ~(GMRF_WITH_HYPER | GMRF_CAPTURE)))
        return fail(GMRF_E_INVALID_ARG, "batch_sweep: NULL batch, negative count or unknown flag");
    if (nsweeps == 0)
        return GMRF_OK;
    if (flags & GMRF_CAPTURE) {
        const auto key = std::make_pair((int)nsweeps, flags & GMRF_WITH_HYPER);
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            if (!b->capture_stream)
                GMRF_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
            GMRF_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
            launch_batch_sweeps(b, nsweeps, flags, b->capture_stream);
            hipGraph_t gdef = nullptr;
            const hipError_t le = hipGetLastError();
            GMRF_HIP(hipStreamEndCapture(b->capture_stream, &gdef));
            if (le != hipSuccess) {
                (void)hipGraphDestroy(gdef);
                return fail(GMRF_E_DEVICE, std::string("batch_sweep: capture: ") +
                                               hipGetErrorString(le));
            }
            hipGraphExec_t exec = nullptr;
            GMRF_HIP(hipGraphInstantiate(&exec, gdef, nullptr, nullptr, 0));
            b->graph_defs.push_back(gdef);
            it = b->graphs.emplace(key, exec).first;
        }
        GMRF_HIP(hipGraphLaunch(it->second, stream));
    } else {
        launch_batch_sweeps(b, nsweeps, flags, stream);
        GMRF_HIP(hipGetLastError());
    }
    for (gmrf_chain *c : b->chains)
        c->host_sweeps += (uint64_t)nsweeps;
    return GMRF_OK;
}

} // extern "C"
