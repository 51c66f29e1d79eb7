/*
 * gmrf.h -- C ABI of libgmrf: chromatic Gibbs sampling of a Gaussian Markov
 * random field (GMRF) with a conditional autoregressive (CAR) prior on an
 * AMD Instinct MI355X (gfx950).
 *
 * Model (Brown, McMahan & Self 2017, Sec. 3.1 image model, Sec. 3.2 proper
 * CAR), written with precisions tau (prior) and lam = 1/sigma^2 (noise):
 *     y | x, lam  ~ N(beta0 1 + x, I / lam)    beta0 = 0 without an intercept
 *     x | tau     ~ N(0, (tau (D - rho W))^-)   rho = 1: intrinsic CAR (IAR)
 *     tau ~ Gamma(a_tau, rate b_tau),  lam ~ Gamma(a_lam, rate b_lam)
 * W is the 0/1 adjacency of an undirected graph (w_ij = I(i ~ j)) and
 * D = diag(row sums of W).
 *
 * One sweep (Sec. 2.3, Algorithm 1) visits the colors 0..k-1 of a proper
 * coloring in order; every site i of the current color is drawn at once from
 * its full conditional (Sec. 2.2 with A = I, Sigma = I/lam; Sec. 3.1 local
 * characteristics):
 *     Qii = tau * D_ii + lam
 *     m_i = (lam * (y_i - beta0) + tau * rho * sum_{j~i} x_j) / Qii
 *     x_i = m_i + z_{t,i} / sqrt(Qii)
 * and then, with hyperparameter updates on, the hyperparameters are redrawn
 * from their conjugate conditionals (Sec. 3.1, precisions as Gamma laws):
 *     beta0 ~ N(mean(y - x), 1 / (n lam))       (intercept only; flat prior)
 *     tau ~ Gamma(a_tau + r/2, b_tau + x'(D - rho W)x / 2),
 *     lam ~ Gamma(a_lam + n/2, b_lam + ||y - beta0 1 - x||^2 / 2)  (new beta0),
 * r = n - #connected components (intrinsic) or n (proper).  Sweeps with index
 * t >= burn_in add phi = beta0 + x and phi^2 to FP64 running sums (posterior
 * mean/variance of the image; with a flat beta0 and an intrinsic prior only
 * phi is identified).
 *
 * Binomial logit model (Sec. 3.2, general graphs, gmrf_chain_create_binomial):
 *     Y_i ~ Bin(m_i, pi_i),  logit(pi_i) = beta0 + x_i,  beta0 ~ N(0, v0)
 * made conditionally Gaussian by Polya-Gamma augmentation (Polson, Scott &
 * Windle 2013): with kappa_i = Y_i - m_i / 2, each site draws
 * psi_i ~ PG(m_i, beta0 + x_i) from its value before its color's pass (a sum
 * of m_i PG(1, .) terms, Devroye's alternating-series sampler).  Since psi_i
 * depends only on beta0 and site i's own value, which no earlier color pass
 * changes, the library draws every psi_i of a sweep before the color passes
 * (one launch for all terms, in chunks of 2, then one sum per site); then
 *     Qii = tau * D_ii + psi_i,
 *     m_i = (kappa_i - psi_i beta0 + tau * rho * sum_{j~i} x_j) / Qii,
 * and after the sweep beta0 ~ N(sum(kappa - psi x) / P, 1/P),
 * P = sum psi + 1/v0 (v0 = 0: flat), then tau as above.  The accumulators
 * collect the linear predictor beta0 + x.
 *
 * Random numbers: Philox4x32-10 keyed by the 64-bit seed with counter
 * (site id, sweep t, instance, tag); tag 0 = site normal (Box-Muller, cosine
 * branch), tags 1/2 = the tau/lam Gamma draws (Marsaglia-Tsang), tag 3 (site
 * id 0) = the beta0 normal; the PG(1, .) term j of site i draws uniform u
 * from half (u & 1) of the block at (i, t, instance, 2^31 | j << 10 | u >> 1).  Site ids are
 * the caller's ORIGINAL ids, so results do not depend on the internal layout,
 * the thread mapping or the color permutation.
 *
 * Conventions
 *   - Every function returns gmrf_status (0 = GMRF_OK).  No C++ exception
 *     crosses the ABI.  gmrf_last_error() returns a thread-local message for
 *     the last failing call on the calling thread.
 *   - Device work is asynchronous on the caller's stream; a kernel fault
 *     surfaces at the next synchronising call.  A chain must be driven from
 *     one stream at a time.
 *   - The library allocates no device memory.  Graphs and chains live in
 *     device workspaces the caller allocates (size from the footprint
 *     queries) and keeps alive until the handle is destroyed.  Workspaces
 *     must be 256-byte aligned.
 *   - "Host" arrays are read during the call and may be freed on return.
 */
#ifndef GMRF_H
#define GMRF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GMRF_OK = 0,
    GMRF_E_INVALID_ARG = 1, /* NULL pointer, bad size, bad flag, bad model value */
    GMRF_E_GRAPH = 2,       /* malformed CSR: non-monotone, out of range, self-loop,
                               duplicate or asymmetric edge, too large for int32 */
    GMRF_E_COLORING = 3,    /* improper coloring; the message names the first bad edge */
    GMRF_E_WORKSPACE = 4,   /* workspace NULL, misaligned or smaller than the footprint */
    GMRF_E_DEVICE = 5,      /* HIP runtime error (message carries hipGetErrorString) */
    GMRF_E_NUMERIC = 6      /* non-finite tau/lam or Gamma attempt cap hit on the device;
                               reported by the next synchronising call */
} gmrf_status;

typedef enum {
    GMRF_FP64 = 0,          /* FP64 state, draws, neighbour sums */
    GMRF_FP32_ACC64 = 1     /* FP32 state, y, draws and neighbour sums; FP64 posterior
                               accumulators, FP64 q/sse reductions, FP64 tau/lam */
} gmrf_precision;

/* gmrf_sweep flags */
#define GMRF_WITH_HYPER 1u  /* draw tau, lam after every sweep (normal MCMC mode) */
#define GMRF_CAPTURE 2u     /* record the nsweeps sweeps once as a HIP graph and replay it */

/* Number of compiled lattice tile shapes (gmrf_chain_set_tile). */
#define GMRF_NUM_TILES 3

/* gmrf_posterior_stats flags */
#define GMRF_PTR_HOST 0u    /* mean / var are host pointers; the call synchronises */
#define GMRF_PTR_DEVICE 1u  /* mean / var are device pointers; asynchronous */

/* Graph description.  Either a general graph (lat_stencil = 0) given as a CSR
 * adjacency plus a proper coloring, or a rows x cols pixel lattice with free
 * boundary (lat_stencil = 4: edge neighbours, checkerboard coloring
 * (r + c) mod 2, k = 2; lat_stencil = 8: edge and diagonal neighbours, 2x2
 * parity coloring 2 (r mod 2) + (c mod 2), k = 4), site id r * cols + c.
 * Lattice colorings are the ones found by inspection (Sec. 2.3, Fig. 1); for a
 * lattice, row_ptr / col_idx / color may be NULL, and if color is given it must
 * equal the parity coloring. */
typedef struct {
    int64_t n;              /* number of sites (lattice: rows * cols) */
    const int64_t *row_ptr; /* host, n + 1 offsets into col_idx (general graph) */
    const int32_t *col_idx; /* host, row_ptr[n] neighbour ids; each row ascending,
                               no self loops, no duplicates, symmetric */
    const int32_t *color;   /* host, n colors in 0 .. num_colors - 1 */
    int32_t num_colors;     /* k (lattice: 2 or 4, or 0 to imply it) */
    int32_t lat_rows, lat_cols;
    int32_t lat_stencil;    /* 0 = general graph, 4 or 8 = lattice */
    double rho;             /* 1 = intrinsic CAR; -1 < rho < 1 proper CAR */
} gmrf_graph_desc;

/* Model constants of one chain. */
typedef struct {
    double a_tau, b_tau;    /* Gamma(shape, rate) prior of the prior precision tau */
    double a_lam, b_lam;    /* Gamma(shape, rate) prior of the noise precision lam */
    double tau0, lam0;      /* initial tau, lam (> 0) */
    int64_t burn_in;        /* sweeps t < burn_in are not accumulated */
    int32_t intercept;      /* 1: the model has an intercept beta0 (Sec. 3.1: flat prior;
                               binomial: N(0, beta0_var)); 0: beta0 = 0 */
    int32_t likelihood;     /* GMRF_GAUSSIAN (gmrf_chain_create) or GMRF_BINOMIAL
                               (gmrf_chain_create_binomial) */
    double beta0;           /* initial beta0 (finite; must be 0 when intercept = 0) */
    double beta0_var;       /* binomial: prior variance of beta0, 0 = flat; Gaussian: 0 */
    int32_t rng_version;    /* random-number contract of the site normals (0 means 1):
                               1: one Philox block per site, cosine branch;
                               2: the sites of each color, ranked by original id, share
                               one block per rank pair (2m, 2m + 1): cosine branch for
                               the first, sine branch for the second (Box-Muller's two
                               independent normals; half the generator work).  Version
                               2 is taken by Gaussian lattice chains whose width is a
                               multiple of 4, swept on their own (not in a batch). */
} gmrf_model;

#define GMRF_GAUSSIAN 0
#define GMRF_BINOMIAL 1

typedef struct gmrf_graph gmrf_graph;
typedef struct gmrf_chain gmrf_chain;

/* Thread-local message of the last failing call ("" if none). */
const char *gmrf_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int gmrf_version(void);

/* ---- graphs (Sec. 2.3: coloring and the per-color site lists) ------------- */

/* Device workspace bytes that gmrf_graph_create needs for d (0 for a
 * lattice, which needs no structure on the device).  For a general graph the
 * call validates d and builds the host form of the graph (coloring slabs and
 * chunk tables, see gmrf_graph_create), so it costs about as much host time
 * as the create itself.  Returns 0 and sets the error message if d is
 * invalid. */
size_t gmrf_graph_footprint(const gmrf_graph_desc *d);

/* Validate d and build the device form of the graph: for a general graph the
 * sites are permuted so that each color is a contiguous slab (color, then the
 * chunk order below), with a permuted CSR (int32) whose neighbour lists stay
 * in ascending ORIGINAL-id order, plus the slab-to-original map.  The sites
 * are also split into chunks of at most about 640 sites (graph-Voronoi
 * cells: a capacity-bounded multi-source breadth-first growth from seeds
 * placed by recursive bisection of hop-distance coordinates), and for each
 * chunk the graph stores its closure R under lower-color neighbours, R's
 * other neighbours, and R's adjacency in chunk-local 16-bit slots: the
 * tables of the chunked sweep (launch shape 1; Sec. 2.3, a sweep as color
 * phases inside each chunk).  A graph whose chunks do not fit the kernel's
 * LDS image or 16-bit slots, or with more than 32 colors, gets no chunk
 * tables.  The permutation is internal: results are keyed by original ids.
 * The
 * arrays are uploaded to d_ws (ws_bytes >= gmrf_graph_footprint(d)) on stream
 * and the call synchronises the stream before returning.  Checks: CSR shape,
 * ranges, symmetry, no self loops / duplicates, proper coloring (Sec. 2.3: no
 * edge inside a color class), -1 < rho <= 1.  Errors: GMRF_E_INVALID_ARG,
 * GMRF_E_GRAPH, GMRF_E_COLORING, GMRF_E_WORKSPACE, GMRF_E_DEVICE. */
int gmrf_graph_create(const gmrf_graph_desc *d, void *d_ws, size_t ws_bytes, hipStream_t stream,
                      gmrf_graph **out);
int gmrf_graph_destroy(gmrf_graph *g);

/* Shape of a created graph: n, number of colors k, number of connected
 * components (sets the rank r = n - components of the intrinsic prior),
 * number of directed adjacency entries (2 |E|). */
int gmrf_graph_info(const gmrf_graph *g, int64_t *n, int32_t *k, int64_t *components,
                    int64_t *nnz);

/* Greedy coloring of the supplementary greedy algorithm (host only): color j
 * is a maximal independent set of the still-uncolored sites grown from the
 * smallest id upward; colors are 0-based in discovery order.  Equivalent to
 * first-fit in ascending id order.  color_out has n entries. */
int gmrf_greedy_coloring(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                         int32_t *color_out, int32_t *k_out);

/* ---- chains -------------------------------------------------------------- */

/* Device workspace bytes of one chain of precision p on g. */
size_t gmrf_chain_footprint(const gmrf_graph *g, gmrf_precision p);

/* Create a chain of the Gibbs sampler of Sec. 2.3 (Algorithm 1) for the
 * hierarchical model of Sec. 3.1 / 3.2: y | x ~ N(beta0 1 + x, I / lam), x a
 * CAR field with precision tau (D - rho W) (Sec. 2.1; rho = 1 the intrinsic
 * prior of Sec. 3.1, rho < 1 the proper prior of Sec. 3.2), Gamma priors on
 * tau and lam.  Upload y (host, n values in original order, FP64; stored as
 * FP32 for GMRF_FP32_ACC64) and x0 (host, original order, or NULL for zeros),
 * set tau = m->tau0, lam = m->lam0, sweep = 0, clear the accumulators.  seed
 * and instance key the chain's random numbers (by m->rng_version).
 * Synchronises the stream.  Errors: GMRF_E_INVALID_ARG (bad model or
 * precision, non-finite y or x0, rng_version other than 0, 1, 2, or 2 on a
 * general graph or a lattice whose width is not a multiple of 4),
 * GMRF_E_WORKSPACE, GMRF_E_DEVICE. */
int gmrf_chain_create(const gmrf_graph *g, const gmrf_model *m, const double *y, const double *x0,
                      gmrf_precision p, uint64_t seed, uint32_t instance, void *d_ws,
                      size_t ws_bytes, hipStream_t stream, gmrf_chain **out);
int gmrf_chain_destroy(gmrf_chain *c);

/* Device workspace bytes of one binomial chain on a general graph g with the
 * given trials (host, n values m_i, original order): the Gaussian layout plus
 * the trials, the Polya-Gamma term chunk tables and sums (about 6 bytes per
 * trial), and a per-site envelope and psi (about 40 bytes per site).
 * Returns 0 and sets the error message on bad input. */
size_t gmrf_binomial_footprint(const gmrf_graph *g, gmrf_precision p, const int32_t *trials);

/* Create a binomial logit chain (Sec. 3.2) on a general graph: successes
 * (host, n values Y_i, integers) and trials (host, n values m_i, 0 <= Y_i <=
 * m_i < 2^21; m_i = 0 marks a site without data, which then needs at least
 * one neighbour), x0 as for gmrf_chain_create, m->likelihood = GMRF_BINOMIAL,
 * m->beta0_var >= 0.  a_lam / b_lam / lam0 are not used by the sampler (lam
 * stays lam0).  Batches do not take binomial chains.  The workspace needs
 * gmrf_binomial_footprint(g, p, trials) bytes.  Synchronises.  Errors as gmrf_chain_create,
 * plus GMRF_E_INVALID_ARG for a lattice graph or invalid counts. */
int gmrf_chain_create_binomial(const gmrf_graph *g, const gmrf_model *m, const double *successes,
                               const int32_t *trials, const double *x0, gmrf_precision p,
                               uint64_t seed, uint32_t instance, void *d_ws, size_t ws_bytes,
                               hipStream_t stream, gmrf_chain **out);

/* Enqueue nsweeps sweeps (Algorithm 1 over all colors, with the fused
 * x'(D - rho W)x and ||y - beta0 1 - x||^2 reductions and the posterior
 * accumulators).  flags: GMRF_WITH_HYPER draws the hyperparameters after
 * every sweep on the device; without it they stay fixed.  GMRF_CAPTURE
 * records the nsweeps sweeps as a HIP graph the first time a (nsweeps, flags)
 * pair is seen on this chain and replays it afterwards.  No host
 * synchronisation.  Launches: a lattice sweep, and a general-graph sweep in
 * launch shape 1 (chunked), is one kernel, which first ends the previous
 * sweep of the call (sums its reductions and draws the hyperparameters, in
 * every block); a one-block commit kernel ends the call's last sweep.  A
 * general graph in shape 0 runs one kernel per color and the commit kernel
 * after every sweep; shape 2 runs the whole call in one launch.  With
 * GMRF_WITH_HYPER a small kernel
 * draws the rate-free parts of the hyperparameter draws (which depend only
 * on the sweep index) before every 128 sweeps.  Sec. 2.3, Algorithm 1; the
 * draws: Sec. 3.1 conjugate conditionals. */
int gmrf_sweep(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream);

/* gmrf_sweep for callers that cannot allocate device memory or must not have
 * the library touch more of it than the chain (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same sweeps,
 * bitwise the same results, but the kernels keep the sweep's scratch (the
 * FP64 partial sums of the blocks and the ring of unit variates drawn ahead)
 * in a fixed device array inside the library -- at most 8192 partial slots
 * per sweep, about 400 KB, one copy per device held until the process ends
 * -- instead of the chain's workspace.  The call allocates nothing.  The
 * current device must be the chain's.  Every call on a device shares that
 * device's array, so calls that overlap on one device (other streams, other
 * host threads) race and must be serialised by the caller; the array keeps
 * the last call's contents, and nothing in it needs to start at zero.
 * flags: GMRF_WITH_HYPER only (no GMRF_CAPTURE; the caller may capture the
 * launches itself).  Errors: GMRF_E_INVALID_ARG (NULL chain, bad flags, a
 * binomial chain, whose Polya-Gamma scratch lives in its workspace, or a
 * chain whose sweep needs more than 8192 partial slots: lattices up to
 * 8192 tiles of the chain's shape, general graphs up to 8192 blocks of 256
 * sites over all colors in shape 0 and up to 8192 chunks in shape 1), GMRF_E_DEVICE. */
int gmrf_sweep_static(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream);

/* Profiling form of gmrf_sweep (plain launches, no capture): the same sweeps,
 * with a pair of HIP events that the dispatches themselves record at the
 * start and the end of the sweep kernels of every sweep (the lattice kernel,
 * which includes the end of the previous sweep; on a general graph, from
 * its first launch, which for the binomial model is the first Polya-Gamma
 * kernel, to the last color pass), excluding the one-block commit kernels
 * and the unit-variate kernels.  Synchronises and returns in *kernel_ms the
 * summed event time of the sweep kernels over the nsweeps sweeps and, if
 * span_ms is not NULL, the elapsed time from the start of the first sweep
 * kernel to the end of the call's last kernel (all events are created
 * before the first launch, so host work is not in the span). */
int gmrf_sweep_timed(gmrf_chain *c, int32_t nsweeps, uint32_t flags, hipStream_t stream,
                     double *kernel_ms, double *span_ms);

/* Draw beta0 (with an intercept), tau and lam (Sec. 3.1 conjugate
 * conditionals) from the reductions of the last completed sweep, with that
 * sweep's index in the random counter;
 * sweeping without GMRF_WITH_HYPER and then calling this is bitwise the same
 * as sweeping with it.  Asynchronous.  Errors: GMRF_E_INVALID_ARG if no sweep
 * has completed. */
int gmrf_hyper_update(gmrf_chain *c, hipStream_t stream);

/* Set tau and lam (> 0, finite).  Asynchronous. */
int gmrf_set_hyper(gmrf_chain *c, double tau, double lam, hipStream_t stream);

/* Posterior mean S1/N and variance (S2 - S1^2/N)/(N - 1) of phi = beta0 + x
 * over the N sweeps accumulated after burn-in (Sec. 3.1: posterior summaries
 * from the draws of the chain), in original site order, FP64.  With
 * GMRF_PTR_HOST the call synchronises, mean / var / n_acc are host pointers
 * (n_acc may be NULL) and N < 2 is refused with GMRF_E_INVALID_ARG (nothing
 * written).  With GMRF_PTR_DEVICE mean / var are device buffers of n
 * doubles, n_acc must be NULL, the call is asynchronous and N is not
 * checked: the values are computed as written, so N = 1 gives an infinite
 * or NaN variance and N = 0 NaN means.  Returns GMRF_E_NUMERIC if a device
 * draw failed. */
int gmrf_posterior_stats(gmrf_chain *c, double *mean, double *var, int64_t *n_acc,
                         uint32_t flags, hipStream_t stream);

/* Read the chain state, the current draw of Algorithm 1 (Sec. 2.3) and of
 * the Sec. 3.1 hyperparameter conditionals: x (host, n doubles, original
 * order), tau, lam and the number of completed sweeps; any output pointer
 * may be NULL.  Synchronises.  Returns GMRF_E_NUMERIC if a device draw
 * failed. */
int gmrf_get_state(gmrf_chain *c, double *x, double *tau, double *lam, uint64_t *sweep,
                   hipStream_t stream);

/* Overwrite the chain state (checkpoint resume, tests): the state of the
 * Markov chain of Algorithm 1 (Sec. 2.3) is x, tau, lam (and beta0, see
 * gmrf_set_intercept) after a completed sweep.  x: host, original order, or
 * NULL to keep x.  The random streams are keyed by (seed, instance, sweep,
 * site), so resuming from a saved state continues the same chain bitwise.
 * Synchronises. */
int gmrf_set_state(gmrf_chain *c, const double *x, double tau, double lam, uint64_t sweep,
                   hipStream_t stream);

/* Read / write the posterior accumulators (host, original order, n doubles
 * each) and the accumulated-sweep count, for checkpointing.  Synchronise. */
int gmrf_get_accumulators(gmrf_chain *c, double *s1, double *s2, int64_t *n_acc,
                          hipStream_t stream);
int gmrf_set_accumulators(gmrf_chain *c, const double *s1, const double *s2, int64_t n_acc,
                          hipStream_t stream);

/* Intercept beta0 of the chain (0 without an intercept).  Synchronises. */
int gmrf_get_intercept(gmrf_chain *c, double *beta0, hipStream_t stream);

/* Set beta0 (finite) of a chain created with an intercept; the stored sse of
 * the last sweep moves to the new beta0.  Asynchronous. */
int gmrf_set_intercept(gmrf_chain *c, double beta0, hipStream_t stream);

/* Hyperparameter trace (for autocorrelation diagnostics, Sec. 3.1 ESS / IAT):
 * d_trace is a device buffer of 3 * capacity doubles that the chain owner
 * keeps alive while the trace is on; after sweep t (0-based) with t <
 * capacity, row t is set to (tau, lam, beta0) after that sweep's draws (a
 * later gmrf_hyper_update rewrites it).  capacity 0 (d_trace may be NULL)
 * turns the trace off.  The setting lives in the chain's device state, so
 * captured sweeps and batches follow it; once this call has returned with
 * the trace off, no later sweep writes the old buffer.  Synchronises. */
int gmrf_set_trace(gmrf_chain *c, double *d_trace, int64_t capacity, hipStream_t stream);

/* Launch shape of a chain.  Lattices (Sec. 2.3: the color phases of a
 * lattice sweep run tile by tile): shape 0 is a 64 x 64 tile with 512
 * threads, shape 1 a 32 x 32 tile with 256 threads; shape 2 (lattices of at
 * most 64 x 64 sites) is shape 0's single tile swept by a persistent
 * one-block kernel that runs all the sweeps of a gmrf_sweep call, with their
 * draws, in one launch (bitwise the results of shape 0).  A new lattice chain
 * starts with shape 2 if the lattice fits one 64 x 64 tile, else with shape 0
 * if that gives at least 512 tiles, else shape 1.  Shapes 0 and 1 group the
 * FP64 reductions differently (results agree to rounding, not bit for bit);
 * the draws of x are keyed by site and do not depend on the shape.
 * General graphs: shape 0 launches one kernel per color (256-thread blocks)
 * and the commit kernel; shape 1 (Gaussian chains on a graph with chunk
 * tables whose largest chunk image fits 64 KB of LDS) sweeps with one
 * 256-thread block per chunk that stages the chunk's closure R and its
 * other neighbours in LDS, runs every color phase of R there and writes the
 * chunk's own sites back (sites of R outside the chunk are recomputed,
 * bitwise as their owner computes them), one launch per sweep, the field
 * alternating between two buffers; shape 2 (a field of at most 122880
 * bytes, at most 32 colors) runs the color passes and the draws in one
 * 512-thread block with the field in LDS -- all the sweeps of a call in one
 * launch, or, for the binomial model, one sweep per launch after the
 * Polya-Gamma launches.  Shape 2 gives bitwise the results of shape 0;
 * shape 1 computes each site's draw the same way but groups the FP64
 * reductions by chunk, so its chains agree with the others to rounding.  A
 * new
 * general-graph chain starts with shape 1 if it fits, else shape 2 if it
 * fits and no color has more than 1024 sites, else shape 0.
 * gmrf_chain_get_tile reports the shape, the tile size (0 x 0 for a general
 * graph) and the threads per block; any output pointer may be NULL.
 * gmrf_chain_set_tile drops the chain's captured sweeps and, when the chain
 * moves to or from shape 1 with the field in the other buffer, copies the
 * field over (synchronising the device); a batch keeps the shapes its chains
 * had when it was created (shape 2 is batched as shape 0).
 * For a shape-2 chain gmrf_sweep_timed reports the duration of the single
 * launch (draws included) as both kernel and span time (binomial: the
 * Polya-Gamma launches and the one-block launch of each sweep).  Host-only
 * calls. */
int gmrf_chain_get_tile(const gmrf_chain *c, int32_t *tile, int32_t *tile_rows, int32_t *tile_cols,
                        int32_t *threads);
int gmrf_chain_set_tile(gmrf_chain *c, int32_t tile);

/* Autotune the launch shape of a chain (a lattice, or a Gaussian chain on a
 * general graph; not binomial chains): time `reps` (1 .. 100000) whole
 * sweeps (draws included) of each shape that fits on the chain itself and
 * keep the fastest.  The timed sweeps run in a dry mode:
 * the draws are computed but not stored, and an accumulating chain's
 * accumulator updates go to its statistics scratch (the same memory traffic),
 * so only scratch (the other state buffer, the partial slots, the statistics
 * area) is written and the chain's state, accumulators, trace and sweep count
 * are unchanged.  us_per_sweep (NULL or
 * GMRF_NUM_TILES doubles) receives the mean time per sweep of each shape in
 * microseconds (0 for a shape that does not fit), best the chosen shape.
 * Synchronises the stream. */
int gmrf_chain_autotune(gmrf_chain *c, int32_t reps, hipStream_t stream, int32_t *best,
                        double *us_per_sweep);

/* Reductions of the last completed sweep: q = x'(D - rho W)x and
 * sse = ||y - beta0 1 - x||^2 (FP64; after a draw of beta0, at the new
 * beta0); for a binomial chain sse is sum_i psi_i.  Synchronises. */
int gmrf_last_reductions(gmrf_chain *c, double *q, double *sse, hipStream_t stream);

/* ---- batches: many chains advanced by shared launches -------------------- */

typedef struct gmrf_batch gmrf_batch;

/* Device workspace bytes of a batch over `count` chains (the job tables of
 * the shared launches, sized for the chains' own tile shapes and for every
 * lattice chain in either tile configuration, as gmrf_batch_autotune lays
 * them out).  Returns 0 and sets the error message if the chains cannot form
 * a batch. */
size_t gmrf_batch_footprint(gmrf_chain *const *chains, int32_t count);

/* Group `count` distinct chains of one precision, each on its own graph or
 * sharing graphs, so that gmrf_batch_sweep advances all of them with shared
 * launches per sweep: one lattice launch per stencil covering the tiles of
 * every lattice chain, one chunked launch (per intercept setting) covering
 * the chunks of every shape-1 general-graph chain (these chains' sweep
 * kernels end their previous sweep; chains with more than 2048 chunks get a
 * launch of their own and end every sweep in the per-sweep commit, as on
 * their own), one launch per color index covering that color's slab of
 * every other general-graph chain followed by one commit launch with a
 * block per such chain, and at the end of the call one commit launch with a
 * block per one-launch (lattice or shape-1) chain
 * (Sec. 2.3, Algorithm 1, for every chain; the independent chains need no
 * communication).  Each chain keeps its own workspace, state, reductions and
 * random streams, so its results equal those of gmrf_sweep on that chain bit
 * for bit.  The tables are uploaded to d_ws (ws_bytes >=
 * gmrf_batch_footprint) and the call synchronises the stream.  The chains
 * must outlive the batch and must not be swept on their own while the batch
 * is in use on another stream.  Errors: GMRF_E_INVALID_ARG (count < 1, NULL
 * or repeated chain, mixed precisions, a binomial or rng_version 2 chain),
 * GMRF_E_WORKSPACE, GMRF_E_DEVICE. */
int gmrf_batch_create(gmrf_chain *const *chains, int32_t count, void *d_ws, size_t ws_bytes,
                      hipStream_t stream, gmrf_batch **out);
int gmrf_batch_destroy(gmrf_batch *b);

/* nsweeps sweeps of every chain of the batch; flags as for gmrf_sweep
 * (GMRF_WITH_HYPER, GMRF_CAPTURE). */
int gmrf_batch_sweep(gmrf_batch *b, int32_t nsweeps, uint32_t flags, hipStream_t stream);

/* Choose the tile shape of the batch's lattice chains for the shared launch:
 * time `reps` (1 .. 100000) passes over the tiles of every lattice chain of
 * the batch with all of them in shape 0 (64 x 64 tiles) and then in shape 1
 * (32 x 32), in the dry mode of gmrf_chain_autotune (only scratch written:
 * the chains' state, accumulators and sweep counts are unchanged), and give every
 * lattice chain the faster shape (as gmrf_chain_set_tile does, also for its
 * own sweeps).  The batch's tables are then laid out again and its captured
 * sweeps dropped.  General-graph chains are not timed or changed.
 * us_per_sweep (NULL or 2 doubles) receives the mean time of one pass in
 * microseconds per shape, best the chosen shape (-1 if the batch has no
 * lattice chain).  Synchronises the stream. */
int gmrf_batch_autotune(gmrf_batch *b, int32_t reps, hipStream_t stream, int32_t *best,
                        double *us_per_sweep);

#ifdef __cplusplus
}
#endif

#endif /* GMRF_H */
