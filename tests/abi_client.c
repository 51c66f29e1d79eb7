/* abi_client.c -- a plain C program on the C ABI of libgmrf (include/gmrf.h),
 * with device memory from hipMalloc: no Python, no torch.  Test helper.
 *
 * usage: abi_client ROWS COLS STENCIL NSWEEPS SEED Y_FILE MEAN_FILE
 *   Y_FILE    ROWS * COLS doubles (row-major), the data y
 *   MEAN_FILE receives the posterior mean after NSWEEPS sweeps of an FP64
 *             chain with hyperparameter draws (Gamma(1, 1) priors, tau0 =
 *             lam0 = 1, x0 = 0, no burn-in)
 * Prints "tau lam sweeps n_acc" on success; exits non-zero with the
 * library's message on any error. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gmrf.h"

static int check(int rc, const char *what)
{
    if (rc != GMRF_OK) {
        fprintf(stderr, "%s: status %d: %s\n", what, rc, gmrf_last_error());
        exit(1);
    }
    return rc;
}

int main(int argc, char **argv)
{
    if (argc != 8) {
        fprintf(stderr, "usage: %s ROWS COLS STENCIL NSWEEPS SEED Y_FILE MEAN_FILE\n", argv[0]);
        return 2;
    }
    const int rows = atoi(argv[1]), cols = atoi(argv[2]), stencil = atoi(argv[3]);
    const int nsweeps = atoi(argv[4]);
    const unsigned long long seed = strtoull(argv[5], NULL, 10);
    const int64_t n = (int64_t)rows * cols;
    if (rows < 1 || cols < 1 || nsweeps < 1)
        return 2;

    double *y = malloc(sizeof(double) * (size_t)n);
    double *mean = malloc(sizeof(double) * (size_t)n);
    double *var = malloc(sizeof(double) * (size_t)n);
    FILE *f = fopen(argv[6], "rb");
    if (!y || !mean || !var || !f || fread(y, sizeof(double), (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "cannot read %s\n", argv[6]);
        return 1;
    }
    fclose(f);

    hipStream_t stream;
    if (hipStreamCreate(&stream) != hipSuccess) {
        fprintf(stderr, "hipStreamCreate failed\n");
        return 1;
    }

    gmrf_graph_desc d;
    memset(&d, 0, sizeof d);
    d.n = n;
    d.lat_rows = rows;
    d.lat_cols = cols;
    d.lat_stencil = stencil;
    d.rho = 1.0;
    gmrf_graph *g = NULL;
    check(gmrf_graph_create(&d, NULL, 0, stream, &g), "graph_create");

    gmrf_model m;
    memset(&m, 0, sizeof m);
    m.a_tau = m.b_tau = m.a_lam = m.b_lam = 1.0;
    m.tau0 = m.lam0 = 1.0;
    m.likelihood = GMRF_GAUSSIAN;
    const size_t need = gmrf_chain_footprint(g, GMRF_FP64);
    if (need == 0) {
        fprintf(stderr, "chain_footprint: %s\n", gmrf_last_error());
        return 1;
    }
    void *ws = NULL;
    if (hipMalloc(&ws, need) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %zu bytes failed\n", need);
        return 1;
    }
    gmrf_chain *c = NULL;
    check(gmrf_chain_create(g, &m, y, NULL, GMRF_FP64, seed, 0u, ws, need, stream, &c),
          "chain_create");
    check(gmrf_sweep(c, nsweeps, GMRF_WITH_HYPER, stream), "sweep");
    int64_t nacc = 0;
    check(gmrf_posterior_stats(c, mean, var, &nacc, GMRF_PTR_HOST, stream), "posterior_stats");
    double tau = 0.0, lam = 0.0;
    uint64_t sweeps = 0;
    check(gmrf_get_state(c, NULL, &tau, &lam, &sweeps, stream), "get_state");

    f = fopen(argv[7], "wb");
    if (!f || fwrite(mean, sizeof(double), (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "cannot write %s\n", argv[7]);
        return 1;
    }
    fclose(f);
    printf("%.17g %.17g %llu %lld\n", tau, lam, (unsigned long long)sweeps, (long long)nacc);

    check(gmrf_chain_destroy(c), "chain_destroy");
    check(gmrf_graph_destroy(g), "graph_destroy");
    (void)hipFree(ws);
    (void)hipStreamDestroy(stream);
    free(y);
    free(mean);
    free(var);
    return 0;
}
