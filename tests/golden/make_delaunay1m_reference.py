"""Write the FP64 oracle reference of the 1,000,000-site Delaunay workload.

Runs the CPU oracle (oracle/, FP64) for 2000 sweeps of the proper CAR
(rho = 0.95) on the Delaunay graph of 1,000,000 uniform points (data seed 3,
the oracle's own greedy coloring in point-index order), Gamma(1,1) priors,
chain seed 5, instance 1, burn-in 0, from x = 0, and stores, for a fixed set
of sites, the posterior mean and variance and the final field, the tau / lam
trajectory after every sweep, the last q / sse, and digests of the inputs
(y and the coloring) so that a test can check it regenerated the same
workload.  Only the oracle and the seeded input generator are used.

    python tests/golden/make_delaunay1m_reference.py [--threads N]
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1702_05518_amd import inputs  # noqa: E402

N = 1_000_000
SWEEPS = 2000
SEED, INSTANCE = 5, 1
OUT = os.path.join(HERE, "delaunay1m_fp64_oracle.npz")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sample_sites(n):
    """8192 seeded random sites and the first and last 256 ids."""
    rng = np.random.Generator(np.random.PCG64(321))
    pick = [np.arange(256), n - 256 + np.arange(256), rng.choice(n, 8192, replace=False)]
    return np.unique(np.concatenate(pick)).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    oracle.build(force=False)
    wl = inputs.delaunay_workload(N, data_seed=3, rho=0.95)
    color, k = oracle.greedy_coloring(wl["row_ptr"], wl["col"])
    ch = oracle.Chain(wl["row_ptr"], wl["col"], color, wl["y"], rho=0.95, seed=SEED,
                      instance=INSTANCE)
    taus, lams = np.empty(SWEEPS), np.empty(SWEEPS)
    t0 = time.time()
    for t in range(SWEEPS):
        ch.sweeps(1, nthreads=args.threads)
        taus[t], lams[t] = ch.tau, ch.lam
        if t % 100 == 99:
            print(f"sweep {t + 1}: tau {ch.tau:.6f} lam {ch.lam:.6f} ({time.time() - t0:.0f} s)",
                  flush=True)
    mean, var = ch.stats()
    sites = sample_sites(N)
    np.savez_compressed(OUT, sites=sites, mean=mean[sites], var=var[sites], x=ch.x[sites],
                        tau=taus, lam=lams, q=ch.q, sse=ch.sse, sweeps=SWEEPS, colors=k,
                        y_sha256=digest(wl["y"]), color_sha256=digest(np.asarray(color, np.int32)),
                        full_mean_abs_max=np.abs(mean).max())
    print("wrote", OUT)


if __name__ == "__main__":
    main()
