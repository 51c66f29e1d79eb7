"""Write the FP64 oracle reference of the 2048 x 2048 lattice workload.

Runs the CPU oracle (oracle/, FP64) for 1000 sweeps of the 8-neighbour
intrinsic CAR on the 2048 x 2048 block image (Gamma(1,1) priors, seed 1,
instance 0, burn-in 0) and stores, for a fixed set of sites, the posterior
mean and variance and the final field, plus the tau / lam trajectory and the
last q / sse.  Only the oracle and the seeded input generator are used.
--rng-version 2 runs the paired random-number contract and writes the
_v2 file.

    python tests/golden/make_lattice2048_reference.py [--threads N] [--rng-version 2]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1702_05518_amd import inputs  # noqa: E402

ROWS = COLS = 2048
SWEEPS = 1000
OUT = {1: os.path.join(HERE, "lattice2048_s8_fp64_oracle.npz"),
       2: os.path.join(HERE, "lattice2048_s8_fp64_oracle_v2.npz")}


def sample_sites(rows, cols):
    """Boundary rows / columns, a middle row, and 4096 seeded random sites."""
    rng = np.random.Generator(np.random.PCG64(123))
    pick = [np.arange(cols), (rows - 1) * cols + np.arange(cols),
            (rows // 2) * cols + np.arange(cols), np.arange(rows) * cols,
            np.arange(rows) * cols + cols - 1, rng.choice(rows * cols, 4096, replace=False)]
    return np.unique(np.concatenate(pick)).astype(np.int64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--rng-version", type=int, default=1, choices=(1, 2))
    args = ap.parse_args()
    oracle.build(force=False)
    wl = inputs.lattice_workload(ROWS, COLS, 8, noise_sd=0.1, data_seed=1)
    ch = oracle.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], rho=1.0, seed=1,
                      instance=0, rng_version=args.rng_version)
    taus, lams = np.empty(SWEEPS), np.empty(SWEEPS)
    t0 = time.time()
    for t in range(SWEEPS):
        ch.sweeps(1, nthreads=args.threads)
        taus[t], lams[t] = ch.tau, ch.lam
        if t % 100 == 99:
            print(f"sweep {t + 1}: tau {ch.tau:.6f} lam {ch.lam:.6f} ({time.time() - t0:.0f} s)",
                  flush=True)
    mean, var = ch.stats()
    sites = sample_sites(ROWS, COLS)
    out = OUT[args.rng_version]
    np.savez_compressed(out, sites=sites, mean=mean[sites], var=var[sites], x=ch.x[sites],
                        tau=taus, lam=lams, q=ch.q, sse=ch.sse, sweeps=SWEEPS,
                        full_mean_abs_max=np.abs(mean).max())
    print("wrote", out)


if __name__ == "__main__":
    main()
