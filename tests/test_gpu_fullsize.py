"""GPU parity at the full workload sizes, in the benchmark's launch configuration.

* 2048 x 2048, 8 neighbours: one FP64 sweep from an injected state against
  one oracle sweep over every site; 1000-sweep FP32 and FP64 runs against the
  stored FP64 oracle reference (tests/golden/, written by the committed
  script make_lattice2048_reference.py, which calls only the oracle):
  posterior mean / variance at ~14k sampled sites and the tau / lam
  trajectory after every sweep (device trace).
* 4096 x 4096, 8 neighbours (4096 tiles, more than the blocks the chip
  holds at once, and a working set beyond the 256 MB Infinity Cache): one
  FP64 sweep from an injected state against one oracle sweep over every site.
* 1500 x 1500, 8 neighbours, in 32 x 32 tiles (2209 tiles: every sweep ends
  in its own commit launch) and in 64 x 64 tiles: six sweeps against the
  oracle, FP64 and FP32.
* Delaunay graph with 1,000,000 sites: one FP64 sweep from an injected
  state against one oracle sweep over every site; the configured 2000-sweep
  run in FP32 and FP64 against the stored FP64 oracle reference
  (make_delaunay1m_reference.py): posterior mean / variance at ~8.7k sampled
  sites, the final field there, and tau / lam after every sweep.
"""
import hashlib
import os

import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REF2048 = os.path.join(HERE, "golden", "lattice2048_s8_fp64_oracle.npz")
REF1M = os.path.join(HERE, "golden", "delaunay1m_fp64_oracle.npz")
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05518_amd import gmrf

    gmrf.lib()
    return gmrf


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def wl2048():
    return inputs.lattice_workload(2048, 2048, 8, noise_sd=0.1, data_seed=1)


def test_lattice2048_one_sweep_fp64_all_sites(G, orc, wl2048):
    wl = wl2048
    n = wl["n"]
    x0 = (np.random.default_rng(3).normal(size=n) * 0.2 + wl["y"]).astype(np.float64)
    g = G.Graph(lattice=(2048, 2048, 8))
    ch = G.Chain(g, wl["y"], precision=G.FP64, seed=1)
    ch.set_state(x0, 45.0, 110.0, 7)
    ch.sweep(1, capture=True)
    x, tau, lam, sw = ch.get_state()
    q, sse = ch.last_reductions()
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=1)
    oc.set_state(x0, 45.0, 110.0, 7)
    oc.sweeps(1, nthreads=THREADS)
    assert sw == 8
    assert rel(x, oc.x) <= 1e-12
    assert rel(q, oc.q) <= 1e-12 and rel(sse, oc.sse) <= 1e-12
    assert rel(tau, oc.tau) <= 1e-12 and rel(lam, oc.lam) <= 1e-12


@pytest.mark.skipif(not os.path.exists(REF2048), reason="reference not generated")
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lattice2048_1000_sweeps_against_reference(G, wl2048, prec):
    ref = np.load(REF2048)
    g = G.Graph(lattice=(2048, 2048, 8))
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    ch = G.Chain(g, wl2048["y"], precision=p, seed=1)
    ch.enable_trace(1000)
    for b in range(10):
        ch.sweep(100, capture=True)
    x, _, _, sw = ch.get_state()
    assert sw == 1000
    tr = ch.trace()
    taus, lams = tr[:, 0], tr[:, 1]
    mean, var, nacc = ch.posterior_stats()
    assert nacc == 1000
    sites = ref["sites"]
    mean_err = np.max(np.abs(mean[sites] - ref["mean"]))
    var_err = np.max(np.abs(var[sites] - ref["var"]))
    print(f"{prec}: posterior mean max abs err {mean_err:.3e}, var max abs err {var_err:.3e}, "
          f"tau rel {rel(taus, ref['tau']):.3e}, lam rel {rel(lams, ref['lam']):.3e}")
    if prec == "fp32":
        assert mean_err <= 1e-4
        assert var_err <= 1e-4 * max(1.0, float(np.max(ref["var"])))
        assert rel(taus, ref["tau"]) <= 1e-3
        assert rel(lams, ref["lam"]) <= 1e-3
    else:
        assert rel(mean[sites], ref["mean"]) <= 1e-12
        assert rel(x[sites], ref["x"]) <= 1e-12
        assert rel(taus, ref["tau"]) <= 1e-12
        assert rel(lams, ref["lam"]) <= 1e-12
        assert np.max(np.abs(var[sites] - ref["var"])) <= 1e-9 * float(np.max(ref["var"]))


def test_lattice4096_one_sweep_fp64_all_sites(G, orc):
    """More tiles (4096 of 64 x 64) than resident blocks, and a working set
    (about 0.7 GB) beyond the Infinity Cache: one FP64 sweep from an injected
    state, every site, q / sse and the draws, at 1e-12."""
    wl = inputs.lattice_workload(4096, 4096, 8, noise_sd=0.1, data_seed=2)
    n = wl["n"]
    x0 = (np.random.default_rng(8).normal(size=n) * 0.3 + wl["y"]).astype(np.float64)
    g = G.Graph(lattice=(4096, 4096, 8))
    ch = G.Chain(g, wl["y"], precision=G.FP64, seed=2, instance=4)
    assert ch.tile[0] == 0
    ch.set_state(x0, 30.0, 95.0, 11)
    ch.sweep(1)
    x, tau, lam, sw = ch.get_state()
    q, sse = ch.last_reductions()
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=2, instance=4)
    oc.set_state(x0, 30.0, 95.0, 11)
    oc.sweeps(1, nthreads=THREADS)
    assert sw == 12
    assert rel(x, oc.x) <= 1e-12
    assert rel(q, oc.q) <= 1e-12 and rel(sse, oc.sse) <= 1e-12
    assert rel(tau, oc.tau) <= 1e-12 and rel(lam, oc.lam) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_many_tiles_sweeps_commit_each(G, orc, prec):
    """A lattice with more tiles (2209 of 32 x 32) than a block sums when it
    ends the previous sweep itself: every sweep ends in its own commit
    launch.  Six sweeps with the hyperparameter draws, every site and tau /
    lam against the oracle (FP64 1e-12; FP32 state: field 1e-4, tau / lam
    1e-4 relative), and the same chain in 64 x 64 tiles (576 tiles, the
    previous sweep ended inside the next sweep's kernel) agreeing to
    rounding."""
    wl = inputs.lattice_workload(1500, 1500, 8, noise_sd=0.1, data_seed=5)
    n = wl["n"]
    p = G.FP64 if prec == "fp64" else G.FP32_ACC64
    g = G.Graph(lattice=(1500, 1500, 8))
    out = {}
    for shape in (1, 0):
        ch = G.Chain(g, wl["y"], precision=p, seed=6, burn_in=2)
        ch.set_tile(shape)
        ch.sweep(4)
        ch.sweep(2, capture=True)
        x, tau, lam, sw = ch.get_state()
        s1, _, nacc = ch.get_accumulators()
        assert sw == 6 and nacc == 4
        out[shape] = (x, tau, lam, s1)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=6, burn_in=2)
    oc.sweeps(6, nthreads=THREADS)
    tol = 1e-12 if prec == "fp64" else 1e-4
    for shape in (1, 0):
        x, tau, lam, s1 = out[shape]
        assert np.max(np.abs(x - oc.x)) <= tol * max(1.0, float(np.max(np.abs(oc.x))))
        assert rel(tau, oc.tau) <= tol and rel(lam, oc.lam) <= tol
        assert np.max(np.abs(s1 - oc.s1)) <= 4 * tol * max(1.0, float(np.max(np.abs(oc.s1))))


def test_delaunay_1m_one_sweep_fp64_all_sites(G, orc):
    wl = inputs.delaunay_workload(1_000_000, data_seed=3, rho=0.95)
    color, k = G.greedy_coloring(wl["row_ptr"], wl["col"])
    assert 5 <= k <= 8
    n = wl["n"]
    x0 = wl["truth"] + 0.05 * np.random.default_rng(4).normal(size=n)
    g = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k, rho=0.95)
    ch = G.Chain(g, wl["y"], precision=G.FP64, seed=5, instance=1)
    ch.set_state(x0, 2.0, 25.0, 3)
    ch.sweep(1)
    x, tau, lam, sw = ch.get_state()
    oc = orc.Chain(wl["row_ptr"], wl["col"], color, wl["y"], rho=0.95, seed=5, instance=1)
    oc.set_state(x0, 2.0, 25.0, 3)
    oc.sweeps(1, nthreads=THREADS)
    assert rel(x, oc.x) <= 1e-12
    assert rel(tau, oc.tau) <= 1e-12 and rel(lam, oc.lam) <= 1e-12


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def wl1m():
    return inputs.delaunay_workload(1_000_000, data_seed=3, rho=0.95)


@pytest.mark.skipif(not os.path.exists(REF1M), reason="reference not generated")
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_delaunay_1m_2000_sweeps_against_reference(G, wl1m, prec):
    """The configured irregular run: 1,000,000 Delaunay sites, proper CAR rho
    0.95, 2000 sweeps from x = 0 with the hyperparameter draws, in FP32 with
    FP64 accumulators (posterior-mean max abs error <= 1e-4 against the FP64
    oracle, the variance and the tau / lam trajectories bounded) and in FP64
    (1e-12 relative)."""
    ref = np.load(REF1M)
    wl = wl1m
    assert digest(wl["y"]) == str(ref["y_sha256"])
    color, k = G.greedy_coloring(wl["row_ptr"], wl["col"])
    assert digest(np.asarray(color, np.int32)) == str(ref["color_sha256"]) and k == int(ref["colors"])
    g = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k, rho=0.95)
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    ch = G.Chain(g, wl["y"], precision=p, seed=5, instance=1)
    ch.enable_trace(2000)
    ch.sweep(1000, capture=True)
    ch.sweep(1000, capture=True)
    x, _, _, sw = ch.get_state()
    assert sw == 2000
    tr = ch.trace()
    mean, var, nacc = ch.posterior_stats()
    assert nacc == 2000
    sites = ref["sites"]
    mean_err = np.max(np.abs(mean[sites] - ref["mean"]))
    var_err = np.max(np.abs(var[sites] - ref["var"]))
    print(f"1M {prec}, 2000 sweeps: posterior mean max abs err {mean_err:.3e}, var max abs err "
          f"{var_err:.3e}, x rel {rel(x[sites], ref['x']):.3e}, tau rel "
          f"{rel(tr[:, 0], ref['tau']):.3e}, lam rel {rel(tr[:, 1], ref['lam']):.3e}")
    if prec == "fp32":
        assert mean_err <= 1e-4
        assert var_err <= 1e-4 * max(1.0, float(np.max(ref["var"])))
        assert rel(tr[:, 0], ref["tau"]) <= 1e-3 and rel(tr[:, 1], ref["lam"]) <= 1e-3
    else:
        assert rel(mean[sites], ref["mean"]) <= 1e-12
        assert rel(x[sites], ref["x"]) <= 1e-12
        assert rel(tr[:, 0], ref["tau"]) <= 1e-12 and rel(tr[:, 1], ref["lam"]) <= 1e-12
        assert var_err <= 1e-9 * float(np.max(ref["var"]))
