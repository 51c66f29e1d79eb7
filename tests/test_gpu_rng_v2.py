"""GPU parity of the paired random-number contract (version 2) on lattices.

Version 2 gives the sites of each color, ranked by original id, one Philox
block per rank pair: the cosine Box-Muller branch for the first site, the
sine branch for the second.  The lattice kernels take the pairs as
(r, c), (r, c + 2) with bit 1 of c clear, which is that ranking when the
lattice width is a multiple of 4 (the only widths version 2 accepts).  Every
test compares the HIP path, through the C ABI, with the oracle's version-2
chain on the same seeded inputs: FP64 within 1e-12 relative (field, tau,
lam, q, sse), FP32 posterior means within 1e-4 of the FP64 oracle after
1000 sweeps.  Lattices span several tiles with ragged tails (150 x 132 in
64 x 64 and 32 x 32 tiles), one-row and one-column-pair lattices, and every
launch shape (tiles of 64 and 32, and the single-block persistent kernel).
"""
import os

import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu

RTOL64 = 1e-12
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


def v2_pair(G, orc, rows, cols, st, precision=None, seed=1, instance=0, rho=1.0, **kw):
    wl = inputs.lattice_workload(rows, cols, st, noise_sd=0.1, data_seed=rows * 1000 + cols)
    g = G.Graph(lattice=(rows, cols, st), rho=rho)
    prec = G.FP64 if precision is None else precision
    ch = G.Chain(g, wl["y"], precision=prec, seed=seed, instance=instance, rng_version=2, **kw)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], rho=rho, seed=seed,
                   instance=instance, rng_version=2, **kw)
    return wl, ch, oc


LATTICES = [(64, 64, 4), (64, 64, 8), (150, 132, 4), (150, 132, 8), (1, 4, 8), (1, 76, 4),
            (77, 4, 8), (2, 4, 8), (129, 68, 8), (3, 8, 4)]


def shapes_for(rows, cols):
    return [0, 1, 2] if rows <= 64 and cols <= 64 else [0, 1]


@pytest.mark.parametrize("rows,cols,st", LATTICES)
def test_one_sweep_from_injected_state(G, orc, rows, cols, st):
    for shape in shapes_for(rows, cols):
        wl, ch, oc = v2_pair(G, orc, rows, cols, st, seed=7, instance=2)
        n = rows * cols
        x0 = np.random.default_rng(n).normal(size=n) * 0.3 + 0.5
        ch.set_tile(shape)
        ch.set_state(x0, 1.7, 60.0, 5)
        oc.set_state(x0, 1.7, 60.0, 5)
        ch.sweep(1, hyper=True)
        oc.sweeps(1, hyper=True)
        x, tau, lam, sw = ch.get_state()
        q, sse = ch.last_reductions()
        assert sw == 6
        assert rel(x, oc.x) <= RTOL64, (shape, rel(x, oc.x))
        assert rel(q, oc.q) <= RTOL64 and rel(sse, oc.sse) <= RTOL64, shape
        assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64, shape


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("st", [4, 8])
def test_version_2_differs_from_version_1_only_on_sine_sites(G, orc, st, prec):
    """One sweep from one state under each version: color 0's sites read only
    the injected state, so on its cosine (key) sites version 2 equals
    version 1 bit for bit, and on its sine sites every value differs."""
    rows, cols = 40, 48
    wl = inputs.lattice_workload(rows, cols, st, noise_sd=0.1, data_seed=3)
    g = G.Graph(lattice=(rows, cols, st))
    n = rows * cols
    x0 = np.random.default_rng(5).normal(size=n)
    out = {}
    for v in (1, 2):
        p = G.FP64 if prec == "fp64" else G.FP32_ACC64
        ch = G.Chain(g, wl["y"], precision=p, seed=9, rng_version=v)
        ch.set_state(x0, 2.0, 30.0, 0)
        ch.sweep(1, hyper=False)
        out[v] = ch.get_state()[0]
    r, c = np.divmod(np.arange(n), cols)
    color0 = wl["color"] == 0
    cos_sites = color0 & (((c >> 1) & 1) == 0)
    sin_sites = color0 & (((c >> 1) & 1) == 1)
    assert np.array_equal(out[1][cos_sites], out[2][cos_sites])
    assert not np.any(out[1][sin_sites] == out[2][sin_sites])


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_trajectory_fp64(G, orc, shape):
    """300 sweeps with hyper draws in calls of 1, 7 and 50 sweeps (the last
    captured): field, tau, lam after each call, posterior mean / variance."""
    rows, cols, st = (64, 64, 8) if shape == 2 else (150, 132, 8)
    wl, ch, oc = v2_pair(G, orc, rows, cols, st, seed=3, burn_in=20)
    ch.set_tile(shape)
    done = 0
    for k, cap in [(1, False), (7, False), (50, True), (42, False), (100, True), (100, False)]:
        ch.sweep(k, capture=cap)
        oc.sweeps(k)
        done += k
        x, tau, lam, sw = ch.get_state()
        assert sw == done
        assert rel(x, oc.x) <= RTOL64, (done, rel(x, oc.x))
        assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64, done
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 280
    assert rel(mean, om) <= RTOL64
    assert np.max(np.abs(var - ov)) <= 1e-9 * np.max(np.abs(ov))


@pytest.mark.parametrize("rho", [1.0, 0.9])
def test_intercept_and_proper_prior(G, orc, rho):
    wl, ch, oc = v2_pair(G, orc, 96, 100, 4, seed=6, rho=rho, intercept=True, beta0=0.4)
    for k in (1, 5, 20):
        ch.sweep(k)
        oc.sweeps(k)
        x, tau, lam, _ = ch.get_state()
        assert rel(x, oc.x) <= RTOL64
        assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64
        assert rel(ch.beta0, oc.beta0) <= RTOL64


def test_fp32_posterior_mean_against_fp64_oracle(G, orc):
    wl, ch, oc = v2_pair(G, orc, 64, 64, 8, precision=G.FP32_ACC64, seed=2)
    ch.sweep(1000)
    oc.sweeps(1000)
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    _, tau, lam, _ = ch.get_state()
    assert nacc == 1000
    assert np.max(np.abs(mean - om)) <= 1e-4
    assert np.max(np.abs(var - ov)) <= 1e-4 * max(1.0, np.max(ov))
    assert rel(tau, oc.tau) <= 1e-3 and rel(lam, oc.lam) <= 1e-3


def test_fp32_multi_tile_against_fp64_oracle(G, orc):
    wl, ch, oc = v2_pair(G, orc, 150, 132, 4, precision=G.FP32_ACC64, seed=8)
    for shape in (0, 1):
        ch.set_tile(shape)
        ch.sweep(250, capture=True)
    oc.sweeps(500)
    mean, _, nacc = ch.posterior_stats()
    om, _ = oc.stats()
    assert nacc == 500
    assert np.max(np.abs(mean - om)) <= 1e-4


def test_checkpoint_resume_autotune_and_timed_sweeps(G, orc):
    """The paired contract's draws are keyed by (seed, instance, sweep, key
    site) like version 1's: a chain resumed from its state and accumulators
    continues bit for bit, the autotuner leaves a chain unchanged, and timed
    sweeps equal plain ones."""
    rows, cols, st = 130, 140, 8
    wl = inputs.lattice_workload(rows, cols, st, noise_sd=0.1, data_seed=4)
    g = G.Graph(lattice=(rows, cols, st))
    kw = dict(precision=G.FP64, seed=21, instance=3, rng_version=2)
    full = G.Chain(g, wl["y"], **kw)
    full.sweep(12)
    part = G.Chain(g, wl["y"], **kw)
    part.sweep(5)
    x, tau, lam, sw = part.get_state()
    s1, s2, nacc = part.get_accumulators()
    res = G.Chain(g, wl["y"], **kw)
    res.set_state(x, tau, lam, sw)
    res.set_accumulators(s1, s2, nacc)
    best, _ = res.autotune(reps=3)
    res.set_tile(full.tile[0])          # the shape of the uninterrupted chain
    ms, span = res.sweep_timed(7, span=True)
    assert 0.0 < ms <= span and best in (0, 1, 2)
    a, b = full.get_state(), res.get_state()
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    assert np.array_equal(full.posterior_stats()[0], res.posterior_stats()[0])


def test_lattice2048_two_sweeps_fp64_all_sites(G, orc):
    """The 2048 x 2048 8-neighbour workload in the benchmark's launch shape:
    two captured FP64 sweeps from an injected state (the first sweep's end
    folded into the second sweep's kernel) against the oracle at every site."""
    wl = inputs.lattice_workload(2048, 2048, 8, noise_sd=0.1, data_seed=1)
    n = wl["n"]
    x0 = np.random.default_rng(3).normal(size=n) * 0.2 + wl["y"]
    ch = G.Chain(G.Graph(lattice=(2048, 2048, 8)), wl["y"], precision=G.FP64, seed=1,
                 rng_version=2)
    ch.set_state(x0, 45.0, 110.0, 7)
    ch.sweep(2, capture=True)
    x, tau, lam, sw = ch.get_state()
    q, sse = ch.last_reductions()
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=1, rng_version=2)
    oc.set_state(x0, 45.0, 110.0, 7)
    oc.sweeps(2, nthreads=THREADS)
    assert sw == 9
    assert rel(x, oc.x) <= RTOL64
    assert rel(q, oc.q) <= RTOL64 and rel(sse, oc.sse) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64


REF2048_V2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "lattice2048_s8_fp64_oracle_v2.npz")


@pytest.mark.skipif(not os.path.exists(REF2048_V2), reason="reference not generated")
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lattice2048_1000_sweeps_against_reference(G, prec):
    """The 2048 x 2048 8-neighbour workload for 1000 captured sweeps under
    the paired contract against the stored FP64 oracle reference
    (make_lattice2048_reference.py --rng-version 2): FP64 field, posterior
    mean and tau / lam after every sweep at 1e-12; FP32 posterior mean
    within 1e-4."""
    ref = np.load(REF2048_V2)
    wl = inputs.lattice_workload(2048, 2048, 8, noise_sd=0.1, data_seed=1)
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    ch = G.Chain(G.Graph(lattice=(2048, 2048, 8)), wl["y"], precision=p, seed=1, rng_version=2)
    ch.enable_trace(1000)
    for _ in range(10):
        ch.sweep(100, capture=True)
    x, _, _, sw = ch.get_state()
    assert sw == 1000
    tr = ch.trace()
    mean, var, nacc = ch.posterior_stats()
    assert nacc == 1000
    sites = ref["sites"]
    mean_err = np.max(np.abs(mean[sites] - ref["mean"]))
    print(f"rng v2 {prec}: posterior mean max abs err {mean_err:.3e}, "
          f"tau rel {rel(tr[:, 0], ref['tau']):.3e}")
    if prec == "fp32":
        assert mean_err <= 1e-4
        assert rel(tr[:, 0], ref["tau"]) <= 1e-3 and rel(tr[:, 1], ref["lam"]) <= 1e-3
    else:
        assert rel(mean[sites], ref["mean"]) <= RTOL64
        assert rel(x[sites], ref["x"]) <= RTOL64
        assert rel(tr[:, 0], ref["tau"]) <= RTOL64 and rel(tr[:, 1], ref["lam"]) <= RTOL64
        assert np.max(np.abs(var[sites] - ref["var"])) <= 1e-9 * float(np.max(ref["var"]))


def test_refusals(G):
    wl = inputs.lattice_workload(8, 6, 4, noise_sd=0.1, data_seed=1)
    with pytest.raises(G.GmrfError):      # width not a multiple of 4
        G.Chain(G.Graph(lattice=(8, 6, 4)), wl["y"], rng_version=2)
    wl = inputs.lattice_workload(8, 8, 4, noise_sd=0.1, data_seed=1)
    g = G.Graph(lattice=(8, 8, 4))
    for bad in (-1, 3):
        with pytest.raises(G.GmrfError):
            G.Chain(g, wl["y"], rng_version=bad)
    gc = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"], num_colors=wl["k"])
    with pytest.raises(G.GmrfError):      # general graphs draw by version 1
        G.Chain(gc, wl["y"], rng_version=2)
    a = G.Chain(g, wl["y"], rng_version=2)
    b = G.Chain(g, wl["y"], seed=2)
    with pytest.raises(G.GmrfError):      # batches take version-1 chains
        G.Batch([b, a])
    G.Chain(g, wl["y"], rng_version=0).sweep(2)   # 0 is version 1
