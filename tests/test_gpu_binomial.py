"""GPU parity of the binomial logit model (Sec. 3.2, Polya-Gamma augmentation)
through the C ABI, against the CPU oracle on the same seeded inputs.

FP64: the field, the Polya-Gamma sums (sum psi), sum (kappa - psi x), q,
tau and beta0 within 1e-12 relative after every checked sweep.  FP32: the
Polya-Gamma draws stay FP64 and their accept/reject tests see the tilt
beta0 + x only through the mixture choice and the left-piece proposal, so
the rounding-level differences of an FP32 state flip a decision only rarely
and the FP32 chain follows the oracle's path: posterior-mean max abs error
<= 1e-4 after 300 sweeps (the FP32 lattice criterion), and, with different
seeds, statistical agreement with an FP64 chain.
"""
import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu

RTOL64 = 1e-12


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


def case(G, n=2000, median=40.0, seed=5, rho=0.995):
    wl = inputs.binomial_workload(n, data_seed=seed, rho=rho, trials_median=median)
    wl["color"], wl["k"] = G.greedy_coloring(wl["row_ptr"], wl["col"])
    return wl


def pair(G, orc, wl, precision=None, seed=3, instance=0, burn_in=0, intercept=True):
    prec = G.FP64 if precision is None else precision
    g = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"], num_colors=wl["k"],
                rho=wl["rho"])
    kw = dict(seed=seed, instance=instance, burn_in=burn_in, intercept=intercept,
              beta0_var=1000.0, trials=wl["trials"])
    ch = G.Chain(g, wl["y"], precision=prec, **kw)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], rho=wl["rho"], **kw)
    return g, ch, oc


@pytest.mark.parametrize("shape", [0, 2])
@pytest.mark.parametrize("rho", [0.995, 1.0])
def test_binomial_one_sweep_from_injected_state(G, orc, rho, shape):
    wl = case(G, rho=rho)
    n = wl["n"]
    x0 = np.random.default_rng(1).normal(size=n) * 0.4
    g, ch, oc = pair(G, orc, wl, seed=11, instance=4)
    ch.set_tile(shape)
    ch.set_state(x0, 2.5, 1.0, 6)
    ch.set_intercept(0.2)
    oc.set_state(x0, 2.5, 1.0, 6, beta0=0.2)
    ch.sweep(1)
    oc.sweeps(1)
    x, tau, _, sw = ch.get_state()
    q, spsi = ch.last_reductions()
    assert sw == 7
    assert rel(x, oc.x) <= RTOL64
    assert rel(q, oc.q) <= RTOL64 and rel(spsi, oc.sse) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(ch.beta0, oc.beta0) <= RTOL64


@pytest.mark.parametrize("shape", [0, 2])
def test_binomial_trajectory_fp64(G, orc, shape):
    wl = case(G, n=1500, median=60.0, seed=8)
    g, ch, oc = pair(G, orc, wl, burn_in=10)
    ch.set_tile(shape)
    worst = 0.0
    for block in range(4):
        for _ in range(10):
            ch.sweep(1)
            oc.sweeps(1)
            _, tau, _, _ = ch.get_state()
            worst = max(worst, rel(tau, oc.tau), rel(ch.beta0, oc.beta0))
        x, _, _, _ = ch.get_state()
        worst = max(worst, rel(x, oc.x))
    assert worst <= RTOL64, worst
    m, v, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 30 and rel(m, om) <= RTOL64 and rel(v, ov) <= 1e-9


@pytest.mark.parametrize("shape", [0, 2])
def test_binomial_without_intercept_and_capture(G, orc, shape):
    wl = case(G, n=800, median=20.0, seed=2)
    g, ch, oc = pair(G, orc, wl, intercept=False, seed=5)
    ch.set_tile(shape)
    ch.sweep(12, capture=True)
    oc.sweeps(12)
    x, tau, _, _ = ch.get_state()
    assert ch.beta0 == 0.0 and oc.beta0 == 0.0
    assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64


def test_binomial_hyper_update_equals_fused(G, orc):
    wl = case(G, n=600, median=30.0, seed=9)
    _, a, _ = pair(G, orc, wl, seed=7)
    _, b, _ = pair(G, orc, wl, seed=7)
    for _ in range(4):
        a.sweep(1, hyper=True)
        b.sweep(1, hyper=False)
        b.hyper_update()
    xa, ta, _, _ = a.get_state()
    xb, tb, _, _ = b.get_state()
    assert np.array_equal(xa, xb) and ta == tb and a.beta0 == b.beta0


def test_binomial_fp32_follows_the_oracle_path(G, orc):
    wl = case(G, n=1500, median=60.0, seed=6)
    _, ch, oc = pair(G, orc, wl, precision=G.FP32_ACC64, burn_in=100, seed=9)
    ch.sweep(300)
    oc.sweeps(300, nthreads=8)
    m, _, nacc = ch.posterior_stats()
    om, _ = oc.stats()
    _, tau, _, _ = ch.get_state()
    assert nacc == 200
    assert np.max(np.abs(m - om)) <= 1e-4
    assert abs(tau - oc.tau) <= 1e-5 * oc.tau and abs(ch.beta0 - oc.beta0) <= 1e-4


def test_binomial_fp32_agrees_statistically(G, orc):
    """FP32 and FP64 chains of the same posterior: the posterior means of
    beta0 + x agree within their Monte Carlo error."""
    wl = case(G, n=1200, median=80.0, seed=4)
    _, c32, _ = pair(G, orc, wl, precision=G.FP32_ACC64, burn_in=200, seed=21)
    _, c64, _ = pair(G, orc, wl, burn_in=200, seed=22)
    c32.sweep(1200)
    c64.sweep(1200)
    m32, v32, n32 = c32.posterior_stats()
    m64, v64, n64 = c64.posterior_stats()
    assert n32 == n64 == 1000
    # independent chains: difference of two means, each with an error below
    # sd / sqrt(N / IAT); IAT of these sites is well under 100
    se = np.sqrt((v32 + v64) / (1000 / 100))
    assert np.mean(np.abs(m32 - m64) < 4 * se) > 0.99
    assert np.corrcoef(m32, wl["truth"])[0, 1] > 0.5


@pytest.mark.parametrize("layout", ["mixed", "no_trials"])
def test_binomial_extreme_trial_counts(G, orc, layout):
    """Sites without trials (psi = 0) next to one site with 5,000 trials,
    whose 1,250 PG term chunks span many wavefronts; and a graph with no
    trials at all (no PG terms to draw)."""
    wl = case(G, n=500, median=10.0, seed=12)
    trials, y = wl["trials"].copy(), wl["y"].copy()
    if layout == "mixed":
        trials[::3], y[::3] = 0, 0.0
        trials[5], y[5] = 5000, 2400.0
        trials[6], y[6] = 130, 70.0       # a run that starts mid-wavefront
    else:
        trials[:], y[:] = 0, 0.0
    wl["trials"], wl["y"] = trials, y
    g, ch, oc = pair(G, orc, wl, seed=13, instance=1)
    for _ in range(3):
        ch.sweep(1)
        oc.sweeps(1)
        x, tau, _, _ = ch.get_state()
        q, spsi = ch.last_reductions()
        assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64
        assert rel(ch.beta0, oc.beta0) <= RTOL64
        if layout == "no_trials":
            assert spsi == 0.0 and oc.sse == 0.0
        else:
            assert rel(spsi, oc.sse) <= RTOL64


def test_binomial_one_block_is_bitwise_color_passes(G, orc):
    wl = case(G, n=2500, median=40.0, seed=14)
    _, a, _ = pair(G, orc, wl, seed=4, burn_in=2)
    _, b, _ = pair(G, orc, wl, seed=4, burn_in=2)
    a.set_tile(0)
    b.set_tile(2)
    assert a.tile[0] == 0 and b.tile[0] == 2
    a.sweep(6)
    b.sweep(6)
    a.sweep(4, capture=True)
    b.sweep(4, capture=True)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:] and a.beta0 == b.beta0
    assert a.last_reductions() == b.last_reductions()
    ma, va, _ = a.posterior_stats()
    mb, vb, _ = b.posterior_stats()
    assert np.array_equal(ma, mb) and np.array_equal(va, vb)


def test_binomial_argument_errors(G):
    wl = case(G, n=300, median=10.0, seed=1)
    g = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"], num_colors=wl["k"],
                rho=0.995)
    bad = wl["y"].copy()
    bad[0] = wl["trials"][0] + 1
    with pytest.raises(G.GmrfError):
        G.Chain(g, bad, trials=wl["trials"], intercept=True)
    frac = wl["y"].copy()
    frac[1] = 0.5
    with pytest.raises(G.GmrfError):
        G.Chain(g, frac, trials=wl["trials"])
    with pytest.raises(G.GmrfError):
        G.Chain(g, wl["y"], trials=wl["trials"], beta0_var=-1.0)
    with pytest.raises(G.GmrfError):
        G.Chain(g, wl["y"], beta0_var=10.0)               # Gaussian chain with beta0_var
    lat = G.Graph(lattice=(8, 8, 4))
    with pytest.raises(G.GmrfError):
        G.Chain(lat, np.zeros(64), trials=np.ones(64, dtype=np.int32))
    ch = G.Chain(g, wl["y"], trials=wl["trials"], intercept=True, beta0_var=1000.0)
    with pytest.raises(G.GmrfError):
        G.Batch([ch])


def test_binomial_full_size_one_sweep(G, orc):
    """The benchmark's binomial workload (n = 14,926, ~5 million trials), one
    FP64 sweep with the hyperparameter draws, against the oracle."""
    wl = inputs.binomial_workload(14926, data_seed=5)
    wl["color"], wl["k"] = G.greedy_coloring(wl["row_ptr"], wl["col"])
    g, ch, oc = pair(G, orc, wl, seed=1)
    ch.sweep(1)
    oc.sweeps(1, nthreads=8)
    x, tau, _, _ = ch.get_state()
    q, spsi = ch.last_reductions()
    assert rel(x, oc.x) <= RTOL64 and rel(spsi, oc.sse) <= RTOL64 and rel(q, oc.q) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(ch.beta0, oc.beta0) <= RTOL64
