"""GPU parity on graphs with hubs: sites whose degree far exceeds the
neighbours a thread gathers in one batch, so the general-graph kernels take
their long-row loops for the neighbour sum and for the q terms.

A wheel (one hub joined to every site of a ring) and a complete bipartite
graph K(3, m) (three hubs of degree m), Gaussian (proper and intrinsic CAR)
and binomial, in the color-pass kernels and the one-block kernel: FP64
field, q, sse and the hyperparameters within 1e-12 relative of the oracle.
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


def wheel(n):
    """Site 0 joined to sites 1 .. n - 1, which form a ring."""
    ring = np.arange(1, n)
    ei = np.concatenate([np.zeros(n - 1, dtype=np.int64), ring])
    ej = np.concatenate([ring, np.roll(ring, -1)])
    return inputs.edges_to_csr(n, ei, ej)


def bipartite(hubs, m):
    """Sites 0 .. hubs - 1 each joined to every site hubs .. hubs + m - 1."""
    ei = np.repeat(np.arange(hubs), m)
    ej = np.tile(np.arange(hubs, hubs + m), hubs)
    return inputs.edges_to_csr(hubs + m, ei, ej)


GRAPHS = {"wheel1201": lambda: wheel(1201), "k3_700": lambda: bipartite(3, 700)}


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("rho", [1.0, 0.95])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_hub_graph_gaussian_sweeps(G, orc, name, rho, shape):
    rp, cl = GRAPHS[name]()
    n = len(rp) - 1
    color, k = G.greedy_coloring(rp, cl)
    assert int(np.max(np.diff(rp))) >= 700
    y = np.sin(np.arange(n) * 0.37) + 0.1 * np.random.default_rng(2).standard_normal(n)
    g = G.Graph(row_ptr=rp, col_idx=cl, color=color, num_colors=k, rho=rho)
    ch = G.Chain(g, y, seed=21, instance=2)
    ch.set_tile(shape)
    oc = orc.Chain(rp, cl, color, y, rho=rho, seed=21, instance=2)
    for _ in range(4):
        ch.sweep(5)
        oc.sweeps(5)
        x, tau, lam, _ = ch.get_state()
        q, sse = ch.last_reductions()
        assert rel(x, oc.x) <= RTOL64
        assert rel(q, oc.q) <= RTOL64 and rel(sse, oc.sse) <= RTOL64
        assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64


@pytest.mark.parametrize("shape", [0, 2])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_hub_graph_binomial_sweeps(G, orc, name, shape):
    rp, cl = GRAPHS[name]()
    n = len(rp) - 1
    color, k = G.greedy_coloring(rp, cl)
    rng = np.random.default_rng(9)
    trials = rng.integers(0, 60, size=n).astype(np.int32)
    yb = rng.binomial(trials, 0.4).astype(np.float64)
    kw = dict(seed=13, instance=1, intercept=True, beta0_var=1000.0, trials=trials)
    g = G.Graph(row_ptr=rp, col_idx=cl, color=color, num_colors=k, rho=0.995)
    ch = G.Chain(g, yb, **kw)
    ch.set_tile(shape)
    oc = orc.Chain(rp, cl, color, yb, rho=0.995, **kw)
    for _ in range(3):
        ch.sweep(2)
        oc.sweeps(2)
        x, tau, _, _ = ch.get_state()
        q, spsi = ch.last_reductions()
        assert rel(x, oc.x) <= RTOL64
        assert rel(q, oc.q) <= RTOL64 and rel(spsi, oc.sse) <= RTOL64
        assert rel(tau, oc.tau) <= RTOL64 and rel(ch.beta0, oc.beta0) <= RTOL64


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("rho", [1.0, 0.95])
def test_graph_without_edges(G, orc, rho, shape):
    """Every site isolated (no column entries at all): x_i ~ N(y_i, 1 / lam)
    each sweep, q = 0, tau drawn from its prior."""
    n = 700
    rp = np.zeros(n + 1, dtype=np.int64)
    cl = np.zeros(0, dtype=np.int32)
    color = np.zeros(n, dtype=np.int32)
    y = np.cos(np.arange(n) * 0.21)
    g = G.Graph(row_ptr=rp, col_idx=cl, color=color, num_colors=1, rho=rho)
    assert g.components == n
    ch = G.Chain(g, y, seed=5)
    ch.set_tile(shape)
    oc = orc.Chain(rp, cl, color, y, rho=rho, seed=5)
    ch.sweep(10)
    oc.sweeps(10)
    x, tau, lam, _ = ch.get_state()
    q, sse = ch.last_reductions()
    assert q == 0.0 and oc.q == 0.0
    assert rel(x, oc.x) <= RTOL64 and rel(sse, oc.sse) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64
