"""Batched sweeps: many independent chains advanced by shared launches.

Every chain of a batch must end bit for bit where the same chain ends when
swept on its own (which the parity tests tie to the oracle), for lattices of
both stencils (ragged sizes included) and general graphs with different
color counts, in both precisions, with plain launches and a captured graph.
"""
import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05518_amd import gmrf

    gmrf.lib()
    return gmrf


def workloads(G):
    out = []
    for rows, cols, st in [(64, 64, 4), (33, 200, 4), (130, 70, 8), (5, 7, 8), (97, 97, 4)]:
        wl = inputs.lattice_workload(rows, cols, st, data_seed=rows)
        out.append((G.Graph(lattice=(rows, cols, st)), wl["y"]))
    for n, ds in [(3000, 1), (800, 2), (12000, 3)]:
        wl = inputs.delaunay_workload(n, data_seed=ds, rho=0.95)
        color, k = G.greedy_coloring(wl["row_ptr"], wl["col"])
        out.append((G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k,
                            rho=0.95), wl["y"]))
    return out


def make_chains(G, wls, prec, seed0):
    return [G.Chain(g, y, precision=prec, seed=seed0 + i, instance=i, burn_in=2)
            for i, (g, y) in enumerate(wls)]


def same(a, b):
    sa, sb = a.get_state(), b.get_state()
    ma, va, na = a.posterior_stats()
    mb, vb, nb = b.posterior_stats()
    return (np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:] and np.array_equal(ma, mb)
            and np.array_equal(va, vb) and na == nb)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("capture", [False, True])
def test_batch_equals_standalone(G, prec, capture):
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    wls = workloads(G)
    solo = make_chains(G, wls, p, 100)
    mixed = make_chains(G, wls, p, 100)
    for c in solo:
        c.sweep(9)
    batch = G.Batch(mixed)
    if capture:
        for _ in range(3):
            batch.sweep(3, capture=True)
    else:
        batch.sweep(9)
    for a, b in zip(solo, mixed):
        assert same(a, b)


def test_batch_subsets_and_fixed_hyper(G):
    wls = workloads(G)[:4]
    solo = make_chains(G, wls, G.FP32_ACC64, 7)
    mixed = make_chains(G, wls, G.FP32_ACC64, 7)
    for c in solo:
        c.sweep(4, hyper=False)
    G.Batch(mixed[:2]).sweep(4, hyper=False)
    G.Batch(mixed[2:]).sweep(4, hyper=False)
    for a, b in zip(solo, mixed):
        assert same(a, b)
        assert a.get_state()[1] == 1.0


def test_batch_errors(G):
    wls = workloads(G)[:2]
    a = make_chains(G, wls, G.FP64, 1)
    b = make_chains(G, wls, G.FP32_ACC64, 1)
    with pytest.raises(G.GmrfError):
        G.Batch([a[0], a[0]])          # repeated chain
    with pytest.raises(G.GmrfError):
        G.Batch([a[0], b[1]])          # mixed precision
    with pytest.raises(G.GmrfError):
        G.Batch([])
