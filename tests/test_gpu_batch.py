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


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_with_a_chunked_chain_of_more_slots_than_the_folded_end(G, prec):
    """A chunked chain with more partial slots (chunks) than every block of
    the next launch can sum commits every sweep, in a batch as on its own:
    the 1M-site Delaunay graph (over 2048 chunks) beside a lattice and a
    small chunked graph, standalone against batched, plain and captured,
    bit for bit."""
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    wl = inputs.delaunay_workload(1_000_000, data_seed=3, rho=0.95)
    color, k = G.greedy_coloring(wl["row_ptr"], wl["col"])
    big = (G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k,
                   rho=0.95), wl["y"])
    wls = [big] + [workloads(G)[i] for i in (2, 5)]
    solo = make_chains(G, wls, p, 300)
    mixed = make_chains(G, wls, p, 300)
    assert solo[0].tile[0] == 1
    for c in solo:
        c.sweep(7)
    batch = G.Batch(mixed)
    batch.sweep(4)
    batch.sweep(3, capture=True)
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


def test_full_512_instance_mix(G, orc):
    """The benchmark's batch: all 512 instances (lattices with side 32..512,
    Delaunay graphs with 1k..50k sites).  FP32: every chain of the batch is
    bitwise its standalone self.  FP64: sampled chains of the batch match the
    oracle after two sweeps."""
    mix = inputs.batch_mix(512, data_seed=4)
    graphs = []
    for wl in mix:
        if wl["kind"] == "lattice":
            graphs.append(G.Graph(lattice=(wl["rows"], wl["cols"], wl["stencil"])))
        else:
            wl["color"], wl["k"] = G.greedy_coloring(wl["row_ptr"], wl["col"])
            graphs.append(G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"],
                                  num_colors=wl["k"], rho=wl["rho"]))
    solo = [G.Chain(g, wl["y"], precision=G.FP32_ACC64, seed=1 + i, instance=i)
            for i, (g, wl) in enumerate(zip(graphs, mix))]
    for c in solo:
        c.sweep(3)
    mixed = [G.Chain(g, wl["y"], precision=G.FP32_ACC64, seed=1 + i, instance=i)
             for i, (g, wl) in enumerate(zip(graphs, mix))]
    G.Batch(mixed).sweep(3, capture=True)
    for a, b in zip(solo, mixed):
        xa, ta, la, _ = a.get_state()
        xb, tb, lb, _ = b.get_state()
        assert np.array_equal(xa, xb) and ta == tb and la == lb
    del solo, mixed
    picks = [0, 200, 256, 511]
    chains = [G.Chain(graphs[i], mix[i]["y"], seed=1 + i, instance=i) for i in range(512)]
    G.Batch(chains).sweep(2)
    for i in picks:
        wl = mix[i]
        if wl["kind"] == "lattice":
            rp, cl = inputs.lattice_csr(wl["rows"], wl["cols"], wl["stencil"])
        else:
            rp, cl = wl["row_ptr"], wl["col"]
        oc = orc.Chain(rp, cl, wl["color"], wl["y"], rho=wl["rho"], seed=1 + i, instance=i)
        oc.sweeps(2, nthreads=8)
        x, tau, lam, _ = chains[i].get_state()
        assert np.max(np.abs(x - oc.x)) <= 1e-12 * np.max(np.abs(oc.x))
        assert abs(tau / oc.tau - 1) <= 1e-12 and abs(lam / oc.lam - 1) <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_autotune_keeps_state_and_equality(G, prec):
    """gmrf_batch_autotune times the lattice tiles in both shapes without
    touching the chains' state, gives every lattice chain the faster shape,
    and the re-laid-out batch still ends where standalone sweeps end."""
    p = G.FP32_ACC64 if prec == "fp32" else G.FP64
    wls = workloads(G)
    chains = make_chains(G, wls, p, 300)
    twins = make_chains(G, wls, p, 300)
    batch = G.Batch(chains)
    batch.sweep(3, capture=True)
    for t in twins:
        t.sweep(3)
    before = [(c.get_state(), c.get_accumulators()) for c in chains]
    best, us = batch.autotune(reps=3)
    assert best in (0, 1) and us[0] > 0.0 and us[1] > 0.0
    assert best == (1 if us[1] < us[0] else 0)
    for c, (st, ps) in zip(chains, before):
        st2, ps2 = c.get_state(), c.get_accumulators()
        assert np.array_equal(st[0], st2[0]) and st[1:] == st2[1:]
        # one accumulated sweep so far (too few for posterior_stats' variance)
        assert np.array_equal(ps[0], ps2[0]) and np.array_equal(ps[1], ps2[1])
        assert ps[2] == ps2[2] == 1
    for c, t, (g, _) in zip(chains, twins, wls):
        if g.lattice is not None:
            assert c.tile[0] == best
            t.set_tile(best)
    batch.sweep(4, capture=True)
    batch.sweep(2)
    for t in twins:
        t.sweep(6)
    for c, t in zip(chains, twins):
        assert same(c, t)
    only_csr = G.Batch(make_chains(G, wls[5:], p, 900))
    assert only_csr.autotune(reps=1) == (-1, [0.0, 0.0])


@pytest.mark.parametrize("kinds", ["lattice", "csr", "mixed"])
def test_batch_workspace_is_the_footprint(G, kinds):
    """gmrf_batch_create accepts a workspace of exactly gmrf_batch_footprint
    bytes and refuses one byte less (lattice-only, general-only and mixed
    batches: the sizing builds the forced tile layouts only with lattices),
    and the autotuner's re-laid-out tables fit the same workspace."""
    import ctypes as C

    import torch

    wls = workloads(G)
    pick = {"lattice": wls[:5], "csr": wls[5:], "mixed": wls}[kinds]
    chains = make_chains(G, pick, G.FP32_ACC64, 7)
    L = G.lib()
    arr = (C.c_void_p * len(chains))(*[c.handle.value for c in chains])
    need = L.gmrf_batch_footprint(arr, len(chains))
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    assert L.gmrf_batch_create(arr, len(chains), C.c_void_p(ws.data_ptr()), need - 1, None,
                               C.byref(h)) == G.E_WORKSPACE
    assert L.gmrf_batch_create(arr, len(chains), C.c_void_p(ws.data_ptr()), need, None,
                               C.byref(h)) == G.OK
    best, us = C.c_int32(), (C.c_double * 2)()
    assert L.gmrf_batch_autotune(h, 2, None, C.byref(best), us) == G.OK
    assert (best.value == -1) == (kinds == "csr")
    assert L.gmrf_batch_sweep(h, 4, G.WITH_HYPER, None) == G.OK   # 2 past the burn-in
    torch.cuda.synchronize()
    assert L.gmrf_batch_destroy(h) == G.OK
    solo = make_chains(G, pick, G.FP32_ACC64, 7)
    for a, b in zip(solo, chains):
        a.set_tile(b.tile[0])          # the shape the autotuner gave the batched chain
        a.sweep(4)
        assert same(a, b)
