"""Lattice tile shapes and their autotuner, and the two general-graph shapes
(through the C ABI).

Both shapes must reproduce the CPU oracle (FP64 within 1e-12 relative over
many sweeps: the shapes differ only in how the FP64 reductions are grouped),
the autotuner must leave the chain's state untouched, and a batch that mixes
shapes must equal standalone sweeps bit for bit.
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


def test_default_shapes(G):
    big = G.Chain(G.Graph(lattice=(2048, 2048, 8)), np.zeros(2048 * 2048),
                  precision=G.FP32_ACC64)
    small = G.Chain(G.Graph(lattice=(200, 300, 4)), np.zeros(60000))
    assert big.tile == (0, 64, 64, 512)
    assert small.tile == (1, 32, 32, 256)
    wl = inputs.delaunay_workload(500, data_seed=2)
    color, k = G.greedy_coloring(wl["row_ptr"], wl["col"])
    csr = G.Chain(G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k,
                          rho=0.95), wl["y"])
    assert csr.tile == (1, 0, 0, 256)          # chunks, one launch per sweep (the default)
    csr.set_tile(0)
    assert csr.tile == (0, 0, 0, 256)          # one launch per color
    csr.set_tile(2)
    assert csr.tile == (2, 0, 0, 512)          # the field fits in LDS: one block
    with pytest.raises(G.GmrfError):
        small.set_tile(2)
    best, us = csr.autotune(reps=2)
    assert csr.tile[0] == best and all(u > 0 for u in us)
    big_wl = inputs.delaunay_workload(20000, data_seed=3)
    bcolor, bk = G.greedy_coloring(big_wl["row_ptr"], big_wl["col"])
    bg = G.Graph(row_ptr=big_wl["row_ptr"], col_idx=big_wl["col"], color=bcolor, num_colors=bk,
                 rho=0.95)
    # 20,000 sites: the chunked one-launch sweep by default; for the one-block
    # shape FP64 (160 KB) does not fit in LDS, FP32 (80 KB) does
    c64 = G.Chain(bg, big_wl["y"])
    c32 = G.Chain(bg, big_wl["y"], precision=G.FP32_ACC64)
    assert c64.tile[0] == 1 and c32.tile[0] == 1
    with pytest.raises(G.GmrfError):
        c64.set_tile(2)
    c32.set_tile(2)
    assert c32.tile == (2, 0, 0, 512)


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("rows,cols,st", [(200, 131, 8), (97, 160, 4)])
def test_shape_trajectory_matches_oracle(G, orc, rows, cols, st, shape):
    wl = inputs.lattice_workload(rows, cols, st)
    ch = G.Chain(G.Graph(lattice=(rows, cols, st)), wl["y"], seed=4, burn_in=20)
    ch.set_tile(shape)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=4, burn_in=20)
    ch.sweep(100, capture=True)
    oc.sweeps(100)
    x, tau, lam, sw = ch.get_state()
    assert sw == 100
    assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64
    m, v, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 80 and rel(m, om) <= RTOL64 and rel(v, ov) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_leaves_state_unchanged(G, prec):
    p = G.FP64 if prec == "fp64" else G.FP32_ACC64
    wl = inputs.lattice_workload(300, 257, 8)
    g = G.Graph(lattice=(300, 257, 8))
    a = G.Chain(g, wl["y"], precision=p, seed=6)
    b = G.Chain(g, wl["y"], precision=p, seed=6)
    for ch in (a, b):
        ch.sweep(7)
    before = a.get_state(), a.get_accumulators(), a.last_reductions()
    best, us = a.autotune(reps=5)
    after = a.get_state(), a.get_accumulators(), a.last_reductions()
    assert best in (0, 1) and len(us) == 3 and all(u > 0 for u in us[:2]) and us[2] == 0.0
    assert a.tile[0] == best
    assert np.array_equal(before[0][0], after[0][0]) and before[0][1:] == after[0][1:]
    assert np.array_equal(before[1][0], after[1][0]) and np.array_equal(before[1][1], after[1][1])
    assert before[1][2] == after[1][2] and before[2] == after[2]
    # the chain continues exactly as an untuned one on the same shape
    b.set_tile(best)
    a.sweep(5)
    b.sweep(5)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


def test_batch_with_mixed_shapes_is_bitwise_standalone(G):
    wls = [inputs.lattice_workload(s, s + 9, st, data_seed=s)
           for s, st in ((70, 4), (130, 8), (45, 8), (260, 4))]
    def make():
        out = []
        for i, wl in enumerate(wls):
            ch = G.Chain(G.Graph(lattice=(wl["rows"], wl["cols"], wl["stencil"])), wl["y"],
                         precision=G.FP32_ACC64, seed=20 + i)
            ch.set_tile(i % 2)
            out.append(ch)
        return out
    alone, batched = make(), make()
    for ch in alone:
        ch.sweep(25)
    G.Batch(batched).sweep(25, capture=True)
    for a, b in zip(alone, batched):
        xa, ta, la, _ = a.get_state()
        xb, tb, lb, _ = b.get_state()
        assert np.array_equal(xa, xb) and ta == tb and la == lb


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("rows,cols,st,intercept", [(50, 50, 8, True), (64, 64, 4, False),
                                                     (17, 40, 8, False), (1, 1, 8, False)])
def test_persistent_shape_is_bitwise_shape0(G, orc, prec, rows, cols, st, intercept):
    """Shape 2 (one launch per gmrf_sweep call) gives bit for bit the state,
    accumulators, reductions and trace of shape 0, plain and captured, across
    the burn-in boundary; FP64 also matches the oracle."""
    p = G.FP64 if prec == "fp64" else G.FP32_ACC64
    wl = inputs.lattice_workload(rows, cols, st, data_seed=rows + cols)
    kw = dict(precision=p, seed=9, burn_in=5, intercept=intercept)
    g = G.Graph(lattice=(rows, cols, st))
    a = G.Chain(g, wl["y"], **kw)
    b = G.Chain(g, wl["y"], **kw)
    a.set_tile(0)
    b.set_tile(2)
    for ch in (a, b):
        ch.enable_trace(64)
        ch.sweep(3)
        ch.sweep(7, capture=True)
        ch.sweep(7, capture=True)
        ch.sweep(1)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:] and sb[3] == 18
    ma, va, na = a.posterior_stats()
    mb, vb, nb = b.posterior_stats()
    assert na == nb == 13 and np.array_equal(ma, mb) and np.array_equal(va, vb)
    assert a.last_reductions() == b.last_reductions() and a.beta0 == b.beta0
    assert np.array_equal(a.trace(), b.trace(), equal_nan=True)
    if prec == "fp64":
        oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=9, burn_in=5,
                       intercept=intercept)
        oc.sweeps(18)
        assert rel(sb[0], oc.x) <= RTOL64 and rel(sb[1], oc.tau) <= RTOL64


def test_persistent_shape_rules_and_autotune(G):
    wl = inputs.lattice_workload(50, 50, 8)
    g = G.Graph(lattice=(50, 50, 8))
    ch = G.Chain(g, wl["y"], seed=3)
    ch.sweep(4)
    before = ch.get_state(), ch.get_accumulators(), ch.last_reductions()
    best, us = ch.autotune(reps=20)
    after = ch.get_state(), ch.get_accumulators(), ch.last_reductions()
    assert len(us) == 3 and all(u > 0 for u in us) and best in (0, 1, 2)
    assert np.array_equal(before[0][0], after[0][0]) and before[0][1:] == after[0][1:]
    assert np.array_equal(before[1][0], after[1][0]) and before[1][2] == after[1][2]
    assert before[2] == after[2]
    big = G.Chain(G.Graph(lattice=(65, 64, 4)), np.zeros(65 * 64))
    with pytest.raises(G.GmrfError):
        big.set_tile(2)
    b2, us2 = big.autotune(reps=3)
    assert us2[2] == 0.0 and b2 in (0, 1)
    # a shape-2 chain batches as shape 0: bitwise equal to standalone shape 2
    a = G.Chain(g, wl["y"], seed=5)
    b = G.Chain(g, wl["y"], seed=5)
    a.set_tile(2)
    b.set_tile(2)
    a.sweep(6)
    G.Batch([b]).sweep(6)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["lattice8_b0", "lattice4", "csr"])
def test_one_block_long_call_is_bitwise(G, orc, kind, prec):
    """One call of 300 sweeps in a one-block kernel (shape 2), which draws
    the rate-free parts of the hyperparameter draws 128 sweeps at a time
    ahead of the sweeps (so the call refills them twice, the last time for
    44 sweeps), ends bitwise where 300 separate sweeps of the multi-launch
    shape end; FP64 also against the oracle."""
    p = G.FP64 if prec == "fp64" else G.FP32_ACC64
    if kind == "csr":
        wl = inputs.delaunay_workload(2000, data_seed=9, rho=0.95)
        wl["color"], wl["k"] = G.greedy_coloring(wl["row_ptr"], wl["col"])
        g = G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"],
                    num_colors=wl["k"], rho=0.95)
        kw = {}
    else:
        st = 8 if kind == "lattice8_b0" else 4
        side = 50 if st == 8 else 64
        wl = inputs.lattice_workload(side, side, st)
        g = G.Graph(lattice=(side, side, st))
        kw = {"intercept": True} if st == 8 else {}
    a = G.Chain(g, wl["y"], precision=p, seed=12, burn_in=40, **kw)
    b = G.Chain(g, wl["y"], precision=p, seed=12, burn_in=40, **kw)
    a.set_tile(2)
    b.set_tile(0)
    a.sweep(300)
    for _ in range(300):
        b.sweep(1)
    sa, sb = a.get_state(), b.get_state()
    assert sa[3] == sb[3] == 300
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:]
    ma, va, na = a.posterior_stats()
    mb, vb, nb = b.posterior_stats()
    assert na == nb == 260 and np.array_equal(ma, mb) and np.array_equal(va, vb)
    if p == G.FP64:
        rho = 0.95 if kind == "csr" else 1.0
        oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], rho=rho, seed=12,
                       burn_in=40, **kw)
        oc.sweeps(300)
        x, tau, lam, _ = a.get_state()
        assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64
