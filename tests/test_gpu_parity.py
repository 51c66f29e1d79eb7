"""GPU parity: the HIP sampler (through the C ABI) against the CPU oracle.

FP64 results must match the oracle within 1e-12 relative (max-norm over the
field, and per scalar for tau, lam, q, sse); FP32 results are compared with
the FP64 oracle at the stated accuracy (posterior-mean max abs error <= 1e-4
after 1000 sweeps).  Inputs are seeded and synthetic (see inputs.py).
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


def lattice_case(rows, cols, st, noise=0.1, data_seed=1):
    return inputs.lattice_workload(rows, cols, st, noise_sd=noise, data_seed=data_seed)


def csr_case(n, data_seed=3, rho=0.95):
    from paper_1702_05518_amd import gmrf

    wl = inputs.delaunay_workload(n, data_seed=data_seed, rho=rho)
    wl["color"], wl["k"] = gmrf.greedy_coloring(wl["row_ptr"], wl["col"])
    return wl


def gpu_graph(G, wl, force_csr=False):
    if wl["kind"] == "lattice" and not force_csr:
        return G.Graph(lattice=(wl["rows"], wl["cols"], wl["stencil"]), rho=wl["rho"])
    return G.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=wl["color"],
                   num_colors=wl["k"], rho=wl["rho"])


def pair(G, orc, wl, precision=None, seed=1, instance=0, burn_in=0, x0=None, force_csr=False,
         **prior):
    prec = G.FP64 if precision is None else precision
    g = gpu_graph(G, wl, force_csr)
    ch = G.Chain(g, wl["y"], precision=prec, seed=seed, instance=instance, burn_in=burn_in,
                 x0=x0, **prior)
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], rho=wl["rho"], seed=seed,
                   instance=instance, burn_in=burn_in, x0=x0, **prior)
    return g, ch, oc


LATTICES = [(64, 64, 4), (64, 64, 8), (150, 133, 4), (150, 133, 8), (1, 1, 8), (1, 77, 4),
            (77, 1, 8), (2, 3, 8), (129, 65, 8)]


@pytest.mark.parametrize("shape", [0, 1])
@pytest.mark.parametrize("rows,cols,st", LATTICES)
def test_lattice_one_sweep_from_injected_state(G, orc, rows, cols, st, shape):
    wl = lattice_case(rows, cols, st)
    n = rows * cols
    x0 = np.random.default_rng(n).normal(size=n) * 0.3 + 0.5
    g, ch, oc = pair(G, orc, wl, seed=7, instance=2)
    ch.set_tile(shape)
    ch.set_state(x0, 1.7, 60.0, 5)
    oc.set_state(x0, 1.7, 60.0, 5)
    ch.sweep(1, hyper=True)
    oc.sweeps(1, hyper=True)
    x, tau, lam, sw = ch.get_state()
    q, sse = ch.last_reductions()
    assert sw == 6
    assert rel(x, oc.x) <= RTOL64
    assert rel(q, oc.q) <= RTOL64 and rel(sse, oc.sse) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("rho", [1.0, 0.95])
def test_csr_one_sweep_from_injected_state(G, orc, rho, shape):
    wl = csr_case(3000, data_seed=5, rho=rho)
    n = wl["n"]
    x0 = np.random.default_rng(1).normal(size=n)
    g, ch, oc = pair(G, orc, wl, seed=11, instance=4)
    ch.set_tile(shape)
    ch.set_state(x0, 2.0, 25.0, 17)
    oc.set_state(x0, 2.0, 25.0, 17)
    ch.sweep(1)
    oc.sweeps(1)
    x, tau, lam, sw = ch.get_state()
    q, sse = ch.last_reductions()
    assert rel(x, oc.x) <= RTOL64
    assert rel(q, oc.q) <= RTOL64 and rel(sse, oc.sse) <= RTOL64
    assert rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64


def test_lattice_trajectory_64x64_fp64(G, orc):
    """64 x 64, 4 neighbours, checkerboard, FP64, 1000 sweeps with hyper draws:
    the field, tau and lam after every sweep, and the posterior mean /
    variance at the end."""
    wl = lattice_case(64, 64, 4)
    g, ch, oc = pair(G, orc, wl, seed=1)
    worst = 0.0
    for t in range(1000):
        ch.sweep(1)
        oc.sweeps(1)
        x, tau, lam, sw = ch.get_state()
        assert sw == t + 1
        worst = max(worst, rel(x, oc.x), rel(tau, oc.tau), rel(lam, oc.lam))
    assert worst <= RTOL64, worst
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 1000
    assert rel(mean, om) <= RTOL64
    assert np.max(np.abs(var - ov)) <= 1e-9 * np.max(np.abs(ov))


def oracle_trajectory(oc, sweeps, every=100, nthreads=8):
    """tau / lam after every sweep of the oracle and its field every `every`
    sweeps."""
    taus, lams, xs = np.empty(sweeps), np.empty(sweeps), {}
    for t in range(sweeps):
        oc.sweeps(1, nthreads=nthreads)
        taus[t], lams[t] = oc.tau, oc.lam
        if (t + 1) % every == 0:
            xs[t + 1] = oc.x.copy()
    return taus, lams, xs


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_csr_trajectory_delaunay_fp64(G, orc, shape):
    """The 15,000-site irregular workload for its 2000 sweeps in FP64: tau and
    lam after every sweep (device trace), the field every 100 sweeps, and the
    posterior mean / variance at the end, against the oracle at 1e-12."""
    wl = csr_case(15000, data_seed=3)
    g, ch, oc = pair(G, orc, wl, seed=3, burn_in=10)
    ch.set_tile(shape)
    ch.enable_trace(2000)
    taus, lams, xs = oracle_trajectory(oc, 2000)
    for t in range(20):
        ch.sweep(100, capture=True)
        x, tau, lam, sw = ch.get_state()
        assert sw == 100 * (t + 1)
        assert rel(x, xs[sw]) <= RTOL64, (sw, rel(x, xs[sw]))
    tr = ch.trace()
    assert rel(tr[:, 0], taus) <= RTOL64 and rel(tr[:, 1], lams) <= RTOL64
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 1990
    assert rel(mean, om) <= RTOL64
    assert np.max(np.abs(var - ov)) <= 1e-9 * np.max(np.abs(ov))


@pytest.mark.parametrize("st", [4, 8])
def test_lattice_path_equals_csr_path(G, orc, st):
    wl = lattice_case(97, 130, st)
    _, a, _ = pair(G, orc, wl, seed=5)
    gc = gpu_graph(G, wl, force_csr=True)
    b = G.Chain(gc, wl["y"], precision=G.FP64, seed=5)
    a.sweep(20)
    b.sweep(20)
    xa, ta, la, _ = a.get_state()
    xb, tb, lb, _ = b.get_state()
    assert rel(xa, xb) <= 1e-13 and rel(ta, tb) <= 1e-13 and rel(la, lb) <= 1e-13


def test_fp32_lattice_posterior_mean_against_fp64_oracle(G, orc):
    wl = lattice_case(64, 64, 8)
    g, ch, oc = pair(G, orc, wl, precision=G.FP32_ACC64, seed=2)
    ch.sweep(1000)
    oc.sweeps(1000)
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    _, tau, lam, _ = ch.get_state()
    assert nacc == 1000
    assert np.max(np.abs(mean - om)) <= 1e-4
    assert np.max(np.abs(var - ov)) <= 1e-4 * max(1.0, np.max(ov))
    assert rel(tau, oc.tau) <= 1e-3 and rel(lam, oc.lam) <= 1e-3


def test_fp32_csr_posterior_mean_against_fp64_oracle(G, orc):
    """The irregular 15,000-site workload in FP32 with FP64 accumulators for
    its 2000 sweeps against the FP64 oracle on the same seeds: posterior-mean
    max abs error within 1e-4 (the stated FP32 accuracy), the variance and the
    tau / lam trajectories (every sweep, device trace) reported and bounded."""
    wl = csr_case(15000, data_seed=3)
    g, ch, oc = pair(G, orc, wl, precision=G.FP32_ACC64, seed=4)
    ch.enable_trace(2000)
    ch.sweep(1000, capture=True)
    ch.sweep(1000, capture=True)
    taus, lams, _ = oracle_trajectory(oc, 2000, every=2000)
    mean, var, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    tr = ch.trace()
    assert nacc == 2000
    mean_err = np.max(np.abs(mean - om))
    var_err = np.max(np.abs(var - ov))
    print(f"15k FP32, 2000 sweeps: posterior mean max abs err {mean_err:.2e}, var {var_err:.2e}, "
          f"tau rel {rel(tr[:, 0], taus):.2e}, lam rel {rel(tr[:, 1], lams):.2e}")
    assert mean_err <= 1e-4
    assert var_err <= 1e-4 * max(1.0, np.max(ov))
    assert rel(tr[:, 0], taus) <= 1e-3 and rel(tr[:, 1], lams) <= 1e-3


def test_run_to_run_bitwise_and_capture(G, orc):
    wl = lattice_case(200, 190, 8)
    g = gpu_graph(G, wl)
    runs = []
    for capture in (False, False, True):
        ch = G.Chain(g, wl["y"], precision=G.FP32_ACC64, seed=9)
        if capture:
            for _ in range(3):
                ch.sweep(10, capture=True)
        else:
            ch.sweep(30)
        runs.append((ch.get_state(), ch.posterior_stats()))
    for other in runs[1:]:
        assert np.array_equal(runs[0][0][0], other[0][0])
        assert runs[0][0][1:] == other[0][1:]
        assert np.array_equal(runs[0][1][0], other[1][0])


def test_hyper_update_equals_fused_draw(G, orc):
    wl = csr_case(2000, data_seed=8)
    g = gpu_graph(G, wl)
    a = G.Chain(g, wl["y"], seed=3)
    b = G.Chain(g, wl["y"], seed=3)
    a.sweep(5)
    for _ in range(5):
        b.sweep(1, hyper=False)
        b.hyper_update()
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:]


def test_fixed_hyper_and_set_hyper(G, orc):
    wl = lattice_case(40, 50, 8)
    g, ch, oc = pair(G, orc, wl, seed=6)
    ch.set_hyper(3.0, 80.0)
    oc.set_state(oc.x, 3.0, 80.0, 0)
    ch.sweep(7, hyper=False)
    oc.sweeps(7, hyper=False)
    x, tau, lam, sw = ch.get_state()
    assert tau == 3.0 and lam == 80.0 and sw == 7
    assert rel(x, oc.x) <= RTOL64


def test_checkpoint_resume_bitwise(G, orc):
    wl = csr_case(2500, data_seed=9)
    g = gpu_graph(G, wl)
    full = G.Chain(g, wl["y"], seed=21, instance=3)
    full.sweep(12)
    part = G.Chain(g, wl["y"], seed=21, instance=3)
    part.sweep(5)
    x, tau, lam, sw = part.get_state()
    s1, s2, nacc = part.get_accumulators()
    res = G.Chain(g, wl["y"], seed=21, instance=3)
    res.set_state(x, tau, lam, sw)
    res.set_accumulators(s1, s2, nacc)
    res.sweep(7)
    a, b = full.get_state(), res.get_state()
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    assert np.array_equal(full.posterior_stats()[0], res.posterior_stats()[0])


def test_device_pointer_stats(G, orc):
    import torch

    wl = lattice_case(33, 47, 4)
    g, ch, oc = pair(G, orc, wl, seed=2)
    ch.sweep(9)
    m = torch.empty(wl["n"], dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    ch.posterior_stats_device(m, v)
    mean, var, _ = ch.posterior_stats()
    assert np.array_equal(m.cpu().numpy(), mean) and np.array_equal(v.cpu().numpy(), var)


@pytest.mark.parametrize("rho", [1.0, 0.9])
@pytest.mark.parametrize("shape", [0, 1, 2])
def test_isolated_sites_and_empty_color(G, orc, shape, rho):
    # 3 components (one isolated site) and a coloring that leaves color 2
    # empty; with rho < 1 the tau shape's rank is n minus the isolated sites
    rp, cl = inputs.edges_to_csr(6, [0, 1, 3], [1, 2, 4])
    color = np.array([0, 1, 0, 0, 1, 3], dtype=np.int32)
    y = np.array([0.1, 0.5, -0.2, 1.0, 0.3, -0.7])
    g = G.Graph(row_ptr=rp, col_idx=cl, color=color, num_colors=4, rho=rho)
    assert g.components == 3
    ch = G.Chain(g, y, seed=4)
    ch.set_tile(shape)
    oc = orc.Chain(rp, cl, color, y, seed=4, rho=rho)
    assert oc.rank == (3 if rho == 1.0 else 5)
    ch.sweep(25)
    oc.sweeps(25)
    x, tau, lam, _ = ch.get_state()
    assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64 and rel(lam, oc.lam) <= RTOL64


def test_chain_argument_errors(G):
    wl = lattice_case(8, 8, 4)
    g = gpu_graph(G, wl)
    with pytest.raises(G.GmrfError) as e:
        G.Chain(g, np.full(64, np.nan))
    assert e.value.status == G.E_INVALID_ARG
    with pytest.raises(G.GmrfError):
        G.Chain(g, wl["y"], tau0=-1.0)
    with pytest.raises(G.GmrfError):
        G.Chain(g, wl["y"], b_tau=0.0)
    ch = G.Chain(g, wl["y"])
    with pytest.raises(G.GmrfError):
        ch.hyper_update()          # no completed sweep
    with pytest.raises(G.GmrfError):
        ch.set_hyper(0.0, 1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lattice_checkpoint_resume_and_burn_in(G, orc, prec):
    """Reading the state and the sums part way, and resuming a new chain from
    them, continues the same chain exactly, across the burn-in boundary."""
    wl = lattice_case(70, 90, 8)
    p = G.FP64 if prec == "fp64" else G.FP32_ACC64
    g = gpu_graph(G, wl)
    full = G.Chain(g, wl["y"], precision=p, seed=13, burn_in=3)
    full.sweep(11)
    part = G.Chain(g, wl["y"], precision=p, seed=13, burn_in=3)
    part.sweep(6)
    x, tau, lam, sw = part.get_state()
    s1, s2, nacc = part.get_accumulators()
    assert nacc == 3
    res = G.Chain(g, wl["y"], precision=p, seed=13, burn_in=3)
    res.set_state(x, tau, lam, sw)
    res.set_accumulators(s1, s2, nacc)
    res.sweep(5)
    part.sweep(5)                  # continuing after get_accumulators
    a, b, c = full.get_state(), res.get_state(), part.get_state()
    assert np.array_equal(a[0], b[0]) and a[1:] == b[1:]
    assert np.array_equal(a[0], c[0]) and a[1:] == c[1:]
    ma, va, na = full.posterior_stats()
    for other in (res, part):
        mb, vb, nb = other.posterior_stats()
        assert na == nb == 8
        assert np.array_equal(ma, mb) and np.array_equal(va, vb)
    if prec == "fp64":
        oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], wl["y"], seed=13, burn_in=3)
        oc.sweeps(11)
        om, ov = oc.stats()
        assert rel(ma, om) <= RTOL64
        s1f, s2f, nf = full.get_accumulators()
        assert nf == 8 and rel(s1f, oc.s1) <= RTOL64 and rel(s2f, oc.s2) <= RTOL64


@pytest.mark.parametrize("kind", ["lattice", "csr", "csr_one_block", "csr_chunked"])
def test_sweep_timed_equals_sweep(G, orc, kind):
    wl = lattice_case(100, 120, 8) if kind == "lattice" else csr_case(4000, data_seed=2)
    g = gpu_graph(G, wl)
    a = G.Chain(g, wl["y"], seed=4)
    b = G.Chain(g, wl["y"], seed=4)
    if kind.startswith("csr"):
        shape = {"csr": 0, "csr_one_block": 2, "csr_chunked": 1}[kind]
        a.set_tile(shape)
        b.set_tile(shape)
    a.sweep(6)
    ms, span = b.sweep_timed(6, span=True)
    if kind == "csr_one_block":     # one launch carries the sweeps and their draws
        assert b.tile[0] == 2 and 0.0 < ms == span
    else:
        assert 0.0 < ms < span
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:]
    assert b.sweep_timed(0, span=True) == (0.0, 0.0)


@pytest.mark.parametrize("prec,n", [("fp64", 5000), ("fp32", 5000), ("fp64", 15000),
                                    ("fp32", 30000)])
@pytest.mark.parametrize("capture", [False, True])
def test_csr_one_block_is_bitwise_color_passes(G, orc, prec, n, capture):
    """The one-block kernel (field in LDS) repeats the color-pass kernels'
    operations in their order, FP64 partial sums and draws included: the
    chains stay bitwise equal, with and without capture, across calls, up to
    the largest fields that fit (15,000 FP64 and 30,000 FP32 sites)."""
    precision = G.FP64 if prec == "fp64" else G.FP32_ACC64
    wl = csr_case(n, data_seed=8, rho=0.95)
    g = gpu_graph(G, wl)
    a = G.Chain(g, wl["y"], precision=precision, seed=6, burn_in=3)
    b = G.Chain(g, wl["y"], precision=precision, seed=6, burn_in=3)
    a.set_tile(0)
    b.set_tile(2)
    assert a.tile[0] == 0 and b.tile[0] == 2
    for n in (1, 7, 12):
        a.sweep(n, capture=capture)
        b.sweep(n, capture=capture)
    a.sweep(5, hyper=False)
    b.sweep(5, hyper=False)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[1:] == sb[1:]
    assert a.last_reductions() == b.last_reductions()
    ma, va, na = a.posterior_stats()
    mb, vb, nb = b.posterior_stats()
    assert na == nb == 22 and np.array_equal(ma, mb) and np.array_equal(va, vb)


def test_library_first_load_order(G):
    """A program that uses the library before it touches torch (a lattice
    graph needs no device memory, so the first chain is the first device
    call) still finds the device: the binding lets torch bring up the HIP
    runtime before loading the library.  Fresh process, so that nothing has
    initialised the device yet."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prog = ("import numpy as np\n"
            "from paper_1702_05518_amd import gmrf\n"
            "g = gmrf.Graph(lattice=(32, 32, 4))\n"
            "ch = gmrf.Chain(g, np.zeros(32 * 32), seed=1)\n"
            "ch.sweep(5)\n"
            "assert ch.get_state()[3] == 5\n"
            "print('first-load ok')\n")
    r = subprocess.run([sys.executable, "-c", prog], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "first-load ok" in r.stdout, r.stderr[-2000:]


def test_numeric_failure_is_reported_through_the_status_word(G, orc):
    """A field so rough that x'(D - W)x overflows to inf: the tau draw at rate
    b + q/2 = inf is not a positive finite number, so the device sets its
    status word (the kernels still end normally) and the next synchronising
    call returns GMRF_E_NUMERIC; the oracle refuses the same draw."""
    rows = cols = 16
    wl = lattice_case(rows, cols, 4)
    r, c = np.divmod(np.arange(rows * cols), cols)
    y = np.where((r + c) % 2 == 0, 1e160, -1e160)
    g = G.Graph(lattice=(rows, cols, 4))
    ch = G.Chain(g, y, precision=G.FP64, seed=1, lam0=1e6)
    ch.sweep(1)
    with pytest.raises(G.GmrfError) as e:
        ch.get_state()
    assert e.value.status == G.E_NUMERIC
    with pytest.raises(G.GmrfError):
        ch.posterior_stats()
    oc = orc.Chain(wl["row_ptr"], wl["col"], wl["color"], y, seed=1, lam0=1e6)
    with pytest.raises(FloatingPointError):
        oc.sweeps(1)



@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_csr_chunked_shape_changes_mid_chain(G, orc, prec):
    """The chunked one-launch sweep (shape 1) keeps the field in the buffer of
    the sweep parity, the other shapes in one buffer: switching shapes after
    an odd number of sweeps moves it, so the chain goes on exactly as the
    oracle's, with plain and captured sweeps."""
    precision = G.FP64 if prec == "fp64" else G.FP32_ACC64
    wl = csr_case(9000, data_seed=6, rho=0.95)
    g, ch, oc = pair(G, orc, wl, precision=precision, seed=12, burn_in=4)
    ref = G.Chain(g, wl["y"], precision=precision, seed=12, burn_in=4)
    ref.set_tile(1)
    steps = [(0, 3, False), (1, 5, True), (2, 1, False), (1, 2, False), (0, 4, True)]
    for shape, n, cap in steps:
        ch.set_tile(shape)
        assert ch.tile[0] == shape
        ch.sweep(n, capture=cap)
        ref.sweep(n)
        oc.sweeps(n, nthreads=8)
        x, tau, lam, _ = ch.get_state()
        if prec == "fp64":
            assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64, (shape, n)
        else:
            assert np.max(np.abs(x - oc.x)) <= 1e-4
    m, v, nacc = ch.posterior_stats()
    om, ov = oc.stats()
    assert nacc == 15 - 4
    if prec == "fp64":
        assert rel(m, om) <= RTOL64
    # the chunked chain swept in one shape ends in the same state as the
    # oracle's too (the same site values, whatever the shape)
    xr, _, _, _ = ref.get_state()
    if prec == "fp64":
        assert rel(xr, oc.x) <= RTOL64


def test_csr_autotune_leaves_state_unchanged(G, orc):
    wl = csr_case(6000, data_seed=7, rho=0.95)
    g, ch, oc = pair(G, orc, wl, seed=14)
    twin = G.Chain(g, wl["y"], seed=14)
    ch.set_tile(1)
    ch.sweep(3)                         # odd: the field sits in the second buffer
    twin.sweep(3)
    before = ch.get_state(), ch.get_accumulators(), ch.last_reductions()
    best, us = ch.autotune(reps=4)
    after = ch.get_state(), ch.get_accumulators(), ch.last_reductions()
    assert best in (0, 1, 2) and all(u > 0 for u in us), us
    assert ch.tile[0] == best
    assert np.array_equal(before[0][0], after[0][0]) and before[0][1:] == after[0][1:]
    assert np.array_equal(before[1][0], after[1][0]) and np.array_equal(before[1][1], after[1][1])
    assert before[1][2] == after[1][2] and before[2] == after[2]
    ch.sweep(5)
    twin.sweep(5)
    oc.sweeps(8)
    for c in (ch, twin):
        x, tau, lam, _ = c.get_state()
        assert rel(x, oc.x) <= RTOL64 and rel(tau, oc.tau) <= RTOL64


@pytest.mark.gpu
def test_posterior_stats_needs_two_accumulated_sweeps(G):
    """The host form of gmrf_posterior_stats refuses N < 2 accumulated sweeps
    (burn-in not yet passed, or one sweep); the device form computes the
    values as written (N = 1: the variance divides by zero)."""
    import torch
    wl = lattice_case(16, 16, 4)
    g = G.Graph(lattice=(16, 16, 4))
    ch = G.Chain(g, wl["y"], precision=G.FP64, seed=2, burn_in=5)
    ch.sweep(5)                                    # all burn-in: N = 0
    with pytest.raises(G.GmrfError) as e:
        ch.posterior_stats()
    assert e.value.status == G.E_INVALID_ARG and "accumulated" in G.last_error()
    ch.sweep(1)                                    # N = 1
    with pytest.raises(G.GmrfError):
        ch.posterior_stats()
    mean = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    var = torch.empty_like(mean)
    ch.posterior_stats_device(mean, var)
    torch.cuda.synchronize()
    s1, _, nacc = ch.get_accumulators()
    assert nacc == 1
    assert np.array_equal(mean.cpu().numpy(), s1)       # a lattice: no permutation
    assert not np.isfinite(var.cpu().numpy()).any()
    ch.sweep(1)                                    # N = 2
    m, v, n = ch.posterior_stats()
    assert n == 2 and np.isfinite(m).all() and np.isfinite(v).all()
