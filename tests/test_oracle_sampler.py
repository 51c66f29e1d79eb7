"""Pins for the oracle's sampler, each against something other than itself.

* The one-sweep map against dense linear algebra of the full conditional
  (Sec. 2.2: x | y ~ N(Qp^{-1} b, Qp^{-1})) applied color by color
  (Sec. 2.3, Algorithm 1), written here from the dense matrix Qp.
* Zero noise turns the sweep into colored Gauss-Seidel for Qp x = b, whose
  fixed point is numpy.linalg.solve (the Gibbs / Gauss-Seidel view cited in
  Sec. 2.1).
* k = n colors is single-site Gibbs (Sec. 2.3).
* The stationary law N(Qp^{-1} b, Qp^{-1}) and the exact finite-t moments of
  the affine-Gaussian sweep map, on tiny graphs.
* Conjugate Gamma conditionals of tau and lam (Sec. 3.1) and a Geweke joint
  "getting it right" test of the whole kernel with proper priors (Sec. 3.2
  proper CAR).
* Greedy coloring (supplementary greedy algorithm) equals first-fit in index
  order; colorings are proper (Sec. 2.3).
"""
import numpy as np
import pytest
from scipy import stats
from scipy.sparse.csgraph import connected_components
import scipy.sparse as sp

from paper_1702_05518_amd import inputs


# --------------------------------------------------------------------------
# dense helpers (written from the definitions, independent of the oracle)
# --------------------------------------------------------------------------
def dense_W(row_ptr, col):
    n = row_ptr.size - 1
    W = np.zeros((n, n))
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            W[i, col[e]] = 1.0
    return W


def dense_Qp(row_ptr, col, tau, lam, rho):
    W = dense_W(row_ptr, col)
    D = np.diag(W.sum(axis=1))
    return tau * (D - rho * W) + lam * np.eye(W.shape[0])


def tiny_graphs():
    out = []
    for st in (4, 8):
        rp, cl = inputs.lattice_csr(4, 4, st)
        color, k = inputs.lattice_coloring(4, 4, st)
        out.append((f"lat4x4s{st}", rp, cl, color))
    rp, cl = inputs.lattice_csr(3, 5, 8)
    color, k = inputs.lattice_coloring(3, 5, 8)
    out.append(("lat3x5s8", rp, cl, color))
    rp, cl = inputs.path_graph(5)
    out.append(("path5", rp, cl, (np.arange(5) % 2).astype(np.int32)))
    _, rp, cl = inputs.delaunay_graph(30, data_seed=7)
    out.append(("delaunay30", rp, cl, None))
    return out


def graph_case(orc, name, rp, cl, color):
    if color is None:
        color, _ = orc.greedy_coloring(rp, cl)
    return rp, cl, color


GRAPHS = tiny_graphs()
IDS = [g[0] for g in GRAPHS]


# --------------------------------------------------------------------------
# colorings and graph utilities
# --------------------------------------------------------------------------
def first_fit(row_ptr, col):
    n = row_ptr.size - 1
    color = -np.ones(n, dtype=np.int64)
    for i in range(n):
        used = {color[j] for j in col[row_ptr[i]:row_ptr[i + 1]] if color[j] >= 0}
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def proper(row_ptr, col, color):
    src = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    return not np.any(color[src] == color[col])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_equals_first_fit_and_is_proper(orc, seed):
    graphs = []
    _, rp, cl = inputs.delaunay_graph(300, data_seed=seed)
    graphs.append((rp, cl))
    rng = np.random.default_rng(seed)
    n = 200
    ei = rng.integers(0, n, 600)
    ej = rng.integers(0, n, 600)
    graphs.append(inputs.edges_to_csr(n, ei, ej))
    graphs.append(inputs.lattice_csr(7, 9, 8))
    for rp, cl in graphs:
        color, k = orc.greedy_coloring(rp, cl)
        assert proper(rp, cl, color)
        assert np.array_equal(color, first_fit(rp, cl))
        assert k == color.max() + 1


def test_greedy_on_lattice_and_planar_color_counts(orc):
    rp, cl = inputs.lattice_csr(16, 16, 4)
    color, k = orc.greedy_coloring(rp, cl)
    assert k == 2 and np.array_equal(color, inputs.lattice_coloring(16, 16, 4)[0])
    _, rp, cl = inputs.delaunay_graph(15000, data_seed=3)
    color, k = orc.greedy_coloring(rp, cl)
    assert proper(rp, cl, color)
    assert 4 <= k <= 8


@pytest.mark.parametrize("st", [4, 8])
def test_lattice_colorings_are_proper(st):
    for rows, cols in [(1, 1), (1, 7), (5, 5), (6, 9), (64, 64)]:
        rp, cl = inputs.lattice_csr(rows, cols, st)
        color, k = inputs.lattice_coloring(rows, cols, st)
        assert proper(rp, cl, color)
        W = dense_W(rp, cl) if rows * cols <= 100 else None
        if W is not None:
            assert np.array_equal(W, W.T)


def test_components(orc):
    rng = np.random.default_rng(5)
    for n, m in [(1, 0), (10, 3), (100, 60), (300, 400)]:
        ei = rng.integers(0, n, m)
        ej = rng.integers(0, n, m)
        rp, cl = inputs.edges_to_csr(n, ei, ej)
        A = sp.csr_matrix((np.ones(cl.size), cl, rp), shape=(n, n))
        ref = connected_components(A, directed=False)[0]
        assert orc.components(rp, cl) == ref


# --------------------------------------------------------------------------
# the sweep map
# --------------------------------------------------------------------------
def dense_sweep(Qp, b, x, color, z):
    """Algorithm 1 from the dense full conditional: site i of color c gets
    (b_i - sum_{j != i} Qp_ij x_j) / Qp_ii + z_i / sqrt(Qp_ii)."""
    x = x.copy()
    for c in range(color.max() + 1):
        for i in np.flatnonzero(color == c):
            off = Qp[i] @ x - Qp[i, i] * x[i]
            x[i] = (b[i] - off) / Qp[i, i] + z[i] / np.sqrt(Qp[i, i])
    return x


@pytest.mark.parametrize("rho", [1.0, 0.9])
@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_one_sweep_equals_dense_conditional(orc, gi, rho):
    name, rp, cl, color = GRAPHS[gi]
    rp, cl, color = graph_case(orc, name, rp, cl, color)
    n = rp.size - 1
    rng = np.random.default_rng(gi)
    y = rng.normal(size=n)
    x0 = rng.normal(size=n)
    tau, lam = 1.7, 0.6
    ch = orc.Chain(rp, cl, color, y, rho=rho, tau0=tau, lam0=lam, seed=9, instance=3, x0=x0)
    ch.set_state(x0, tau, lam, sweep=11)
    ch.sweeps(1, hyper=False)
    z = orc.site_normals(9, 11, 3, n)
    ref = dense_sweep(dense_Qp(rp, cl, tau, lam, rho), lam * y, x0, color, z)
    assert np.max(np.abs(ch.x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    assert ch.sweep_count == 12 and ch.tau == tau and ch.lam == lam


@pytest.mark.parametrize("gi", range(len(GRAPHS)), ids=IDS)
def test_zero_noise_is_colored_gauss_seidel(orc, gi):
    name, rp, cl, color = GRAPHS[gi]
    rp, cl, color = graph_case(orc, name, rp, cl, color)
    n = rp.size - 1
    rng = np.random.default_rng(100 + gi)
    y = rng.normal(size=n)
    tau, lam, rho = 2.0, 0.5, 1.0
    Qp = dense_Qp(rp, cl, tau, lam, rho)
    b = lam * y
    ch = orc.Chain(rp, cl, color, y, rho=rho, tau0=tau, lam0=lam)
    # first iterates equal a textbook Gauss-Seidel in color order
    xg = np.zeros(n)
    for _ in range(3):
        ch.sweeps(1, hyper=False, zero_noise=True)
        xg = dense_sweep(Qp, b, xg, color, np.zeros(n))
        assert np.max(np.abs(ch.x - xg)) <= 1e-13 * max(1.0, np.max(np.abs(xg)))
    ch.sweeps(3000, hyper=False, zero_noise=True)
    ref = np.linalg.solve(Qp, b)
    assert np.max(np.abs(ch.x - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_k_equals_n_is_single_site(orc):
    # single-site Gibbs = chromatic Gibbs with one color per site (Sec. 2.3)
    rp, cl = inputs.lattice_csr(4, 5, 8)
    n = 20
    rng = np.random.default_rng(1)
    y = rng.normal(size=n)
    tau, lam = 1.3, 2.1
    ch = orc.Chain(rp, cl, np.arange(n, dtype=np.int32), y, tau0=tau, lam0=lam, seed=4)
    ch.sweeps(3, hyper=False)
    x = np.zeros(n)
    for t in range(3):
        for i in range(n):        # sequential scalar draws, site by site
            s = 0.0
            for e in range(rp[i], rp[i + 1]):
                s += x[cl[e]]
            Q = tau * float(rp[i + 1] - rp[i]) + lam
            m = (lam * y[i] + tau * 1.0 * s) / Q
            x[i] = m + orc.normal(4, i, t, 0, 0) / np.sqrt(Q)
    assert np.array_equal(ch.x, x)


def test_visit_order_and_threads_do_not_matter(orc):
    _, rp, cl = inputs.delaunay_graph(500, data_seed=11)
    color, k = orc.greedy_coloring(rp, cl)
    n = rp.size - 1
    y = np.random.default_rng(2).normal(size=n)
    a = orc.Chain(rp, cl, color, y, rho=0.95, seed=3).sweeps(5)
    perm = np.random.default_rng(3).permutation(n)
    b = orc.Chain(rp, cl, color, y, rho=0.95, seed=3).sweeps(5, visit=perm)
    c = orc.Chain(rp, cl, color, y, rho=0.95, seed=3).sweeps(5, nthreads=4)
    for other in (b, c):
        assert np.array_equal(a.x, other.x)
        assert a.tau == other.tau and a.lam == other.lam


@pytest.mark.parametrize("rho", [1.0, 0.95, 0.3])
def test_quadratic_form_matches_dense(orc, rho):
    _, rp, cl = inputs.delaunay_graph(60, data_seed=1)
    color, k = orc.greedy_coloring(rp, cl)
    n = rp.size - 1
    rng = np.random.default_rng(4)
    y = rng.normal(size=n)
    x = rng.normal(size=n) + 3.0
    ch = orc.Chain(rp, cl, color, y, rho=rho)
    q, sse = ch.quadratic_terms(x)
    W = dense_W(rp, cl)
    R = np.diag(W.sum(1)) - rho * W
    assert abs(q - x @ R @ x) <= 1e-13 * abs(x @ R @ x)
    assert abs(sse - np.sum((y - x) ** 2)) <= 1e-13 * sse


def test_rank_of_intrinsic_prior(orc):
    rp, cl = inputs.lattice_csr(4, 4, 4)
    color, _ = inputs.lattice_coloring(4, 4, 4)
    assert orc.Chain(rp, cl, color, np.zeros(16)).rank == 15
    assert orc.Chain(rp, cl, color, np.zeros(16), rho=0.9).rank == 16
    rp2, cl2 = inputs.edges_to_csr(6, [0, 1, 3], [1, 2, 4])   # 3 components
    assert orc.Chain(rp2, cl2, np.array([0, 1, 0, 0, 1, 0]), np.zeros(6)).rank == 3


@pytest.mark.parametrize("rho", [1.0, 0.9, 0.5])
def test_rank_matches_the_dense_precision(orc, rho):
    """The tau shape's r is the rank of D - rho W (Sec. 2.1; proper prior of
    Sec. 3.2): numpy's SVD rank of the dense matrix, on graphs with isolated
    sites and several components."""
    cases = [inputs.edges_to_csr(6, [0, 1, 3], [1, 2, 4]),        # site 5 isolated
             inputs.edges_to_csr(9, [0, 2, 2, 6], [1, 3, 4, 7]),  # sites 5, 8 isolated
             inputs.lattice_csr(4, 5, 8)]
    for rp, cl in cases:
        color, _ = orc.greedy_coloring(rp, cl)
        W = dense_W(rp, cl)
        R = np.diag(W.sum(1)) - rho * W
        ch = orc.Chain(rp, cl, color, np.zeros(rp.size - 1), rho=rho)
        assert ch.rank == np.linalg.matrix_rank(R)


# --------------------------------------------------------------------------
# distributional pins (fixed tau, lam)
# --------------------------------------------------------------------------
def run_instances(orc, rp, cl, color, y, tau, lam, rho, M, T, seed=21):
    n = rp.size - 1
    X = np.empty((M, n))
    for m in range(M):
        ch = orc.Chain(rp, cl, color, y, rho=rho, tau0=tau, lam0=lam, seed=seed, instance=m)
        ch.sweeps(T, hyper=False)
        X[m] = ch.x
    return X


def moments_close(X, mu, Sigma, nsig=5.0):
    M = X.shape[0]
    d = np.sqrt(np.diag(Sigma))
    err_mu = np.abs(X.mean(0) - mu) / (d / np.sqrt(M))
    S = np.cov(X, rowvar=False)
    se = np.sqrt((np.outer(d ** 2, d ** 2) + Sigma ** 2) / M)
    err_S = np.abs(S - Sigma) / se
    return err_mu.max(), err_S.max()


@pytest.mark.parametrize("gi", [0, 1, 4], ids=[IDS[0], IDS[1], IDS[4]])
def test_stationary_law(orc, gi):
    name, rp, cl, color = GRAPHS[gi]
    rp, cl, color = graph_case(orc, name, rp, cl, color)
    n = rp.size - 1
    y = np.random.default_rng(gi).normal(size=n) + 1.0
    tau, lam, rho = 2.0, 1.0, 1.0
    Qp = dense_Qp(rp, cl, tau, lam, rho)
    X = run_instances(orc, rp, cl, color, y, tau, lam, rho, M=3000, T=60)
    e_mu, e_S = moments_close(X, np.linalg.solve(Qp, lam * y), np.linalg.inv(Qp))
    assert e_mu < 5.0 and e_S < 5.5


@pytest.mark.parametrize("T", [1, 2, 5])
def test_finite_t_moments(orc, T):
    rp, cl = inputs.lattice_csr(3, 4, 8)
    color, k = inputs.lattice_coloring(3, 4, 8)
    n = 12
    y = np.linspace(-1.0, 2.0, n)
    tau, lam, rho = 3.0, 0.7, 1.0
    Qp = dense_Qp(rp, cl, tau, lam, rho)
    b = lam * y
    # x' = M^{-1} (b - U x + Dg^{1/2} z), M = Dg + L (L: lower colors, U: higher)
    ci, cj = np.meshgrid(color, color, indexing="ij")
    L = np.where(ci > cj, Qp, 0.0)
    U = np.where(ci < cj, Qp, 0.0)
    Dg = np.diag(np.diag(Qp))
    Minv = np.linalg.inv(Dg + L)
    mu, S = np.zeros(n), np.zeros((n, n))
    for _ in range(T):
        mu = Minv @ (b - U @ mu)
        S = Minv @ (U @ S @ U.T + Dg) @ Minv.T
    X = run_instances(orc, rp, cl, color, y, tau, lam, rho, M=4000, T=T, seed=5)
    e_mu, e_S = moments_close(X, mu, S)
    assert e_mu < 5.0 and e_S < 5.5


def test_two_site_chain_autocorrelation(orc):
    # n = 2, one edge: x2 follows AR(1) with coefficient a^2, a = tau / (tau + lam)
    rp, cl = inputs.path_graph(2)
    tau, lam = 3.0, 1.0
    ch = orc.Chain(rp, cl, np.array([0, 1]), np.array([0.5, -0.5]), tau0=tau, lam0=lam, seed=8)
    T = 40000
    xs = np.empty(T)
    for t in range(T):
        ch.sweeps(1, hyper=False)
        xs[t] = ch.x[1]
    xs = xs[100:]
    a = tau / (tau + lam)
    r1 = np.corrcoef(xs[:-1], xs[1:])[0, 1]
    # SE of a lag-1 autocorrelation of an AR(1) with coefficient phi
    phi = a * a
    se = np.sqrt((1 - phi ** 2) / xs.size)
    assert abs(r1 - phi) < 5 * se


# --------------------------------------------------------------------------
# hyperparameters
# --------------------------------------------------------------------------
@pytest.mark.parametrize("rho", [1.0, 0.9])
def test_hyper_conditionals_are_conjugate_gammas(orc, rho):
    _, rp, cl = inputs.delaunay_graph(40, data_seed=2)
    color, k = orc.greedy_coloring(rp, cl)
    n = rp.size - 1
    rng = np.random.default_rng(6)
    y = rng.normal(size=n)
    x = rng.normal(size=n)
    ch = orc.Chain(rp, cl, color, y, rho=rho, a_tau=1.5, b_tau=0.5, a_lam=2.0, b_lam=3.0)
    W = dense_W(rp, cl)
    q = x @ (np.diag(W.sum(1)) - rho * W) @ x
    sse = np.sum((y - x) ** 2)
    ch.set_state(x, 1.0, 1.0, 1)
    ch.sweeps(0)
    ch._s.q, ch._s.sse = ch.quadratic_terms(x)
    N = 6000
    taus, lams = np.empty(N), np.empty(N)
    for t in range(N):
        ch._s.sweep = t + 1
        ch.hyper()
        taus[t], lams[t] = ch.tau, ch.lam
    r = n - 1 if rho == 1.0 else n
    assert stats.kstest(taus, stats.gamma(1.5 + r / 2, scale=1 / (0.5 + q / 2)).cdf).pvalue > 1e-4
    assert stats.kstest(lams, stats.gamma(2.0 + n / 2, scale=1 / (3.0 + sse / 2)).cdf).pvalue > 1e-4


def test_geweke_joint_distribution(orc):
    """Successive-conditional simulator: alternate the oracle's Gibbs kernel
    (x, tau, lam | y) with y | x, lam; the (tau, lam) marginals must stay at
    their Gamma(1, 1) priors under the proper CAR prior."""
    rp, cl = inputs.path_graph(5)
    n, rho = 5, 0.8
    color = (np.arange(n) % 2).astype(np.int32)
    rng = np.random.default_rng(17)
    W = dense_W(rp, cl)
    R = np.diag(W.sum(1)) - rho * W
    tau, lam = rng.gamma(1.0), rng.gamma(1.0)
    x = rng.multivariate_normal(np.zeros(n), np.linalg.inv(tau * R))
    y = x + rng.normal(size=n) / np.sqrt(lam)
    ch = orc.Chain(rp, cl, color, y, rho=rho, tau0=tau, lam0=lam, x0=x, seed=23)
    T = 60000
    taus, lams = np.empty(T), np.empty(T)
    for t in range(T):
        ch.sweeps(1, hyper=True)
        y = ch.x + rng.normal(size=n) / np.sqrt(ch.lam)
        ch.set_y(y)
        taus[t], lams[t] = ch.tau, ch.lam

    def batch_se(v, nb=60):
        b = v[: v.size // nb * nb].reshape(nb, -1).mean(1)
        return b.std(ddof=1) / np.sqrt(nb)

    for v in (taus, lams):
        assert abs(v.mean() - 1.0) < 5 * batch_se(v)
        assert abs(np.mean(v < 1.0) - (1 - np.exp(-1.0))) < 5 * batch_se((v < 1.0) * 1.0)


# --------------------------------------------------------------------------
# accumulators, burn-in, resume
# --------------------------------------------------------------------------
def test_stats_match_trajectory_and_burn_in(orc):
    rp, cl = inputs.lattice_csr(5, 6, 4)
    color, _ = inputs.lattice_coloring(5, 6, 4)
    y = np.random.default_rng(3).normal(size=30)
    ch = orc.Chain(rp, cl, color, y, burn_in=4, seed=12)
    traj = []
    for _ in range(15):
        ch.sweeps(1)
        traj.append(ch.x.copy())
    traj = np.array(traj[4:])
    mean, var = ch.stats()
    assert ch.n_acc == 11
    assert np.allclose(mean, traj.mean(0), rtol=1e-13, atol=1e-14)
    assert np.allclose(var, traj.var(0, ddof=1), rtol=1e-9, atol=1e-13)


def test_checkpoint_resume_is_bitwise(orc):
    _, rp, cl = inputs.delaunay_graph(200, data_seed=4)
    color, k = orc.greedy_coloring(rp, cl)
    y = np.random.default_rng(9).normal(size=200)
    full = orc.Chain(rp, cl, color, y, rho=0.95, seed=31, instance=2).sweeps(20)
    part = orc.Chain(rp, cl, color, y, rho=0.95, seed=31, instance=2).sweeps(8)
    res = orc.Chain(rp, cl, color, y, rho=0.95, seed=31, instance=2)
    res.set_state(part.x, part.tau, part.lam, part.sweep_count)
    res.s1[:], res.s2[:] = part.s1, part.s2
    res._s.n_acc = part.n_acc
    res.sweeps(12)
    assert np.array_equal(full.x, res.x) and full.tau == res.tau and full.lam == res.lam
    assert np.array_equal(full.s1, res.s1) and np.array_equal(full.s2, res.s2)


def test_hyper_after_plain_sweep_equals_fused(orc):
    rp, cl = inputs.lattice_csr(6, 6, 8)
    color, _ = inputs.lattice_coloring(6, 6, 8)
    y = np.random.default_rng(1).normal(size=36)
    a = orc.Chain(rp, cl, color, y, seed=2).sweeps(4)
    b = orc.Chain(rp, cl, color, y, seed=2)
    for _ in range(4):
        b.sweeps(1, hyper=False)
        b.hyper()
    assert np.array_equal(a.x, b.x) and a.tau == b.tau and a.lam == b.lam


# --------------------------------------------------------------------------
# the image model with an intercept (Sec. 3.1: y = 1 b0 + x + e, flat prior)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("gi", [0, 1, 4], ids=[IDS[0], IDS[1], IDS[4]])
def test_intercept_sweep_equals_dense_conditional(orc, gi):
    name, rp, cl, color = GRAPHS[gi]
    rp, cl, color = graph_case(orc, name, rp, cl, color)
    n = rp.size - 1
    rng = np.random.default_rng(40 + gi)
    y = rng.normal(size=n) + 3.0
    x0 = rng.normal(size=n)
    tau, lam, b0 = 1.3, 0.8, 2.4
    ch = orc.Chain(rp, cl, color, y, tau0=tau, lam0=lam, seed=5, intercept=True)
    ch.set_state(x0, tau, lam, sweep=3, beta0=b0)
    ch.sweeps(1, hyper=False)
    z = orc.site_normals(5, 3, 0, n)
    ref = dense_sweep(dense_Qp(rp, cl, tau, lam, 1.0), lam * (y - b0), x0, color, z)
    assert np.max(np.abs(ch.x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    assert ch.beta0 == b0


def test_intercept_conditionals(orc):
    """b0 | x, lam ~ N(mean(y - x), 1/(n lam)); then lam | x, b0 ~
    Gamma(a + n/2, b + ||y - b0 - x||^2 / 2) with the NEW b0 (probability
    integral transform, since the rate changes with every b0)."""
    rp, cl = inputs.lattice_csr(6, 7, 8)
    color, _ = inputs.lattice_coloring(6, 7, 8)
    n = 42
    rng = np.random.default_rng(8)
    y = rng.normal(size=n) + 5.0
    x = rng.normal(size=n)
    tau, lam = 2.0, 3.0
    ch = orc.Chain(rp, cl, color, y, intercept=True, a_lam=0.5, b_lam=0.25)
    N = 6000
    b0s, u = np.empty(N), np.empty(N)
    for t in range(N):
        ch.set_state(x, tau, lam, sweep=t + 1, beta0=0.0)
        ch.hyper()
        b0s[t] = ch.beta0
        sse = np.sum((y - ch.beta0 - x) ** 2)
        u[t] = stats.gamma(0.5 + n / 2, scale=1 / (0.25 + sse / 2)).cdf(ch.lam)
    assert stats.kstest(b0s, stats.norm(np.mean(y - x), 1 / np.sqrt(n * lam)).cdf).pvalue > 1e-4
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_intercept_accumulates_the_image(orc):
    rp, cl = inputs.lattice_csr(5, 5, 4)
    color, _ = inputs.lattice_coloring(5, 5, 4)
    y = np.random.default_rng(2).normal(size=25) + 1.0
    ch = orc.Chain(rp, cl, color, y, intercept=True, seed=9)
    imgs = []
    for _ in range(12):
        b0 = ch.beta0                   # the intercept the coming sweep uses
        ch.sweeps(1)
        imgs.append(ch.x + b0)
    mean, var = ch.stats()
    imgs = np.array(imgs)
    assert np.allclose(mean, imgs.mean(0), rtol=1e-13, atol=1e-14)
    assert np.allclose(var, imgs.var(0, ddof=1), rtol=1e-9, atol=1e-12)
    assert ch.beta0 != 0.0
