"""Pins for the oracle's Polya-Gamma sampler and binomial logit model
(Sec. 3.2 with the augmentation of Polson, Scott & Windle 2013), each
against something other than the oracle itself:

* PG(1, 0) = J*(1)/4 against the exact CDF of J*(1), written from its two
  series (the small-x erfc series and the large-x exponential series, which
  are checked against each other first);
* the Laplace transform E exp(-s PG(b, c)) = cosh(c/2)^b / cosh(sqrt(c^2/4 + s/2))^b
  and the closed-form mean b tanh(c/2) / (2c) and variance of PG(1, c);
* the binomial sweep against dense linear algebra of the augmented
  conditional (Qp = tau (D - rho W) + diag(psi), b = kappa - psi b0), with
  psi_i = PG(m_i, b0 + old x_i) recomputed from the sampler's public draw;
* the b0 and tau conditionals (KS), and a Geweke successive-conditional
  test of the whole binomial kernel under proper priors.
"""
import numpy as np
import pytest
from scipy import stats
from scipy.special import erfc

from paper_1702_05518_amd import inputs


def jstar_cdf(x, terms=60):
    """CDF of J*(1): small-x series sum_n (-1)^n 2 erfc((2n+1)/sqrt(2x)),
    large-x series 1 - sum_n (-1)^n 4/(pi(2n+1)) exp(-(2n+1)^2 pi^2 x / 8)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = np.arange(terms)[:, None]
    sgn = (-1.0) ** n
    small = np.sum(sgn * 2.0 * erfc((2 * n + 1) / np.sqrt(2.0 * np.maximum(x, 1e-300))), 0)
    large = 1.0 - np.sum(sgn * 4.0 / (np.pi * (2 * n + 1))
                         * np.exp(-((2 * n + 1) ** 2) * np.pi ** 2 * x / 8.0), 0)
    return np.where(x <= 1.0, small, large)


def test_jstar_series_agree():
    for x in (0.3, 0.64, 1.0, 1.5):
        n = np.arange(60)
        small = np.sum((-1.0) ** n * 2.0 * erfc((2 * n + 1) / np.sqrt(2.0 * x)))
        large = 1.0 - np.sum((-1.0) ** n * 4.0 / (np.pi * (2 * n + 1))
                             * np.exp(-((2 * n + 1) ** 2) * np.pi ** 2 * x / 8.0))
        assert abs(small - large) < 1e-12


def draws(orc, c, N, b=1, seed=3, sweep=0):
    if b == 1:
        return np.array([orc.pg1(c, seed, i % 1000, sweep + i // 1000, 0, 0) for i in range(N)])
    return np.array([orc.pg(b, c, seed, i, sweep, 0) for i in range(N)])


def test_pg1_zero_tilt_law(orc):
    w = draws(orc, 0.0, 20000)
    assert stats.kstest(w, lambda y: jstar_cdf(4.0 * y)).pvalue > 1e-3


@pytest.mark.parametrize("c", [0.0, 0.7, 2.0, -3.5, 9.0])
def test_pg1_moments_and_laplace_transform(orc, c):
    N = 20000
    w = draws(orc, c, N, seed=11)
    if c == 0.0:
        mean, var = 0.25, 1.0 / 24.0
    else:
        a = abs(c)
        mean = np.tanh(a / 2) / (2 * a)
        var = (np.sinh(a) - a) / (4 * a ** 3 * np.cosh(a / 2) ** 2)
    se = np.sqrt(var / N)
    assert abs(w.mean() - mean) < 5 * se
    assert abs(w.var() / var - 1) < 0.06
    for s in (1.0, 6.0):
        lt = np.cosh(c / 2) / np.cosh(np.sqrt(c * c / 4 + s / 2))
        v = np.exp(-s * w)
        assert abs(v.mean() - lt) < 5 * v.std() / np.sqrt(N)


def test_pg_integer_b_is_a_sum(orc):
    """PG(b, c) is the sum of the b terms' PG(1, c) draws; its Laplace
    transform is the b-th power of PG(1, c)'s."""
    b, c = 7, -1.5
    assert orc.pg(b, c, 5, 3, 2, 1) == sum(orc.pg1(c, 5, 3, 2, 1, j) for j in range(b))
    assert orc.pg(0, c, 5, 3, 2, 1) == 0.0
    N = 4000
    w = draws(orc, c, N, b=b, seed=8)
    s = 0.8
    lt = (np.cosh(c / 2) / np.cosh(np.sqrt(c * c / 4 + s / 2))) ** b
    v = np.exp(-s * w)
    assert abs(v.mean() - lt) < 5 * v.std() / np.sqrt(N)
    assert abs(w.mean() - b * np.tanh(0.75) / 3.0) < 5 * w.std() / np.sqrt(N)


# --------------------------------------------------------------------------
# the binomial model
# --------------------------------------------------------------------------
def dense_W(rp, cl):
    n = rp.size - 1
    W = np.zeros((n, n))
    for i in range(n):
        W[i, cl[rp[i]:rp[i + 1]]] = 1.0
    return W


def small_binomial(seed=0, n_pts=40):
    _, rp, cl = inputs.delaunay_graph(n_pts, data_seed=seed)
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 9, size=n_pts).astype(np.int32)
    y = rng.binomial(m, 0.4).astype(np.float64)
    return rp, cl, m, y


@pytest.mark.parametrize("rho", [0.995, 1.0])
def test_binomial_sweep_equals_dense_conditional(orc, rho):
    rp, cl, m, y = small_binomial(1)
    n = m.size
    color, _ = orc.greedy_coloring(rp, cl)
    x0 = np.random.default_rng(2).normal(size=n) * 0.5
    tau, b0 = 1.7, 0.35
    ch = orc.Chain(rp, cl, color, y, rho=rho, trials=m, intercept=True, beta0_var=1000.0,
                   seed=6, instance=2)
    ch.set_state(x0, tau, 1.0, sweep=9, beta0=b0)
    ch.sweeps(1, hyper=False)
    psi = np.array([orc.pg(m[i], b0 + x0[i], 6, i, 9, 2) for i in range(n)])
    assert np.array_equal(ch.psi[:n], psi)
    W = dense_W(rp, cl)
    Qp = tau * (np.diag(W.sum(1)) - rho * W) + np.diag(psi)
    kappa = y - m / 2.0
    z = orc.site_normals(6, 9, 2, n)
    x = x0.copy()
    for c in range(color.max() + 1):
        for i in np.flatnonzero(color == c):
            off = Qp[i] @ x - Qp[i, i] * x[i]
            x[i] = (kappa[i] - psi[i] * b0 - off) / Qp[i, i] + z[i] / np.sqrt(Qp[i, i])
    assert np.max(np.abs(ch.x - x)) <= 1e-12 * max(1.0, np.max(np.abs(x)))
    # the sums the b0 draw uses
    assert abs(ch.sse - psi.sum()) <= 1e-12 * psi.sum()
    assert abs(ch.rsum - np.sum(kappa - psi * ch.x)) <= 1e-12 * max(1.0, np.abs(kappa).sum())


def test_binomial_hyper_conditionals(orc):
    """After a sweep: b0 ~ N(sum(kappa - psi x)/P, 1/P), P = sum psi + 1/v0,
    and tau ~ Gamma(a + n/2, b + x'(D - rho W)x / 2) (proper prior, rank n)."""
    rp, cl, m, y = small_binomial(3)
    n = m.size
    color, _ = orc.greedy_coloring(rp, cl)
    ch = orc.Chain(rp, cl, color, y, rho=0.995, trials=m, intercept=True, beta0_var=4.0,
                   a_tau=2.0, b_tau=0.5, seed=4)
    ch.sweeps(3)
    ch.sweeps(1, hyper=False)
    x, psi, t = ch.x.copy(), ch.psi[:n].copy(), ch.sweep_count
    P = psi.sum() + 0.25
    mean = np.sum((y - m / 2.0) - psi * x) / P
    q, _ = ch.quadratic_terms(x)
    b0s, taus = [], []
    for k in range(4000):
        ch.set_state(x, 1.0, 1.0, sweep=t + k)
        ch._s.sse, ch._s.rsum, ch._s.q = psi.sum(), np.sum((y - m / 2.0) - psi * x), q
        ch.hyper()
        b0s.append(ch.beta0)
        taus.append(ch.tau)
    assert stats.kstest(b0s, stats.norm(mean, 1 / np.sqrt(P)).cdf).pvalue > 1e-4
    assert stats.kstest(taus, stats.gamma(2.0 + n / 2, scale=1 / (0.5 + q / 2)).cdf).pvalue > 1e-4


def test_binomial_geweke_joint_distribution(orc):
    """Successive-conditional simulator on a path of 6 sites: alternate the
    oracle's binomial kernel (psi, x, b0, tau | Y) with Y | x, b0 ~ Bin(m,
    logistic(b0 + x)); b0 and tau must keep their N(0, 1) and Gamma(2, 1)
    priors."""
    rp, cl = inputs.path_graph(6)
    n, rho = 6, 0.7
    color = (np.arange(n) % 2).astype(np.int32)
    m = np.array([3, 0, 5, 2, 4, 1], dtype=np.int32)
    rng = np.random.default_rng(31)
    W = dense_W(rp, cl)
    R = np.diag(W.sum(1)) - rho * W
    tau, b0 = rng.gamma(2.0), rng.normal()
    x = rng.multivariate_normal(np.zeros(n), np.linalg.inv(tau * R))
    y = rng.binomial(m, 1 / (1 + np.exp(-(b0 + x)))).astype(np.float64)
    ch = orc.Chain(rp, cl, color, y, rho=rho, trials=m, intercept=True, beta0_var=1.0,
                   a_tau=2.0, b_tau=1.0, tau0=tau, x0=x, beta0=b0, seed=41)
    T = 40000
    b0s, taus = np.empty(T), np.empty(T)
    for t in range(T):
        ch.sweeps(1, hyper=True)
        y = rng.binomial(m, 1 / (1 + np.exp(-(ch.beta0 + ch.x)))).astype(np.float64)
        ch.set_y(y)
        b0s[t], taus[t] = ch.beta0, ch.tau

    def batch_se(v, nb=50):
        b = v[: v.size // nb * nb].reshape(nb, -1).mean(1)
        return b.std(ddof=1) / np.sqrt(nb)

    assert abs(b0s.mean()) < 5 * batch_se(b0s)
    assert abs(np.mean(b0s < 0.5) - stats.norm.cdf(0.5)) < 5 * batch_se((b0s < 0.5) * 1.0)
    assert abs(taus.mean() - 2.0) < 5 * batch_se(taus)
    assert abs(np.mean(taus < 1.0) - stats.gamma(2.0).cdf(1.0)) < 5 * batch_se((taus < 1.0) * 1.0)


@pytest.mark.parametrize("c", [2.9, 3.3])
def test_pg1_mean_high_power_near_the_switch(orc, c):
    """Close to z = 1/t on either side (the two samplers of the left piece),
    200,000 draws resolve the mean to 0.2%: a tilt error in the left piece
    of the envelope moves it by about 1%."""
    N = 200_000
    w = np.array([orc.pg1(c, 17, i % 2000, i // 2000, 3, 1) for i in range(N)])
    mean = np.tanh(c / 2) / (2 * c)
    assert abs(w.mean() / mean - 1) < 5 * w.std() / np.sqrt(N) / mean
    s = 3.0
    lt = np.cosh(c / 2) / np.cosh(np.sqrt(c * c / 4 + s / 2))
    v = np.exp(-s * w)
    assert abs(v.mean() - lt) < 5 * v.std() / np.sqrt(N)
