"""Pins for the oracle's random-number contract version 2 (paired site normals).

Version 2 pairs the sites of each color by their rank in ascending original
id, ranks (2m, 2m + 1), and gives both sites of a pair the two Box-Muller
branches of the one Philox block keyed by the lower-ranked site (Box & Muller
1958: the cosine and sine of the same angle with the same radius are two
independent standard normals).  Each pin checks the oracle against something
other than its own formula:

* the pairing against a sort-and-pair of every color (brute force) and, on
  lattices whose width is a multiple of 4, against the closed form the lattice
  kernels use: (r, c) and (r, c + 2) with bit 1 of c clear form a pair;
* the cosine branch against the version-1 normal of the key site, bitwise;
* the pair's law: both branches N(0, 1), the squared radius chi-square with
  two degrees of freedom, the angle uniform, the branches uncorrelated;
* sweeps: one color per site has no pairs, so version 2 equals version 1
  bitwise; a one-color edgeless graph exposes every site's normal; the
  stationary law N(Qp^{-1} b, Qp^{-1}) of Sec. 2.2 still holds.
"""
import numpy as np
import pytest
from scipy import stats

from paper_1702_05518_amd import inputs


def sort_and_pair(color):
    """Brute force of the definition: sort each color's sites, pair
    neighbours in that order."""
    n = color.size
    key = np.arange(n)
    branch = np.zeros(n, dtype=np.int64)
    for c in np.unique(color):
        sites = sorted(int(i) for i in np.flatnonzero(color == c))
        for m in range(0, len(sites) - 1, 2):
            key[sites[m + 1]] = sites[m]
            branch[sites[m + 1]] = 1
    return key, branch


@pytest.mark.parametrize("seed", range(6))
def test_pairs_are_sorted_neighbours_within_each_color(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    k = int(rng.integers(1, 9))
    color = rng.integers(0, k, size=n).astype(np.int32)
    color[rng.integers(0, n)] = k - 1          # every color 0..k-1 may be empty but k-1
    key, branch = orc.rng_pairs(color)
    ek, eb = sort_and_pair(color)
    assert np.array_equal(key, ek) and np.array_equal(branch, eb)
    # every key is a branch-0 site of the same color with a lower id
    assert np.all(branch[key] == 0)
    assert np.all(color[key] == color)
    assert np.all(key <= np.arange(n))
    # each color has floor(count / 2) pairs
    for c in range(k):
        cnt = int(np.count_nonzero(color == c))
        assert int(np.count_nonzero(branch[color == c])) == cnt // 2


@pytest.mark.parametrize("st", [4, 8])
@pytest.mark.parametrize("rows,cols", [(4, 4), (5, 8), (7, 12), (3, 20)])
def test_lattice_pairs_closed_form(orc, st, rows, cols):
    """Width a multiple of 4: every row holds an even number of sites of each
    of its colors, so pairs stay in a row and are (c, c + 2) with bit 1 of c
    clear, the key the lower column."""
    color, _ = inputs.lattice_coloring(rows, cols, st)
    key, branch = orc.rng_pairs(color)
    r, c = np.divmod(np.arange(rows * cols), cols)
    assert np.array_equal(key, r * cols + (c & ~2))
    assert np.array_equal(branch, (c >> 1) & 1)


def test_lattice_pairs_straddle_rows_when_width_is_2_mod_4(orc):
    # 4-neighbour coloring of width 6: color 0 of row 0 is c = 0, 2, 4 (three
    # sites), so its third site pairs with the first color-0 site of row 1
    color, _ = inputs.lattice_coloring(3, 6, 4)
    key, branch = orc.rng_pairs(color)
    assert key[1 * 6 + 1] == 4 and branch[1 * 6 + 1] == 1
    assert np.array_equal(key, sort_and_pair(color)[0])


def test_pairs_edge_cases(orc):
    key, branch = orc.rng_pairs(np.zeros(0, dtype=np.int32))
    assert key.size == 0 and branch.size == 0
    key, branch = orc.rng_pairs(np.array([0], dtype=np.int32))
    assert key.tolist() == [0] and branch.tolist() == [0]
    key, branch = orc.rng_pairs(np.array([2, 1, 0], dtype=np.int32))   # one site per color
    assert key.tolist() == [0, 1, 2] and branch.tolist() == [0, 0, 0]
    with pytest.raises(ValueError):
        orc.rng_pairs(np.array([0, -1], dtype=np.int32))


def test_cosine_branch_is_the_version_1_normal(orc):
    rng = np.random.default_rng(3)
    for _ in range(2000):
        seed = int(rng.integers(0, 2 ** 63))
        key, t, inst = (int(v) for v in rng.integers(0, 2 ** 32, size=3))
        assert orc.normal_pair(seed, key, 0, t, inst, 0) == orc.normal(seed, key, t, inst, 0)


def test_pair_law(orc):
    seed, t, inst = 77, 5, 2
    N = 100000
    zc = np.array([orc.normal_pair(seed, i, 0, t, inst, 0) for i in range(N)])
    zs = np.array([orc.normal_pair(seed, i, 1, t, inst, 0) for i in range(N)])
    assert not np.any(zc == zs)
    for z in (zc, zs):
        assert stats.kstest(z, "norm").pvalue > 1e-4
        assert abs(z.mean()) < 5 / np.sqrt(N)
    # radius^2 ~ chi^2(2), angle ~ U(0, 1) independent of it
    r2 = zc * zc + zs * zs
    assert stats.kstest(r2, "chi2", args=(2,)).pvalue > 1e-4
    ang = np.mod(np.arctan2(zs, zc) / (2 * np.pi), 1.0)
    assert stats.kstest(ang, "uniform").pvalue > 1e-4
    assert abs(np.corrcoef(zc, zs)[0, 1]) < 5 / np.sqrt(N)
    assert abs(np.corrcoef(r2, ang)[0, 1]) < 5 / np.sqrt(N)
    # products of the pair have mean 0: a sine branch built from a different
    # angle (or the cosine twice) would not
    assert abs(np.mean(zc * zs)) < 5 / np.sqrt(N)
    assert abs(np.mean(zc * zc * zs * zs) - 1.0) < 6 * np.sqrt(8.0 / N)


def test_pair_radius_is_the_block_radius(orc):
    # z_cos^2 + z_sin^2 = -2 ln u1 with u1 from the first two words of the block
    for (seed, key, t) in [(1, 0, 0), (99, 17, 4), (2 ** 40 + 3, 5, 1)]:
        w = orc.philox([key, t, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u1 = orc.uniform52(int(w[0]), int(w[1]))
        r2 = orc.normal_pair(seed, key, 0, t, 0, 0) ** 2 + orc.normal_pair(seed, key, 1, t, 0, 0) ** 2
        assert abs(r2 + 2.0 * np.log(u1)) <= 1e-14 * max(1.0, r2)


def test_sine_branch_is_box_muller_of_block(orc):
    # z = sqrt(-2 ln u1) sin(2 pi u2), numpy's sine of the block's angle
    for (seed, key, t) in [(1, 0, 0), (99, 17, 4), (2 ** 40 + 3, 5, 1), (7, 2 ** 32 - 1, 9)]:
        w = orc.philox([key, t, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u1 = orc.uniform52(int(w[0]), int(w[1]))
        u2 = orc.uniform52(int(w[2]), int(w[3]))
        ref = np.sqrt(-2.0 * np.log(u1)) * np.sin(2.0 * np.pi * u2)
        assert abs(orc.normal_pair(seed, key, 1, t, 0, 0) - ref) <= 1e-15 * max(1.0, abs(ref))


def test_one_color_per_site_equals_version_1(orc):
    rp, cl = inputs.lattice_csr(4, 5, 8)
    n = 20
    y = np.random.default_rng(1).normal(size=n)
    col = np.arange(n, dtype=np.int32)
    a = orc.Chain(rp, cl, col, y, seed=4).sweeps(4)
    b = orc.Chain(rp, cl, col, y, seed=4, rng_version=2).sweeps(4)
    assert np.array_equal(a.x, b.x) and a.tau == b.tau and a.lam == b.lam


def test_edgeless_one_color_sweep_exposes_the_pair_normals(orc):
    # no edges: x_i = y_i + z_i / sqrt(lam) exactly in distribution, so the
    # sweep's z_i = (x_i - y_i) sqrt(lam) must be the paired normals
    n = 9
    rp = np.zeros(n + 1, dtype=np.int64)
    cl = np.zeros(0, dtype=np.int32)
    y = np.linspace(-1.0, 1.0, n)
    lam = 4.0
    ch = orc.Chain(rp, cl, np.zeros(n, dtype=np.int32), y, tau0=1.0, lam0=lam, seed=12,
                   instance=3, rng_version=2)
    ch.sweeps(1, hyper=False)
    z = (ch.x - y) * np.sqrt(lam)
    for i in range(n):
        key, br = (i - 1, 1) if i % 2 else (i, 0)
        assert abs(z[i] - orc.normal_pair(12, key, br, 0, 3, 0)) <= 1e-14
    # the last site (odd count) is unpaired: its version-1 normal
    assert abs(z[8] - orc.normal(12, 8, 0, 3, 0)) <= 1e-14


@pytest.mark.parametrize("st", [4, 8])
def test_stationary_law_version_2(orc, st):
    rp, cl = inputs.lattice_csr(4, 4, st)
    color, _ = inputs.lattice_coloring(4, 4, st)
    n = 16
    y = np.random.default_rng(st).normal(size=n) + 1.0
    tau, lam, rho = 2.0, 1.0, 1.0
    W = np.zeros((n, n))
    for i in range(n):
        W[i, cl[rp[i]:rp[i + 1]]] = 1.0
    Qp = tau * (np.diag(W.sum(1)) - rho * W) + lam * np.eye(n)
    M, T = 3000, 60
    X = np.empty((M, n))
    for m in range(M):
        ch = orc.Chain(rp, cl, color, y, rho=rho, tau0=tau, lam0=lam, seed=21, instance=m,
                       rng_version=2)
        ch.sweeps(T, hyper=False)
        X[m] = ch.x
    mu, Sigma = np.linalg.solve(Qp, lam * y), np.linalg.inv(Qp)
    d = np.sqrt(np.diag(Sigma))
    assert (np.abs(X.mean(0) - mu) / (d / np.sqrt(M))).max() < 5.0
    se = np.sqrt((np.outer(d ** 2, d ** 2) + Sigma ** 2) / M)
    assert (np.abs(np.cov(X, rowvar=False) - Sigma) / se).max() < 5.5


def test_rng_version_is_validated(orc):
    rp, cl = inputs.lattice_csr(2, 4, 4)
    color, _ = inputs.lattice_coloring(2, 4, 4)
    with pytest.raises(ValueError):
        orc.Chain(rp, cl, color, np.zeros(8), rng_version=3)
