"""Seeded synthetic inputs: graphs, colorings by inspection, observations.

This module is shared by the GPU path, the oracle tests and the benchmark.
It holds none of the sampler's arithmetic: it only builds adjacency
structures, the lattice colorings that the paper finds by inspection
(Sec. 2.3, Fig. 1), and synthetic data with the shapes of the paper's
workloads (Sec. 3.1 images, Sec. 3.2 irregular lattice).  Data randomness
uses numpy's PCG64 generator seeded by ``data_seed``; the sampler's own
random numbers come from the counter-based generator on each side.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# Adjacency structures
# --------------------------------------------------------------------------
def _offsets(stencil: int):
    if stencil == 4:
        return [(-1, 0), (0, -1), (0, 1), (1, 0)]
    if stencil == 8:
        return [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
    raise ValueError("stencil must be 4 or 8")


def lattice_csr(rows: int, cols: int, stencil: int):
    """CSR adjacency of a rows x cols pixel lattice with free boundary.

    Site id = r * cols + c.  ``stencil`` 4 joins edge neighbours, 8 also
    diagonal ones; every weight is 1 (w_ij = I(i ~ j), Sec. 3.1) and border
    pixels simply have fewer neighbours.  Neighbour lists come out ascending
    because the offsets are listed in ascending id order.
    """
    n = rows * cols
    r = np.repeat(np.arange(rows, dtype=np.int64), cols)
    c = np.tile(np.arange(cols, dtype=np.int64), rows)
    nbrs = []
    for dr, dc in _offsets(stencil):
        rr, cc = r + dr, c + dc
        ok = (rr >= 0) & (rr < rows) & (cc >= 0) & (cc < cols)
        nbrs.append(np.where(ok, rr * cols + cc, -1))
    nb = np.stack(nbrs, axis=1)            # n x S, ascending per row, -1 = absent
    deg = (nb >= 0).sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = nb[nb >= 0].astype(np.int32)
    return row_ptr, col


def lattice_coloring(rows: int, cols: int, stencil: int):
    """Colorings by inspection: checkerboard (r + c) mod 2 for 4 neighbours,
    2x2 parity 2 (r mod 2) + (c mod 2) for 8 neighbours (Sec. 2.3, Fig. 1)."""
    r = np.repeat(np.arange(rows), cols)
    c = np.tile(np.arange(cols), rows)
    if stencil == 4:
        return ((r + c) % 2).astype(np.int32), 2
    if stencil == 8:
        return (2 * (r % 2) + (c % 2)).astype(np.int32), 4
    raise ValueError("stencil must be 4 or 8")


def edges_to_csr(n: int, ei, ej):
    """Symmetric CSR (neighbours ascending, no duplicates) from an edge list."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    a = np.concatenate([ei, ej])
    b = np.concatenate([ej, ei])
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    src = key // n
    dst = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32)


def delaunay_graph(n: int, data_seed: int = 3):
    """n uniform points in the unit square and their Delaunay adjacency."""
    from scipy.spatial import Delaunay

    rng = np.random.Generator(np.random.PCG64(data_seed))
    pts = rng.random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    ei = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    ej = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    row_ptr, col = edges_to_csr(n, ei, ej)
    return pts, row_ptr, col


def path_graph(n: int):
    return edges_to_csr(n, np.arange(n - 1), np.arange(1, n))


# --------------------------------------------------------------------------
# Synthetic observations
# --------------------------------------------------------------------------
def block_image(rows: int, cols: int, blocks: int = 8, data_seed: int = 1):
    """Piecewise-constant truth: a blocks x blocks grid of constant patches,
    each value U(0, 1); patch edges at floor(i * rows / blocks)."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    vals = rng.random((blocks, blocks))
    bi = (np.arange(rows) * blocks) // rows
    bj = (np.arange(cols) * blocks) // cols
    return vals[bi][:, bj].reshape(-1), rng


def image_observations(rows: int, cols: int, noise_sd: float = 0.1, data_seed: int = 1,
                       blocks: int = 8):
    """y = truth + N(0, noise_sd^2) for the block image (flattened, row-major)."""
    truth, rng = block_image(rows, cols, blocks, data_seed)
    y = truth + noise_sd * rng.standard_normal(truth.size)
    return truth, y


def gaussian_bump_image(p: int):
    """The paper's simulated truth: 5 exp(-|v|^2 / 2) / pi at evenly spaced
    pixel centres of [-3, 3]^2 (Sec. 3.1)."""
    edges = np.linspace(-3.0, 3.0, p + 1)
    v = 0.5 * (edges[:-1] + edges[1:])
    vi, vj = np.meshgrid(v, v, indexing="ij")
    return (5.0 * np.exp(-(vi ** 2 + vj ** 2) / 2.0) / np.pi).reshape(-1)


def _dot(a, b) -> float:
    """Inner product by numpy's pairwise summation, whose order of operations
    is fixed by numpy itself (np.dot hands the sum to the BLAS, whose kernels,
    and so whose rounding, depend on the CPU)."""
    return float(np.add.reduce(a * b))


def conjugate_gradients(A, b, rtol: float = 1e-12, maxiter: int = 100000):
    """Solve A x = b for a symmetric positive definite sparse A by conjugate
    gradients (Hestenes-Stiefel), stopping at ||r|| <= rtol ||b||.  Every
    operation is a CSR product (sequential rows), an elementwise one or _dot,
    so the result is the same on every machine that runs the same numpy and
    scipy builds."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _dot(r, r)
    stop = (rtol * np.sqrt(_dot(b, b))) ** 2
    for _ in range(maxiter):
        if rr <= stop:
            return x
        Ap = A @ p
        alpha = rr / _dot(p, Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = _dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    raise RuntimeError("CG did not converge while drawing the prior field")


def proper_car_prior_draw(row_ptr, col, tau: float, rho: float, rng, rtol: float = 1e-12):
    """Exact draw x ~ N(0, (tau (D - rho W))^{-1}) for 0 <= rho < 1.

    With B the signed edge incidence, D - rho W = (1 - rho) D + rho B'B, so
    w = sqrt(tau) [sqrt(1 - rho) D^{1/2} z1 + sqrt(rho) B' z2] ~ N(0, Q) and
    x = Q^{-1} w ~ N(0, Q^{-1}); Q x = w is solved by conjugate gradients
    (conjugate_gradients, reproducible across machines).
    """
    import scipy.sparse as sp

    n = row_ptr.size - 1
    deg = np.diff(row_ptr).astype(np.float64)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    upper = src < col
    ei, ej = src[upper], col[upper].astype(np.int64)
    m = ei.size
    z1 = rng.standard_normal(n)
    z2 = rng.standard_normal(m)
    btz = np.bincount(ei, weights=z2, minlength=n) - np.bincount(ej, weights=z2, minlength=n)
    w = np.sqrt(tau) * (np.sqrt(1.0 - rho) * np.sqrt(deg) * z1 + np.sqrt(rho) * btz)
    W = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), row_ptr), shape=(n, n))
    Q = tau * (sp.diags(deg) - rho * W)
    return conjugate_gradients(Q.tocsr(), w, rtol=rtol, maxiter=20 * n)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
def lattice_workload(rows: int, cols: int, stencil: int, noise_sd: float = 0.1,
                     data_seed: int = 1, with_csr: bool = True):
    """Image-restoration workload on a lattice: graph, coloring, y, truth."""
    color, k = lattice_coloring(rows, cols, stencil)
    truth, y = image_observations(rows, cols, noise_sd, data_seed)
    out = dict(kind="lattice", rows=rows, cols=cols, stencil=stencil, n=rows * cols,
               color=color, k=k, y=y, truth=truth, rho=1.0)
    if with_csr:
        out["row_ptr"], out["col"] = lattice_csr(rows, cols, stencil)
    return out


def bump_image_workload(p: int, noise_sd: float = 1.0, data_seed: int = 1, stencil: int = 8):
    """The paper's simulated image (Sec. 3.1): p x p Gaussian-bump truth plus
    N(0, noise_sd^2) noise (noise_sd 1 for the low-noise case, 50 for the
    high-noise one), on a lattice of `stencil` neighbours with its parity
    coloring.  The model fitted to it has an intercept and an intrinsic
    prior."""
    color, k = lattice_coloring(p, p, stencil)
    truth = gaussian_bump_image(p)
    rng = np.random.Generator(np.random.PCG64(data_seed))
    y = truth + noise_sd * rng.standard_normal(truth.size)
    row_ptr, col = lattice_csr(p, p, stencil)
    return dict(kind="lattice", rows=p, cols=p, stencil=stencil, n=p * p, color=color, k=k,
                y=y, truth=truth, rho=1.0, row_ptr=row_ptr, col=col)


def delaunay_workload(n: int, data_seed: int = 3, rho: float = 0.95, tau_true: float = 2.0,
                      noise_sd: float = 0.2):
    """Irregular-lattice workload: Delaunay adjacency of uniform points, truth
    drawn from the proper CAR prior with precision tau_true (D - rho W), and
    y = x + N(0, noise_sd^2).  The coloring is left to the caller."""
    pts, row_ptr, col = delaunay_graph(n, data_seed)
    rng = np.random.Generator(np.random.PCG64(data_seed + 1000))
    truth = proper_car_prior_draw(row_ptr, col, tau_true, rho, rng)
    y = truth + noise_sd * rng.standard_normal(n)
    return dict(kind="csr", n=n, points=pts, row_ptr=row_ptr, col=col, y=y, truth=truth,
                rho=rho)


def binomial_workload(n: int, data_seed: int = 5, rho: float = 0.995, tau_true: float = 4.0,
                      beta0_true: float = 0.3, trials_median: float = 250.0,
                      missing: float = 0.022):
    """Binomial areal counts shaped like the paper's election example
    (Sec. 3.2: n precincts, a Delaunay-like irregular adjacency, counts Y_i of
    m_i trials, about 2.2% of areas without data).  Truth: gamma from the
    proper CAR prior with precision tau_true (D - rho W), logit(pi_i) =
    beta0_true + gamma_i; m_i = ceil(lognormal) with the given median (sd 0.8
    on the log scale), m_i = 0 for the missing areas; Y_i ~ Bin(m_i, pi_i).
    The coloring is left to the caller."""
    pts, row_ptr, col = delaunay_graph(n, data_seed)
    rng = np.random.Generator(np.random.PCG64(data_seed + 2000))
    gamma = proper_car_prior_draw(row_ptr, col, tau_true, rho, rng)
    eta = beta0_true + gamma
    trials = np.ceil(np.exp(np.log(trials_median) + 0.8 * rng.standard_normal(n))).astype(np.int32)
    trials[rng.random(n) < missing] = 0
    y = rng.binomial(trials, 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    return dict(kind="csr", n=n, points=pts, row_ptr=row_ptr, col=col, y=y, trials=trials,
                truth=eta, rho=rho)


def smooth_field(points):
    """A smooth synthetic truth on the unit square (used where an exact prior
    draw would be too slow to generate for many graphs)."""
    u, v = points[:, 0], points[:, 1]
    return np.sin(2 * np.pi * 1.5 * u) * np.cos(2 * np.pi * v) + 0.5 * u


def _delaunay_job(args):
    n, seed = args
    return delaunay_graph(n, data_seed=seed)


def batch_mix(count: int = 512, data_seed: int = 4, side=(32, 512), nrange=(1000, 50000),
              noise_lattice: float = 0.1, noise_graph: float = 0.2, workers: int = 1):
    """Many independent instances of uneven sizes: the first half lattices with
    side ~ U{side} (4 neighbours, checkerboard), the second half Delaunay
    graphs with n ~ U{nrange} (smooth truth plus noise, proper CAR rho 0.95).
    Returns a list of workload dicts (graphs without colorings).  workers > 1
    builds the Delaunay graphs in that many processes (the same result: the
    random draws are taken in the same order beforehand)."""
    rng = np.random.Generator(np.random.PCG64(data_seed))
    out = []
    nlat = count // 2
    for i in range(nlat):
        s = int(rng.integers(side[0], side[1] + 1))
        wl = lattice_workload(s, s, 4, noise_sd=noise_lattice,
                              data_seed=int(rng.integers(1 << 30)), with_csr=False)
        out.append(wl)
    jobs, noise = [], []
    for i in range(count - nlat):
        n = int(rng.integers(nrange[0], nrange[1] + 1))
        jobs.append((n, int(rng.integers(1 << 30))))
        noise.append(noise_graph * rng.standard_normal(n))
    if workers > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor

        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
            graphs = list(ex.map(_delaunay_job, jobs, chunksize=4))
    else:
        graphs = [_delaunay_job(j) for j in jobs]
    for (n, _), (pts, row_ptr, col), e in zip(jobs, graphs, noise):
        truth = smooth_field(pts)
        out.append(dict(kind="csr", n=n, row_ptr=row_ptr, col=col, y=truth + e, truth=truth,
                        rho=0.95))
    return out
