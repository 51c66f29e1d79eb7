"""CPU oracle for the chromatic Gibbs sampler (ctypes front end of gmrf_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library; the two meet only through the seeded input generators.

The arithmetic lives in ``gmrf_oracle.c`` (plain C, FP64, no fast-math, no FP
contraction).  This module only builds it, marshals arrays and wraps the
chain state.  Every function cites the part of the paper it follows in the C
source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmrf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WITH_HYPER = 1
ZERO_NOISE = 2
GAMMA_MAX_ATTEMPTS = 64
GAUSSIAN, BINOMIAL = 0, 1

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall"]


def build(force: bool = True) -> str:
    """Compile gmrf_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("row_ptr", C.POINTER(C.c_int64)),
        ("col", C.POINTER(C.c_int32)),
        ("color", C.POINTER(C.c_int32)),
        ("k", C.c_int32),
        ("rho", C.c_double),
        ("y", C.POINTER(C.c_double)),
        ("a_tau", C.c_double),
        ("b_tau", C.c_double),
        ("a_lam", C.c_double),
        ("b_lam", C.c_double),
        ("rank", C.c_int64),
        ("burn_in", C.c_int64),
        ("seed", C.c_uint64),
        ("instance", C.c_uint32),
        ("intercept", C.c_int32),
        ("likelihood", C.c_int32),
        ("trials", C.POINTER(C.c_int32)),
        ("beta0_var", C.c_double),
        ("rng_version", C.c_int32),
        ("pair_key", C.POINTER(C.c_int32)),
        ("pair_branch", C.POINTER(C.c_uint8)),
    ]


class _Chain(C.Structure):
    _fields_ = [
        ("x", C.POINTER(C.c_double)),
        ("s1", C.POINTER(C.c_double)),
        ("s2", C.POINTER(C.c_double)),
        ("tau", C.c_double),
        ("lam", C.c_double),
        ("sweep", C.c_int64),
        ("n_acc", C.c_int64),
        ("q", C.c_double),
        ("sse", C.c_double),
        ("status", C.c_int32),
        ("beta0", C.c_double),
        ("psi", C.POINTER(C.c_double)),
        ("rsum", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        u32, u64, i32, i64, dbl = C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_double
        L.orc_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform52.argtypes = [u32, u32]
        L.orc_uniform52.restype = dbl
        L.orc_normal.argtypes = [u64, u32, u32, u32, u32]
        L.orc_normal.restype = dbl
        L.orc_normal_pair.argtypes = [u64, u32, u32, u32, u32, u32]
        L.orc_normal_pair.restype = dbl
        L.orc_rng_pairs.argtypes = [i64, C.POINTER(i32), i32, C.POINTER(i32),
                                    C.POINTER(C.c_uint8)]
        L.orc_rng_pairs.restype = i32
        L.orc_gamma.argtypes = [dbl, dbl, u64, u32, u32, u32, C.c_int, C.POINTER(dbl)]
        L.orc_gamma.restype = C.c_int
        L.orc_pg1.argtypes = [dbl, u64, u32, u32, u32, u32, C.POINTER(dbl)]
        L.orc_pg1.restype = C.c_int
        L.orc_pg.argtypes = [i32, dbl, u64, u32, u32, u32, C.POINTER(dbl)]
        L.orc_pg.restype = C.c_int
        L.orc_greedy_coloring.argtypes = [i64, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]
        L.orc_greedy_coloring.restype = i32
        L.orc_components.argtypes = [i64, C.POINTER(i64), C.POINTER(i32)]
        L.orc_components.restype = i64
        L.orc_quadratic_terms.argtypes = [C.POINTER(_Problem), C.POINTER(dbl), C.POINTER(dbl),
                                          C.POINTER(dbl)]
        L.orc_quadratic_terms.restype = None
        L.orc_hyper.argtypes = [C.POINTER(_Problem), C.POINTER(_Chain)]
        L.orc_hyper.restype = C.c_int
        L.orc_sweeps.argtypes = [C.POINTER(_Problem), C.POINTER(_Chain), i64, u32,
                                 C.POINTER(i64), i32]
        L.orc_sweeps.restype = C.c_int
        L.orc_stats.argtypes = [C.POINTER(_Chain), i64, C.POINTER(dbl), C.POINTER(dbl)]
        L.orc_stats.restype = None
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def uniform52(hi: int, lo: int) -> float:
    return lib().orc_uniform52(hi, lo)


def normal(seed: int, c0: int, c1: int, c2: int, c3: int) -> float:
    """Box-Muller normal of the Philox block at counter (c0, c1, c2, c3)."""
    return lib().orc_normal(seed, c0, c1, c2, c3)


def normal_pair(seed: int, key: int, branch: int, c1: int, c2: int, c3: int) -> float:
    """Cosine (branch 0) or sine (branch 1) Box-Muller normal of the Philox
    block at counter (key, c1, c2, c3): the version-2 site normal."""
    return lib().orc_normal_pair(seed, key, branch, c1, c2, c3)


def rng_pairs(color):
    """Version-2 pairing of a coloring: (key, branch) per site, key the id
    of the lower-ranked site of its pair within its color, branch 1 for the
    higher-ranked site."""
    color = np.ascontiguousarray(color, dtype=np.int32)
    n = color.size
    k = int(color.max()) + 1 if n else 0
    key = np.zeros(max(n, 1), dtype=np.int32)
    branch = np.zeros(max(n, 1), dtype=np.uint8)
    if lib().orc_rng_pairs(n, _ptr(color, C.c_int32), k, _ptr(key, C.c_int32),
                           _ptr(branch, C.c_uint8)) != 0:
        raise ValueError("color outside 0 .. k-1")
    return key[:n], branch[:n]


def site_normals(seed: int, sweep: int, instance: int, n: int) -> np.ndarray:
    """The site normals z_{t,i} of one sweep, i = 0..n-1 (tag 0)."""
    L = lib()
    return np.array([L.orc_normal(seed, i, sweep, instance, 0) for i in range(n)])


def gamma(shape: float, rate: float, seed: int, sweep: int, instance: int, tag: int,
          max_attempts: int = GAMMA_MAX_ATTEMPTS):
    """Marsaglia-Tsang Gamma(shape, rate) draw; returns (value, attempts)."""
    out = C.c_double(0.0)
    a = lib().orc_gamma(shape, rate, seed, sweep, instance, tag, max_attempts, C.byref(out))
    if a == -2:
        raise ValueError("gamma: shape must be >= 1 and rate > 0")
    return (out.value if a > 0 else float("nan")), a


def pg1(c: float, seed: int, site: int, sweep: int, instance: int, j: int) -> float:
    """PG(1, c) draw from the uniform stream of term j of (site, sweep)."""
    out = C.c_double(0.0)
    if lib().orc_pg1(float(c), seed, site, sweep, instance, j, C.byref(out)):
        raise FloatingPointError("pg1: uniform stream exhausted")
    return out.value


def pg(b: int, c: float, seed: int, site: int, sweep: int, instance: int) -> float:
    """PG(b, c) for integer b: the sum of the PG(1, c) terms j = 0 .. b-1."""
    out = C.c_double(0.0)
    if lib().orc_pg(int(b), float(c), seed, site, sweep, instance, C.byref(out)):
        raise FloatingPointError("pg: uniform stream exhausted")
    return out.value


# --------------------------------------------------------------------------
# Graph utilities
# --------------------------------------------------------------------------
def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return rp, cl


def greedy_coloring(row_ptr, col):
    """Greedy coloring by peeling maximal independent sets (min-index first)."""
    rp, cl = _csr(row_ptr, col)
    n = rp.size - 1
    color = np.zeros(max(n, 1), dtype=np.int32)
    k = lib().orc_greedy_coloring(n, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                  _ptr(color, C.c_int32))
    return color[:n].copy(), int(k)


def components(row_ptr, col) -> int:
    rp, cl = _csr(row_ptr, col)
    return int(lib().orc_components(rp.size - 1, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32)))


# --------------------------------------------------------------------------
# Sampler
# --------------------------------------------------------------------------
class Chain:
    """One chromatic Gibbs chain on the CPU oracle.

    Parameters mirror the model: a CSR adjacency (neighbours ascending), a
    proper coloring, observations y, rho (1 = intrinsic), Gamma(a, rate b)
    priors on tau and lam, burn-in, seed and instance.
    """

    def __init__(self, row_ptr, col, color, y, rho=1.0, a_tau=1.0, b_tau=1.0, a_lam=1.0,
                 b_lam=1.0, tau0=1.0, lam0=1.0, burn_in=0, seed=1, instance=0, x0=None,
                 rank=None, intercept=False, beta0=0.0, trials=None, beta0_var=0.0,
                 rng_version=1):
        """With ``trials`` (m_i, integers >= 0) the chain samples the binomial
        logit model: y holds the successes Y_i, the Polya-Gamma psi_i of the
        last sweep are in ``psi``, and beta0_var is the prior variance of b0
        (0 = flat).  rng_version 2 draws the site normals by the paired
        contract (``rng_pairs``), 1 one Philox block per site."""
        self.row_ptr, self.col = _csr(row_ptr, col)
        self.n = n = self.row_ptr.size - 1
        self.color = np.ascontiguousarray(color, dtype=np.int32)
        if self.color.size != n:
            raise ValueError("color must have n entries")
        self.k = int(self.color.max()) + 1 if n else 0
        self.y = np.ascontiguousarray(y, dtype=np.float64).copy()
        if rank is None:
            # rank of D - rho W (Sec. 2.1, Sec. 3.2): n minus the number of
            # connected components for the intrinsic prior (rho = 1); for the
            # proper prior (rho < 1) only the rows of isolated sites vanish
            isolated = int(np.count_nonzero(np.diff(self.row_ptr) == 0))
            rank = (n - components(self.row_ptr, self.col) if rho == 1.0 else n - isolated)
        self.rank = int(rank)
        self.x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
        self.s1 = np.zeros(n)
        self.s2 = np.zeros(n)
        self.psi = np.zeros(max(n, 1))
        binom = trials is not None
        self.trials = (np.ascontiguousarray(trials, dtype=np.int32) if binom
                       else np.zeros(1, dtype=np.int32))
        if binom and self.trials.size != n:
            raise ValueError("trials must have n entries")
        if rng_version not in (1, 2):
            raise ValueError("rng_version must be 1 or 2")
        self.rng_version = int(rng_version)
        if self.rng_version == 2:
            self.pair_key, self.pair_branch = rng_pairs(self.color)
        else:
            self.pair_key = np.zeros(1, dtype=np.int32)
            self.pair_branch = np.zeros(1, dtype=np.uint8)
        self.pair_key = np.ascontiguousarray(self.pair_key)
        self.pair_branch = np.ascontiguousarray(self.pair_branch)
        self._p = _Problem(n, _ptr(self.row_ptr, C.c_int64), _ptr(self.col, C.c_int32),
                           _ptr(self.color, C.c_int32), self.k, float(rho),
                           _ptr(self.y, C.c_double), a_tau, b_tau, a_lam, b_lam, self.rank,
                           int(burn_in), int(seed), int(instance), 1 if intercept else 0,
                           BINOMIAL if binom else GAUSSIAN, _ptr(self.trials, C.c_int32),
                           float(beta0_var), self.rng_version,
                           _ptr(self.pair_key, C.c_int32), _ptr(self.pair_branch, C.c_uint8))
        self._s = _Chain(_ptr(self.x, C.c_double), _ptr(self.s1, C.c_double),
                         _ptr(self.s2, C.c_double), float(tau0), float(lam0), 0, 0, 0.0, 0.0, 0,
                         float(beta0), _ptr(self.psi, C.c_double), 0.0)

    # state ----------------------------------------------------------------
    @property
    def tau(self):
        return self._s.tau

    @property
    def lam(self):
        return self._s.lam

    @property
    def sweep_count(self):
        return self._s.sweep

    @property
    def n_acc(self):
        return self._s.n_acc

    @property
    def q(self):
        return self._s.q

    @property
    def sse(self):
        return self._s.sse

    @property
    def status(self):
        return self._s.status

    @property
    def beta0(self):
        return self._s.beta0

    @property
    def rsum(self):
        return self._s.rsum

    def set_state(self, x, tau, lam, sweep, beta0=None):
        self.x[:] = x
        self._s.tau = float(tau)
        self._s.lam = float(lam)
        self._s.sweep = int(sweep)
        if beta0 is not None:
            self._s.beta0 = float(beta0)

    def set_y(self, y):
        self.y[:] = y

    # work -----------------------------------------------------------------
    def sweeps(self, nsweeps: int, hyper: bool = True, zero_noise: bool = False, visit=None,
               nthreads: int = 1):
        flags = (WITH_HYPER if hyper else 0) | (ZERO_NOISE if zero_noise else 0)
        vp = None
        if visit is not None:
            self._visit = np.ascontiguousarray(visit, dtype=np.int64)
            vp = _ptr(self._visit, C.c_int64)
        rc = lib().orc_sweeps(C.byref(self._p), C.byref(self._s), int(nsweeps), flags, vp,
                              int(nthreads))
        if rc != 0:
            raise FloatingPointError("oracle: Gamma attempt cap hit or non-finite draw")
        return self

    def hyper(self):
        if self._s.sweep < 1:
            raise RuntimeError("hyper needs a completed sweep")
        if lib().orc_hyper(C.byref(self._p), C.byref(self._s)) != 0:
            raise FloatingPointError("oracle: Gamma attempt cap hit or non-finite draw")

    def quadratic_terms(self, x=None):
        xx = self.x if x is None else np.ascontiguousarray(x, dtype=np.float64)
        q, s = C.c_double(), C.c_double()
        lib().orc_quadratic_terms(C.byref(self._p), _ptr(xx, C.c_double), C.byref(q), C.byref(s))
        return q.value, s.value

    def stats(self):
        mean = np.zeros(self.n)
        var = np.zeros(self.n)
        lib().orc_stats(C.byref(self._s), self.n, _ptr(mean, C.c_double), _ptr(var, C.c_double))
        return mean, var
