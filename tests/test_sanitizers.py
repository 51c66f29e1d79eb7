"""Sanitizer builds of the host code (CPU only): AddressSanitizer and
UndefinedBehaviorSanitizer, built with gcc / g++ (no device code).

* The graph builder (graph_host.cpp) under tests/sanitize/graph_check.cpp,
  which also checks the invariants of the color slabs and the chunk tables
  on Delaunay (up to 60,000 sites, where some chunks exceed the LDS caps
  and split), lattice, hub and isolated-site graphs.
* The oracle (gmrf_oracle.c), loaded through its own Python wrapper in a
  child process with the sanitizer runtime preloaded, over Gaussian,
  intercept, proper-CAR and binomial chains.
"""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from paper_1702_05518_amd import gmrf, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1702_05518_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} is not installed")
    return path


def write_graphs(path, graphs):
    with open(path, "wb") as f:
        for rp, cl, color, k, rho in graphs:
            rp = np.ascontiguousarray(rp, dtype=np.int64)
            cl = np.ascontiguousarray(cl, dtype=np.int32)
            n = rp.size - 1
            f.write(np.array([n, cl.size], dtype=np.int64).tobytes())
            f.write(np.array([k], dtype=np.int32).tobytes())
            f.write(np.array([rho], dtype=np.float64).tobytes())
            f.write(rp.tobytes())
            f.write(cl.tobytes())
            f.write(np.ascontiguousarray(color, dtype=np.int32).tobytes())


def colored(rp, cl, rho=1.0):
    color, k = gmrf.greedy_coloring(rp, cl)
    return rp, cl, color, k, rho


def test_graph_builder_under_sanitizers(tmp_path):
    runtime("libasan.so")
    exe = str(tmp_path / "graph_check")
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include",
                    os.path.join(ROOT, "tests", "sanitize", "graph_check.cpp"),
                    os.path.join(CSRC, "graph_host.cpp"), "-o", exe], check=True)
    rng = np.random.default_rng(5)
    star = inputs.edges_to_csr(301, np.zeros(300, np.int64), np.arange(1, 301))
    a, b = rng.integers(0, 400, 900), rng.integers(0, 400, 900)
    keep = (a < 350) & (b < 350)                     # sites 350 .. 399 isolated
    graphs = [colored(*inputs.delaunay_graph(3000, data_seed=2)[1:]),
              colored(*inputs.delaunay_graph(60000, data_seed=9)[1:], rho=0.95),
              colored(*inputs.delaunay_graph(700, data_seed=4)[1:], rho=0.9),
              colored(*inputs.lattice_csr(37, 29, 8)),
              colored(*inputs.lattice_csr(20, 20, 4)),
              colored(*star),
              colored(*inputs.edges_to_csr(400, a[keep], b[keep]), rho=0.5),
              colored(*inputs.path_graph(9))]
    data = str(tmp_path / "graphs.bin")
    write_graphs(data, graphs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, data], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert f"checked {len(graphs)} graphs, {len(graphs)} with chunk tables" in r.stdout


ORACLE_RUN = textwrap.dedent("""
    import sys
    import numpy as np
    import oracle
    from paper_1702_05518_amd import inputs
    oracle._LIB = sys.argv[1]
    assert oracle.lib()._name == sys.argv[1]
    rp, cl = inputs.lattice_csr(12, 12, 8)
    color, k = oracle.greedy_coloring(rp, cl)
    y = np.random.default_rng(1).normal(size=144)
    for kw in ({}, {"intercept": True, "beta0": 0.5}, {"rho": 0.9}, {"rng_version": 2}):
        ch = oracle.Chain(rp, cl, color, y, seed=3, burn_in=2, **kw)
        ch.sweeps(12)
        m, v = ch.stats()
        assert np.isfinite(m).all() and np.isfinite(v).all()
    assert oracle.components(rp, cl) == 1
    key, br = oracle.rng_pairs(color)
    assert key.size == 144 and int(br.sum()) > 0
    _, rp2, cl2 = inputs.delaunay_graph(200, data_seed=6)
    color2, _ = oracle.greedy_coloring(rp2, cl2)
    trials = np.random.default_rng(2).integers(0, 30, 200).astype(np.int32)
    succ = np.minimum(trials, np.random.default_rng(3).integers(0, 20, 200)).astype(float)
    bc = oracle.Chain(rp2, cl2, color2, succ, seed=7, trials=trials, intercept=True,
                      beta0_var=4.0)
    bc.sweeps(6)
    assert np.isfinite(bc.x).all()
    print("oracle ok")
""")


def test_oracle_under_sanitizers(tmp_path):
    asan = runtime("libasan.so")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                    "-ffp-contract=off", *SAN, "-o", so,
                    os.path.join(ROOT, "oracle", "gmrf_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", ORACLE_RUN, so], capture_output=True, text=True,
                       env=env, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr
