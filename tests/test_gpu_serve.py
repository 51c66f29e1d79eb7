"""Continuous batching: jobs join and leave the shared launches at step
boundaries, admission respects the memory budget, and every job's posterior
mean and variance equal a standalone run of the same job bit for bit and the
CPU oracle's run of it (FP64 jobs at 1e-12 relative, FP32 jobs at the stated
posterior-mean accuracy, max abs error <= 1e-4)."""
import numpy as np
import pytest

from paper_1702_05518_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_05518_amd import gmrf, serve

    gmrf.lib()
    return gmrf, serve


ORACLE_INPUTS = {}      # id(graph) -> (row_ptr, col, color, rho) for the oracle


def pool(gmrf):
    graphs = []
    wl = inputs.lattice_workload(40, 50, 8, data_seed=2)
    g = gmrf.Graph(lattice=(40, 50, 8))
    ORACLE_INPUTS[id(g)] = (wl["row_ptr"], wl["col"], wl["color"], 1.0)
    graphs.append((g, wl["y"]))
    for n, ds in [(2000, 5), (700, 6)]:
        wl = inputs.delaunay_workload(n, data_seed=ds, rho=0.95)
        color, k = gmrf.greedy_coloring(wl["row_ptr"], wl["col"])
        g = gmrf.Graph(row_ptr=wl["row_ptr"], col_idx=wl["col"], color=color, num_colors=k,
                       rho=0.95)
        ORACLE_INPUTS[id(g)] = (wl["row_ptr"], wl["col"], color, 0.95)
        graphs.append((g, wl["y"]))
    return graphs


def check_against_oracle(orc, job, fp64):
    """The job's posterior mean / variance against the FP64 oracle's run of
    the same job (same graph, data, seed, instance and sweeps)."""
    rp, cl, color, rho = ORACLE_INPUTS[id(job.graph)]
    oc = orc.Chain(rp, cl, color, job.y, rho=rho, seed=job.seed, instance=job.instance)
    oc.sweeps(job.nsweeps, nthreads=8)
    om, ov = oc.stats()
    err = np.max(np.abs(job.mean - om))
    if fp64:
        assert err <= 1e-12 * np.max(np.abs(om)), err
        assert np.max(np.abs(job.var - ov)) <= 1e-9 * np.max(np.abs(ov))
    else:
        assert err <= 1e-4, err
        assert np.max(np.abs(job.var - ov)) <= 1e-4 * max(1.0, np.max(ov))
    return err


def jobs_for(serve, graphs, prec):
    out = []
    for i in range(9):
        g, y = graphs[i % len(graphs)]
        out.append(serve.Job(i, g, y, seed=50 + i, instance=i, nsweeps=[20, 40, 30][i % 3],
                             arrival=0.0, precision=prec))
    return out


@pytest.mark.parametrize("overlap", [False, True])
@pytest.mark.parametrize("prec_name", ["fp32", "fp64"])
def test_served_results_equal_standalone(S, orc, prec_name, overlap):
    gmrf, serve = S
    prec = gmrf.FP32_ACC64 if prec_name == "fp32" else gmrf.FP64
    graphs = pool(gmrf)
    jobs = jobs_for(serve, graphs, prec)
    one = serve.chain_bytes(graphs[0][0], prec)
    server = serve.Server(budget_bytes=3 * one + 1, step_sweeps=10, max_active=3,
                          overlap=overlap)
    server.run(jobs, realtime=False)
    assert len(server.finished) == len(jobs)
    assert server.rebuilds > 2            # the mix changed while jobs were running
    for job in jobs:
        ch = gmrf.Chain(job.graph, job.y, precision=prec, seed=job.seed, instance=job.instance)
        ch.sweep(job.nsweeps)
        mean, var, nacc = ch.posterior_stats()
        assert nacc == job.nsweeps
        assert np.array_equal(mean, job.mean) and np.array_equal(var, job.var)
        check_against_oracle(orc, job, prec == gmrf.FP64)


@pytest.mark.parametrize("overlap", [False, True])
def test_admission_respects_budget(S, overlap):
    gmrf, serve = S
    graphs = pool(gmrf)
    jobs = jobs_for(serve, graphs, gmrf.FP32_ACC64)
    budget = max(serve.chain_bytes(g, gmrf.FP32_ACC64) for g, _ in graphs) * 2
    server = serve.Server(budget_bytes=budget, step_sweeps=10, overlap=overlap)
    orig_step = server.step
    seen = []

    def step(clock):
        r = orig_step(clock)
        assert server.used <= budget
        seen.append(len(server.active))
        return r

    server.step = step
    server.run(jobs, realtime=False)
    assert len(server.finished) == len(jobs)
    assert max(seen) >= 2                  # several jobs shared the launches
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=10).submit(jobs[0])
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=budget, step_sweeps=7).submit(jobs[0])


@pytest.mark.parametrize("overlap", [False, True])
def test_full_config_stream_equals_standalone(S, orc, overlap):
    """The benchmark's serving configuration: Poisson arrivals at 200/s for
    2 s of 1000-sweep jobs on Delaunay graphs of 15,000 sites (probability
    0.98) or 1,000,000 sites (0.02), served in real time with continuous
    batching (host work overlapped with the sweeps, or synchronised after
    every step); sampled jobs (every 1M-site job among them) equal a
    standalone run bit for bit, and three sampled 15,000-site jobs are held
    against the FP64 oracle's run of the same job (posterior-mean max abs
    error <= 1e-4, the FP32 accuracy)."""
    gmrf, serve = S
    graphs = []
    for n, ds in [(15000, 11), (15000, 12), (15000, 13), (1_000_000, 14)]:
        pts, rp, cl = inputs.delaunay_graph(n, data_seed=ds)
        y = inputs.smooth_field(pts) + 0.2 * np.random.default_rng(ds).standard_normal(n)
        color, k = gmrf.greedy_coloring(rp, cl)
        g = gmrf.Graph(row_ptr=rp, col_idx=cl, color=color, num_colors=k, rho=0.95)
        ORACLE_INPUTS[id(g)] = (rp, cl, color, 0.95)
        graphs.append((g, y))
    rng = np.random.default_rng(7)
    t, jobs = 0.0, []
    while True:
        t += rng.exponential(1 / 200.0)
        if t > 2.0:
            break
        g, y = graphs[3] if rng.random() < 0.02 else graphs[int(rng.integers(0, 3))]
        jobs.append(serve.Job(len(jobs), g, y, seed=1000 + len(jobs), instance=len(jobs),
                              nsweeps=1000, arrival=t, precision=gmrf.FP32_ACC64))
    import torch

    free, _ = torch.cuda.mem_get_info()
    server = serve.Server(budget_bytes=int(0.5 * free), step_sweeps=10, max_active=1024,
                          overlap=overlap)
    server.run(jobs, realtime=True)
    assert len(server.finished) == len(jobs) > 300
    big = [j for j in jobs if j.sites == 1_000_000]
    picks = big + [jobs[i] for i in rng.choice(len(jobs), 5, replace=False)]
    for job in picks:
        ch = gmrf.Chain(job.graph, job.y, precision=job.precision, seed=job.seed,
                        instance=job.instance)
        ch.sweep(job.nsweeps, capture=True)
        mean, var, nacc = ch.posterior_stats()
        assert nacc == 1000
        assert np.array_equal(mean, job.mean) and np.array_equal(var, job.var)
    small = [j for j in jobs if j.sites == 15000]
    errs = [check_against_oracle(orc, small[i], False)
            for i in rng.choice(len(small), 3, replace=False)]
    print(f"served FP32 jobs vs the FP64 oracle: posterior-mean max abs err {max(errs):.2e}")
