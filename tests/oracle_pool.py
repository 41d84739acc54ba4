"""Oracle runs of benchmark instances in worker processes (spawned, so they hold no GPU state):
the live references of the benchmark-size parity tests.  Test infrastructure only."""
import multiprocessing as mp
import os


def oracle_workers():
    """FFT threads the oracle may use on this host (the GPU machine grants one GPU's share, 16)."""
    return max(1, min(16, os.cpu_count() or 1))


def _moments_at(args):
    from oracle import model, spectral
    from paper_1403_3746_amd import workloads as W
    name, k, steps, workers = args
    spectral.set_workers(workers)
    insts, _ = W.config(name)
    p, ic = insts[k]
    f = model.run(model.init_equilibrium(*ic, p), p, steps)
    return k, model.moments(f, p)


def moments_at(name, instances, steps, procs=8):
    """{k: (rho, ux, uy, T)} of the oracle after `steps` RK2 steps of instances k of workload
    `name`, largest grids first, in up to `procs` spawned processes sharing the host's cores."""
    from paper_1403_3746_amd import workloads as W
    insts, _ = W.config(name)
    order = sorted(instances, key=lambda k: -insts[k][1][0].size)
    procs = max(1, min(procs, len(order)))
    workers = max(1, oracle_workers() // procs)
    with mp.get_context("spawn").Pool(procs) as pool:
        return dict(pool.imap_unordered(_moments_at, [(name, k, steps, workers) for k in order]))
