"""Write oracle reference samples for the GPU parity tests at benchmark sizes.

Runs only the FP64 CPU oracle (oracle/) on the seeded benchmark inputs (workloads.config) and
stores, per instance, the moments rho, ux, uy, T at a fixed random sample of cells together with
each field's max |value| over the whole grid (the parity norm's denominators):

  quench512_oracle.npz  : 512x512 quench, steps 10 and 100
  ragged64_oracle.npz   : every instance of the 64-instance ragged batch, step 50
  quench2048_oracle.npz : 2048x2048 quench, step 5

Usage: python tests/golden/make_oracle_samples.py [--procs N] [--only NAME]
(about 15 minutes on 8 cores, and 10 more for quench2048)
"""
import argparse
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SAMPLE_SEED = 424242


def sample_cells(n_cells, k, key):
    rng = np.random.default_rng(SAMPLE_SEED + key)
    return np.sort(rng.choice(n_cells, size=min(k, n_cells), replace=False))


def run_instance(args):
    from oracle import model, spectral
    from paper_1403_3746_amd import workloads as W
    name, k, checkpoints, nsample, workers = args
    spectral.set_workers(workers)
    insts, _ = W.config(name)
    p, ic = insts[k]
    f = model.init_equilibrium(*ic, p)
    idx = sample_cells(ic[0].size, nsample, k)
    out = {}
    step = 0
    for cp in sorted(checkpoints):
        f = model.run(f, p, cp - step)
        step = cp
        mom = model.moments(f, p)
        for fname, g in zip(("rho", "ux", "uy", "T"), mom):
            out[f"s{cp}_{fname}"] = g.reshape(-1)[idx]
            out[f"s{cp}_{fname}_absmax"] = np.abs(g).max()
    out["idx"] = idx
    return k, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    from paper_1403_3746_amd import workloads as W
    jobs = []
    if a.only in ("", "quench512"):
        jobs.append(("quench512", [("quench512", 0, [10, 100], 16384, a.procs)]))
    if a.only in ("", "quench2048"):
        jobs.append(("quench2048", [("quench2048", 0, [5], 16384, a.procs)]))
    if a.only in ("", "ragged64"):
        insts, _ = W.config("ragged64")
        # largest first so the pool finishes evenly
        order = sorted(range(len(insts)), key=lambda k: -insts[k][1][0].size)
        jobs.append(("ragged64", [("ragged64", k, [50], 2048, 1) for k in order]))
    for name, tasks in jobs:
        with mp.Pool(min(a.procs, len(tasks))) as pool:
            res = dict(pool.imap_unordered(run_instance, tasks))
        flat = {}
        for k, d in res.items():
            for key, v in d.items():
                flat[f"i{k}_{key}"] = v
        path = os.path.join(HERE, f"{name}_oracle.npz")
        np.savez_compressed(path, **flat)
        print("wrote", path, os.path.getsize(path), "bytes", flush=True)


if __name__ == "__main__":
    main()
