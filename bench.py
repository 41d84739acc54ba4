"""Benchmark of the D2V16 windowed-FFT thermal LB step on one MI355X.

Prints ONE JSON line.  The headline workload is the 512x512 thermal quench (rho = rho_c (1 +
0.001 U(-1,1)), u = 0, T = 0.9 T_c, seed 2000) in FP64; the FP32 form of the same grid and the
FP32 batch of 256 independent 128x128 quenches (per-instance T in [0.85, 0.98] T_c) are reported
as variants.  A "step" is one full RK2 step of every instance (two evaluations of R(f): moments,
macroscopic spectral derivatives, forcing, population x and y passes).  Inputs are resident in
HBM before timing starts; the timed region replays the captured step graph.

roofline: algorithmic HBM words per cell of each pass times cells, over the pass's mean launch
duration from HIP events recorded on the library's stream during a second run of steps
(lb_step_timed); the dominant pass (largest time per step) is reported, priced at the reference
word count (REF_WORDS) and at this design's own (ALG_WORDS), and beside it the HBM bytes per
launch the rocprofv3 counters measured (profiles/traffic.json) over the same time.
cpu_baseline: the FP64 CPU oracle stepping the same 512x512 initial condition for a bounded number
of steps on all host cores, and on one core.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (cells×RK2 steps/s) FP32-batched vs FP64-plain; % of HBM roofline"
HBM_PEAK_GBS = 8000.0

# Algorithmic words per cell of one launch of each pass in this design (q = 0), averaged over the
# two RK stages (only pop_x differs: 39 words in stage 1, 55 in stage 2 where the base f^n is read).
ALG_WORDS = {
    "moments": 20,     # read 16 f, write rho, ux, uy, T
    "macro_x1": 9,     # read rho, T, ux, uy; write d_x rho, d_xx rho, d_x T, d_x ux, d_x uy
    "macro_y1": 9,     # read rho, T, ux, uy; write the five y counterparts
    "stress": 17,      # read 12 derivative/moment fields; write S_xx, S_xy, S_yy, div u, C0
    "macro_x2": 6,     # read S_xx, S_xy, div u; write their x-derivatives
    "macro_y2": 6,     # read S_xy, S_yy, div u; write their y-derivatives
    "finalize": 14,    # read rho, T, grad rho, 4 S derivatives, grad div u, C0; write B_x, B_y, C
    "pop_x": 47,       # read 16 f + 7 coefficients (+16 base in stage 2); write 16
    "pop_y": 36,       # read 12 f + 12 partials; write 12
}
WORDS_PER_STEP = 2 * sum(ALG_WORDS.values())   # 328

# The reference count the roofline fraction is priced on: a design with the fewest passes the
# method allows moves 262 words per cell per RK2 step -- an x population pass over the 12
# populations with v_x != 0 (12 f + 7 coefficients read, 4 final + 8 partial writes: 31 words; 47
# in stage 2 with 16 base reads), a y population pass that also sums the next stage's moments
# (12 f + 8 partials + 7 coefficients + 4 x-final populations read, 12 populations + 4 moments
# written), and macroscopic passes X1 (4 read + 5 written), Y1 (9 + 7, the stress formed in it),
# X2 (3 + 3) and Y2 (11 + 3, B and C formed in it).  Each pass here is priced at the words that
# design spends on the same work, never more than this design's own count: the moments at the
# y pass's 4 + 4 moment words, the stress and finalize kernels at the words Y1 and Y2 spend beyond
# 9 and 6, the population x pass at the x pass's 31 / 47 (39 on average).
REF_WORDS = {
    "moments": 8, "macro_x1": 9, "macro_y1": 9, "stress": 7, "macro_x2": 6, "macro_y2": 6,
    "finalize": 8, "pop_x": 39, "pop_y": 36,
}
REF_WORDS_PER_STEP = 262
# On square grids the x and y macroscopic passes of a stage run as one fused launch, timed in the
# x slot: its words are those of both.
FUSED = {"macro_x1": ("macro_xy1", "macro_y1"), "macro_x2": ("macro_xy2", "macro_y2")}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lb_kernels.h", "lb_fft.h", "lb_lines.inc", "lb_lines_xy.inc", "lb_pointwise.hip"):
        h.update(open(os.path.join(ROOT, "paper_1403_3746_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload, pass_name, pops_per_block=None):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources (else None).  The population x pass is looked up for the plan the run
    used (populations per block), which the counter runs force one at a time."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        ent = d.get(workload, {}).get(pass_name)
        if ent and "plans" in ent:
            ent = ent["plans"].get(str(pops_per_block))
        if ent and ent.get("kernel_source_hash") == kernel_source_hash():
            return ent["bytes_per_launch"]
    except Exception:
        return None
    return None


def run_gpu(instances, precision, steps, warmup, timed_steps, settle=None):
    import torch
    from paper_1403_3746_amd.lbfft import Sim

    sim = Sim(instances, precision)
    cells = sum(ic[0].size for _, ic in instances)
    if settle is not None:
        settle(sim)   # GPU clocks up again after the context's set-up, before its warm-up steps
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes = sim.step_timed(timed_steps)
    sim.sync()
    plan = sim.plan(0)
    c = sim.conservation(0)
    sim.close()
    if not np.all(np.isfinite(c)):
        raise RuntimeError("non-finite state after the benchmark")
    dt = t1 - t0
    return dict(mlups=cells * steps / dt / 1e6, ms_per_step=1e3 * dt / steps, cells=cells,
                passes=passes, plan=plan)


def spin(sim, seconds):
    """Step `sim` untimed for about `seconds` of wall time: a GPU that has just come out of idle (or
    has sat through a context's set-up on the host) runs its first tenths of a second a few per
    cent slower than at its settled clocks."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.step(64)
        sim.sync()
    return time.perf_counter() - t0


class GpuWarmer:
    """A throwaway 512x512 FP64 context stepped untimed right before each timed run."""

    def __init__(self):
        from paper_1403_3746_amd import workloads as W
        from paper_1403_3746_amd.lbfft import Sim

        insts, _ = W.config("quench512")
        self.sim = Sim(insts, "fp64")
        self.total = 0.0

    def spin(self, seconds):
        self.total += spin(self.sim, seconds)

    def close(self):
        self.sim.close()


def roofline(res, word_bytes, workload):
    """Roofline of the dominant pass (largest time per step).  `achieved` / `frac` price it at the
    reference count (REF_WORDS), `achieved_design` / `frac_design` at this design's own words."""
    cells = res["cells"]
    passes = res["passes"]
    # a batch of several size classes launches each pass once per class: the pass's time per
    # stage is the mean launch duration times the number of classes, its bytes those of all cells
    nclass = res["plan"].get("size_classes", 1)
    per_pass = {}
    for name, ms in passes.items():
        if ms <= 0:
            continue
        words, ref = ALG_WORDS[name], REF_WORDS[name]
        if name in FUSED and passes.get(FUSED[name][1], 0.0) <= 0:
            other = FUSED[name][1]
            name, words, ref = FUSED[name][0], words + ALG_WORDS[other], ref + REF_WORDS[other]
        alg = ref * word_bytes * cells
        own = words * word_bytes * cells
        ms = ms * nclass
        per_pass[name] = dict(ms=ms, alg_bytes=alg, own_bytes=own, gbs=alg / (ms * 1e-3) / 1e9,
                              gbs_design=own / (ms * 1e-3) / 1e9)
    dom = max(per_pass, key=lambda k: per_pass[k]["ms"])
    d = per_pass[dom]
    traffic = load_traffic(workload, dom, res["plan"]["pops_per_block_x"]) if nclass == 1 else None
    # the same launch priced by the HBM bytes the rocprofv3 counters measured (when they were
    # taken on the current kernel sources)
    measured = None if traffic is None else traffic / (d["ms"] * 1e-3) / 1e9
    step_bytes = res["mlups"] * 1e6 * word_bytes / 1e9
    return dict(bound="hbm", kernel=dom, achieved=round(d["gbs"], 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(d["gbs"] / HBM_PEAK_GBS, 4), traffic=traffic,
                achieved_design=round(d["gbs_design"], 1),
                frac_design=round(d["gbs_design"] / HBM_PEAK_GBS, 4),
                measured_gbs=None if measured is None else round(measured, 1),
                measured_frac=None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                alg_bytes_per_launch=d["alg_bytes"] if nclass == 1 else None,
                alg_bytes_per_pass=d["alg_bytes"], design_bytes_per_pass=d["own_bytes"],
                launches_per_pass=nclass, mean_launch_ms=round(d["ms"] / nclass, 5),
                passes={k: dict(ms=round(v["ms"], 5), gbs=round(v["gbs"], 1),
                                gbs_design=round(v["gbs_design"], 1)) for k, v in per_pass.items()},
                step_frac=round(step_bytes * REF_WORDS_PER_STEP / HBM_PEAK_GBS, 4),
                step_frac_design=round(step_bytes * WORDS_PER_STEP / HBM_PEAK_GBS, 4))


def _oracle_rate(instances, workers, budget_s):
    """MLUPS of the FP64 oracle stepping the first instance on the host with `workers` FFT
    threads: one warm-up step, then as many steps as fit in about budget_s (1..20)."""
    from oracle import model, spectral

    spectral.set_workers(workers)
    try:
        p, ic = instances[0]
        f = model.init_equilibrium(*ic, p)
        t0 = time.perf_counter()
        f = model.rk2_step(f, p)
        t1 = time.perf_counter() - t0
        n = int(max(1, min(20, budget_s / max(t1, 1e-3))))
        t0 = time.perf_counter()
        for _ in range(n):
            f = model.rk2_step(f, p)
        dt = time.perf_counter() - t0
    finally:
        spectral.set_workers(1)
    return ic[0].size * n / dt / 1e6, n


def cpu_baseline(instances, budget_s=15.0, budget_1core_s=8.0):
    workers = os.cpu_count() or 1
    rate, n = _oracle_rate(instances, workers, budget_s)
    rate1, n1 = _oracle_rate(instances, 1, budget_1core_s)
    model_name = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model_name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    shape = instances[0][1][0].shape
    return dict(value=round(rate, 4), unit="MLUPS", cores=workers, kind="oracle",
                cpu=model_name,
                sample=f"FP64 oracle, {shape[1]}x{shape[0]} quench, {n} RK2 steps after 1 "
                       f"warm-up step, scipy.fft workers={workers}",
                single_core=dict(value=round(rate1, 4), unit="MLUPS", cores=1,
                                 sample=f"the same, {n1} RK2 steps, scipy.fft workers=1"))


def calib_copy():
    """A plain device copy of exactly 256 MiB (read 256 MiB, write 256 MiB), three times: the
    reference dispatch for scaling the HBM byte counters."""
    import torch
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--timed-steps", type=int, default=50)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--gpu-warm", type=float, default=0.5,
                    help="seconds of untimed stepping of a throwaway context before each timed run")
    ap.add_argument("--only", choices=("quench512_fp64", "quench512_fp32", "batch128x256_fp32",
                                       "ragged64_fp32", "quench2048_fp32", "slab64_fp64"),
                    help="run one workload only and print its summary (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with a 256 MiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not built"}))
        sys.exit(2)

    from paper_1403_3746_amd import workloads as W

    if args.only:
        # profiling runs: the measured context itself is stepped untimed first, so that the
        # profiler sees only this workload's kernels, at settled clocks
        name, prec = args.only.rsplit("_", 1)
        insts, _ = W.config(name)
        settle = (lambda sim: spin(sim, args.gpu_warm)) if args.gpu_warm > 0 else None
        r = run_gpu(insts, prec, args.steps, args.warmup, args.timed_steps, settle)
        print(json.dumps({"workload": args.only, "mlups": round(r["mlups"], 2),
                          "ms_per_step": round(r["ms_per_step"], 5), "plan": r["plan"],
                          "roofline": roofline(r, 8 if prec == "fp64" else 4, args.only)}))
        if args.calib_copy:
            calib_copy()
        return

    insts, _ = W.config("quench512")
    # every timed run starts on a GPU at its settled clocks (the variants also run before the
    # headline), so that a short timed region measures the steady rate of a long run
    warmer = GpuWarmer() if args.gpu_warm > 0 else None
    settle = (lambda sim: warmer.spin(args.gpu_warm)) if warmer else None
    var, rb = {}, None
    if not args.no_variants:

        def variant(name, prec, steps, warmup, timed):
            vi, _ = W.config(name)
            r = run_gpu(vi, prec, steps, warmup, timed, settle)
            key = f"{name}_{prec}"
            return r, dict(mlups=round(r["mlups"], 2), ms_per_step=round(r["ms_per_step"], 5),
                           steps=steps, roofline=roofline(r, 8 if prec == "fp64" else 4, key),
                           plan=r["plan"])

        _, var["quench512_fp32"] = variant("quench512", "fp32", args.steps, args.warmup, args.timed_steps)
        rb, var["batch128x256_fp32"] = variant("batch128x256", "fp32", args.steps, args.warmup,
                                               max(1, args.timed_steps // 4))
        # the large single domain with its per-step FP64 conservation history, and the ragged batch
        # (fewer steps: each step is 8-16x the work of the headline's)
        big_steps, big_warm = max(10, args.steps // 8), max(2, args.warmup // 4)
        _, var["quench2048_fp32"] = variant("quench2048", "fp32", big_steps, big_warm, 2)
        _, var["ragged64_fp32"] = variant("ragged64", "fp32", big_steps, big_warm, 2)
    main_res = run_gpu(insts, "fp64", args.steps, args.warmup, args.timed_steps, settle)
    warm_s = 0.0
    if warmer:
        warm_s = round(warmer.total, 3)
        warmer.close()
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "quench512: 512x512 periodic thermal quench, FP64, one instance",
                   "grid": [512, 512], "instances": 1, "precision": "fp64",
                   "params": "dx=1 dt=1e-3 tau=1e-2 K=1e-2 a=9/49 b_w=2/21 T=0.9T_c b=2 H=zeta=q=0"},
        "roofline": roofline(main_res, 8, "quench512_fp64"),
        "plan": main_res["plan"],
        "gpu_warm_s": warm_s,
    }
    if var:
        var["fp32_batched_over_fp64_plain"] = round(rb["mlups"] / main_res["mlups"], 3)
        out["variants"] = var
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(insts)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
