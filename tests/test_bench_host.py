"""bench.py's bookkeeping without a GPU: algorithmic words, the fused x+y passes, the roofline
fields of the JSON line, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_words_per_step():
    # stage 1 and stage 2 together; pop_x averages its 39 (stage 1) and 55 (stage 2) words
    assert bench.WORDS_PER_STEP == 2 * sum(bench.ALG_WORDS.values()) == 328
    assert bench.ALG_WORDS["pop_x"] == (39 + 55) // 2


def test_reference_words_never_exceed_the_design_count():
    # the reference count prices the x population pass at its 31 / 47 words (39 on average) and
    # no pass above this design's own words; the passes together stay within the 262 words per
    # step of the reference design
    assert bench.REF_WORDS["pop_x"] == (31 + 47) // 2
    assert set(bench.REF_WORDS) == set(bench.ALG_WORDS)
    for k, v in bench.REF_WORDS.items():
        assert 0 < v <= bench.ALG_WORDS[k]
    assert 2 * sum(bench.REF_WORDS.values()) <= bench.REF_WORDS_PER_STEP == 262


def test_roofline_of_fused_and_separate_passes():
    cells = 512 * 512
    passes = {"moments": 0.0074, "macro_x1": 0.0142, "macro_y1": 0.0, "stress": 0.0057,
              "macro_x2": 0.0104, "macro_y2": 0.0, "finalize": 0.0048, "pop_x": 0.0213,
              "pop_y": 0.0148}
    res = dict(cells=cells, passes=passes, mlups=1500.0, plan=dict(pops_per_block_x=2))
    r = bench.roofline(res, 8, "no_such_workload")
    assert r["kernel"] == "pop_x" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    # fused launches are reported under their own names with both passes' words
    assert "macro_xy1" in r["passes"] and "macro_x1" not in r["passes"]
    xy1 = 18 * 8 * cells / (0.0142e-3) / 1e9
    assert abs(r["passes"]["macro_xy1"]["gbs"] - round(xy1, 1)) < 0.2
    alg = 39 * 8 * cells
    assert r["alg_bytes_per_launch"] == alg
    assert abs(r["achieved"] - alg / 0.0213e-3 / 1e9) < 0.2
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4
    assert abs(r["achieved_design"] - 47 * 8 * cells / 0.0213e-3 / 1e9) < 0.2
    assert r["traffic"] is None and r["measured_frac"] is None   # no counters for this workload
    assert abs(r["step_frac"] - 1500e6 * 262 * 8 / 1e9 / 8000) < 1e-4
    assert abs(r["step_frac_design"] - 1500e6 * 328 * 8 / 1e9 / 8000) < 1e-4
    # separate launches (non-square grids) keep the x and y names
    passes.update(macro_y1=0.0107, macro_y2=0.0079)
    r = bench.roofline(dict(res, passes=passes), 8, "no_such_workload")
    assert {"macro_x1", "macro_y1", "macro_x2", "macro_y2"} <= set(r["passes"])


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip().splitlines()[-1])["error"]


def test_measured_traffic_fraction(monkeypatch):
    monkeypatch.setattr(bench, "load_traffic", lambda w, p, ppb: 119_000_000 if ppb == 2 else None)
    res = dict(cells=512 * 512, passes={"pop_x": 0.0211, "pop_y": 0.0147}, mlups=1500.0,
               plan=dict(pops_per_block_x=2))
    r = bench.roofline(res, 8, "quench512_fp64")
    assert r["traffic"] == 119_000_000
    assert abs(r["measured_gbs"] - 119e6 / 0.0211e-3 / 1e9) < 0.1
    assert abs(r["measured_frac"] - r["measured_gbs"] / 8000.0) < 1e-4


def test_traffic_is_looked_up_for_the_plan_and_sources(tmp_path, monkeypatch):
    # the population x pass's counters are kept per plan; another plan or other kernel sources
    # give no traffic figure
    h = bench.kernel_source_hash()
    d = {"w": {"moments": {"bytes_per_launch": 5, "kernel_source_hash": h},
               "pop_x": {"plans": {"2": {"bytes_per_launch": 7, "kernel_source_hash": h},
                                   "4": {"bytes_per_launch": 9, "kernel_source_hash": "other"}}}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.load_traffic("w", "moments", 1) == 5
    assert bench.load_traffic("w", "pop_x", 2) == 7
    assert bench.load_traffic("w", "pop_x", 4) is None     # taken on other sources
    assert bench.load_traffic("w", "pop_x", 1) is None     # plan not measured
    assert bench.load_traffic("x", "pop_x", 2) is None


def test_roofline_of_a_batch_of_several_size_classes():
    # each pass runs once per class: per stage its time is the mean launch times the class count,
    # its bytes those of every cell of the batch; no single-launch traffic figure applies
    cells = 64 * 64 + 128 * 128
    passes = {"moments": 0.002, "macro_x1": 0.004, "macro_y1": 0.0, "stress": 0.002,
              "macro_x2": 0.003, "macro_y2": 0.0, "finalize": 0.002, "pop_x": 0.006, "pop_y": 0.005}
    res = dict(cells=cells, passes=passes, mlups=500.0, plan=dict(pops_per_block_x=2, size_classes=2))
    r = bench.roofline(res, 4, "quench512_fp32")
    assert r["kernel"] == "pop_x" and r["launches_per_pass"] == 2
    assert abs(r["achieved"] - 39 * 4 * cells / (2 * 0.006e-3) / 1e9) < 0.2
    assert r["mean_launch_ms"] == 0.006 and r["alg_bytes_per_launch"] is None
    assert r["traffic"] is None and r["measured_frac"] is None
