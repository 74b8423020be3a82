"""Host-side parts of the benchmark (CPU): the one-GPU refusal of --gpus N > 1, the drift study's
frames generated in worker processes (equal to the scene's own frames), the CPU-baseline leg,
which runs the oracle and reports the record the benchmark line carries, and the batched-assembly
summary of a kernel trace."""
import csv
import json
import os
import subprocess
import sys

import numpy as np

from paper_2007_08576_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_worker_generated_frames_equal_the_scene_frames():
    sc = synth.make_config2(n_frames=300)
    got = synth.config2_arrays(2, 300, [1, 7])
    for (depth, fx, fd, gt), t in zip(got, (1, 7)):
        f = sc.frame(t)
        assert np.array_equal(depth, f.depth) and np.array_equal(fd, f.feat_desc)
        assert np.array_equal(fx, f.feat_xyz, equal_nan=True) and np.array_equal(gt, f.gt_vertices)


def test_cpu_baseline_record():
    sys.path.insert(0, ROOT)
    import bench
    sc = synth.make_config1(1)
    rec, verts = bench.cpu_baseline(sc, sc.frame(1), 2)
    assert rec["kind"] == "oracle" and rec["unit"] == "frames/s" and rec["cores"] == 1
    assert rec["value"] > 0 and "LM iterations" in rec["sample"]
    assert verts.shape == (sc.pts.shape[0], 3) and np.isfinite(verts).all()


def test_assembly_batched_summary_windows(tmp_path):
    """Per LM round, the window runs from the first assembly kernel's start to the last one's end
    before the round's factorisation, whichever launch form the round used: per-stream kernels,
    the first iteration's multi-system kernels, or the later iterations' fused ones. The first
    frame's ten rounds are left out."""
    sys.path.insert(0, ROOT)
    import bench
    rows, t = [], 0
    plan = {0: ["k_data_rows", "k_arap_assemble", "k_data_assemble"],  # warm frame, per-stream kernels
            10: ["k_rows_multi", "k_scalars_multi", "k_arap_multi", "k_data_multi", "k_damp_multi"]}
    later = ["k_rows_arap_multi", "k_data_multi", "k_damp_multi"]
    expect = []
    for r in range(20):
        names = plan.get(r, plan[0] if r < 10 else later)
        start = t
        end = None
        for k in names:
            rows.append({"Kernel_Name": f"void (anonymous namespace)::{k}(args)", "Start_Timestamp": t,
                         "End_Timestamp": t + 7000})
            if k in ("k_data_rows", "k_arap_assemble", "k_data_assemble", "k_rows_multi", "k_arap_multi",
                     "k_data_multi", "k_rows_arap_multi"):
                end = t + 7000
            t += 10000
        if r >= 10:
            expect.append((end - start) / 1e3)
        rows.append({"Kernel_Name": "void (anonymous namespace)::k_chol_dataflow(args)", "Start_Timestamp": t,
                     "End_Timestamp": t + 50000})
        t += 60000
    trace = tmp_path / "t_kernel_trace.csv"
    with open(trace, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    run = tmp_path / "run.json"
    run.write_text(json.dumps({"assembly_batched": {"config": 4, "streams": [{"N": 100, "M": 1000, "K": 100}],
                                                    "frames": 2}}) + "\n")
    out = tmp_path / "out.json"
    bench.assembly_batched_summary(str(trace), str(run), str(out), "cmd")
    rec = json.loads(out.read_text())
    assert rec["rounds"] == 10
    assert abs(rec["mean_window_us"] - float(np.mean(expect))) < 1e-9
    assert abs(rec["min_window_us"] - min(expect)) < 1e-9 and abs(rec["max_window_us"] - max(expect)) < 1e-9
