"""Host-side parts of the benchmark (CPU): the one-GPU refusal of --gpus N > 1, the drift study's
frames generated in worker processes (equal to the scene's own frames), and the CPU-baseline leg,
which runs the oracle and reports the record the benchmark line carries."""
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
