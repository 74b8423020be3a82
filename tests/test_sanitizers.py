"""Host-code sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer), CPU only.

The oracle (plain C) is rebuilt with gcc -fsanitize=address,undefined and runs a config-1 frame with
every debug tap and its library routines in a subprocess that preloads the ASan runtime. The HIP
library is rebuilt with the sanitizers on its host code only (-Xarch_host before each -fsanitize=;
device code is not instrumented) and its argument checks, defaults and error strings run the same
way: there is no GPU here, so every call that would reach the device is left out. Any sanitizer
report, or a non-zero exit, fails the test.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(script, env_extra, tmp_path):
    path = tmp_path / "run.py"
    path.write_text(textwrap.dedent(script))
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, str(path)], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error:" not in report, report[-4000:]
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "libtt_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", *SAN, "-o", str(lib),
                    os.path.join(ROOT, "oracle", "tt_oracle.c"), "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    out = _run("""
        import numpy as np
        from oracle import oracle as O
        from paper_2007_08576_amd import synth
        # a small sequence, two frames in a row (the second warm-started), every debug tap
        sc = synth.make_sequence(seed=5, M=900, N=24, K1=120, width=96, height=72, n_frames=3, name="san")
        K = sc.intr
        s = O.Stream(O.default_params(num_control_points=sc.num_control_points, seed=1, lm_iters=3),
                     O.intrinsics(K.width, K.height, K.fx, K.fy, K.cx, K.cy))
        s.set_template(sc.pts, sc.feat_xyz, sc.feat_desc)
        for t in (1, 2):
            fr = sc.frame(t)
            v, q, d = s.track_frame(fr.depth, fr.feat_xyz, fr.feat_desc, debug=True)
            assert np.isfinite(v).all()
        s.close()
        idx, dist = O.hamming_match(sc.feat_desc, fr.feat_desc)
        A = np.random.default_rng(0).standard_normal((40, 40))
        A = A @ A.T + 40 * np.eye(40)
        L, rc = O.cholesky(A)
        assert rc == 0
        x = O.cholesky_solve(L, np.ones(40))
        assert np.allclose(A @ x, 1.0)
        print("oracle ok")
    """, {"TT_ORACLE_LIB": str(lib), "LD_PRELOAD": f"{asan}:{ubsan}"}, tmp_path)
    assert "oracle ok" in out


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("hipcc or the clang ASan runtime is not installed")
    from paper_2007_08576_amd import build as B
    host_san = [f for flag in SAN for f in ("-Xarch_host", flag)]
    objs = []
    procs = []
    for src in B.sources():
        obj = tmp_path / (os.path.basename(src) + ".o")
        objs.append(str(obj))
        procs.append(subprocess.Popen([hipcc] + B.FLAGS + host_san + ["-g", "-c", src, "-o", str(obj)],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-3000:]
    lib = tmp_path / "libtt_san.so"
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *host_san, "-shared-libasan", "-o", str(lib)]
                   + objs, check=True, capture_output=True)
    out = _run(f"""
        import ctypes as C
        from paper_2007_08576_amd import tt
        tt.LIB_PATH = {str(lib)!r}
        L = tt.lib()
        p = tt.default_params(num_control_points=40)
        K = tt.intrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)
        h = C.c_void_p()
        for field, bad in (("knn", 3), ("ransac_refs", 0), ("lm_iters", -1), ("H", 0.0), ("precision", 7),
                           ("solver", 5), ("arap_knn", 99), ("graph", 2), ("ir_iters", 9)):
            q = tt.default_params(num_control_points=40)
            setattr(q, field, bad)
            assert L.tt_create_stream(C.byref(q), C.byref(K), None, C.byref(h)) == tt.TT_EINVAL, field
        badK = tt.intrinsics(2, 120, 150.0, 150.0, 80.0, 60.0)
        assert L.tt_create_stream(C.byref(p), C.byref(badK), None, C.byref(h)) == tt.TT_EINVAL
        assert L.tt_create_stream(None, C.byref(K), None, C.byref(h)) == tt.TT_EINVAL
        for code in range(-6, 1):
            assert L.tt_strerror(code)
        assert L.tt_destroy(None) == tt.TT_EINVAL and L.tt_sync(None) == tt.TT_EINVAL
        sp = tt.ServerParams()
        L.tt_server_default_params(C.byref(sp))
        sp.max_rounds_ahead = 99
        assert L.tt_server_create(C.byref(sp), None, C.byref(h)) == tt.TT_EINVAL
        assert L.tt_server_submit(None, None, None, None) == tt.TT_EINVAL
        assert L.tt_server_destroy(None) == tt.TT_EINVAL
        op = tt.OrbParams()
        L.tt_orb_default_params(C.byref(op))
        print("library host ok")
    """, {"LD_PRELOAD": rt[-1]}, tmp_path)
    assert "library host ok" in out
