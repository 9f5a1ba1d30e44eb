"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc) and
run through every entry point on a ragged scene (partial tiles, off-screen and unrendered
Gaussians) in both binning modes, plus the projection; its sums must equal those of the regular
build. A sanitizer report fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gsinputs
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-ffp-contract=off",
           os.path.join(HERE, "native", "oracle_sanitize.c"),
           os.path.join(os.path.dirname(HERE), "oracle", "gsoracle.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)

    s = gsinputs.make_scene("C1", seed=51, n=900, width=70, height=37)
    s["means2d"][:10] -= np.float32(30.0)
    s["radii"][10:20] = 0
    s["opacity"][20:30] = 0.002
    W, H, n = s["width"], s["height"], len(s["radii"])
    g = gsinputs.make_dloss(W, H, 52)
    s3 = gsinputs.make_scene3d(n=700, seed=53, width=70, height=37)
    K, deg = 16, 3
    arrays = {"means2d": s["means2d"], "conics": s["conics"], "opacity": s["opacity"],
              "colors": s["colors"], "depths": s["depths"], "dloss": g,
              "means3d": s3["means3d"], "scales": s3["scales"], "quats": s3["quats"],
              "sh": s3["sh"], "cam": oracle.camera_array(s3["camera"])}
    for k, a in arrays.items():
        np.ascontiguousarray(a, np.float64).tofile(tmp_path / k)
    np.ascontiguousarray(s["radii"], np.int32).tofile(tmp_path / "radii")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe), str(tmp_path), str(W), str(H), str(n), "700", str(K), str(deg)],
                       capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]

    # the sanitized build computes what the regular build computes
    lines = dict((ln.split()[0] + (ln.split()[1] if ln.startswith("mode") else ""), ln.split())
                 for ln in r.stdout.strip().splitlines())
    for mode in (0, 1):
        f = lines[f"mode{mode}"]
        pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                                  s["opacity"], mode)
        fw = oracle.forward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"],
                            (0.1, 0.2, 0.3))
        bw = oracle.backward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"],
                             g, (0.1, 0.2, 0.3))
        assert int(f[3]) == len(pl) == int(f[4])
        np.testing.assert_allclose(float(f[6]), fw["image"].sum(), rtol=1e-12)
        np.testing.assert_allclose(float(f[8]), fw["final_T"].sum(), rtol=1e-12)
        for idx, k in ((10, "dmeans2d"), (12, "dconics"), (14, "dopacity"), (16, "dcolors")):
            np.testing.assert_allclose(float(f[idx]), bw[k].sum(), rtol=1e-9, atol=1e-12)
    p = lines["project"]
    pr = oracle.project(s3)
    np.testing.assert_allclose(float(p[2]), pr["means2d"].sum(), rtol=1e-12)
    np.testing.assert_allclose(float(p[4]), pr["conics"].sum(), rtol=1e-12)
    np.testing.assert_allclose(float(p[6]), pr["colors"].sum(), rtol=1e-12)
    assert int(p[8]) == int(pr["radii"].sum())
