"""The benchmark's CPU baseline product (eigenvalues taken once, rfft2 / irfft2) against the
oracle's FFT2 products, and the benchmark's byte accounting (CPU only)."""
import numpy as np
import pytest

import bench
import synth
from oracle import bttb as obttb
from oracle import prism as oprism


@pytest.mark.parametrize("g", [synth.SMALL, synth.Grid(7, 9, 11, 5, 3, 40.0, 30.0, 25.0, decl=20.0)])
def test_cpu_baseline_operator_equals_oracle(g):
    og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field)
    r = np.random.default_rng(4)
    x = r.uniform(0.0, 1.0, g.model_shape)
    v = r.standard_normal(g.data_shape)
    for kind in (oprism.GRAVITY, oprism.MAGNETIC):
        T = obttb.kernel_array(kind, og)
        op = bench.CpuFFTOperator(T, g.sx, g.sy, workers=1)
        y, z = op.matvec(x), op.rmatvec(v)
        y_ref, z_ref = obttb.fft_matvec(T, x, g.sx, g.sy), obttb.fft_rmatvec(T, v, g.sx, g.sy)
        assert np.linalg.norm(y - y_ref) <= 1e-13 * np.linalg.norm(y_ref)
        assert np.linalg.norm(z - z_ref) <= 1e-13 * np.linalg.norm(z_ref)


def test_b_alg_matches_the_formula():
    # 2 nz Px (Py/2+1) 2b + 2 nx ny nz b + 2 sx sy b: 84.67 MB (FP32) and 169.35 MB (FP64) at
    # 256x256x32 with 512-point transforms
    info = dict(nz=32, nx=256, ny=256, sx=256, sy=256, Px=512, Py=512)
    assert bench.b_alg(info, 4) == 84_672_512
    assert bench.b_alg(info, 8) == 2 * 84_672_512
    # the solver's product launches: method bytes exclude the row spectra U
    info.update(eig_bytes=32 * 257 * 512 * 8)
    alg, inter = bench.group_kernel_bytes([info], 4)
    n = 32 * 256 * 256
    assert alg["fwd_row_r2c"] == 4 * n * 4 and inter["fwd_row_r2c"] == 32 * 257 * 256 * 8
    assert alg["fwd_col_eig_sum"] == info["eig_bytes"]


def test_more_than_one_gpu_is_refused():
    # one GPU only: --gpus N > 1 exits with status 2 and says so, before touching a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=root)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_launch_shape_option():
    # --launch fixes the timed solve's launch shape; malformed values fail at parsing
    assert bench.parse(["--launch", "512,128,128,2"]).launch == [512, 128, 128, 2]
    assert bench.parse([]).launch is None
    for bad in ("512,128,128", "512,128,x,2", "512,0,128,2"):
        with pytest.raises(SystemExit):
            bench.parse(["--launch", bad])


def test_dense_baseline_runs_both_sizes():
    out = bench.cpu_dense_baselines(budget_s=0.05)
    assert set(out) == {"16x16x8", "12x12x6"}
    assert all(v["op_pairs_per_s"] > 0 and v["pairs"] >= 2 for v in out.values())
