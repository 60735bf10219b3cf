"""GPU joint RRCG through the C ABI vs the FP64 oracle (run on an MI355X)."""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import bttb as obttb
from oracle import prism as oprism
from oracle import rrcg as orrcg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


def ogeom(g):
    return oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field,
                           ox=g.ox, oy=g.oy)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


_PROBLEMS = {}


def problem(g, dense: bool):
    """Oracle operators, kernel arrays and noisy data of a random-box model on grid g."""
    key = (g, dense)
    if key in _PROBLEMS:
        return _PROBLEMS[key]
    og = ogeom(g)
    T = [obttb.kernel_array(k, og) for k in (oprism.GRAVITY, oprism.MAGNETIC)]
    if dense:
        ops = [obttb.DenseOperator(oprism.dense_matrix(k, og), og) for k in (oprism.GRAVITY, oprism.MAGNETIC)]
    else:
        ops = [obttb.FFTOperator(T[i], g.sx, g.sy, workers=8) for i in range(2)]
    rho, kap = synth.random_boxes(g, nbodies=3, seed_workload=2, index=g.nx)
    if rho.max() == 0:
        rho[g.nz // 3, 2:5, 2:5] = 0.5
        kap[g.nz // 3, 2:5, 2:5] = 0.03
    d = [ops[0].matvec(rho), ops[1].matvec(kap)]
    sig = [synth.noise_sigma(d[0], 0.02, 0.01 * np.abs(d[0]).max()),
           synth.noise_sigma(d[1], 0.02, 0.01 * np.abs(d[1]).max())]
    dobs = [d[i] + sig[i] * synth.normal_like(d[i].shape, 3, 20 + i) for i in range(2)]
    data = orrcg.Data(dobs=dobs, wd=[1.0 / s for s in sig],
                      wdepth=[synth.depth_weight(g, 2.0), synth.depth_weight(g, 3.0)])
    _PROBLEMS[key] = (ops, T, data, (rho, kap))
    return _PROBLEMS[key]


def gpu_solver(pk, g, T, data, prm, dtype, state=None, use_graph=True):
    ops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=dtype) for i in range(2)]
    m0 = state.m if state is not None else None
    s = pk.JointRRCG(ops, data.dobs, data.wd, data.wdepth, lo=prm.lo, hi=prm.hi, alpha0=prm.alpha0, q=prm.q,
                     alpha_min=prm.alpha_min, lam=prm.lam, eps2=prm.eps2, coupled=prm.coupled,
                     restart=prm.restart, p_norm=prm.p_norm, gramian=prm.gramian, anchor=prm.anchor, m0=m0,
                     use_graph=use_graph)
    if state is not None:
        for i in range(2):
            s.p[i].copy_(torch.as_tensor(state.p[i], dtype=dtype, device="cuda"))
            if prm.anchor == "prev":
                s.mprev[i].copy_(torch.as_tensor(state.m_prev[i], dtype=dtype, device="cuda"))
        s.set_scalars(alpha=state.alpha, L_prev=state.L_prev, frozen=state.frozen, k=state.k)
        s.refresh()
    return s, ops


BASE = dict(alpha0=(2000.0, 5000.0), q=(0.8, 0.85), lam=(2.0, 100.0), lo=(0.0, 0.0), hi=(1.0, 0.1))
VARIANTS = [
    dict(n_inner=1, restart=False),                       # the printed single loop
    dict(n_inner=6, restart=True),                        # nested reading
    dict(n_inner=4, restart=True, coupled=False, lam=(0.0, 0.0)),   # stand-alone
    dict(n_inner=4, restart=True, p_norm=2, alpha_min=(500.0, 500.0)),  # joint minimum length
    dict(n_inner=3, restart=False, gramian="weighted", lam=(1e-3, 1e-1)),
    dict(n_inner=1, restart=False, anchor="prev"),        # RRCG:4 as printed, single loop
    dict(n_inner=4, restart=True, anchor="prev", gramian="weighted", lam=(1e-3, 1e-1)),
]


# SMALL (transform 32) and SUB (transform 24 = 8 3, a radix-3 pass): the CG pieces ride on the
# products' row transforms (group path); RAGGED (24 x 16 with 9 stations per 16-point row, which
# has no half form): the general kernels and separate elementwise kernels
RAGGED = synth.Grid(7, 9, 11, 5, 3, 40.0, 30.0, 25.0, decl=20.0)


@pytest.mark.parametrize("g", [synth.SMALL, synth.SUB, RAGGED], ids=["pow2-fused", "radix3-fused", "general"])
@pytest.mark.parametrize("var", range(len(VARIANTS)))
def test_single_outer_step_parity_fp64(pk, var, g):
    ops, T, data, _ = problem(g, dense=True)
    v = dict(VARIANTS[var])
    n_inner = v.pop("n_inner")
    kw = dict(BASE)
    kw.update(v)
    prm = orrcg.Params(**kw)
    # a mid-solve state: two oracle outer steps from the start
    st, _ = orrcg.run(ops, data, prm, n_outer=2, n_inner=n_inner)
    ref, rec = orrcg.outer_step(ops, data, prm, st, n_inner)
    s, gops = gpu_solver(pk, g, T, data, prm, torch.float64, state=st)
    s.step(n_inner)
    sc = s.scalars()
    for i in range(2):
        assert rel(host(s.m[i]), ref.m[i]) <= 1e-12
        # p is the CG direction (an intermediate, O(100) in size), not a result
        assert rel(host(s.p[i]), ref.p[i]) <= 1e-11
        if prm.anchor == "prev":
            assert rel(host(s.mprev[i]), ref.m_prev[i]) <= 1e-12
        assert sc["alpha"][i] == pytest.approx(ref.alpha[i], rel=1e-15)
        assert sc["phi"][i] == pytest.approx(rec["phi"][i], rel=1e-12)
        assert sc["L_prev"][i] == pytest.approx(ref.L_prev[i], rel=1e-12)
        assert sc["frozen"][i] == ref.frozen[i]
    assert sc["k"] == ref.k
    assert sc["converged"] == rec["converged"]
    assert sc["gramian"] == pytest.approx(rec["gramian"], rel=1e-10)
    assert not sc["nonfinite"]
    s.close()


def test_full_solve_divergence_curve_fp64(pk):
    g = synth.SMALL
    ops, T, data, _ = problem(g, dense=True)
    prm = orrcg.Params(**BASE)
    st = orrcg.initial_state(data, prm, g.model_shape)
    s, _ = gpu_solver(pk, g, T, data, prm, torch.float64)
    curve = []
    for k in range(8):
        st, rec = orrcg.outer_step(ops, data, prm, st, 10)
        s.step(10)
        curve.append(max(rel(host(s.m[i]), st.m[i]) for i in range(2)))
    print("divergence per outer step:", " ".join(f"{c:.2e}" for c in curve), flush=True)
    assert max(curve) <= 1e-8
    s.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_mid_grid_single_step(pk, dtype, tol):
    g = synth.MID
    ops, T, data, _ = problem(g, dense=False)
    prm = orrcg.Params(**BASE)
    st, _ = orrcg.run(ops, data, prm, n_outer=1, n_inner=5)
    ref, rec = orrcg.outer_step(ops, data, prm, st, 5)
    s, _ = gpu_solver(pk, g, T, data, prm, dtype, state=st)
    s.step(5)
    sc = s.scalars()
    errs = [rel(host(s.m[i]), ref.m[i]) for i in range(2)]
    print(f"{dtype}: model rel err {errs}, phi {sc['phi']} vs {rec['phi']}", flush=True)
    assert max(errs) <= tol
    for i in range(2):
        assert sc["phi"][i] == pytest.approx(rec["phi"][i], rel=tol)
    s.close()


def test_checkpoint_resume_is_bitwise(pk):
    g = synth.SUB
    _, T, data, _ = problem(g, dense=True)
    prm = orrcg.Params(**BASE)
    s, _ = gpu_solver(pk, g, T, data, prm, torch.float64)
    s.run(2, 4)
    ck = s.state_dict()
    s.run(2, 4)
    a = [host(x) for x in s.m] + [host(x) for x in s.p]
    sa = s.scalars()
    s2, _ = gpu_solver(pk, g, T, data, prm, torch.float64)
    s2.load_state_dict(ck)
    s2.run(2, 4)
    b = [host(x) for x in s2.m] + [host(x) for x in s2.p]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert s2.scalars()["alpha"] == sa["alpha"] and s2.scalars()["k"] == sa["k"]
    s.close()
    s2.close()


def test_repeatable_and_bounded(pk):
    g = synth.SUB
    _, T, data, _ = problem(g, dense=True)
    prm = orrcg.Params(**BASE)
    outs = []
    for _ in range(2):
        s, _ = gpu_solver(pk, g, T, data, prm, torch.float64)
        s.run(3, 5)
        m = [host(x) for x in s.m]
        assert m[0].min() >= 0.0 and m[0].max() <= 1.0 and m[1].min() >= 0.0 and m[1].max() <= 0.1
        outs.append(m)
        s.close()
    assert all(np.array_equal(x, y) for x, y in zip(*outs))


def test_nonfinite_flag_from_host_data(pk):
    g = synth.SUB
    _, T, data, _ = problem(g, dense=True)
    bad = orrcg.Data(dobs=[data.dobs[0].copy(), data.dobs[1]], wd=data.wd, wdepth=data.wdepth)
    bad.dobs[0][3, 4] = math.nan
    prm = orrcg.Params(**BASE)
    s, _ = gpu_solver(pk, g, T, bad, prm, torch.float64)
    s.step(2)
    assert s.scalars()["nonfinite"]
    from paper_2112_15562_amd import BTTBError
    with pytest.raises(BTTBError):
        s.run(1, 1, stop_on_chi2=True)
    s.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_graph_replay_equals_eager(pk, dtype):
    # the captured step graphs are replayed many times, with eager kernels and host
    # synchronisations in between; every outer step must match the eager launches bitwise
    g = synth.SMALL
    _, T, data, _ = problem(g, dense=True)
    prm = orrcg.Params(**dict(BASE, restart=True))
    sg, ops = gpu_solver(pk, g, T, data, prm, dtype, use_graph=True)
    se, _ = gpu_solver(pk, g, T, data, prm, dtype, use_graph=False)
    x = torch.rand(g.model_shape, dtype=dtype, device="cuda")
    for k in range(5):
        sg.step(4)
        ops[0].matvec(x)            # unrelated eager work between replays
        torch.cuda.synchronize()
        se.step(4)
        for i in range(2):
            assert np.array_equal(host(sg.m[i]), host(se.m[i]))
            assert np.array_equal(host(sg.p[i]), host(se.p[i]))
            assert np.array_equal(host(sg.resid[i]), host(se.resid[i]))
        a, b = sg.scalars(), se.scalars()
        assert a["phi"] == b["phi"] and a["alpha"] == b["alpha"] and a["k"] == b["k"] == k + 1
    sg.close()
    se.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_autotune_mid_solve_keeps_the_trajectory(pk, dtype, tol):
    # tuning times CG steps on the live solver and must restore its state exactly; only the
    # grouping of partial sums changes with the launch shape
    g = synth.MID
    ops, T, data, _ = problem(g, dense=False)
    prm = orrcg.Params(**BASE)
    a, _ = gpu_solver(pk, g, T, data, prm, dtype)
    b, _ = gpu_solver(pk, g, T, data, prm, dtype)
    a.step(5)
    b.step(5)
    res = b.autotune(reps=2)
    assert res["tried"] >= 4
    for _ in range(2):
        a.step(5)
        b.step(5)
    for i in range(2):
        assert rel(host(b.m[i]), host(a.m[i])) <= tol
    assert b.scalars()["k"] == a.scalars()["k"] == 3
    a.close()
    b.close()


# ------------------------------------------------------------------------------------
# the benchmarked solve: 256x256 stations over 256x256x32 prisms (512-point transforms, the
# fused N = 512 forms of the group path), the bench's model, noise and parameters
# ------------------------------------------------------------------------------------
_LARGE = {}
LARGE_INNER = 3


def large_reference():
    """Oracle state after one outer step from the start, and the oracle's next outer step
    from it (FFT2 products on the host cores)."""
    if _LARGE:
        return _LARGE["v"]
    g = synth.LARGE
    og = ogeom(g)
    workers = min(16, os.cpu_count() or 1)
    T = [obttb.kernel_array(k, og) for k in (oprism.GRAVITY, oprism.MAGNETIC)]
    ops = [obttb.FFTOperator(T[i], g.sx, g.sy, workers=workers) for i in range(2)]
    rho, kap = synth.dyke_and_block(g)
    d = [ops[0].matvec(rho), ops[1].matvec(kap)]
    sig = [synth.noise_sigma(d[0], 0.02, 0.02), synth.noise_sigma(d[1], 0.02, 1.0)]
    dobs = [d[i] + sig[i] * synth.normal_like(d[i].shape, 3, 100 + i) for i in range(2)]
    data = orrcg.Data(dobs=dobs, wd=[1.0 / x for x in sig],
                      wdepth=[synth.depth_weight(g, 2.0), synth.depth_weight(g, 3.0)])
    prm = orrcg.Params(alpha0=(20000.0, 20000.0), q=(0.95, 0.95), lam=(2.0, 100.0), eps2=1e-9, lo=(0.0, 0.0),
                       hi=(1.0, 0.1), coupled=True, restart=True, p_norm=1)
    st, _ = orrcg.outer_step(ops, data, prm, orrcg.initial_state(data, prm, g.model_shape), LARGE_INNER)
    ref, rec = orrcg.outer_step(ops, data, prm, st, LARGE_INNER)
    _LARGE["v"] = (T, data, prm, st, ref, rec)
    return _LARGE["v"]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("shape", [None, (512, 64, 128, 2)], ids=["default-shape", "bench-shape"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_large_grid_outer_step_parity(pk, dtype, tol, shape):
    g = synth.LARGE
    T, data, prm, st, ref, rec = large_reference()
    s, ops = gpu_solver(pk, g, T, data, prm, dtype, state=st)
    if shape is not None:   # the launch shape the bench's tuner picks (set before the first capture)
        s.products().set_launch(*shape)
    print(f"256x256x32 {dtype} shape {shape}: launch {s.products().info()}", flush=True)
    s.step(LARGE_INNER)
    sc = s.scalars()
    errs = [rel(host(s.m[i]), ref.m[i]) for i in range(2)]
    print(f"  model rel err {errs}; phi {sc['phi']} vs {rec['phi']}; S_G {sc['gramian']} vs {rec['gramian']}",
          flush=True)
    assert max(errs) <= tol
    for i in range(2):
        assert sc["phi"][i] == pytest.approx(rec["phi"][i], rel=tol)
        assert sc["alpha"][i] == pytest.approx(ref.alpha[i], rel=1e-15)
    assert sc["gramian"] == pytest.approx(rec["gramian"], rel=100 * tol)
    assert sc["similarity"] == pytest.approx(orrcg.similarity(ref.m[0], ref.m[1]), rel=tol)
    s.close()
    for op in ops:
        op.close()


def test_timed_solver_steps_like_an_untimed_one(pk):
    # per-kernel event timing repeats each product launch; the repeats of the fused direction
    # update write to scratch, so the solver's trajectory is bitwise that of an untimed solver
    g = synth.SMALL
    _, T, data, _ = problem(g, dense=True)
    prm = orrcg.Params(**BASE)
    a, _ = gpu_solver(pk, g, T, data, prm, torch.float64, use_graph=False)
    b, _ = gpu_solver(pk, g, T, data, prm, torch.float64, use_graph=False)
    prod = b.products()
    prod.timing_enable(200, 10)
    for _ in range(2):
        a.step(4)
        b.step(4)
    tm = prod.timing_read()
    prod.timing_enable(0)
    # 8 CG steps (fused forms) and 2 residual products (plain) of the forward row transform
    assert tm["fwd_row_r2c"][1] == 10 * (8 + 2) and tm["adj_row_c2r"][1] == 10 * 8
    for i in range(2):
        assert np.array_equal(host(a.m[i]), host(b.m[i]))
        assert np.array_equal(host(a.p[i]), host(b.p[i]))
    sa, sb = a.scalars(), b.scalars()
    assert sa["phi"] == sb["phi"] and sa["beta"] == sb["beta"] and sa["step"] == sb["step"]
    a.close()
    b.close()


@pytest.mark.parametrize("coupled", [True, False], ids=["joint_step", "per_data_set_step"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_zero_data_and_prior_stay_at_zero(pk, dtype, coupled):
    # the degenerate problem whose every objective vanishes at m = 0: zero gradient, zero
    # direction, the step length's 0/0 taken as 0 (as the oracle does), no non-finite flag
    g = synth.SMALL
    _, T, data, _ = problem(g, dense=True)
    zero = orrcg.Data(dobs=[np.zeros_like(d) for d in data.dobs], wd=data.wd, wdepth=data.wdepth)
    prm = orrcg.Params(**BASE, coupled=coupled)
    s, _ = gpu_solver(pk, g, T, zero, prm, dtype)
    s.run(3, 4)
    sc = s.scalars()
    assert not sc["nonfinite"]
    for k in range(2):
        assert not host(s.m[k]).any()
        assert sc["phi"][k] == 0.0 and sc["step"][k] == 0.0
    assert sc["similarity"] == 0.0
    s.close()
