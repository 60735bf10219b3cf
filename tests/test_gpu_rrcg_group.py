"""Group solver (many joint inversions stepped together, one launch per phase) vs the FP64
oracle and vs one-inversion solvers (run on an MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import rrcg as orrcg
from test_gpu_rrcg import BASE, host, problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


# uneven inversions (transforms 32 after power-of-two padding, ragged 7 x 9 over 11 x 5 x 3)
GRIDS = [synth.SMALL, synth.SUB, synth.Grid(7, 9, 11, 5, 3, 40.0, 30.0, 25.0, decl=20.0),
         synth.Grid(10, 14, 10, 14, 4, 50.0, 40.0, 30.0), synth.Grid(16, 12, 16, 12, 3, 50.0, 50.0, 40.0)]
# one solver variant per inversion: nested with restart, stand-alone, joint minimum length,
# weighted Gramian without restart, the printed previous-iterate anchor of RRCG:4
VARIANTS = [
    dict(restart=True),
    dict(restart=True, coupled=False, lam=(0.0, 0.0)),
    dict(restart=True, p_norm=2, alpha_min=(500.0, 500.0)),
    dict(restart=False, gramian="weighted", lam=(1e-3, 1e-1)),
    dict(restart=False, anchor="prev"),
]
N_INNER = 3


def params(v):
    kw = dict(BASE)
    kw.update(v)
    return orrcg.Params(**kw)


def solver_kwargs(prm):
    return dict(lo=prm.lo, hi=prm.hi, alpha0=prm.alpha0, q=prm.q, alpha_min=prm.alpha_min, lam=prm.lam,
                eps2=prm.eps2, coupled=prm.coupled, restart=prm.restart, p_norm=prm.p_norm, gramian=prm.gramian,
                anchor=prm.anchor)


def ops_for(pk, g, T, dtype):
    return [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=dtype, pad_pow2=True)
            for i in range(2)]


def build_group(pk, dtype, use_graph=True):
    probs, refs = [], []
    for g, v in zip(GRIDS, VARIANTS):
        ops, T, data, _ = problem(g, dense=True)
        prm = params(v)
        probs.append(dict(ops=ops_for(pk, g, T, dtype), dobs=data.dobs, wd=data.wd, wdepth=data.wdepth,
                          **solver_kwargs(prm)))
        refs.append((g, ops, T, data, prm))
    return pk.JointRRCGGroup(probs, use_graph=use_graph), refs


def set_state(grp, i, st, dtype):
    for k in range(2):
        grp.inv[i].m[k].copy_(torch.as_tensor(st.m[k], dtype=dtype, device="cuda"))
        grp.inv[i].p[k].copy_(torch.as_tensor(st.p[k], dtype=dtype, device="cuda"))
        if grp.inv[i].mprev is not None:
            grp.inv[i].mprev[k].copy_(torch.as_tensor(st.m_prev[k], dtype=dtype, device="cuda"))
    grp.set_scalars(i, alpha=st.alpha, L_prev=st.L_prev, frozen=st.frozen, k=st.k)


# p, the CG direction, is an intermediate: in FP32 it carries the rounding of the gradient
# l = A~^T r~ + alpha m~ + ..., whose terms cancel more and more as the inner CG converges
# (1e-3 relative after three steps here), so only the FP64 run checks it; the results -- the
# models and the misfits -- are held to the precision bounds in both.
@pytest.mark.parametrize("dtype,tol_m,tol_p", [(torch.float64, 1e-12, 1e-11), (torch.float32, 1e-5, None)])
def test_group_step_parity_per_inversion(pk, dtype, tol_m, tol_p):
    grp, refs = build_group(pk, dtype)
    expected = []
    for i, (g, ops, T, data, prm) in enumerate(refs):
        st, _ = orrcg.run(ops, data, prm, n_outer=2, n_inner=N_INNER)   # a mid-solve state
        ref, rec = orrcg.outer_step(ops, data, prm, st, N_INNER)
        set_state(grp, i, st, dtype)
        expected.append((ref, rec))
    grp.refresh()
    grp.step(N_INNER)
    for i, (ref, rec) in enumerate(expected):
        sc = grp.scalars(i)
        for k in range(2):
            assert rel(host(grp.inv[i].m[k]), ref.m[k]) <= tol_m, (i, k)
            if tol_p is not None:
                assert rel(host(grp.inv[i].p[k]), ref.p[k]) <= tol_p, (i, k)
            assert sc["alpha"][k] == pytest.approx(ref.alpha[k], rel=1e-15)
            assert sc["phi"][k] == pytest.approx(rec["phi"][k], rel=tol_m * 10)
            assert sc["frozen"][k] == ref.frozen[k]
        assert sc["k"] == ref.k
        assert not sc["nonfinite"]
    grp.close()


def test_group_equals_one_inversion_solvers_and_graphs(pk):
    grp, refs = build_group(pk, torch.float64, use_graph=True)
    eager, _ = build_group(pk, torch.float64, use_graph=False)
    singles = []
    for g, ops, T, data, prm in refs:
        singles.append(pk.JointRRCG(ops_for(pk, g, T, torch.float64), data.dobs, data.wd, data.wdepth,
                                    **solver_kwargs(prm)))
    for _ in range(3):
        grp.step(N_INNER)
        eager.step(N_INNER)
        for s in singles:
            s.step(N_INNER)
    for i, s in enumerate(singles):
        for k in range(2):
            a, b = host(grp.inv[i].m[k]), host(eager.inv[i].m[k])
            assert np.array_equal(a, b), (i, k)          # graph replay == eager
            assert rel(a, host(s.m[k])) <= 1e-12, (i, k)  # same arithmetic, other partial sums
        assert grp.scalars(i)["k"] == s.scalars()["k"] == 3
        s.close()
    grp.close()
    eager.close()


@pytest.mark.parametrize("how", ["set_launch", "narrow", "autotune"])
def test_group_launch_shape_recaptures(pk, how):
    grp, _ = build_group(pk, torch.float64)
    ref, _ = build_group(pk, torch.float64)
    if how == "set_launch":
        grp.set_launch(model_row_threads=64, data_row_threads=64, col_threads=64, layer_chunks=2)
        info = grp.launch_info()
        assert (info["model_row_threads"], info["col_threads"], info["layer_chunks"]) == (64, 64, 2)
    elif how == "narrow":
        # blocks below one wave (8 threads): the fused forms' partial sums take the lane-shuffle
        # butterfly instead of the full-wave DPP sum
        grp.set_launch(model_row_threads=8, data_row_threads=8, col_threads=8, layer_chunks=1)
        info = grp.launch_info()
        assert (info["model_row_threads"], info["data_row_threads"], info["col_threads"]) == (8, 8, 8)
    else:
        res = grp.autotune(reps=2)
        assert res["col_threads"] == grp.launch_info()["col_threads"]
    grp.step(N_INNER)
    ref.step(N_INNER)
    for i in range(len(grp)):
        for k in range(2):
            assert rel(host(grp.inv[i].m[k]), host(ref.inv[i].m[k])) <= 1e-12
    grp.close()
    ref.close()


# five inversions whose plans keep their 5-smooth transform sizes (24, 40, 72 x 64, 32, 120):
# every phase one launch per size class, the CG pieces fused into the 5-smooth transforms too
MIXED_GRIDS = [synth.SUB, synth.Grid(20, 20, 20, 20, 4, 40.0, 40.0, 25.0),
               synth.Grid(36, 30, 36, 30, 5, 40.0, 45.0, 25.0, decl=15.0), synth.SMALL,
               synth.Grid(60, 60, 60, 60, 5, 40.0, 40.0, 25.0)]


@pytest.mark.parametrize("dtype,tol_m", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_group_step_parity_at_5smooth_sizes(pk, dtype, tol_m):
    probs, expected = [], []
    for idx, (g, v) in enumerate(zip(MIXED_GRIDS, VARIANTS)):
        ops, T, data, _ = problem(g, dense=g.nx <= 36)
        prm = params(v)
        gops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=dtype) for i in range(2)]
        probs.append(dict(ops=gops, dobs=data.dobs, wd=data.wd, wdepth=data.wdepth, **solver_kwargs(prm)))
        st, _ = orrcg.run(ops, data, prm, n_outer=2, n_inner=N_INNER)
        ref, rec = orrcg.outer_step(ops, data, prm, st, N_INNER)
        expected.append((st, ref, rec, gops))
    assert [op.info()["Px"] for _, _, _, ops in expected for op in ops[:1]] == [24, 40, 72, 32, 120]
    grp = pk.JointRRCGGroup(probs)
    for i, (st, _, _, _) in enumerate(expected):
        set_state(grp, i, st, dtype)
    grp.refresh()
    grp.step(N_INNER)
    for i, (_, ref, rec, _) in enumerate(expected):
        sc = grp.scalars(i)
        errs = [rel(host(grp.inv[i].m[k]), ref.m[k]) for k in range(2)]
        print(f"{dtype} inversion {i}: model rel err {errs}", flush=True)
        assert max(errs) <= tol_m, (i, errs)
        for k in range(2):
            assert sc["phi"][k] == pytest.approx(rec["phi"][k], rel=tol_m * 10)
            assert sc["alpha"][k] == pytest.approx(ref.alpha[k], rel=1e-15)
        assert sc["k"] == ref.k and not sc["nonfinite"]
    grp.close()


# four inversions at 5-smooth sizes the cost-model padding picks (288: 8 9 4, 320: 8 5 8,
# 576: 8 9 8, 640: 8 10 8), the radix-9 / -5 / -10 LDS passes with a register last pass,
# stepped together by the group solver as the batched bench runs them
AUTO_GRIDS = [synth.Grid(n, n, n, n, 2, 40.0, 40.0, 25.0) for n in (136, 160, 266, 314)]
_AUTO_REF = {}


def auto_reference():
    if not _AUTO_REF:
        for idx, g in enumerate(AUTO_GRIDS):
            ops, T, data, _ = problem(g, dense=False)
            prm = params(VARIANTS[idx])
            st, _ = orrcg.run(ops, data, prm, n_outer=1, n_inner=N_INNER)
            ref, rec = orrcg.outer_step(ops, data, prm, st, N_INNER)
            _AUTO_REF[idx] = (g, T, data, prm, st, ref, rec)
    return _AUTO_REF


@pytest.mark.parametrize("dtype,tol_m", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_group_step_parity_at_auto_padded_sizes(pk, dtype, tol_m):
    refs = auto_reference()
    probs = []
    for idx in range(len(AUTO_GRIDS)):
        g, T, data, prm, _, _, _ = refs[idx]
        gops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=dtype, pad="auto")
                for i in range(2)]
        probs.append(dict(ops=gops, dobs=data.dobs, wd=data.wd, wdepth=data.wdepth, **solver_kwargs(prm)))
    assert [p["ops"][0].info()["Px"] for p in probs] == [288, 320, 576, 640]
    grp = pk.JointRRCGGroup(probs)
    for idx in range(len(AUTO_GRIDS)):
        set_state(grp, idx, refs[idx][4], dtype)
    grp.refresh()
    grp.step(N_INNER)
    for idx in range(len(AUTO_GRIDS)):
        _, _, _, _, _, ref, rec = refs[idx]
        sc = grp.scalars(idx)
        errs = [rel(host(grp.inv[idx].m[k]), ref.m[k]) for k in range(2)]
        print(f"{dtype} inversion {idx} (P = {probs[idx]['ops'][0].info()['Px']}): model rel err {errs}", flush=True)
        assert max(errs) <= tol_m, (idx, errs)
        for k in range(2):
            assert sc["phi"][k] == pytest.approx(rec["phi"][k], rel=tol_m * 10)
        assert sc["k"] == ref.k and not sc["nonfinite"]
    grp.close()
    for p in probs:
        for op in p["ops"]:
            op.close()


def test_group_solver_inversion_limit(pk):
    # up to 32 joint inversions per group solver: 32 small ones step together, each as its own
    # one-inversion solver steps; a 33rd is refused
    from paper_2112_15562_amd import _lib as L
    g = synth.SMALL
    _, T, data, _ = problem(g, dense=True)
    prm = params(VARIANTS[0])
    probs = []
    for k in range(33):
        ops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=torch.float64) for i in range(2)]
        probs.append(dict(ops=ops, dobs=data.dobs, wd=data.wd, wdepth=data.wdepth, **solver_kwargs(prm)))
    with pytest.raises(L.BTTBError) as e:
        pk.JointRRCGGroup(probs)
    assert e.value.status == L.BTTB_EINVAL
    grp = pk.JointRRCGGroup(probs[:32])
    grp.step(N_INNER)
    one = pk.JointRRCG(probs[32]["ops"], data.dobs, data.wd, data.wdepth, **solver_kwargs(prm))
    one.step(N_INNER)
    for i in (0, 17, 31):
        for k in range(2):
            assert rel(host(grp.inv[i].m[k]), host(one.m[k])) <= 1e-13
    one.close()
    grp.close()
    for p in probs:
        for op in p["ops"]:
            op.close()


def test_graph_replays_equal_eager_steps_with_several_size_classes(pk):
    # the four auto-sized inversions (four transform sizes, so every phase is four launches,
    # FP32 with the first transform riding in the update): each outer step replayed from its HIP
    # graph equals the eager launches bit for bit, checked after every replay, with host reads
    # and eager work between the replays
    refs = auto_reference()

    def build(use_graph):
        probs = []
        for idx in range(len(AUTO_GRIDS)):
            g, T, data, prm, st, _, _ = refs[idx]
            ops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=torch.float32, pad="auto")
                   for i in range(2)]
            probs.append(dict(ops=ops, dobs=data.dobs, wd=data.wd, wdepth=data.wdepth, **solver_kwargs(prm)))
        grp = pk.JointRRCGGroup(probs, use_graph=use_graph)
        for idx in range(len(AUTO_GRIDS)):
            set_state(grp, idx, refs[idx][4], torch.float32)
        grp.refresh()
        return grp, probs

    gg, gp = build(True)
    ge, ep = build(False)
    for step in range(3):
        gg.step(N_INNER)
        ge.step(N_INNER)
        for idx in range(len(AUTO_GRIDS)):
            for k in range(2):
                assert np.array_equal(host(gg.inv[idx].m[k]), host(ge.inv[idx].m[k])), (step, idx, k)
            assert gg.scalars(idx)["phi"] == ge.scalars(idx)["phi"]
    for grp, probs in ((gg, gp), (ge, ep)):
        grp.close()
        for p in probs:
            for op in p["ops"]:
                op.close()
