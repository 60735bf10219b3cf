"""Library calls captured into the caller's graph (torch.cuda.graph) and replayed: one-plan
products (power-of-two and 5-smooth plans, weighted), a group product, the allocation-free
products and a joint RRCG outer step without the solver's own graphs.  These calls only launch
kernels (no allocation, copy, memset or synchronisation), so a capture records them.  Each replay
is compared bit for bit with the same calls made eagerly, after new inputs are written eagerly
between the replays (run on an MI355X)."""
import ctypes as C

import pytest
import torch

import synth
from oracle import rrcg as orrcg
from test_gpu_rrcg import BASE, problem

pytestmark = pytest.mark.gpu

REPLAYS = 4


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


def capture(fn):
    """fn run once eagerly on a side stream (warm-up), then captured into a graph."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph


def _noalloc(L, op, kind, x, out, winv, wd):
    p = lambda t: C.c_void_p(t.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.lib().bttb_apply_noalloc(op.plan, kind, p(x), p(out), p(winv), p(wd), stream)


# 128x128x20 (256-point transforms), 12x12 over 12x12x6 (24 points, 5-smooth) in FP32,
# 16x16x8 (32 points) in FP64
CASES = [(synth.MID, torch.float32), (synth.SUB, torch.float32), (synth.SMALL, torch.float64)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_products_replay_from_a_captured_graph(pk, case):
    from paper_2112_15562_amd import _lib as L
    from paper_2112_15562_amd.operator import pointer_array
    F, A = L.BTTB_OP_FORWARD, L.BTTB_OP_ADJOINT
    g, dt = CASES[case]
    print(f"case {case}: {g.sx}x{g.sy} over {g.nx}x{g.ny}x{g.nz}, {dt}", flush=True)
    r = synth.rng(11, case)
    new = lambda shape, lo=None: torch.tensor(r.uniform(lo, 2.0, shape) if lo else r.standard_normal(shape),
                                              dtype=dt, device="cuda")
    ops = [pk.Operator.from_geometry(k, g, dtype=dt) for k in (pk.GRAVITY, pk.MAGNETIC)]
    grp = pk.Group(ops)
    x, v = new(g.model_shape), new(g.data_shape)
    winv, wd = new(g.model_shape, 0.5), new(g.data_shape, 0.5)
    zeros = lambda shape: [torch.zeros(shape, dtype=dt, device="cuda") for _ in ops]
    y, z, gy, gz, ny, nz = (zeros(g.data_shape), zeros(g.model_shape), zeros(g.data_shape), zeros(g.model_shape),
                            zeros(g.data_shape), zeros(g.model_shape))
    ptr = lambda ts: pointer_array(ts, x.device)
    xs, vs, ws, ds = ptr([x, x]), ptr([v, v]), ptr([winv, winv]), ptr([wd, wd])
    gyp, gzp = ptr(gy), ptr(gz)

    def run():
        for i, op in enumerate(ops):
            op.matvec(x, winv=winv, wd=wd, out=y[i])
            op.rmatvec(v, winv=winv, wd=wd, out=z[i])
        grp.apply_ptrs(F, xs, gyp, ws, ds)
        grp.apply_ptrs(A, vs, gzp, ws, ds)
        for i, op in enumerate(ops):
            assert _noalloc(L, op, F, x, ny[i], winv, wd) == L.BTTB_OK
            assert _noalloc(L, op, A, v, nz[i], winv, wd) == L.BTTB_OK

    graph = capture(run)
    for k in range(REPLAYS):
        x.copy_(new(g.model_shape))   # eager work between the replays
        v.copy_(new(g.data_shape))
        graph.replay()
        ref_y = [op.matvec(x, winv=winv, wd=wd) for op in ops]
        ref_z = [op.rmatvec(v, winv=winv, wd=wd) for op in ops]
        ref_gy = grp.apply(F, [x, x], winv=[winv, winv], wd=[wd, wd])
        ref_gz = grp.apply(A, [v, v], winv=[winv, winv], wd=[wd, wd])
        ref_ny, ref_nz = zeros(g.data_shape), zeros(g.model_shape)
        for i, op in enumerate(ops):
            assert _noalloc(L, op, F, x, ref_ny[i], winv, wd) == L.BTTB_OK
            assert _noalloc(L, op, A, v, ref_nz[i], winv, wd) == L.BTTB_OK
        torch.cuda.synchronize()
        for name, got, ref in (("matvec", y, ref_y), ("rmatvec", z, ref_z), ("group matvec", gy, ref_gy),
                               ("group rmatvec", gz, ref_gz), ("noalloc matvec", ny, ref_ny),
                               ("noalloc rmatvec", nz, ref_nz)):
            for i in range(2):
                assert torch.equal(got[i], ref[i]), (k, name, i)
        assert torch.isfinite(y[0]).all() and float(torch.linalg.vector_norm(y[0])) > 0.0
    del graph
    grp.close()
    for op in ops:
        op.close()


def test_solver_step_replays_from_a_captured_graph(pk):
    # two identical FP32 solvers without their own graphs; one outer step of the first is
    # captured and replayed, the second steps eagerly: the iterates agree bit for bit
    g = synth.SMALL
    _, T, data, _ = problem(g, dense=False)
    prm = orrcg.Params(**BASE)

    def make():
        ops = [pk.Operator(torch.as_tensor(T[i], device="cuda"), (g.sx, g.sy), dtype=torch.float32)
               for i in range(2)]
        s = pk.JointRRCG(ops, data.dobs, data.wd, data.wdepth, lo=prm.lo, hi=prm.hi, alpha0=prm.alpha0, q=prm.q,
                         lam=prm.lam, use_graph=False)
        return s, ops

    (s1, o1), (s2, o2) = make(), make()
    graph = capture(lambda: s1.step(2))
    s2.step(2)   # the warm-up step of s1
    for k in range(REPLAYS):
        graph.replay()
        s2.step(2)
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(s1.m[i], s2.m[i]), (k, "m", i)
            assert torch.equal(s1.p[i], s2.p[i]), (k, "p", i)
        a, b = s1.scalars(), s2.scalars()
        assert a == b, k
        assert not a["nonfinite"]
    del graph
    for s, ops in ((s1, o1), (s2, o2)):
        s.close()
        for op in ops:
            op.close()
