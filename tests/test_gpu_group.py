"""Group products (one launch per stage over many uneven plans) vs the FP64 oracle and vs
the one-plan products (run on an MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import bttb as obttb
from oracle import prism as oprism

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


# uneven members: transform sizes 32 .. 512 after power-of-two padding, ragged shapes,
# sx < nx, both operators.  With the default shapes the smallest members run 64 row
# transforms per block: row tiles of 128 rows over 12 rows padded to 16.
MEMBERS = [
    (oprism.GRAVITY, synth.Grid(12, 10, 12, 10, 5, 50.0, 50.0, 50.0)),
    (oprism.MAGNETIC, synth.Grid(12, 10, 12, 10, 5, 50.0, 50.0, 50.0)),
    (oprism.MAGNETIC, synth.Grid(30, 21, 33, 20, 7, 40.0, 45.0, 25.0, decl=15.0)),
    (oprism.GRAVITY, synth.Grid(64, 64, 64, 64, 16, 40.0, 40.0, 25.0)),
    (oprism.MAGNETIC, synth.Grid(40, 57, 40, 50, 9, 40.0, 40.0, 25.0)),
    (oprism.GRAVITY, synth.Grid(100, 100, 100, 100, 12, 40.0, 40.0, 25.0)),
    (oprism.MAGNETIC, synth.Grid(190, 130, 200, 120, 6, 40.0, 40.0, 25.0)),
]

_CACHE = {}


def oracle_case(idx):
    """Oracle kernel array, inputs and FP64 FFT2 products of member idx."""
    if idx in _CACHE:
        return _CACHE[idx]
    kind, g = MEMBERS[idx]
    og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field)
    T = obttb.kernel_array(kind, og)
    x = synth.rng(6, idx).uniform(0.0, 1.0, g.model_shape)
    r = synth.rng(6, 100 + idx).standard_normal(g.data_shape)
    winv = synth.rng(6, 200 + idx).uniform(0.5, 2.0, g.model_shape)
    wd = synth.rng(6, 300 + idx).uniform(0.5, 2.0, g.data_shape)
    y = obttb.fft_matvec(T, x, g.sx, g.sy)
    z = obttb.fft_rmatvec(T, r, g.sx, g.sy)
    yw = obttb.weighted_matvec(T, x, winv, wd, g.sx, g.sy)
    zw = obttb.weighted_rmatvec(T, r, winv, wd, g.sx, g.sy)
    _CACHE[idx] = (T, x, r, winv, wd, y, z, yw, zw)
    return _CACHE[idx]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def make(pk, dtype, idxs=None):
    idxs = list(range(len(MEMBERS))) if idxs is None else idxs
    ops = []
    for i in idxs:
        T = oracle_case(i)[0]
        g = MEMBERS[i][1]
        ops.append(pk.Operator(torch.as_tensor(T, device="cuda"), (g.sx, g.sy), dtype=dtype, pad_pow2=True))
    return ops, pk.Group(ops)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_group_products_match_oracle(pk, dtype, tol):
    ops, grp = make(pk, dtype)
    cases = [oracle_case(i) for i in range(len(MEMBERS))]
    dev = lambda a: torch.as_tensor(a, dtype=dtype, device="cuda").contiguous()
    xs = [dev(c[1]) for c in cases]
    rs = [dev(c[2]) for c in cases]
    ys = grp.matvec(xs)
    zs = grp.rmatvec(rs)
    yw = grp.matvec(xs, winv=[dev(c[3]) for c in cases], wd=[dev(c[4]) for c in cases])
    zw = grp.rmatvec(rs, winv=[dev(c[3]) for c in cases], wd=[dev(c[4]) for c in cases])
    for i, c in enumerate(cases):
        assert rel(host(ys[i]), c[5]) <= tol, (i, "forward")
        assert rel(host(zs[i]), c[6]) <= tol, (i, "transpose")
        assert rel(host(yw[i]), c[7]) <= tol, (i, "weighted forward")
        assert rel(host(zw[i]), c[8]) <= tol, (i, "weighted transpose")
    # the same plans one at a time: the same operations per element, but the one-plan and the
    # group kernels are separate instantiations, in which the compiler may fuse different
    # products of a sum into an FMA (and the forward layer sums may group differently), so
    # they agree to a few units in the last place, not bit for bit
    same = 1e-14 if dtype == torch.float64 else 1e-6
    for i, op in enumerate(ops):
        assert rel(host(op.matvec(xs[i])), host(ys[i])) <= same
        assert rel(host(op.rmatvec(rs[i])), host(zs[i])) <= same
    grp.close()
    for op in ops:
        op.close()


def test_group_launch_shapes(pk):
    ops, grp = make(pk, torch.float64)
    cases = [oracle_case(i) for i in range(len(MEMBERS))]
    dev = lambda a: torch.as_tensor(a, device="cuda").contiguous()
    xs = [dev(c[1]) for c in cases]
    rs = [dev(c[2]) for c in cases]
    y0 = [host(y) for y in grp.matvec(xs)]
    z0 = [host(z) for z in grp.rmatvec(rs)]
    info = grp.info()
    for rm, rd, cc, nch in [(64, 64, 64, 1), (512, 128, 256, 4), (128, 512, 128, 2)]:
        grp.set_launch(rm, rd, cc, nch)
        got = grp.info()
        assert (got["model_row_threads"], got["data_row_threads"], got["col_threads"]) == (rm, rd, cc)
        for i, y in enumerate(grp.matvec(xs)):
            assert rel(host(y), y0[i]) <= 1e-14
        for i, z in enumerate(grp.rmatvec(rs)):
            assert np.array_equal(host(z), z0[i])
    grp.set_launch(info["model_row_threads"], info["data_row_threads"], info["col_threads"], info["layer_chunks"])
    grp.close()
    for op in ops:
        op.close()


def test_group_autotune(pk):
    ops, grp = make(pk, torch.float32)
    cases = [oracle_case(i) for i in range(len(MEMBERS))]
    dev = lambda a: torch.as_tensor(a, dtype=torch.float32, device="cuda").contiguous()
    res = grp.autotune(reps=2)
    info = grp.info()
    assert res["tried"] >= 4 and res["us_per_pair"] > 0
    assert [info[k] for k in ("model_row_threads", "data_row_threads", "col_threads", "layer_chunks")] == \
        [res[k] for k in ("model_row_threads", "data_row_threads", "col_threads", "layer_chunks")]
    ys = grp.matvec([dev(c[1]) for c in cases])
    zs = grp.rmatvec([dev(c[2]) for c in cases])
    for i, c in enumerate(cases):
        assert rel(host(ys[i]), c[5]) <= 1e-5
        assert rel(host(zs[i]), c[6]) <= 1e-5
    grp.close()
    for op in ops:
        op.close()


def test_group_rejects_bad_members_and_shapes(pk):
    from paper_2112_15562_amd import _lib as L
    T = torch.as_tensor(oracle_case(0)[0], device="cuda")
    g = MEMBERS[0][1]
    # 16 stations over 8 prism columns on a 24-point circle: 2 sx > 24, so no half form
    radix3 = pk.Operator(torch.zeros((2, 23, 23), dtype=torch.float64, device="cuda"), (16, 16))
    a = pk.Operator(T, (g.sx, g.sy), dtype=torch.float64, pad_pow2=True)
    b = pk.Operator(T, (g.sx, g.sy), dtype=torch.float32, pad_pow2=True)
    assert a.info()["Px"] == 32 and radix3.info()["Px"] == 24
    for members in ([radix3], [a, b]):
        with pytest.raises(L.BTTBError) as e:
            pk.Group(members)
        assert e.value.status == L.BTTB_ESTATE
    grp = pk.Group([a])
    for bad in [(3, 0, 0, 0), (0, 1024, 0, 0), (0, 0, 512, 0), (2, 0, 0, 0)]:
        with pytest.raises(L.BTTBError) as e:
            grp.set_launch(*bad)
        assert e.value.status == L.BTTB_EINVAL
    with pytest.raises(ValueError):
        grp.matvec([torch.zeros((2,) + g.model_shape, dtype=torch.float64, device="cuda")])
    grp.close()
    for op in (radix3, a, b):
        op.close()


def test_group_apply_checks_every_vector(pk):
    # the library gets bare device pointers per member, so the binding checks every list:
    # one tensor per member, of that member's shape, dtype and device, contiguous
    ops, grp = make(pk, torch.float64, [0, 2])
    dev = "cuda"
    x = [torch.rand(o.model_shape, dtype=torch.float64, device=dev) for o in ops]
    r = [torch.randn(o.data_shape, dtype=torch.float64, device=dev) for o in ops]
    wi = [torch.rand(o.model_shape, dtype=torch.float64, device=dev) + 0.5 for o in ops]
    wd = [torch.rand(o.data_shape, dtype=torch.float64, device=dev) + 0.5 for o in ops]
    F, A = 0, 1
    bad = [
        dict(op=F, xs=x[:1]),                                            # short input list
        dict(op=F, xs=x, outs=[torch.empty(ops[0].data_shape, dtype=torch.float64, device=dev)]),
        dict(op=F, xs=x, outs=[torch.empty(o.model_shape, dtype=torch.float64, device=dev) for o in ops]),
        dict(op=A, xs=r, outs=[torch.empty(o.data_shape, dtype=torch.float64, device=dev) for o in ops]),
        dict(op=F, xs=x, winv=wi[:1]),
        dict(op=F, xs=x, winv=[wd[0], wi[1]]),                           # wrong shape
        dict(op=F, xs=x, wd=wi),
        dict(op=F, xs=x, wd=[w.float() for w in wd]),                    # wrong dtype
        dict(op=F, xs=x, winv=[wi[0].cpu(), wi[1]]),                     # wrong device
        dict(op=F, xs=[x[0], x[1].transpose(1, 2)]),                     # not contiguous / shape
        dict(op=F, xs=[x[0].unsqueeze(0), x[1]]),                        # a batch, not one vector
        dict(op=A, xs=r, outs=[None, None]),
        dict(op=7, xs=x),
    ]
    for kw in bad:
        with pytest.raises((ValueError, TypeError)):
            grp.apply(**kw)
    # the pointer-array form: int64 arrays of one address per member, on the device
    px, py = pk.pointer_array(x, dev), pk.pointer_array([torch.empty(o.data_shape, dtype=torch.float64, device=dev)
                                                         for o in ops], dev)
    for a, b in [(px[:1], py), (px, py.cpu()), (px.to(torch.int32), py), (px, None)]:
        with pytest.raises(ValueError):
            grp.apply_ptrs(F, a, b)
    # entries of the diagonals may be None (identity for that member)
    ys = grp.apply(F, x, winv=[None, wi[1]], wd=[wd[0], None])
    ref0 = ops[0].matvec(x[0], wd=wd[0])
    ref1 = ops[1].matvec(x[1], winv=wi[1])
    assert rel(host(ys[0]), host(ref0)) <= 1e-12 and rel(host(ys[1]), host(ref1)) <= 1e-12
    grp.close()
    for op in ops:
        op.close()


# ------------------------------------------------------------------------------------
# 5-smooth transform sizes (no power-of-two padding): radix-3 and radix-5 passes
# ------------------------------------------------------------------------------------
MIXED = [
    (oprism.GRAVITY, synth.Grid(12, 12, 12, 12, 6, 50.0, 50.0, 50.0)),                # 24 = 8 3
    (oprism.MAGNETIC, synth.Grid(20, 20, 20, 20, 4, 40.0, 40.0, 25.0)),               # 40 = 8 5
    (oprism.MAGNETIC, synth.Grid(36, 30, 36, 30, 5, 40.0, 45.0, 25.0, decl=15.0)),    # 72 x 64
    (oprism.GRAVITY, synth.Grid(16, 16, 16, 16, 8, 50.0, 50.0, 50.0)),                # 32: a power of two
    (oprism.GRAVITY, synth.Grid(60, 60, 60, 60, 5, 40.0, 40.0, 25.0)),                # 120 = 8 3 5
    (oprism.MAGNETIC, synth.Grid(100, 100, 100, 100, 6, 40.0, 40.0, 25.0)),           # 200 = 8 5 5
    (oprism.MAGNETIC, synth.Grid(108, 108, 108, 108, 4, 40.0, 40.0, 25.0)),           # 216 = 8 27
    (oprism.GRAVITY, synth.Grid(144, 144, 144, 144, 3, 40.0, 40.0, 25.0)),            # 288: 8, 9, 4
    (oprism.MAGNETIC, synth.Grid(192, 192, 192, 192, 3, 40.0, 40.0, 25.0)),           # 384: 8, 6, 8
    (oprism.MAGNETIC, synth.Grid(288, 288, 288, 288, 2, 40.0, 40.0, 25.0)),           # 576: 8, 9, 8
    (oprism.GRAVITY, synth.Grid(320, 320, 320, 320, 2, 40.0, 40.0, 25.0)),            # 640: 8, 10, 8
]
_MCACHE = {}


def mixed_case(idx):
    if idx in _MCACHE:
        return _MCACHE[idx]
    kind, g = MIXED[idx]
    og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field)
    T = obttb.kernel_array(kind, og)
    x = synth.rng(7, idx).uniform(0.0, 1.0, g.model_shape)
    r = synth.rng(7, 100 + idx).standard_normal(g.data_shape)
    winv = synth.rng(7, 200 + idx).uniform(0.5, 2.0, g.model_shape)
    wd = synth.rng(7, 300 + idx).uniform(0.5, 2.0, g.data_shape)
    _MCACHE[idx] = (T, x, r, winv, wd, obttb.fft_matvec(T, x, g.sx, g.sy), obttb.fft_rmatvec(T, r, g.sx, g.sy),
                    obttb.weighted_matvec(T, x, winv, wd, g.sx, g.sy),
                    obttb.weighted_rmatvec(T, r, winv, wd, g.sx, g.sy))
    return _MCACHE[idx]


@pytest.mark.parametrize("shape", [None, (512, 256, 512, 2), (128, 128, 128, 1)], ids=["default", "wide", "narrow"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_group_products_at_5smooth_sizes(pk, dtype, tol, shape):
    ops = []
    for i, (kind, g) in enumerate(MIXED):
        ops.append(pk.Operator(torch.as_tensor(mixed_case(i)[0], device="cuda"), (g.sx, g.sy), dtype=dtype))
    sizes = [(op.info()["Px"], op.info()["Py"]) for op in ops]
    assert sizes == [(24, 24), (40, 40), (72, 64), (32, 32), (120, 120), (200, 200), (216, 216), (288, 288),
                     (384, 384), (576, 576), (640, 640)]
    grp = pk.Group(ops)
    if shape is not None:
        if dtype == torch.float64:
            shape = (shape[0], shape[1], min(shape[2], 256), shape[3])
        grp.set_launch(*shape)
    # 640-point rows take 80 lanes, padded to 128: fewer threads per block are refused
    with pytest.raises(pk.BTTBError):
        grp.set_launch(128, 64, 128, 1)
    print(f"{dtype} launch {grp.info()}", flush=True)
    dev = lambda a: torch.as_tensor(a, dtype=dtype, device="cuda")
    xs = [dev(mixed_case(i)[1]) for i in range(len(ops))]
    rs = [dev(mixed_case(i)[2]) for i in range(len(ops))]
    wi = [dev(mixed_case(i)[3]) for i in range(len(ops))]
    wd = [dev(mixed_case(i)[4]) for i in range(len(ops))]
    ys, zs = grp.matvec(xs), grp.rmatvec(rs)
    yw, zw = grp.matvec(xs, winv=wi, wd=wd), grp.rmatvec(rs, winv=wi, wd=wd)
    for i in range(len(ops)):
        c = mixed_case(i)
        errs = [rel(host(ys[i]), c[5]), rel(host(zs[i]), c[6]), rel(host(yw[i]), c[7]), rel(host(zw[i]), c[8])]
        print(f"  member {i} {sizes[i]}: rel errs {['%.1e' % e for e in errs]}", flush=True)
        assert max(errs) <= tol, (i, errs)
    grp.close()
    for op in ops:
        op.close()


def test_auto_padding_chooses_cheaper_sizes(pk):
    # BTTB_PAD_AUTO: per axis the power of two or a 5-smooth size of least estimated cost; for
    # grids just above a power of two the 5-smooth sizes with one pass through LDS win
    # (n = 300: 600 points are cheaper than 1024, and 640 cheaper still)
    expect = {178: 512, 101: 256, 266: 576, 320: 640, 136: 288, 160: 320, 192: 512, 244: 512, 300: 640}
    for n, P in expect.items():
        T = torch.zeros((1, 2 * n - 1, 2 * n - 1), dtype=torch.float64, device="cuda")
        op = pk.Operator(T, (n, n), dtype=torch.float32, pad="auto")
        assert (op.info()["Px"], op.info()["Py"]) == (P, P), n
        op.close()
    with pytest.raises(ValueError):
        pk.Operator(torch.zeros((1, 7, 7), dtype=torch.float64, device="cuda"), (4, 4), pad="bad")


# every 5-smooth size with compiled group kernels, as a column transform (Px) and as a row
# transform (Py): member j has Px = SIZES[j], Py = SIZES[22 - j] (stations over prism centres,
# n = P / 2, so the plans keep these sizes), in two groups of at most 14 sizes per stage
ALL_MIXED = [24, 40, 48, 72, 80, 96, 120, 144, 160, 192, 200, 216, 240, 288, 320, 360, 384, 400, 432, 480, 576,
             600, 640]
_ACACHE = {}


def all_mixed_case(j):
    if j not in _ACACHE:
        Px, Py = ALL_MIXED[j], ALL_MIXED[len(ALL_MIXED) - 1 - j]
        g = synth.Grid(Px // 2, Py // 2, Px // 2, Py // 2, 2, 40.0, 40.0, 25.0, decl=5.0 * j)
        kind = oprism.GRAVITY if j % 2 == 0 else oprism.MAGNETIC
        og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field)
        T = obttb.kernel_array(kind, og)
        x = synth.rng(8, j).uniform(0.0, 1.0, g.model_shape)
        r = synth.rng(8, 100 + j).standard_normal(g.data_shape)
        _ACACHE[j] = (g, T, x, r, obttb.fft_matvec(T, x, g.sx, g.sy), obttb.fft_rmatvec(T, r, g.sx, g.sy))
    return _ACACHE[j]


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_group_products_at_every_compiled_5smooth_size(pk, dtype, tol):
    assert len(ALL_MIXED) == 23
    for part in (range(0, 12), range(12, 23)):
        ops, cases = [], []
        for j in part:
            g, T, x, r, y, z = all_mixed_case(j)
            op = pk.Operator(torch.as_tensor(T, device="cuda"), (g.sx, g.sy), dtype=dtype)
            assert (op.info()["Px"], op.info()["Py"]) == (ALL_MIXED[j], ALL_MIXED[22 - j])
            ops.append(op)
            cases.append((x, r, y, z))
        grp = pk.Group(ops)
        ys = grp.matvec([torch.as_tensor(c[0], dtype=dtype, device="cuda") for c in cases])
        zs = grp.rmatvec([torch.as_tensor(c[1], dtype=dtype, device="cuda") for c in cases])
        for k, j in enumerate(part):
            errs = [rel(host(ys[k]), cases[k][2]), rel(host(zs[k]), cases[k][3])]
            print(f"  {dtype} Px {ALL_MIXED[j]} Py {ALL_MIXED[22 - j]}: {['%.1e' % e for e in errs]}", flush=True)
            assert max(errs) <= tol, (j, errs)
        grp.close()
        for op in ops:
            op.close()


def test_group_member_limit(pk):
    # a group holds up to 64 members (the gravity and magnetic operators of 32 inversions): 64
    # small uneven members give every member's own products; a 65th is refused
    from paper_2112_15562_amd import _lib as L
    grids = [synth.Grid(16 + (k % 9), 16 + (k * 5) % 9, 16 + (k % 9), 16 + (k * 5) % 9, 1 + k % 3, 40.0, 40.0, 25.0)
             for k in range(65)]
    ops = [pk.Operator.from_geometry(pk.GRAVITY if k % 2 == 0 else pk.MAGNETIC, g, dtype=torch.float32,
                                     pad="pow2")
           for k, g in enumerate(grids)]
    with pytest.raises(L.BTTBError) as e:
        pk.Group(ops)
    assert e.value.status == L.BTTB_EINVAL
    grp = pk.Group(ops[:64])
    xs = [torch.rand(op.model_shape, dtype=torch.float32, device="cuda") for op in ops[:64]]
    rs = [torch.randn(op.data_shape, dtype=torch.float32, device="cuda") for op in ops[:64]]
    ys, zs = grp.matvec(xs), grp.rmatvec(rs)
    for k in range(64):
        assert rel(host(ys[k]), host(ops[k].matvec(xs[k]))) <= 1e-6
        assert rel(host(zs[k]), host(ops[k].rmatvec(rs[k]))) <= 1e-6
    grp.close()
    for op in ops:
        op.close()
