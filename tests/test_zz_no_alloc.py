"""bttb_apply_noalloc -- the one-plan products with their intermediates in the library's fixed
device array instead of the plan's scratch -- called through the C ABI and compared with
bttb_apply (run on an MI355X).  Same kernels and launch shape, so the results are equal bit for
bit; the calls come in a row, a large plan first and then smaller ones, so a call finds the
previous call's intermediates in the array."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _noalloc(L, op, kind, x, out, winv=None, wd=None):
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.lib().bttb_apply_noalloc(op.plan, kind, _ptr(x), _ptr(out), _ptr(winv), _ptr(wd), stream)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# 128x128x20 in FP32 (power-of-two transforms, 20 layers), then 16x16x8 in FP64 and the 12x12x6
# subcase (24-point transforms of the general 5-smooth path) in FP32
CASES = [(synth.MID, torch.float32), (synth.SMALL, torch.float64), (synth.SUB, torch.float32)]


def test_noalloc_products_equal_bttb_apply(pk):
    from paper_2112_15562_amd import _lib as L
    F, A = L.BTTB_OP_FORWARD, L.BTTB_OP_ADJOINT
    for idx, (g, dt) in enumerate(CASES):
        print(f"case {idx}: {g.sx}x{g.sy} over {g.nx}x{g.ny}x{g.nz}, {dt}", flush=True)
        r = synth.rng(9, idx)
        x = torch.tensor(r.uniform(0.0, 1.0, g.model_shape), dtype=dt, device="cuda")
        v = torch.tensor(r.standard_normal(g.data_shape), dtype=dt, device="cuda")
        winv = torch.tensor(r.uniform(0.5, 2.0, g.model_shape), dtype=dt, device="cuda")
        wd = torch.tensor(r.uniform(0.5, 2.0, g.data_shape), dtype=dt, device="cuda")
        for kind in (pk.GRAVITY, pk.MAGNETIC):
            op = pk.Operator.from_geometry(kind, g, dtype=dt)
            for w in ((None, None), (winv, wd)):
                y_ref = _host(op.matvec(x, winv=w[0], wd=w[1]))
                z_ref = _host(op.rmatvec(v, winv=w[0], wd=w[1]))
                y = torch.full(g.data_shape, float("nan"), dtype=dt, device="cuda")
                z = torch.full(g.model_shape, float("nan"), dtype=dt, device="cuda")
                assert _noalloc(L, op, F, x, y, *w) == L.BTTB_OK
                assert _noalloc(L, op, A, v, z, *w) == L.BTTB_OK
                assert np.array_equal(_host(y), y_ref)
                assert np.array_equal(_host(z), z_ref)
            op.close()


def test_noalloc_rejects_plans_beyond_the_fixed_array(pk):
    from paper_2112_15562_amd import _lib as L
    g = synth.LARGE   # FP64 intermediates: about 51 MB
    op = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=torch.float64)
    x = torch.zeros(g.model_shape, dtype=torch.float64, device="cuda")
    y = torch.zeros(g.data_shape, dtype=torch.float64, device="cuda")
    assert _noalloc(L, op, L.BTTB_OP_FORWARD, x, y) == L.BTTB_ESIZE
    assert b"scratch" in L.lib().bttb_last_error()
    assert _noalloc(L, op, 5, x, y) == L.BTTB_EINVAL
    op.close()
