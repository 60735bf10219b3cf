"""Differentiation through the BTTB operators (autograd Functions whose backward is the
hand-written transpose product), checked against finite differences and the dense oracle."""
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


TINY3 = synth.Grid(6, 5, 6, 5, 3, 50.0, 40.0, 25.0, decl=15.0)


def test_gradcheck_and_gradgradcheck_fp64(pk):
    # the products are linear, so a large step leaves only rounding in the differences;
    # the absolute tolerance scales with the largest kernel entry (mGal or nT per unit)
    for kind in (pk.GRAVITY, pk.MAGNETIC):
        scale = float(pk.prism_kernels(kind, TINY3).abs().max().item())
        tol = dict(eps=1e-3, atol=1e-10 * scale, rtol=1e-8)
        op = pk.Operator.from_geometry(kind, TINY3, dtype=torch.float64, max_batch=2)
        m = torch.rand((2,) + TINY3.model_shape, dtype=torch.float64, device="cuda", requires_grad=True)
        r = torch.randn((2,) + TINY3.data_shape, dtype=torch.float64, device="cuda", requires_grad=True)
        f = lambda x: pk.BTTBFunction.apply(x, op)
        g = lambda x: pk.BTTBTransposeFunction.apply(x, op)
        assert torch.autograd.gradcheck(f, (m,), **tol)
        assert torch.autograd.gradcheck(g, (r,), **tol)
        assert torch.autograd.gradgradcheck(f, (m,), **tol)
        op.close()


def test_batched_fp32_backward_vs_fp64_finite_differences(pk):
    # 8 models on 128x128x24 prisms through the gravity (G) and magnetic (T) operators;
    # the FP32 gradient of <u, A m> is the hand-written A^T u
    g = synth.BATCH
    B = 8
    models = np.stack([synth.random_boxes(g, seed_workload=4, index=b)[0] for b in range(B)])
    u_np = synth.normal_like((B,) + g.data_shape, 4, 100)
    dirs = synth.rng(4, 200).standard_normal((32,) + g.model_shape)
    dirs /= np.linalg.norm(dirs.reshape(32, -1), axis=1)[:, None, None, None]
    T = [pk.prism_kernels(k, g) for k in (pk.GRAVITY, pk.MAGNETIC)]
    for i in range(2):
        op32 = pk.Operator(T[i], (g.sx, g.sy), dtype=torch.float32, max_batch=B)
        op64 = pk.Operator(T[i], (g.sx, g.sy), dtype=torch.float64, max_batch=B)
        m32 = torch.tensor(models, dtype=torch.float32, device="cuda", requires_grad=True)
        u32 = torch.tensor(u_np, dtype=torch.float32, device="cuda")
        loss = (pk.BTTBFunction.apply(m32, op32) * u32).sum()
        loss.backward()
        g32 = m32.grad.double()
        m64 = torch.tensor(models, dtype=torch.float64, device="cuda", requires_grad=True)
        u64 = torch.tensor(u_np, dtype=torch.float64, device="cuda")
        (pk.BTTBFunction.apply(m64, op64) * u64).sum().backward()
        g64 = m64.grad
        rel = (torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64)).item()
        assert rel <= 1e-5, rel
        # the FP32 batched gradient of two batch members against the oracle's FP64 A^T u
        # (FFT2 products on the host), from the oracle's own kernel array
        og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl,
                             g.field)
        To = obttb.kernel_array((oprism.GRAVITY, oprism.MAGNETIC)[i], og)
        for b in (0, B - 1):
            ref = obttb.fft_rmatvec(To, u_np[b], g.sx, g.sy, workers=8)
            got = g32[b].cpu().numpy()
            e = float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
            print(f"operator {i} member {b}: FP32 gradient vs oracle rel err {e:.2e}", flush=True)
            assert e <= 1e-5
        # central differences of f(m) = <u, A m> (FP64) along 32 unit directions of one model;
        # f is linear, so a moderate step leaves only rounding
        h = 1e-3
        f = lambda x: float((op64.matvec(x) * u64[0]).sum().item())
        m0 = m64.detach()[0]
        for d in range(32):
            v = torch.tensor(dirs[d], dtype=torch.float64, device="cuda")
            fd = (f(m0 + h * v) - f(m0 - h * v)) / (2 * h)
            an = float((g64[0] * v).sum().item())
            scale = float(torch.linalg.vector_norm(g64[0]).item())
            assert abs(fd - an) <= 1e-7 * scale, (d, fd, an)
        op32.close()
        op64.close()


def test_gradient_matches_dense_oracle(pk):
    # loss = 1/2 ||A m - d||^2 on 12x12x6 (a radix-3 transform size): grad = A^T (A m - d)
    g = synth.SUB
    og = oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field)
    rho, kap = synth.uniform_models(g, 4, 3)
    for kind, m in ((pk.GRAVITY, rho), (pk.MAGNETIC, kap)):
        A = oprism.dense_matrix(kind, og)
        d = A @ (0.5 * m.ravel()) + 0.01 * synth.normal_like(g.sx * g.sy, 4, 4)
        op = pk.Operator.from_geometry(kind, g, dtype=torch.float64)
        mt = torch.tensor(m, dtype=torch.float64, device="cuda", requires_grad=True)
        dt = torch.tensor(d.reshape(g.data_shape), dtype=torch.float64, device="cuda")
        (0.5 * ((pk.BTTBFunction.apply(mt, op) - dt) ** 2).sum()).backward()
        ref = (A.T @ (A @ m.ravel() - d)).reshape(g.model_shape)
        got = mt.grad.cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        op.close()


def test_forward_model_module(pk):
    g = synth.SMALL
    op = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=torch.float32, max_batch=4)
    mod = pk.ForwardModel(op)
    m = torch.rand((4,) + g.model_shape, dtype=torch.float32, device="cuda", requires_grad=True)
    y = mod(m)
    assert y.shape == (4,) + g.data_shape
    y.sum().backward()
    ones = torch.ones((4,) + g.data_shape, dtype=torch.float32, device="cuda")
    assert torch.allclose(m.grad, op.rmatvec(ones), rtol=1e-6, atol=0)
    op.close()
