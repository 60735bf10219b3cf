"""GPU BTTB products through the C ABI vs the FP64 oracle (run on an MI355X)."""
import numpy as np
import pytest
import torch

import synth
from oracle import bttb as obttb
from oracle import dft as odft
from oracle import prism as oprism

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module")
def pk():
    import paper_2112_15562_amd as pk
    assert torch.cuda.is_available()
    return pk


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def ogeom(g: synth.Grid) -> oprism.Geometry:
    return oprism.Geometry(g.sx, g.sy, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.h, g.top, g.incl, g.decl, g.field,
                           ox=g.ox, oy=g.oy)


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


RAGGED = synth.Grid(7, 9, 11, 5, 3, 40.0, 30.0, 25.0, decl=20.0)
TINY = synth.Grid(1, 1, 1, 1, 1, 50.0, 50.0, 50.0)
ODD = synth.Grid(3, 5, 2, 7, 2, 30.0, 20.0, 10.0, h=2.0, top=5.0, incl=40.0, decl=-30.0)
# a padded model domain: 6x5 stations over the interior of 10x9x3 prisms, offset (2, 3)
PADDED = synth.Grid(6, 5, 10, 9, 3, 40.0, 30.0, 25.0, ox=2, oy=3)
# transforms with radix-5 (and 3) passes: 39 -> 40 = 8 5, 119 -> 120 = 8 3 5, 199 -> 200 = 8 5 5
R5 = synth.Grid(20, 20, 20, 20, 4, 40.0, 40.0, 25.0)
R35 = synth.Grid(60, 60, 60, 60, 5, 40.0, 40.0, 25.0, decl=10.0)
R55 = synth.Grid(100, 100, 100, 100, 8, 40.0, 40.0, 25.0)


# ------------------------------------------------------------------------------------
# setup transform: eigenvalues = brute-force DFT2 of the circular kernel array
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("L", [(24, 24), (17, 40), (45, 48), (80, 33), (120, 200), (250, 300)])
def test_eigenvalues_equal_bruteforce_dft(pk, L):
    Lx, Ly = L
    sx, sy = (Lx + 1) // 2, (Ly + 1) // 2
    nx, ny = Lx - sx + 1, Ly - sy + 1
    nz = 2
    rng = np.random.default_rng(Lx * 1000 + Ly)
    T = rng.standard_normal((nz, Lx, Ly))
    op = pk.Operator(dev(T), (sx, sy), dtype=torch.float64)
    info = op.info()
    Px, Py = info["Px"], info["Py"]
    assert Px % 8 == 0 and Py % 8 == 0 and Px >= Lx and Py >= Ly
    eig = op.eigenvalues().cpu().numpy()
    for r in range(nz):
        C = np.zeros((Px, Py))
        for i in range(Lx):
            for j in range(Ly):
                C[(i - (nx - 1)) % Px, (j - (ny - 1)) % Py] = T[r, i, j]
        ref = odft.dft2(C)[:, : Py // 2 + 1] / (Px * Py)   # [Px][K2]
        got = eig[r].T                                    # stored [K2][Px]
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    op.close()


# ------------------------------------------------------------------------------------
# prism kernel generator vs the oracle's closed forms
# ------------------------------------------------------------------------------------
def gravity_term_scale(g):
    """Per entry of the gravity kernel array: G times the summed magnitudes of the 24 terms of
    its 8-corner closed form (Z atan(XY/(ZR)), X ln(Y+R), Y ln(X+R) at each corner).  For
    distant cells the signed sum cancels to far below its terms, so rounding of the size of the
    terms, not of the entry, is what either evaluation carries."""
    og = ogeom(g)
    u = np.arange(-(g.nx - 1), g.sx).reshape(-1, 1)
    v = np.arange(-(g.ny - 1), g.sy).reshape(1, -1)
    x0, y0, z0 = oprism.station_xyz(og, u, v)
    S = np.empty((g.nz, u.shape[0], v.shape[1]))
    for r in range(g.nz):
        xb, yb, zb = oprism.prism_bounds(og, 0, 0, r)
        acc = 0.0
        for i in (0, 1):
            for j in (0, 1):
                for k in (0, 1):
                    X, Y, Z = xb[i] - x0, yb[j] - y0, zb[k] - z0
                    R = np.sqrt(X * X + Y * Y + Z * Z)
                    acc = acc + np.abs(Z * np.arctan(X * Y / (Z * R))) + np.abs(X * np.log(np.abs(Y) + R)) \
                        + np.abs(Y * np.log(np.abs(X) + R))
        S[r] = oprism.C_G * acc
    return S


@pytest.mark.parametrize("g", [synth.SMALL, synth.SUB, RAGGED, ODD, PADDED, synth.MID])
def test_prism_kernels_match_oracle(pk, g):
    for kind in (pk.GRAVITY, pk.MAGNETIC):
        got = host(pk.prism_kernels(kind, g))
        ref = obttb.kernel_array(kind, ogeom(g))
        assert got.shape == ref.shape
        rel = np.abs(got - ref).max() / np.abs(ref).max()
        if kind == pk.GRAVITY:
            # each entry within a few ulps of its terms' magnitudes (the sum cancels for
            # distant and deep cells, by more the larger the grid)
            ratio = (np.abs(got - ref) / (np.finfo(np.float64).eps * gravity_term_scale(g))).max()
            print(f"gravity {g.nx}x{g.ny}x{g.nz}: max err / (eps terms) = {ratio:.2f}, "
                  f"max err / max |T| = {rel:.2e}", flush=True)
            assert ratio <= 4.0
        else:
            # the magnetic closed forms keep their size at distance: relative to the array
            print(f"magnetic {g.nx}x{g.ny}x{g.nz}: max err / max |T| = {rel:.2e}", flush=True)
            assert rel <= 1e-14


# ------------------------------------------------------------------------------------
# products vs the dense oracle (small grids, GPU-generated kernels end to end)
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("g", [synth.SMALL, synth.SUB, RAGGED, ODD, TINY, PADDED, R5])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_products_match_dense_oracle(pk, g, dtype):
    og = ogeom(g)
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    rho, kap = synth.uniform_models(g, 1, 0)
    rough = synth.normal_like(g.data_shape, 1, 1)
    for kind, m in ((pk.GRAVITY, rho), (pk.MAGNETIC, kap)):
        A = oprism.dense_matrix(kind, og)
        op = pk.Operator.from_geometry(kind, g, dtype=dtype)
        y = host(op.matvec(dev(m, dtype)))
        y_ref = (A @ m.ravel()).reshape(g.data_shape)
        assert relerr(y, y_ref) <= tol
        # transpose on a smooth (data-like) and a rough residual
        for r in (y_ref / np.abs(y_ref).max(), rough):
            z = host(op.rmatvec(dev(r, dtype)))
            z_ref = (A.T @ r.ravel()).reshape(g.model_shape)
            assert relerr(z, z_ref) <= tol
        op.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_weighted_and_batched_products(pk, dtype):
    g = synth.SMALL
    og = ogeom(g)
    tol = F64_TOL if dtype == torch.float64 else F32_TOL
    r = synth.rng(1, 7)
    B = 3
    x = r.uniform(0, 1, (B,) + g.model_shape)
    v = r.standard_normal((B,) + g.data_shape)
    winv = r.uniform(0.5, 2.0, g.model_shape)
    wd = r.uniform(0.5, 2.0, g.data_shape)
    for kind in (pk.GRAVITY, pk.MAGNETIC):
        A = oprism.dense_matrix(kind, og)
        At = np.diag(wd.ravel()) @ A @ np.diag(winv.ravel())
        op = pk.Operator.from_geometry(kind, g, dtype=dtype, max_batch=2)   # batch 3 runs in 2 slices
        y = host(op.matvec(dev(x, dtype), winv=dev(winv, dtype), wd=dev(wd, dtype)))
        z = host(op.rmatvec(dev(v, dtype), winv=dev(winv, dtype), wd=dev(wd, dtype)))
        for b in range(B):
            assert relerr(y[b], (At @ x[b].ravel()).reshape(g.data_shape)) <= tol
            assert relerr(z[b], (At.T @ v[b].ravel()).reshape(g.model_shape)) <= tol
            # a batch member is computed exactly as a single call
            ys = host(op.matvec(dev(x[b], dtype), winv=dev(winv, dtype), wd=dev(wd, dtype)))
            assert np.array_equal(ys, y[b])
        op.close()


# ------------------------------------------------------------------------------------
# larger grids vs the oracle's FFT2 products (oracle kernels fed to the GPU setup)
# ------------------------------------------------------------------------------------
_REF_CACHE = {}


def _fft_refs(g, kind, m, rough):
    """Oracle kernel array and FFT2 products, computed once per grid and kind."""
    key = (g, kind)
    if key not in _REF_CACHE:
        T = obttb.kernel_array(kind, ogeom(g))
        y = obttb.fft_matvec(T, m, g.sx, g.sy, workers=8)
        smooth = y / np.abs(y).max()
        zr = obttb.fft_rmatvec(T, rough, g.sx, g.sy, workers=8)
        zs = obttb.fft_rmatvec(T, smooth, g.sx, g.sy, workers=8)
        _REF_CACHE[key] = (T, y, smooth, zr, zs)
    return _REF_CACHE[key]


def _fft_case(pk, g, models, dtype, tol):
    rough = synth.normal_like(g.data_shape, 3, 9)
    for kind, m in zip((pk.GRAVITY, pk.MAGNETIC), models):
        T, y_ref, smooth, zr_ref, zs_ref = _fft_refs(g, kind, m, rough)
        op = pk.Operator(dev(T), (g.sx, g.sy), dtype=dtype)
        print(f"grid {g.sx}x{g.sy}x{g.nz} kind {kind} {dtype}", flush=True)
        assert relerr(host(op.matvec(dev(m, dtype))), y_ref) <= tol
        assert relerr(host(op.rmatvec(dev(rough, dtype))), zr_ref) <= tol
        assert relerr(host(op.rmatvec(dev(smooth, dtype))), zs_ref) <= tol
        op.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mid_grid_matches_fft_oracle(pk, dtype):
    g = synth.MID
    _fft_case(pk, g, synth.random_boxes(g), dtype, F64_TOL if dtype == torch.float64 else F32_TOL)


@pytest.mark.parametrize("g", [R5, R35, R55], ids=["P40", "P120", "P200"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_radix5_transforms_match_fft_oracle(pk, g, dtype):
    # 5-smooth transform sizes with radix-5 passes in every product kernel (rows and columns)
    P = {R5: 40, R35: 120, R55: 200}[g]
    T = obttb.kernel_array(pk.GRAVITY, ogeom(g))
    op = pk.Operator(dev(T), (g.sx, g.sy), dtype=dtype)
    assert op.info()["Px"] == P and op.info()["Py"] == P
    op.close()
    _fft_case(pk, g, synth.random_boxes(g, seed_workload=2, index=P), dtype,
              F64_TOL if dtype == torch.float64 else F32_TOL)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_large_grid_matches_fft_oracle(pk, dtype):
    g = synth.LARGE
    _fft_case(pk, g, synth.dyke_and_block(g), dtype, F64_TOL if dtype == torch.float64 else F32_TOL)


def test_fp32_forward_error_at_256x256x32(pk):
    # The FP32 forward product sums its 32 layers' spectra in FP32 inside the column pass.
    # Its error against the FP64 oracle stays at FP32 rounding: about 2^-24 sqrt(log2 of the
    # 512 x 512 transform) per transform, plus sqrt(nz) 2^-24 = 3.4e-7 for the layer sum;
    # held to 1e-6, ten times below the FP32 parity bound.
    g = synth.LARGE
    rough = synth.normal_like(g.data_shape, 3, 9)
    for kind, m in zip((pk.GRAVITY, pk.MAGNETIC), synth.dyke_and_block(g)):
        T, y_ref, _, _, _ = _fft_refs(g, kind, m, rough)
        op = pk.Operator(dev(T), (g.sx, g.sy), dtype=torch.float32)
        e = relerr(host(op.matvec(dev(m, torch.float32))), y_ref)
        print(f"kind {kind}: FP32 forward rel err at 256x256x32 (32-layer FP32 sum) {e:.2e}", flush=True)
        assert e <= 1e-6
        op.close()


# ------------------------------------------------------------------------------------
# symmetric operators: the real, x-even eigenvalue store
# ------------------------------------------------------------------------------------
def _same_products(a, b, shape_m, shape_d, dtype, tol):
    rng = np.random.default_rng(11)
    x = dev(rng.uniform(0.0, 1.0, shape_m), dtype)
    r = dev(rng.standard_normal(shape_d), dtype)
    winv = dev(rng.uniform(0.5, 2.0, shape_m), dtype)
    wd = dev(rng.uniform(0.5, 2.0, shape_d), dtype)
    assert relerr(host(a.matvec(x)), host(b.matvec(x))) <= tol
    assert relerr(host(a.rmatvec(r)), host(b.rmatvec(r))) <= tol
    assert relerr(host(a.matvec(x, winv=winv, wd=wd)), host(b.matvec(x, winv=winv, wd=wd))) <= tol
    assert relerr(host(a.rmatvec(r, winv=winv, wd=wd)), host(b.rmatvec(r, winv=winv, wd=wd))) <= tol


def _store_checks(even, full, nz, dtype):
    ie, ifu = even.info(), full.info()
    assert (ie["eig_real_even"], ifu["eig_real_even"]) == (1, 0)
    esz = 8 if dtype == torch.float64 else 4
    K2, Px = ie["Py"] // 2 + 1, ie["Px"]
    assert ie["eig_bytes"] == nz * K2 * (Px // 2 + 1) * esz
    assert ifu["eig_bytes"] == nz * K2 * Px * 2 * esz
    # the expanded store is the complex one to rounding: real, lambda[Px - k] = lambda[k]
    eg, ef = even.eigenvalues().cpu().numpy(), full.eigenvalues().cpu().numpy()
    assert np.abs(eg.imag).max() == 0.0
    assert np.abs(eg - ef).max() <= (1e-14 if dtype == torch.float64 else 1e-6) * np.abs(ef).max()


# Stations above the prism centres (sx = nx, sy = ny): the gravity kernel is even in both
# lags, so its eigenvalues are real and lambda[Px - k] = lambda[k]; the magnetic kernel at
# I = 65 deg, D = 2 deg is not.  FP32 plans take the real store (the two stores differ by the
# FP32 rounding of Lambda[Px - k] against Lambda[k]).  FP64 plans of these kernels keep the
# complex store: their closed forms evaluate T(i, j) and T(-i, j) with different rounding,
# which the far-field cancellation amplifies to |Im lambda| ~ 6e-13 (16^2) .. 1e-10 (128^2) of
# max |lambda|, above the FP64 test (1e-14).
@pytest.mark.parametrize("g", [synth.SMALL, synth.MID, synth.SUB, R35], ids=["P32", "P256", "P24", "P120"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_symmetric_gravity_operator_store(pk, g, dtype):
    # (the 5-smooth sizes 24 and 120 take the real store through the one-plan LDS kernels too)
    grav = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=dtype)
    full = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=dtype, full_eig=True)
    mag = pk.Operator.from_geometry(pk.MAGNETIC, g, dtype=dtype)
    assert mag.info()["eig_real_even"] == 0
    if dtype == torch.float64:
        assert grav.info()["eig_real_even"] == 0
    else:
        _store_checks(grav, full, g.nz, dtype)
        _same_products(grav, full, g.model_shape, g.data_shape, dtype, 1e-6)
    for op in (grav, full, mag):
        op.close()


# An FP64 kernel array symmetric bit for bit, T(i, j) = T(-i, j) = T(i, -j): the FP64 plan takes
# the real store, and its products agree with the complex store's to rounding.
@pytest.mark.parametrize("n", [(16, 12, 3), (100, 60, 4)])
def test_exactly_symmetric_kernel_fp64_store(pk, n):
    sx, sy, nz = n
    rng = np.random.default_rng(sx)
    h = rng.standard_normal((nz, sx, sy))     # lags 0 .. s-1 in each direction
    T = np.zeros((nz, 2 * sx - 1, 2 * sy - 1))
    for i in range(-(sx - 1), sx):
        for j in range(-(sy - 1), sy):
            T[:, i + sx - 1, j + sy - 1] = h[:, abs(i), abs(j)]
    even = pk.Operator(dev(T), (sx, sy), dtype=torch.float64, pad_pow2=True)
    full = pk.Operator(dev(T), (sx, sy), dtype=torch.float64, pad_pow2=True, full_eig=True)
    _store_checks(even, full, nz, torch.float64)
    _same_products(even, full, (nz, sx, sy), (sx, sy), torch.float64, 1e-13)
    even.close()
    full.close()


# ------------------------------------------------------------------------------------
# structural properties
# ------------------------------------------------------------------------------------
def test_adjoint_identity_fp64(pk):
    for g in (synth.SMALL, RAGGED, synth.MID):
        r = synth.rng(4, g.nx)
        x = r.standard_normal(g.model_shape)
        v = r.standard_normal(g.data_shape)
        for kind in (pk.GRAVITY, pk.MAGNETIC):
            op = pk.Operator.from_geometry(kind, g, dtype=torch.float64)
            y = host(op.matvec(dev(x)))
            z = host(op.rmatvec(dev(v)))
            assert abs(np.sum(y * v) - np.sum(x * z)) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(v)
            op.close()


def test_impulse_response_is_dense_column(pk):
    g = RAGGED
    A = oprism.dense_matrix(oprism.MAGNETIC, ogeom(g))
    op = pk.Operator.from_geometry(pk.MAGNETIC, g, dtype=torch.float64)
    for (a, b, rr) in [(0, 0, 0), (g.nx - 1, g.ny - 1, g.nz - 1), (5, 2, 1)]:
        e = np.zeros(g.model_shape)
        e[rr, a, b] = 1.0
        y = host(op.matvec(dev(e)))
        col = A[:, (rr * g.nx + a) * g.ny + b].reshape(g.data_shape)
        assert np.abs(y - col).max() <= 1e-12 * np.abs(col).max()
    op.close()


def test_launch_shape_and_repeatability(pk):
    g = synth.MID
    x, _ = synth.random_boxes(g)
    v = synth.normal_like(g.data_shape, 2, 3)
    op = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=torch.float64)
    y0 = host(op.matvec(dev(x)))
    z0 = host(op.rmatvec(dev(v)))
    assert np.array_equal(y0, host(op.matvec(dev(x))))           # repeatable
    assert np.array_equal(z0, host(op.rmatvec(dev(v))))
    info = op.info()
    op.set_launch(row_fft_per_block=1)                              # same arithmetic per element
    assert np.array_equal(y0, host(op.matvec(dev(x))))
    assert np.array_equal(z0, host(op.rmatvec(dev(v))))
    op.set_launch(col_fft_per_block=1)                              # layers grouped differently
    assert relerr(host(op.matvec(dev(x))), y0) <= 1e-14
    assert np.array_equal(z0, host(op.rmatvec(dev(v))))
    op.set_launch(col_fft_per_block=info["col_fft_per_block"], row_fft_per_block=info["row_fft_per_block"])
    op.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autotune_keeps_results(pk, dtype):
    g = synth.MID
    x, _ = synth.random_boxes(g)
    v = synth.normal_like(g.data_shape, 2, 3)
    op = pk.Operator.from_geometry(pk.GRAVITY, g, dtype=dtype)
    y0, z0 = host(op.matvec(dev(x, dtype))), host(op.rmatvec(dev(v, dtype)))
    res = op.autotune(reps=2)
    info = op.info()
    assert res["tried"] >= 8 and res["us_per_pair"] > 0
    assert (info["col_fft_per_block"], info["row_fft_per_block"], info["layer_chunks"]) == \
        (res["col_fft_per_block"], res["row_fft_per_block"], res["layer_chunks"])
    tol = 1e-14 if dtype == torch.float64 else 1e-6
    assert relerr(host(op.matvec(dev(x, dtype))), y0) <= tol
    assert np.array_equal(host(op.rmatvec(dev(v, dtype))), z0)
    op.close()


@pytest.mark.parametrize("g", [synth.MID, synth.SUB])
def test_timing_with_repeats_leaves_results_unchanged(pk, g):
    # power-of-two (register FFT) and radix-3 (generic) paths
    x, _ = synth.random_boxes(g)
    v = synth.normal_like(g.data_shape, 2, 3)
    op = pk.Operator.from_geometry(pk.MAGNETIC, g, dtype=torch.float32)
    y0 = host(op.matvec(dev(x, torch.float32)))
    z0 = host(op.rmatvec(dev(v, torch.float32)))
    op.timing_enable(64, repeat=3)
    assert np.array_equal(y0, host(op.matvec(dev(x, torch.float32))))
    assert np.array_equal(z0, host(op.rmatvec(dev(v, torch.float32))))
    t = op.timing_read()
    assert all(n == 3 for ms, n in t.values()), t
    assert all(ms > 0 for ms, n in t.values()), t
    op.timing_enable(0)
    assert all(n == 0 for ms, n in op.timing_read().values())
    op.close()


def test_error_paths(pk):
    from paper_2112_15562_amd import _lib as L
    with pytest.raises(L.BTTBError) as e:
        pk.Operator(torch.zeros((1, 2049, 3), dtype=torch.float64, device="cuda"), (1, 1))
    assert e.value.status == L.BTTB_ESIZE
    op = pk.Operator.from_geometry(pk.GRAVITY, synth.SUB, dtype=torch.float64)
    with pytest.raises(TypeError):
        op.matvec(torch.zeros(synth.SUB.model_shape, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        op.matvec(torch.zeros((6, 12, 11), dtype=torch.float64, device="cuda"))
    with pytest.raises(L.BTTBError) as e:
        op.set_launch(row_fft_per_block=3)
    assert e.value.status == L.BTTB_EINVAL
    # misaligned pointer
    buf = torch.zeros(synth.SUB.nz * 144 + 1, dtype=torch.float64, device="cuda")
    out = torch.zeros(144, dtype=torch.float64, device="cuda")
    import ctypes as C
    rc = L.lib().bttb_matvec(op.plan, C.c_void_p(buf.data_ptr() + 4), C.c_void_p(out.data_ptr()), None)
    assert rc == L.BTTB_EINVAL
    op.close()


# ------------------------------------------------------------------------------------
# the largest transform (BTTB_MAX_TRANSFORM = 2048 points) along either axis
# ------------------------------------------------------------------------------------
LONG = [synth.Grid(1000, 16, 1000, 16, 2, 40.0, 40.0, 25.0), synth.Grid(16, 1000, 16, 1000, 2, 40.0, 40.0, 25.0, decl=20.0)]


@pytest.mark.parametrize("g", LONG, ids=["Px2048", "Py2048"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_products_at_the_largest_transform(pk, g, dtype, tol):
    og = ogeom(g)
    rng = np.random.default_rng(g.nx)
    x = rng.uniform(0.0, 1.0, g.model_shape)
    r = rng.standard_normal(g.data_shape)
    ops, refs = [], []
    for kind in (oprism.GRAVITY, oprism.MAGNETIC):
        T = obttb.kernel_array(kind, og)
        op = pk.Operator(torch.as_tensor(T, device="cuda"), (g.sx, g.sy), dtype=dtype, pad="pow2")
        assert max(op.info()["Px"], op.info()["Py"]) == pk.MAX_TRANSFORM == 2048
        ops.append(op)
        refs.append((obttb.fft_matvec(T, x, g.sx, g.sy), obttb.fft_rmatvec(T, r, g.sx, g.sy)))
    xd, rd = torch.as_tensor(x, dtype=dtype, device="cuda"), torch.as_tensor(r, dtype=dtype, device="cuda")
    for op, (y, z) in zip(ops, refs):
        errs = [relerr(host(op.matvec(xd)), y), relerr(host(op.rmatvec(rd)), z)]
        print(f"{dtype} {g.nx}x{g.ny} one plan: {errs}", flush=True)
        assert max(errs) <= tol
    grp = pk.Group(ops)
    ys, zs = grp.matvec([xd, xd]), grp.rmatvec([rd, rd])
    for i, (y, z) in enumerate(refs):
        errs = [relerr(host(ys[i]), y), relerr(host(zs[i]), z)]
        print(f"{dtype} {g.nx}x{g.ny} group member {i}: {errs}", flush=True)
        assert max(errs) <= tol
    grp.close()
    for op in ops:
        op.close()


def test_empty_and_chunked_batches(pk):
    from paper_2112_15562_amd import _lib as L
    g = synth.SUB
    op = pk.Operator.from_geometry(pk.MAGNETIC, g, dtype=torch.float64, max_batch=2)
    # an empty batch gives an empty result without a library call
    y = op.matvec(torch.zeros((0,) + tuple(op.model_shape), dtype=torch.float64, device="cuda"))
    z = op.rmatvec(torch.zeros((0, 3) + tuple(op.data_shape), dtype=torch.float64, device="cuda"))
    assert tuple(y.shape) == (0,) + tuple(op.data_shape) and tuple(z.shape) == (0, 3) + tuple(op.model_shape)
    # the C entry point refuses batch 0
    x = torch.rand((5,) + tuple(op.model_shape), dtype=torch.float64, device="cuda")
    out = torch.empty((5,) + tuple(op.data_shape), dtype=torch.float64, device="cuda")
    nin, nout = x[0].numel(), out[0].numel()
    assert L.lib().bttb_apply(op.plan, L.BTTB_OP_FORWARD, 0, x.data_ptr(), nin, out.data_ptr(), nout,
                              None, None, None) == L.BTTB_EINVAL
    # a batch above max_batch runs max_batch members at a time: every member as alone
    ys = op.matvec(x)
    zs = op.rmatvec(ys)
    for b in range(5):
        assert relerr(host(ys[b]), host(op.matvec(x[b].contiguous()))) <= 1e-15
        assert relerr(host(zs[b]), host(op.rmatvec(ys[b].contiguous()))) <= 1e-15
    op.close()
