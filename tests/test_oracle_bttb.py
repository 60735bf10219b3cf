"""Pins of the oracle's BTTB layout and FFT2 products against the dense matrix (CPU)."""
import numpy as np
import pytest

from oracle import bttb, dft, prism


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_dft_definition_matches_numpy_and_parseval():
    r = np.random.default_rng(7)
    for N in (24, 32, 40, 45, 64):
        x = r.standard_normal(N) + 1j * r.standard_normal(N)
        X = dft.dft(x)
        assert np.allclose(X, np.fft.fft(x), rtol=0, atol=1e-12 * np.abs(X).max())
        assert abs(np.vdot(X, X).real - N * np.vdot(x, x).real) <= 1e-12 * N * np.vdot(x, x).real
        xi = dft.dft(X, sign=+1) / N
        assert np.allclose(xi, x, atol=1e-13)
    x2 = r.standard_normal((12, 10))
    assert np.allclose(dft.dft2(x2), np.fft.fft2(x2), atol=1e-12)


GEOMS = [
    prism.Geometry(16, 16, 16, 16, 8, 50.0, 50.0, 50.0),        # 16x16 over 16x16x8
    prism.Geometry(12, 12, 12, 12, 6, 50.0, 50.0, 50.0),        # 12x12x6 subcase
    prism.Geometry(7, 9, 11, 5, 3, 40.0, 30.0, 25.0, decl=20.0),  # ragged, sx != nx
    prism.Geometry(5, 4, 9, 8, 2, 40.0, 30.0, 25.0, ox=2, oy=3),  # stations over an interior part
]


@pytest.fixture(scope="module", params=range(len(GEOMS)))
def setup(request):
    g = GEOMS[request.param]
    out = {}
    for kind in (prism.GRAVITY, prism.MAGNETIC):
        out[kind] = (prism.dense_matrix(kind, g), bttb.kernel_array(kind, g))
    return g, out


def test_kernel_array_holds_dense_entries(setup):
    g, ops = setup
    for kind, (A, T) in ops.items():
        assert T.shape == (g.nz, g.sx + g.nx - 1, g.sy + g.ny - 1)
        r = np.random.default_rng(3)
        for _ in range(50):
            p, q = r.integers(g.sx), r.integers(g.sy)
            a, b, z = r.integers(g.nx), r.integers(g.ny), r.integers(g.nz)
            dense = A[p * g.sy + q, (z * g.nx + a) * g.ny + b]
            tv = T[z, p - a + g.nx - 1, q - b + g.ny - 1]
            assert abs(dense - tv) <= 1e-12 * np.abs(T[z]).max()


def test_fft_products_equal_dense_products(setup):
    g, ops = setup
    r = np.random.default_rng(11)
    for kind, (A, T) in ops.items():
        x = r.uniform(0, 1, (g.nz, g.nx, g.ny))
        v = r.standard_normal((g.sx, g.sy))
        y_d = (A @ x.ravel()).reshape(g.sx, g.sy)
        z_d = (A.T @ v.ravel()).reshape(g.nz, g.nx, g.ny)
        assert relerr(bttb.fft_matvec(T, x, g.sx, g.sy), y_d) <= 1e-12
        assert relerr(bttb.fft_rmatvec(T, v, g.sx, g.sy), z_d) <= 1e-12


def test_impulse_columns_and_rows(setup):
    g, ops = setup
    for kind, (A, T) in ops.items():
        for (a, b, z) in [(0, 0, 0), (g.nx - 1, g.ny - 1, g.nz - 1), (g.nx // 2, 1, g.nz // 2)]:
            e = np.zeros((g.nz, g.nx, g.ny))
            e[z, a, b] = 1.0
            col = A[:, (z * g.nx + a) * g.ny + b].reshape(g.sx, g.sy)
            got = bttb.fft_matvec(T, e, g.sx, g.sy)
            assert np.abs(got - col).max() <= 1e-13 * np.abs(col).max()
        for (p, q) in [(0, 0), (g.sx - 1, g.sy - 1), (g.sx // 2, 2)]:
            e = np.zeros((g.sx, g.sy))
            e[p, q] = 1.0
            row = A[p * g.sy + q, :].reshape(g.nz, g.nx, g.ny)
            got = bttb.fft_rmatvec(T, e, g.sx, g.sy)
            assert np.abs(got - row).max() <= 1e-13 * np.abs(row).max()


def test_adjoint_identity(setup):
    g, ops = setup
    r = np.random.default_rng(5)
    for kind, (A, T) in ops.items():
        x = r.standard_normal((g.nz, g.nx, g.ny))
        v = r.standard_normal((g.sx, g.sy))
        y = bttb.fft_matvec(T, x, g.sx, g.sy)
        z = bttb.fft_rmatvec(T, v, g.sx, g.sy)
        lhs = float(np.sum(y * v))
        rhs = float(np.sum(x * z))
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(v)


def test_weighted_products(setup):
    g, ops = setup
    r = np.random.default_rng(9)
    for kind, (A, T) in ops.items():
        x = r.standard_normal((g.nz, g.nx, g.ny))
        v = r.standard_normal((g.sx, g.sy))
        winv = r.uniform(0.5, 2.0, x.shape)
        wd = r.uniform(0.5, 2.0, v.shape)
        At = np.diag(wd.ravel()) @ A @ np.diag(winv.ravel())      # W_d A W^-1
        assert relerr(bttb.weighted_matvec(T, x, winv, wd, g.sx, g.sy),
                      (At @ x.ravel()).reshape(v.shape)) <= 1e-12
        assert relerr(bttb.weighted_rmatvec(T, v, winv, wd, g.sx, g.sy),
                      (At.T @ v.ravel()).reshape(x.shape)) <= 1e-12


def test_gravity_block_symmetric_magnetic_not():
    # Sec. 2.7.1: the gravity BTTB blocks are symmetric, the magnetic ones are not
    g = prism.Geometry(9, 9, 9, 9, 2, 50.0, 50.0, 50.0)
    for kind, sym in ((prism.GRAVITY, True), (prism.MAGNETIC, False)):
        A = prism.dense_matrix(kind, g)
        blk = A[:, :g.nx * g.ny]
        d = np.abs(blk - blk.T).max() / np.abs(blk).max()
        assert (d <= 1e-12) if sym else (d > 1e-3)
