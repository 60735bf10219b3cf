"""Pins of the oracle's prism kernels and dense sensitivity matrix (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import prism

HERE = os.path.dirname(os.path.abspath(__file__))


def _gl_nodes(a, b, n):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * t + 0.5 * (a + b), 0.5 * (b - a) * w


def _cubature(x0, y0, z0, xb, yb, zb, f, n=48):
    X, wx = _gl_nodes(*xb, n)
    Y, wy = _gl_nodes(*yb, n)
    Z, wz = _gl_nodes(*zb, n)
    XX, YY, ZZ = np.meshgrid(X - x0, Y - y0, Z - z0, indexing="ij")
    W = wx[:, None, None] * wy[None, :, None] * wz[None, None, :]
    return float(np.sum(W * f(XX, YY, ZZ)))


BOX = ((0.0, 50.0), (0.0, 40.0), (100.0, 125.0))
STATIONS = [(23.0, 18.5, -1.0), (210.0, -85.0, -1.0), (-310.0, 45.0, -3.0), (75.0, 60.0, -20.0)]


@pytest.mark.parametrize("st", STATIONS)
def test_gravity_matches_cubature_of_definition(st):
    # g_z = C_G * int Z / R^3 dV, evaluated by 48^3-point Gauss-Legendre cubature
    def f(X, Y, Z):
        return Z / np.sqrt(X * X + Y * Y + Z * Z) ** 3
    ref = prism.C_G * _cubature(*st, *BOX, f)
    got = prism.gravity_prism(*st, *BOX)
    assert abs(got - ref) <= 1e-11 * abs(ref)
    assert got > 0  # positive density below the station attracts downward


@pytest.mark.parametrize("st", STATIONS)
def test_hessian_matches_cubature_of_definition(st):
    # H_ab = int d_a d_b (1/R) dV = int (3 X_a X_b - delta_ab R^2) / R^5 dV
    H = prism.prism_hessian(*st, *BOX)
    comps = {
        "xx": lambda X, Y, Z: 3 * X * X - (X * X + Y * Y + Z * Z),
        "yy": lambda X, Y, Z: 3 * Y * Y - (X * X + Y * Y + Z * Z),
        "zz": lambda X, Y, Z: 3 * Z * Z - (X * X + Y * Y + Z * Z),
        "xy": lambda X, Y, Z: 3 * X * Y,
        "xz": lambda X, Y, Z: 3 * X * Z,
        "yz": lambda X, Y, Z: 3 * Y * Z,
    }
    scale = max(abs(v) for v in H.values())
    for k, num in comps.items():
        ref = _cubature(*st, *BOX, lambda X, Y, Z: num(X, Y, Z) / np.sqrt(X * X + Y * Y + Z * Z) ** 5)
        assert abs(H[k] - ref) <= 1e-10 * scale, k


def _split(b):
    mid = 0.5 * (b[0] + b[1])
    return [(b[0], mid), (mid, b[1])]


@pytest.mark.parametrize("st", STATIONS)
def test_additivity_over_subprisms(st):
    xb, yb, zb = BOX
    g = prism.gravity_prism(*st, xb, yb, zb)
    m = prism.magnetic_prism(*st, xb, yb, zb, 65.0, 2.0, 50000.0)
    gs = ms = 0.0
    for xs in _split(xb):
        for ys in _split(yb):
            for zs in _split(zb):
                gs += prism.gravity_prism(*st, xs, ys, zs)
                ms += prism.magnetic_prism(*st, xs, ys, zs, 65.0, 2.0, 50000.0)
    assert abs(g - gs) <= 1e-12 * abs(g)
    assert abs(m - ms) <= 1e-11 * abs(m)


def _point_mass_error(D_over_s, s=10.0):
    x0, y0, z0 = 0.0, 0.0, 0.0
    c = np.array([0.6, 0.3, 1.0]) / np.linalg.norm([0.6, 0.3, 1.0]) * D_over_s * s
    xb = (c[0] - s / 2, c[0] + s / 2)
    yb = (c[1] - s / 2, c[1] + s / 2)
    zb = (c[2] - s / 2, c[2] + s / 2)
    got = prism.gravity_prism(x0, y0, z0, xb, yb, zb)
    r = np.linalg.norm(c)
    ref = prism.C_G * s ** 3 * c[2] / r ** 3
    return abs(got - ref) / abs(ref)


def test_gravity_far_field_point_mass_fourth_order():
    # a cube has no quadrupole moment, so the point-mass error falls as (s/D)^4
    e10 = _point_mass_error(10.0)
    e30 = _point_mass_error(30.0)
    assert e30 < 1e-6
    assert 40.0 < e10 / e30 < 120.0   # 3^4 = 81


def test_magnetic_far_field_dipole():
    s = 10.0
    I, D, F = 65.0, 2.0, 50000.0
    fh = prism.field_direction(I, D)
    for Ds in (30.0, 60.0):
        c = np.array([0.5, -0.4, 1.0]) / np.linalg.norm([0.5, -0.4, 1.0]) * Ds * s
        xb = (c[0] - s / 2, c[0] + s / 2)
        yb = (c[1] - s / 2, c[1] + s / 2)
        zb = (c[2] - s / 2, c[2] + s / 2)
        got = prism.magnetic_prism(0.0, 0.0, 0.0, xb, yb, zb, I, D, F)
        r = np.linalg.norm(c)
        rh = c / r
        ref = F * s ** 3 * (3.0 * np.dot(fh, rh) ** 2 - 1.0) / (4.0 * np.pi * r ** 3)
        assert abs(got - ref) <= 1e-5 * abs(ref)


@pytest.mark.parametrize("st", STATIONS)
def test_laplace_trace_vanishes_outside(st):
    H = prism.prism_hessian(*st, *BOX)
    assert abs(H["xx"] + H["yy"] + H["zz"]) <= 1e-12


@pytest.mark.parametrize("st", STATIONS)
def test_poisson_relation_vertical_field(st):
    # at I = 90 deg: 4 pi K_m / F = H_zz = -d(g_z / C_G)/dh  (station height h = -z0)
    F = 50000.0
    km = prism.magnetic_prism(*st, *BOX, 90.0, 0.0, F)
    x0, y0, z0 = st

    def central(dh):
        gp = prism.gravity_prism(x0, y0, z0 - dh, *BOX) / prism.C_G   # h + dh
        gm = prism.gravity_prism(x0, y0, z0 + dh, *BOX) / prism.C_G   # h - dh
        return -(gp - gm) / (2 * dh)
    fd = (4 * central(0.1) - central(0.2)) / 3     # Richardson: O(dh^4)
    assert abs(4 * np.pi * km / F - fd) <= 1e-7 * abs(fd)


def test_mirror_symmetries():
    g = prism.Geometry(8, 8, 8, 8, 3, 50.0, 40.0, 25.0, incl=60.0, decl=0.0)
    # the alternating corner sum cancels more with distance, so the tolerance is
    # relative to the largest (near-field) entry of the layer
    for (u, v) in [(3, 2), (1, 5), (7, 7), (2, 0)]:
        for r in range(3):
            kg = [prism.sensitivity(prism.GRAVITY, g, uu, vv, 0, 0, r)
                  for uu, vv in [(u, v), (-u, v), (u, -v)]]
            sg = abs(prism.sensitivity(prism.GRAVITY, g, 0, 0, 0, 0, r))
            assert abs(kg[1] - kg[0]) <= 1e-12 * sg
            assert abs(kg[2] - kg[0]) <= 1e-12 * sg
            # D = 0: the field lies in the y-z plane, so the response is even in x
            km = [prism.sensitivity(prism.MAGNETIC, g, uu, v, 0, 0, r) for uu in (u, -u)]
            sm = abs(prism.sensitivity(prism.MAGNETIC, g, 0, 0, 0, 0, r))
            assert abs(km[1] - km[0]) <= 1e-12 * sm
    # with a declination the magnetic kernel is not even in x (unsymmetric BTTB)
    g2 = prism.Geometry(8, 8, 8, 8, 3, 50.0, 40.0, 25.0, incl=65.0, decl=20.0)
    a = prism.sensitivity(prism.MAGNETIC, g2, 3, 2, 0, 0, 0)
    b = prism.sensitivity(prism.MAGNETIC, g2, -3, 2, 0, 0, 0)
    assert abs(a - b) > 1e-3 * abs(a)


def test_bouguer_slab_limit():
    # an L x L layer of thickness dz tends to the infinite slab 2 pi G rho dz
    dz = 25.0
    slab = 2 * np.pi * prism.C_G * dz
    errs = []
    for L in (400.0, 1600.0, 6400.0):
        g = prism.gravity_prism(0.0, 0.0, -1.0, (-L / 2, L / 2), (-L / 2, L / 2), (0.0, dz))
        errs.append(abs(g - slab) / slab)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_dense_matrix_shift_invariance_and_layout():
    g = prism.Geometry(6, 5, 7, 4, 3, 50.0, 40.0, 25.0)
    for kind in (prism.GRAVITY, prism.MAGNETIC):
        A = prism.dense_matrix(kind, g)
        assert A.shape == (g.sx * g.sy, g.nx * g.ny * g.nz)
        row = lambda p, q: p * g.sy + q
        col = lambda a, b, r: (r * g.nx + a) * g.ny + b
        scale = np.abs(A).max()
        for (p, q, a, b, r) in [(0, 0, 0, 0, 0), (2, 3, 1, 0, 1), (4, 1, 5, 2, 2), (1, 2, 3, 3, 0)]:
            for (dp, dq) in [(1, 0), (0, 1), (1, 1)]:
                if p + dp < g.sx and q + dq < g.sy and a + dp < g.nx and b + dq < g.ny:
                    x = A[row(p, q), col(a, b, r)]
                    y = A[row(p + dp, q + dq), col(a + dp, b + dq, r)]
                    assert abs(x - y) <= 1e-12 * scale
        # entry = closed form at the absolute coordinates
        x0, y0, z0 = prism.station_xyz(g, 4, 1)
        xb, yb, zb = prism.prism_bounds(g, 5, 2, 2)
        ref = (prism.gravity_prism(x0, y0, z0, xb, yb, zb) if kind == prism.GRAVITY else
               prism.magnetic_prism(x0, y0, z0, xb, yb, zb, g.incl, g.decl, g.field))
        assert A[row(4, 1), col(5, 2, 2)] == pytest.approx(float(ref), rel=1e-14)


def test_printed_storage_figures():
    with open(os.path.join(HERE, "golden", "storage.json")) as f:
        gold = json.load(f)
    d1 = gold["dense_one"]
    assert round(d1["m"] * d1["n"] * d1["bytes_per_real"] / 1e9) == d1["printed_GB"]
    d2 = gold["dense_two"]
    assert d2["m"] * d2["n"] * 8 * d2["operators"] == d2["printed_bytes"]
    t = gold["transform"]
    # 299 x 199 = (150+150-1) x (100+100-1): the T size of Sec. 2.7.1 for the 150x100 grid
    assert (t["Lx"], t["Ly"]) == (150 + 150 - 1, 100 + 100 - 1)
    tb = t["operators"] * t["nz"] * t["Lx"] * t["Ly"] * t["bytes_per_complex"]
    assert round(tb / 1e6) == t["printed_MB"]
    assert round(d2["printed_bytes"] / tb) == t["printed_reduction"]


def test_station_offset_selects_rows_of_the_full_grid():
    # stations over an interior part of the prism grid (offset ox, oy) see the same
    # sensitivities as the matching stations of a station grid covering every column
    full = prism.Geometry(8, 7, 8, 7, 2, 40.0, 30.0, 25.0, incl=55.0, decl=10.0)
    part = prism.Geometry(4, 3, 8, 7, 2, 40.0, 30.0, 25.0, incl=55.0, decl=10.0, ox=2, oy=3)
    for kind in (prism.GRAVITY, prism.MAGNETIC):
        A = prism.dense_matrix(kind, full).reshape(8, 7, -1)
        B = prism.dense_matrix(kind, part).reshape(4, 3, -1)
        assert np.array_equal(B, A[2:6, 3:6])
