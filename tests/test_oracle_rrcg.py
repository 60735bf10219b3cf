"""Pins of the oracle's Gramian and RRCG iteration (CPU only)."""
import math

import numpy as np
import pytest

from oracle import bttb, prism, rrcg

G6 = prism.Geometry(6, 6, 6, 6, 3, 50.0, 50.0, 50.0)   # n = 108 unknowns, m = 36 data


def _ops(g):
    return [bttb.DenseOperator(prism.dense_matrix(k, g), g) for k in (prism.GRAVITY, prism.MAGNETIC)]


@pytest.fixture(scope="module")
def ops6():
    return _ops(G6)


def test_gramian_identities():
    r = np.random.default_rng(1)
    m1 = r.standard_normal(50)
    for gamma in (0.3, -2.0, 7.5):
        m2 = gamma * m1
        s = rrcg.gramian(m1, m2)
        assert abs(s) <= 1e-12 * rrcg.dot(m1, m1) * rrcg.dot(m2, m2)
        l1, l2 = rrcg.gramian_ascent(m1, m2)
        assert np.abs(l1).max() <= 1e-12 * np.abs(m1).max() * rrcg.dot(m2, m2)
        assert np.abs(l2).max() <= 1e-12 * np.abs(m2).max() * rrcg.dot(m1, m1)
    for _ in range(5):
        a, b = r.standard_normal(30), r.standard_normal(30)
        assert rrcg.gramian(a, b) >= 0.0
        # gradient of S_G by central differences equals 2 l_G (l_G is the half-gradient)
        l1, l2 = rrcg.gramian_ascent(a, b)
        h = 1e-6
        for j in (0, 7, 29):
            e = np.zeros(30)
            e[j] = h
            g1 = (rrcg.gramian(a + e, b) - rrcg.gramian(a - e, b)) / (2 * h)
            g2 = (rrcg.gramian(a, b + e) - rrcg.gramian(a, b - e)) / (2 * h)
            assert abs(g1 - 2 * l1[j]) <= 1e-6 * max(1.0, abs(g1))
            assert abs(g2 - 2 * l2[j]) <= 1e-6 * max(1.0, abs(g2))
    # scalar weights: S~_G = (w1 w2)^2 S_G
    a, b = r.standard_normal(30), r.standard_normal(30)
    w1, w2 = 2.5, 0.7
    assert rrcg.gramian(w1 * a, w2 * b) == pytest.approx((w1 * w2) ** 2 * rrcg.gramian(a, b), rel=1e-12)


def test_l1_weight():
    eps2 = 1e-9
    m = np.array([0.0, 1e-3, 0.2, -0.5])
    w = rrcg.l1_weight(m, np.zeros(4), eps2)
    assert w[0] == pytest.approx(eps2 ** -0.25, rel=1e-15)     # = 177.83
    assert w[0] == pytest.approx(177.8279410038923, rel=1e-12)
    # ||W_L1 (m - m_apr)||^2 -> ||m - m_apr||_1 as eps -> 0
    assert np.sum((w * m) ** 2) == pytest.approx(np.abs(m).sum(), rel=1e-5)


def _data(g, ops, seed=0, noise=0.0, wdepth=None):
    r = np.random.default_rng(seed)
    m_true = [np.zeros((g.nz, g.nx, g.ny)) for _ in range(2)]
    m_true[0][1:3, 2:4, 1:4] = 0.8
    m_true[1][1:3, 2:4, 1:4] = 0.08
    d = [ops[i].matvec(m_true[i]) for i in range(2)]
    sig = [0.02 * np.abs(d[i]) + 0.01 * np.abs(d[i]).max() for i in range(2)]
    dobs = [d[i] + noise * sig[i] * r.standard_normal(d[i].shape) for i in range(2)]
    if wdepth is None:
        wdepth = [np.ones(m_true[0].shape), np.ones(m_true[0].shape)]
    return rrcg.Data(dobs=dobs, wd=[1.0 / s for s in sig], wdepth=wdepth), m_true


def test_cg_reduces_to_tikhonov_normal_equations(ops6):
    # lambda = 0, W_L1 = I (p = 2), fixed W, q = 1, no bounds: one outer step of n
    # inner CG steps solves (A~^T A~ + alpha I) m~ = A~^T d~ (normal equations); a few
    # outer steps (restarts from the true residual) remove the recurrence's drift
    g = G6
    r = np.random.default_rng(2)
    wdepth = [r.uniform(0.5, 2.0, (g.nz, g.nx, g.ny)) for _ in range(2)]
    data, _ = _data(g, ops6, noise=1.0, wdepth=wdepth)
    alpha = (3.0, 0.5)
    prm = rrcg.Params(alpha0=alpha, q=(1.0, 1.0), lam=(0.0, 0.0), p_norm=2, restart=True)
    st0 = rrcg.initial_state(data, prm, (g.nz, g.nx, g.ny))
    st1, _ = rrcg.run(ops6, data, prm, n_outer=4, n_inner=2 * g.n, state=st0)
    for i in range(2):
        A = ops6[i].A
        W = wdepth[i].ravel()
        At = np.diag(data.wd[i].ravel()) @ A @ np.diag(1.0 / W)
        mt = np.linalg.solve(At.T @ At + alpha[i] * np.eye(g.n), At.T @ (data.wd[i] * data.dobs[i]).ravel())
        ref = mt / W
        assert np.linalg.norm(st1.m[i].ravel() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_objective_decreases_within_inner_cycle(ops6):
    g = G6
    data, _ = _data(g, ops6, noise=1.0)
    prm = rrcg.Params(alpha0=(10.0, 10.0), q=(1.0, 1.0), p_norm=2, restart=True)
    st0 = rrcg.initial_state(data, prm, (g.nz, g.nx, g.ny))

    def objective(m):
        val = 0.0
        for i in range(2):
            rr = data.wd[i] * (ops6[i].matvec(m[i]) - data.dobs[i])
            val += rrcg.dot(rr, rr) + prm.alpha0[i] * rrcg.dot(data.wdepth[i] * m[i], data.wdepth[i] * m[i])
        return val
    vals = [objective(st0.m)]
    for J in range(1, 12):
        st, _ = rrcg.outer_step(ops6, data, prm, st0, n_inner=J)
        vals.append(objective(st.m))
    assert all(vals[j + 1] <= vals[j] * (1 + 1e-12) for j in range(len(vals) - 1))
    assert vals[-1] < 0.5 * vals[0]


def test_gramian_term_reaches_stationary_point_of_objective(ops6):
    # W = I, lambda1 = lambda2: l is half the gradient of
    # sum ||W_d(A m - d)||^2 + alpha ||m||^2 + lambda S_G, so the iteration's limit is a
    # stationary point of that objective.  The residual gradient there must be small
    # next to the Gramian part of the gradient: a dropped, halved or sign-flipped
    # coupling term leaves a residual of the same size as that part.
    g = G6
    data, _ = _data(g, ops6, noise=0.5)
    lam, alpha = 1e3, 20.0
    prm = rrcg.Params(alpha0=(alpha, alpha), q=(1.0, 1.0), lam=(lam, lam), p_norm=2, restart=True)
    st = rrcg.initial_state(data, prm, (g.nz, g.nx, g.ny))
    for _ in range(160):
        st, _ = rrcg.outer_step(ops6, data, prm, st, n_inner=20)
    A = [ops6[i].A for i in range(2)]
    Wd = [data.wd[i].ravel() for i in range(2)]
    d = [data.dobs[i].ravel() for i in range(2)]
    m1, m2 = st.m[0].ravel(), st.m[1].ravel()
    r1 = Wd[0] * (A[0] @ m1 - d[0])
    r2 = Wd[1] * (A[1] @ m2 - d[1])
    l1, l2 = rrcg.gramian_ascent(m1, m2)
    grad = np.concatenate([2 * A[0].T @ (Wd[0] * r1) + 2 * alpha * m1 + 2 * lam * l1,
                           2 * A[1].T @ (Wd[1] * r2) + 2 * alpha * m2 + 2 * lam * l2])
    coupling = np.concatenate([2 * lam * l1, 2 * lam * l2])
    assert np.linalg.norm(grad) <= 0.1 * np.linalg.norm(coupling)
    assert rrcg.gramian(m1, m2) > 0


def test_bounds_hold_and_alpha_schedule(ops6):
    g = G6
    data, _ = _data(g, ops6, noise=1.0)
    prm = rrcg.Params(alpha0=(100.0, 100.0), q=(0.5, 0.8), alpha_min=(10.0, 0.0), lam=(1e-3, 1e-1),
                      lo=(0.0, 0.0), hi=(1.0, 0.1), restart=False)
    st = rrcg.initial_state(data, prm, (g.nz, g.nx, g.ny))
    thr = g.sx * g.sy + math.sqrt(2 * g.sx * g.sy)
    for _ in range(12):
        new, rec = rrcg.outer_step(ops6, data, prm, st, n_inner=1)
        assert new.m[0].min() >= 0.0 and new.m[0].max() <= 1.0
        assert new.m[1].min() >= 0.0 and new.m[1].max() <= 0.1
        assert rec["threshold"] == pytest.approx(thr)
        for i in range(2):
            if new.frozen[i]:
                assert new.alpha[i] == st.alpha[i]
            else:
                assert new.alpha[i] == max(prm.q[i] * st.alpha[i], prm.alpha_min[i])
            assert new.frozen[i] == (st.frozen[i] or rec["phi"][i] <= thr)
        st = new
    assert st.k == 12


def test_swap_symmetry(ops6):
    g = G6
    data, _ = _data(g, ops6, noise=1.0)
    prm = rrcg.Params(alpha0=(50.0, 20.0), q=(0.9, 0.8), lam=(1e-2, 3e-1), lo=(0.0, 0.0), hi=(1.0, 0.1))
    st, _ = rrcg.run(ops6, data, prm, n_outer=4, n_inner=3)
    sw = lambda x: [x[1], x[0]]
    data_s = rrcg.Data(dobs=sw(data.dobs), wd=sw(data.wd), wdepth=sw(data.wdepth))
    prm_s = rrcg.Params(alpha0=sw(prm.alpha0), q=sw(prm.q), lam=sw(prm.lam), lo=sw(prm.lo), hi=sw(prm.hi))
    st_s, _ = rrcg.run(sw(ops6), data_s, prm_s, n_outer=4, n_inner=3)
    assert np.array_equal(st.m[0], st_s.m[1]) and np.array_equal(st.m[1], st_s.m[0])


def test_standalone_equals_two_separate_inversions(ops6):
    # coupled=False with lambda = 0 runs two independent RRCGs (Sec. 3.1.1)
    g = G6
    data, _ = _data(g, ops6, noise=1.0)
    prm = rrcg.Params(alpha0=(50.0, 20.0), q=(0.9, 0.8), coupled=False, lo=(0.0, 0.0), hi=(1.0, 0.1))
    st, _ = rrcg.run(ops6, data, prm, n_outer=3, n_inner=4)
    # the same data set twice gives the same answer whatever the other one is
    data2 = rrcg.Data(dobs=[data.dobs[0], data.dobs[0]], wd=[data.wd[0], data.wd[0]],
                      wdepth=data.wdepth)
    prm2 = rrcg.Params(alpha0=(50.0, 50.0), q=(0.9, 0.9), coupled=False, lo=(0.0, 0.0), hi=(1.0, 1.0))
    st2, _ = rrcg.run([ops6[0], ops6[0]], data2, prm2, n_outer=3, n_inner=4)
    assert np.array_equal(st.m[0], st2.m[0]) and np.array_equal(st2.m[0], st2.m[1])


# ------------------------------------------------------------------------------------
# the Lagrange-parameter scan (Sec. 3.1.3, Sec. 5): similarity and the choice rule
# ------------------------------------------------------------------------------------
def test_similarity_closed_forms():
    r = np.random.default_rng(5)
    a = r.standard_normal((3, 4, 5))
    assert rrcg.similarity(a, a) == pytest.approx(1.0, abs=1e-15)
    assert rrcg.similarity(a, -3.0 * a) == pytest.approx(1.0, abs=1e-15)      # sign-blind
    e1, e2 = np.zeros(6), np.zeros(6)
    e1[1], e2[4] = 2.0, -5.0
    assert rrcg.similarity(e1, e2) == 0.0                                   # orthogonal
    assert rrcg.similarity(np.array([1.0, 0.0]), np.array([1.0, 1.0])) == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert rrcg.similarity(np.zeros(4), np.ones(4)) == 0.0
    # two directions 60 degrees apart in a plane of a larger space, scaled
    u = np.zeros(10)
    v = np.zeros(10)
    u[3], v[3], v[7] = 7.0, 0.5, 0.5 * math.sqrt(3.0)
    assert rrcg.similarity(u, v) == pytest.approx(0.5, rel=1e-15)


def test_lambda_choice_rule():
    rec = lambda c, s: dict(converged=c, similarity=s)
    runs = [rec(True, 0.5), rec(False, 0.95), rec(True, 0.91), rec(True, 0.99)]
    assert rrcg.select_lambda(runs, 0.9) == 2          # smallest pair that fits and is similar
    assert rrcg.select_lambda(runs, 0.995) is None     # none similar enough
    assert rrcg.select_lambda(runs, 0.4) == 0
    assert rrcg.select_lambda([rec(False, 1.0)], 0.0) is None   # a run stopped by the limit
    assert rrcg.select_lambda([], 0.5) is None


# ------------------------------------------------------------------------------------
# branches of RRCG:4-5 that the W = I pins above cannot tell apart
# ------------------------------------------------------------------------------------
def _half_grad_fd(f, a, b, h=1e-5):
    """Half the gradient of f(a, b) with respect to a and to b, by central differences
    (written out here, independent of the oracle's ascent directions)."""
    ga, gb = np.zeros(a.size), np.zeros(b.size)
    for j in range(a.size):
        e = np.zeros(a.size)
        e[j] = h
        e = e.reshape(a.shape)
        ga[j] = (f(a + e, b) - f(a - e, b)) / (4 * h)
        gb[j] = (f(a, b + e) - f(a, b - e)) / (4 * h)
    return ga, gb


def _gram_det(a, b):
    a, b = a.ravel(), b.ravel()
    return float(np.dot(a, a) * np.dot(b, b) - np.dot(a, b) ** 2)


@pytest.mark.parametrize("branch", ["original", "weighted"])
def test_gramian_branch_fixed_point_with_nonuniform_weights(ops6, branch):
    # With a non-uniform, fixed W (p = 2, depth weights in [0.5, 2]) the two Gramian readings
    # have different limits: RRCG:4 vanishes at the limit, with l_G the half-gradient of
    # S_G(m1, m2) at m = m~/W ("original", eqs. RRCG:2-3) or of S_G(m~1, m~2) ("weighted",
    # eqs. steepestascenta/b).  Both half-gradients are taken here by finite differences of
    # the Gramian determinant; the other branch's equation must be far from satisfied.
    g = G6
    r = np.random.default_rng(3)
    wdepth = [r.uniform(0.5, 2.0, (g.nz, g.nx, g.ny)) for _ in range(2)]
    data, _ = _data(g, ops6, noise=0.5, wdepth=wdepth)
    lam, alpha = (1e3, 3e2), (20.0, 5.0)
    prm = rrcg.Params(alpha0=alpha, q=(1.0, 1.0), lam=lam, p_norm=2, restart=True, gramian=branch)
    st = rrcg.initial_state(data, prm, (g.nz, g.nx, g.ny))
    for _ in range(300):
        st, _ = rrcg.outer_step(ops6, data, prm, st, n_inner=50)
    m = st.m
    mt = [wdepth[i] * m[i] for i in range(2)]
    base = []
    for i in range(2):
        A, W, wd = ops6[i].A, wdepth[i].ravel(), data.wd[i].ravel()
        rt = wd * (A @ m[i].ravel() - data.dobs[i].ravel())
        base.append((A.T @ (wd * rt)) / W + alpha[i] * mt[i].ravel())
    lg = {"weighted": _half_grad_fd(_gram_det, mt[0], mt[1]), "original": _half_grad_fd(_gram_det, m[0], m[1])}

    def residual(which):
        res = np.concatenate([base[i] + lam[i] * lg[which][i] for i in range(2)])
        coup = np.concatenate([lam[i] * lg[which][i] for i in range(2)])
        return np.linalg.norm(res) / np.linalg.norm(coup)
    other = "weighted" if branch == "original" else "original"
    assert residual(branch) <= 0.1
    assert residual(other) >= 0.5


def test_printed_single_loop_reaches_tikhonov_solution(ops6):
    # The printed iteration: one CG step per reweighting, beta carried over (RRCG:5 with
    # p_0 = l_0 only at the very start).  With lambda = 0, W fixed, q = 1 and no bounds it is
    # CG on (A~^T A~ + alpha I) m~ = A~^T d~ with the residual taken exactly every step, so
    # 3n steps reach the normal equations' solution (numpy.linalg.solve); the same number
    # of steps with beta reset every step (steepest descent) stays far from it.
    g = G6
    r = np.random.default_rng(2)
    wdepth = [r.uniform(0.5, 2.0, (g.nz, g.nx, g.ny)) for _ in range(2)]
    data, _ = _data(g, ops6, noise=1.0, wdepth=wdepth)
    alpha = (3.0, 0.5)
    ref = []
    for i in range(2):
        A, W = ops6[i].A, wdepth[i].ravel()
        At = np.diag(data.wd[i].ravel()) @ A @ np.diag(1.0 / W)
        mt = np.linalg.solve(At.T @ At + alpha[i] * np.eye(g.n), At.T @ (data.wd[i] * data.dobs[i]).ravel())
        ref.append(mt / W)
    err = {}
    for restart in (False, True):
        prm = rrcg.Params(alpha0=alpha, q=(1.0, 1.0), lam=(0.0, 0.0), p_norm=2, restart=restart)
        st, _ = rrcg.run(ops6, data, prm, n_outer=3 * g.n, n_inner=1)
        err[restart] = max(np.linalg.norm(st.m[i].ravel() - ref[i]) / np.linalg.norm(ref[i]) for i in range(2))
    assert err[False] <= 1e-8
    assert err[True] >= 1e-3


G81 = prism.Geometry(8, 8, 8, 8, 1, 50.0, 50.0, 50.0)   # one layer: a square, invertible system


@pytest.mark.parametrize("n_inner,restart", [(1, False), (5, True)])
def test_previous_iterate_anchor_limit_drops_the_regulariser(n_inner, restart):
    # RRCG:4 as printed, alpha (m~_k - m~_{k-1}): at a limit m~_k = m~_{k-1}, so the term
    # vanishes and the limit solves A~^T (A~ m~ - d~) = 0, i.e. A m = d for this square,
    # invertible system with exact data; the gradient-consistent anchor m~_apr = 0 converges
    # to the Tikhonov solution instead.
    g = G81
    ops = _ops(g)
    A = [ops[i].A for i in range(2)]
    r = np.random.default_rng(2)
    wdepth = [r.uniform(0.8, 1.25, (g.nz, g.nx, g.ny)) for _ in range(2)]
    rr = np.random.default_rng(0)
    m_true = [rr.uniform(0.0, 1.0, (g.nz, g.nx, g.ny)), rr.uniform(0.0, 0.05, (g.nz, g.nx, g.ny))]
    d = [ops[i].matvec(m_true[i]) for i in range(2)]
    # W_d scales each A~ to unit largest singular value, so that alpha = 0.3 matters
    wd = [np.full(d[i].shape, 1.0 / np.linalg.norm(A[i], 2)) for i in range(2)]
    data = rrcg.Data(dobs=d, wd=wd, wdepth=wdepth)
    exact = [np.linalg.solve(A[i], d[i].ravel()) for i in range(2)]
    steps = 200 if n_inner == 1 else 60
    res = {}
    for anchor in ("prev", "apr"):
        prm = rrcg.Params(alpha0=(0.3, 0.3), q=(1.0, 1.0), p_norm=2, restart=restart, anchor=anchor)
        st, _ = rrcg.run(ops, data, prm, n_outer=steps, n_inner=n_inner)
        res[anchor] = max(np.linalg.norm(st.m[i].ravel() - exact[i]) / np.linalg.norm(exact[i]) for i in range(2))
    assert res["prev"] <= 1e-10
    assert res["apr"] >= 0.1


def test_previous_iterate_anchor_first_step_and_state(ops6):
    # m_{-1} := m_0: the first CG step of a run has no anchor term, so from m_0 = 0 it equals
    # the step of the m~_apr = 0 anchor; the state then carries the start of its last CG step.
    g = G6
    data, _ = _data(g, ops6, noise=1.0)
    kw = dict(alpha0=(50.0, 20.0), q=(0.9, 0.8), lam=(1e-2, 3e-1), restart=True)
    st_p, _ = rrcg.run(ops6, data, rrcg.Params(anchor="prev", **kw), n_outer=1, n_inner=1)
    st_a, _ = rrcg.run(ops6, data, rrcg.Params(anchor="apr", **kw), n_outer=1, n_inner=1)
    for i in range(2):
        assert np.array_equal(st_p.m[i], st_a.m[i])
        assert np.array_equal(st_p.m_prev[i], np.zeros_like(st_p.m[i]))
    st2, _ = rrcg.outer_step(ops6, data, rrcg.Params(anchor="prev", **kw), st_p, n_inner=3)
    st3, _ = rrcg.outer_step(ops6, data, rrcg.Params(anchor="apr", **kw), st_p, n_inner=3)
    assert not np.array_equal(st2.m[0], st3.m[0])


@pytest.mark.parametrize("coupled", [True, False])
def test_zero_data_and_prior_stay_at_zero(ops6, coupled):
    # with zero data and a zero prior every reweighted objective (misfit, regulariser and
    # Gramian term, all non-negative) vanishes at m = 0, so the iteration must stay there:
    # the first gradient is zero, the direction is zero, and the step length of RRCG:6 (0/0)
    # is taken as 0
    g = G6
    data, _ = _data(g, ops6)
    zero = rrcg.Data(dobs=[np.zeros_like(d) for d in data.dobs], wd=data.wd, wdepth=data.wdepth)
    prm = rrcg.Params(alpha0=(50.0, 50.0), q=(0.9, 0.9), lam=(2.0, 100.0), lo=(0.0, 0.0), hi=(1.0, 0.1),
                      coupled=coupled, restart=True)
    st, recs = rrcg.run(ops6, zero, prm, n_outer=3, n_inner=4)
    assert all(np.array_equal(m, np.zeros_like(m)) for m in st.m)
    assert all(s == [0.0, 0.0] for rec in recs for s in rec["s"])
    assert recs[-1]["phi"] == [0.0, 0.0]
    assert rrcg.similarity(st.m[0], st.m[1]) == 0.0
