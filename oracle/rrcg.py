"""Joint RRCG with L1 reweighting and the Gramian constraint (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. 2.2-2.6 and 2.8 of the paper in its own notation:

* eq. (WL):     W_L1 = diag(((m - m_apr)^2 + eps^2)^(-1/4)), from the previous iterate.
* eq. (W):      W = W_depth W_hard W_L1.
* eq. (weighting): A~ = W_d A W^-1, m~ = W m, d~ = W_d d, m~_apr = W m_apr.
* eq. (Gramian): S_G = ||m1||^2 ||m2||^2 - (m1, m2)^2.
* eqs. (RRCG:1-8): residual, Gramian ascent directions in the original space,
  regularised gradient, Fletcher-Reeves direction, step length, update, back-transform.
* Sec. 2.5:     projection onto [lo, hi] at every outer iteration.
* eq. (chi2):   Phi_i = ||W_d (A m - d)||^2 <= m + sqrt(2m); eq. (regpara): alpha <- q alpha
  until the data set's chi^2 test is met, then alpha is frozen (Sec. 2.8).

Readings where the paper is silent or inconsistent (each listed in the design notes):
* RRCG:4 prints alpha (m~_k - m~_{k-1}); the gradient of eq. (GlobalFunction2) is
  alpha (m~ - m~_apr).  The default anchor is the gradient-consistent m~_apr;
  anchor="prev" takes the printed form, with m~_{k-1} read as W_k m_{k-1}: the model at
  the start of the previous CG step, in the current weighted space (m_{-1} := m_0, so the
  term vanishes at the first step).  Inside one reweighting W is fixed and the term is
  -alpha s_{k-1} p_{k-1}.
* The printed iteration is a single loop (one CG step per reweighting, beta carried
  over).  ``outer_step(n_inner=J)`` runs J CG steps at a frozen W, alpha, with the
  residual updated by the recurrence r~ <- r~ - s A~ p after the first, then the
  outer update (RRCG:8, bounds, chi^2, alpha).  J = 1 without restart is the printed
  loop; J > 1 with restart is the nested reading.
* l_G enters RRCG:4 without the W^-1 factor of eq. (descentrelaS), as the paper does.
* RRCG:6 block scalars: alpha-bar ||p-bar||^2 = sum_i alpha_i ||p_i||^2, same for lambda.
* "coupled=False" gives the stand-alone form (Sec. 3.1.1): beta and s per data set.
* gramian="weighted" uses the ascent directions of eqs. (steepestascenta/b) on m~.
* RRCG:6 with a zero denominator (p = 0, where (p, l) = 0 too) takes s = 0: the step's
  quadratic is at its minimum.

Pins (tests/test_oracle_rrcg.py): Gramian identities (S_G of collinear models is 0,
l_G vanishes there, S_G >= 0, finite-difference gradient = 2 l_G, the scalar-weight
relation S~_G = (w1 w2)^2 S_G); with lambda = 0, W fixed, no bounds, q = 1 one outer
step of n inner steps reaches (A~^T A~ + alpha I)^-1 A~^T d~ (normal equations solved
by numpy.linalg.solve); bounds hold after every outer step; exchanging the two data
sets exchanges the result; the objective decreases within an inner cycle (lambda = 0);
with non-uniform W the iteration's limit satisfies RRCG:4 with l_G the finite-difference
half-gradient of the Gramian on m (gramian="original") or on m~ ("weighted"), and not the
other; the printed single loop (beta carried over) reaches the Tikhonov solution in 3n
steps; the anchor="prev" limit solves the unregularised system (A m = d on a square one)
while the m~_apr anchor's is the Tikhonov solution; zero data with a zero prior, whose
objectives all vanish at m = 0, leave the iteration at m = 0 exactly.
Full multi-step trajectories are pinned only against these properties.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np


def dot(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.dot(np.ravel(a), np.ravel(b)))


def gramian(m1: np.ndarray, m2: np.ndarray) -> float:
    """S_G(m1, m2) = det [[(m1,m1),(m1,m2)],[(m2,m1),(m2,m2)]]  (eq. Gramian)."""
    return dot(m1, m1) * dot(m2, m2) - dot(m1, m2) ** 2


def gramian_ascent(u1: np.ndarray, u2: np.ndarray):
    """(l_G^(1), l_G^(2)) = (||u2||^2 u1 - (u1,u2) u2, ||u1||^2 u2 - (u1,u2) u1)
    (eqs. RRCG:2-3 on m, eqs. steepestascenta/b on m~); half of grad S_G."""
    g11 = dot(u1, u1)
    g22 = dot(u2, u2)
    g12 = dot(u1, u2)
    return g22 * u1 - g12 * u2, g11 * u2 - g12 * u1


def l1_weight(m: np.ndarray, m_apr: np.ndarray, eps2: float) -> np.ndarray:
    """Diagonal of W_L1 = ((m - m_apr)^2 + eps^2)^(-1/4)  (eq. WL)."""
    return 1.0 / ((m - m_apr) ** 2 + eps2) ** 0.25


@dataclass
class Params:
    alpha0: Sequence[float] = (20000.0, 20000.0)
    q: Sequence[float] = (0.95, 0.95)
    alpha_min: Sequence[float] = (0.0, 0.0)
    lam: Sequence[float] = (0.0, 0.0)
    eps2: float = 1e-9
    lo: Sequence[float] = (-math.inf, -math.inf)
    hi: Sequence[float] = (math.inf, math.inf)
    coupled: bool = True
    restart: bool = True
    p_norm: int = 1
    gramian: str = "original"
    anchor: str = "apr"


@dataclass
class Data:
    dobs: List[np.ndarray]
    wd: List[np.ndarray]                    # diagonal of W_d = 1/sigma, [sx][sy]
    wdepth: List[np.ndarray]                # [nz][nx][ny]
    whard: Optional[List[np.ndarray]] = None
    mapr: Optional[List[np.ndarray]] = None


@dataclass
class State:
    m: List[np.ndarray]                     # m_k in the original space
    p: List[np.ndarray]                     # previous search direction (weighted space)
    L_prev: List[float]                     # ||l^(i)||^2 of the previous CG step (0: none)
    alpha: List[float]
    frozen: List[bool] = field(default_factory=lambda: [False, False])
    k: int = 0
    m_prev: Optional[List[np.ndarray]] = None   # model at the start of the last CG step

    def copy(self) -> "State":
        mp = None if self.m_prev is None else [x.copy() for x in self.m_prev]
        return State([x.copy() for x in self.m], [x.copy() for x in self.p],
                     list(self.L_prev), list(self.alpha), list(self.frozen), self.k, mp)


def initial_state(data: Data, prm: Params, shape) -> State:
    """m_0 = m_apr, p = 0, no previous gradient, alpha = alpha_0, m_{-1} = m_0."""
    mapr = data.mapr or [np.zeros(shape), np.zeros(shape)]
    return State([mapr[0].copy(), mapr[1].copy()], [np.zeros(shape), np.zeros(shape)],
                 [0.0, 0.0], [float(prm.alpha0[0]), float(prm.alpha0[1])],
                 m_prev=[mapr[0].copy(), mapr[1].copy()])


def model_weight(i: int, m: np.ndarray, data: Data, prm: Params) -> np.ndarray:
    """Diagonal of W^(i) = W_depth W_hard W_L1 (eq. W) at the current iterate."""
    w = data.wdepth[i].copy()
    if data.whard is not None:
        w = w * data.whard[i]
    if prm.p_norm == 1:
        mapr = data.mapr[i] if data.mapr is not None else np.zeros_like(m)
        w = w * l1_weight(m, mapr, prm.eps2)
    return w


def outer_step(ops, data: Data, prm: Params, st: State, n_inner: int):
    """One reweighting step: n_inner CG steps at frozen W, alpha; then RRCG:8, bounds,
    chi^2 test and alpha schedule.  Returns (new state, record)."""
    A = ops
    W = [model_weight(i, st.m[i], data, prm) for i in range(2)]
    mapr = data.mapr or [np.zeros_like(st.m[0]), np.zeros_like(st.m[1])]
    mt = [W[i] * st.m[i] for i in range(2)]                    # m~ = W m
    mt_apr = [W[i] * mapr[i] for i in range(2)]                # m~_apr = W m_apr
    p = [st.p[0].copy(), st.p[1].copy()]
    L_prev = list(st.L_prev)
    m_prev = [x.copy() for x in (st.m_prev if st.m_prev is not None else st.m)]
    rt = None
    rec = dict(beta=[], s=[], L=[])
    for j in range(n_inner):
        m = [mt[i] / W[i] for i in range(2)]                   # RRCG:8 applied to m~
        if j == 0:                                             # RRCG:1, r~ = A~ m~ - d~
            rt = [data.wd[i] * (A[i].matvec(m[i]) - data.dobs[i]) for i in range(2)]
        u = m if prm.gramian == "original" else mt
        lG = gramian_ascent(u[0], u[1])                        # RRCG:2-3
        # RRCG:4: l = A~^T r~ + alpha (m~ - anchor) + lambda l_G, A~^T r~ = W^-1 A^T W_d r~
        anchor = mt_apr if prm.anchor == "apr" else [W[i] * m_prev[i] for i in range(2)]
        l = [A[i].rmatvec(data.wd[i] * rt[i]) / W[i]
             + st.alpha[i] * (mt[i] - anchor[i])
             + prm.lam[i] * lG[i] for i in range(2)]
        L = [dot(l[i], l[i]) for i in range(2)]
        restart_now = (j == 0 and prm.restart)
        if prm.coupled:                                        # RRCG:5, joint norms
            Lp = L_prev[0] + L_prev[1]
            b = 0.0 if (restart_now or Lp == 0.0) else (L[0] + L[1]) / Lp
            beta = [b, b]
        else:
            beta = [0.0 if (restart_now or L_prev[i] == 0.0) else L[i] / L_prev[i]
                    for i in range(2)]
        p = [l[i] + beta[i] * p[i] for i in range(2)]
        q = [data.wd[i] * A[i].matvec(p[i] / W[i]) for i in range(2)]   # A~ p
        num = [dot(p[i], l[i]) for i in range(2)]
        den = [dot(q[i], q[i]) + (st.alpha[i] + prm.lam[i]) * dot(p[i], p[i])
               for i in range(2)]
        # RRCG:6.  Reading: a zero denominator means p = 0 (for alpha + lambda > 0), where
        # (p, l) = 0 as well: the quadratic of this reweighting step is at its minimum, and the
        # step is 0 (the iterate stays), the usual end of a CG iteration.
        if prm.coupled:
            D = den[0] + den[1]
            s_ = 0.0 if D == 0.0 else (num[0] + num[1]) / D
            s = [s_, s_]
        else:
            s = [0.0 if den[i] == 0.0 else num[i] / den[i] for i in range(2)]
        m_prev = m                                             # start of this CG step
        mt = [mt[i] - s[i] * p[i] for i in range(2)]           # RRCG:7
        rt = [rt[i] - s[i] * q[i] for i in range(2)]
        L_prev = L
        rec["beta"].append(beta)
        rec["s"].append(s)
        rec["L"].append(L)
    m_new = [np.clip(mt[i] / W[i], prm.lo[i], prm.hi[i]) for i in range(2)]   # RRCG:8 + bounds
    r_new = [data.wd[i] * (A[i].matvec(m_new[i]) - data.dobs[i]) for i in range(2)]
    phi = [dot(r_new[i], r_new[i]) for i in range(2)]
    nd = data.dobs[0].size
    thr = nd + math.sqrt(2.0 * nd)                             # eq. chi2
    passed = [phi[i] <= thr for i in range(2)]
    frozen = [st.frozen[i] or passed[i] for i in range(2)]
    alpha = [st.alpha[i] if frozen[i] else max(prm.q[i] * st.alpha[i], prm.alpha_min[i])
             for i in range(2)]                                # eq. regpara
    new = State(m_new, p, L_prev, alpha, frozen, st.k + 1, m_prev)
    rec.update(phi=phi, threshold=thr, converged=all(passed), frozen=frozen,
               alpha_used=list(st.alpha), alpha_next=alpha,
               gramian=gramian(m_new[0], m_new[1]))
    return new, rec


def run(ops, data: Data, prm: Params, n_outer: int, n_inner: int,
        state: Optional[State] = None, stop_on_chi2: bool = False):
    """Run n_outer outer steps; returns (final state, list of records)."""
    st = state.copy() if state is not None else initial_state(data, prm, data.wdepth[0].shape)
    recs = []
    for _ in range(n_outer):
        st, rec = outer_step(ops, data, prm, st, n_inner)
        recs.append(rec)
        if stop_on_chi2 and rec["converged"]:
            break
    return st, recs


def similarity(m1: np.ndarray, m2: np.ndarray) -> float:
    """|(m1, m2)| / (||m1|| ||m2||): the cosine between the two models in the original space,
    the quantity the Gramian constraint drives to one (S_G = ||m1||^2 ||m2||^2 (1 - cos^2)).
    A single number standing for the paper's cross-correlation plots (reading: the plots are
    scatter plots of m1 against m2; aligned points give a cosine near one).  0 when a model
    is zero."""
    n1, n2 = dot(m1, m1), dot(m2, m2)
    if n1 == 0.0 or n2 == 0.0:
        return 0.0
    return abs(dot(m1, m2)) / math.sqrt(n1 * n2)


def select_lambda(records: Sequence[dict], sim_min: float) -> Optional[int]:
    """The Lagrange-parameter choice of Sec. 3.1.3 and Sec. 5 (conclusions): runs with fixed
    lambda, in increasing order; the first (smallest) pair whose run met both chi^2 tests
    (good predictions of both data sets; a run stopped by the iteration limit is rejected,
    as the paper rejects its non-converged large-lambda run) and whose models are similar
    (similarity >= sim_min).  None when no run qualifies."""
    for i, r in enumerate(records):
        if r["converged"] and r["similarity"] >= sim_min:
            return i
    return None


def lambda_scan(ops, data: Data, prm: Params, lams: Sequence, n_outer: int, n_inner: int,
                sim_min: float = 0.9) -> dict:
    """One run per lambda pair (stopped at the chi^2 test or after n_outer outer steps), each
    from the initial state; returns the per-run records and the selected index."""
    records = []
    for lam in lams:
        st, recs = run(ops, data, replace(prm, lam=(float(lam[0]), float(lam[1]))), n_outer, n_inner,
                       stop_on_chi2=True)
        records.append(dict(lam=(float(lam[0]), float(lam[1])), m=[st.m[0].copy(), st.m[1].copy()],
                            similarity=similarity(st.m[0], st.m[1]), converged=bool(recs[-1]["converged"]),
                            k=len(recs), phi=list(recs[-1]["phi"])))
    return dict(records=records, selected=select_lambda(records, sim_min))


def relative_error(m_exact: np.ndarray, m_rec: np.ndarray) -> float:
    """RE = ||m_exact - m_K|| / ||m_exact||  (eq. RE)."""
    return float(np.linalg.norm(np.ravel(m_exact - m_rec)) / np.linalg.norm(np.ravel(m_exact)))
