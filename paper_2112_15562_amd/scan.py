"""Choice of the Lagrange parameters by a scan over fixed pairs (Sec. 2.8, Sec. 3.1.3, Sec. 5).

The paper keeps lambda^(1), lambda^(2) fixed during a run and chooses them by running the
joint inversion for increasing pairs: the first (smallest) pair whose run fits both data
sets at the noise level and whose models are similar is kept.  Here every pair of a scan
is one inversion of a JointRRCGGroup, so all the runs advance together, one launch per
phase for all of them.

Readings (the paper shows similarity only as cross-correlation plots):
* similarity is |(m1, m2)| / (||m1|| ||m2||), the cosine in the original space that the
  Gramian drives to one (S_G = ||m1||^2 ||m2||^2 (1 - cos^2)), computed on the device with the
  Gramian after every outer step (the solver's scalars); a pair qualifies when it reaches
  ``sim_min``;
* a run fits when it met both chi^2 tests (eq. chi2) within ``n_outer`` outer steps; a run
  stopped by the limit is rejected, as the paper rejects its non-converged run with the
  largest pair;
* each run is recorded at the outer step where it met both tests (the group keeps stepping
  the others).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from .operator import Operator
from .rrcg import JointRRCGGroup

MAX_GROUP = 32  # inversions per group solver


def choose(records: Sequence[dict], sim_min: float) -> Optional[int]:
    """Index of the first record (in scan order) that fits both data sets and reaches
    sim_min, else None."""
    return next((i for i, r in enumerate(records) if r["converged"] and r["similarity"] >= sim_min), None)


def lambda_scan(kernels, data_shape, dobs, wd, wdepth, lams, *, n_outer: int, n_inner: int = 1,
                sim_min: float = 0.9, dtype=torch.float32, whard=None, mapr=None, use_graph: bool = True,
                **solver) -> dict:
    """Run one joint inversion per (lambda^(1), lambda^(2)) pair of ``lams`` (in increasing
    order) and choose the pair.

    kernels: the gravity and magnetic kernel arrays [nz][sx+nx-1][sy+ny-1] (FP64, host or
    device), data_shape (sx, sy); dobs, wd, wdepth (and optional whard, mapr): per data set,
    as JointRRCG takes them; ``solver``: the other JointRRCG parameters, shared by the runs.
    Each run gets its own operator plans (a plan holds its products' intermediates).

    Returns {"records": [{"lam", "similarity", "converged", "k", "phi", "m"}...],
    "selected": index or None}; "m" holds the run's two models (device tensors).
    """
    lams = [(float(l[0]), float(l[1])) for l in lams]
    dev = torch.device("cuda")
    ktens = [torch.as_tensor(k, dtype=torch.float64).to(dev) for k in kernels]
    records = []
    for c0 in range(0, len(lams), MAX_GROUP):
        part = lams[c0:c0 + MAX_GROUP]
        ops_all = [[Operator(ktens[i], tuple(data_shape), dtype=dtype) for i in range(2)]
                   for _ in part]
        probs = [dict(ops=ops, dobs=dobs, wd=wd, wdepth=wdepth, whard=whard, mapr=mapr, lam=lam)
                 for ops, lam in zip(ops_all, part)]
        grp = JointRRCGGroup(probs, use_graph=use_graph, **solver)
        done = [None] * len(part)
        try:
            for _ in range(n_outer):
                grp.step(n_inner)
                for i in range(len(part)):
                    if done[i] is None:
                        sc = grp.scalars(i)
                        if sc["converged"]:
                            done[i] = (sc, [t.clone() for t in grp.m(i)])
                if all(d is not None for d in done):
                    break
            for i, lam in enumerate(part):
                sc, m = done[i] if done[i] is not None else (grp.scalars(i), [t.clone() for t in grp.m(i)])
                records.append(dict(lam=lam, similarity=sc["similarity"], converged=bool(sc["converged"]),
                                    k=int(sc["k"]), phi=list(sc["phi"]), m=m))
        finally:
            grp.close()
            for ops in ops_all:
                for op in ops:
                    op.close()
    return dict(records=records, selected=choose(records, sim_min))
