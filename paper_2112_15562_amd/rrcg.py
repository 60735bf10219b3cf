"""Joint RRCG solver (Sec. 2.4-2.8) behind the C ABI.

The solver state vectors m, p and the residual are PyTorch tensors owned here; every
step runs in the HIP library (rrcg_step) with all scalars kept on the device.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import torch

from . import _lib as L
from .operator import Group, Operator, _ptr, _stream


def _pair(v):
    if isinstance(v, (list, tuple)):
        return (float(v[0]), float(v[1]))
    return (float(v), float(v))


class _Inversion:
    """Device state and C description of one joint inversion (tensors owned here)."""

    def __init__(self, ops: Sequence[Operator], dobs, wd, wdepth, whard=None, mapr=None, *,
                 lo=-math.inf, hi=math.inf, alpha0=20000.0, q=0.95, alpha_min=0.0, lam=0.0,
                 eps2=1e-9, coupled=True, restart=True, p_norm=1, gramian="original", anchor="apr", m0=None,
                 use_graph=True):
        if anchor not in ("apr", "prev"):
            raise ValueError("anchor must be 'apr' or 'prev'")
        if gramian not in ("original", "weighted"):
            raise ValueError("gramian must be 'original' or 'weighted'")
        self.ops = tuple(ops)
        o = self.ops[0]
        self.dtype, self.device = o.dtype, o.device
        conv = lambda t: None if t is None else torch.as_tensor(t).to(self.device, self.dtype).contiguous()
        self.dobs = [conv(x) for x in dobs]
        self.wd = [conv(x) for x in wd]
        self.wdepth = [conv(x) for x in wdepth]
        self.whard = [conv(x) for x in whard] if whard is not None else [None, None]
        self.mapr = [conv(x) for x in mapr] if mapr is not None else [None, None]
        shape = o.model_shape
        if m0 is not None:
            self.m = [conv(x).clone() for x in m0]
        elif mapr is not None:
            self.m = [x.clone() for x in self.mapr]
        else:
            self.m = [torch.zeros(shape, dtype=self.dtype, device=self.device) for _ in range(2)]
        self.p = [torch.zeros(shape, dtype=self.dtype, device=self.device) for _ in range(2)]
        # previous-iterate anchor: the model at the start of the last CG step, m_{-1} = m_0
        self.mprev = [x.clone() for x in self.m] if anchor == "prev" else None
        self.resid = [torch.empty(o.data_shape, dtype=self.dtype, device=self.device) for _ in range(2)]
        for t in self.dobs + self.wd + self.resid:
            if tuple(t.shape) != tuple(o.data_shape):
                raise ValueError("data vectors must be [sx][sy]")
        for t in self.wdepth + [x for x in self.whard + self.mapr if x is not None] + self.m:
            if tuple(t.shape) != tuple(shape):
                raise ValueError("model vectors must be [nz][nx][ny]")
        d = L.RrcgDesc()
        for i in range(2):
            d.plan[i] = self.ops[i].plan.value
            d.m[i] = self.m[i].data_ptr()
            d.p[i] = self.p[i].data_ptr()
            d.resid[i] = self.resid[i].data_ptr()
            d.dobs[i] = self.dobs[i].data_ptr()
            d.wd[i] = self.wd[i].data_ptr()
            d.wdepth[i] = self.wdepth[i].data_ptr()
            d.whard[i] = self.whard[i].data_ptr() if self.whard[i] is not None else None
            d.mapr[i] = self.mapr[i].data_ptr() if self.mapr[i] is not None else None
        d.lo[:] = _pair(lo)
        d.hi[:] = _pair(hi)
        d.alpha0[:] = _pair(alpha0)
        d.q[:] = _pair(q)
        d.alpha_min[:] = _pair(alpha_min)
        d.lambda_[:] = _pair(lam)
        d.eps2 = float(eps2)
        d.coupled = int(bool(coupled))
        d.restart = int(bool(restart))
        d.p_norm = int(p_norm)
        d.gramian_weighted = 1 if gramian == "weighted" else 0
        d.use_graph = int(bool(use_graph))
        d.anchor = L.BTTB_ANCHOR_PREV if anchor == "prev" else L.BTTB_ANCHOR_APR
        for i in range(2):
            d.mprev[i] = self.mprev[i].data_ptr() if self.mprev is not None else None
        self.desc = d


def _scalars_dict(s: L.RrcgScalars) -> dict:
    return dict(alpha=list(s.alpha), L_prev=list(s.L_prev), phi=list(s.phi), threshold=s.threshold,
                beta=list(s.beta), step=list(s.step), gramian=s.gramian, frozen=[bool(x) for x in s.frozen],
                k=s.k, converged=bool(s.converged), nonfinite=bool(s.nonfinite), similarity=s.similarity)


def _apply_scalars(s: L.RrcgScalars, kw: dict) -> None:
    for k, v in kw.items():
        if k in ("alpha", "L_prev", "phi", "beta", "step"):
            getattr(s, k)[:] = [float(x) for x in v]
        elif k == "frozen":
            s.frozen[:] = [int(bool(x)) for x in v]
        elif k in ("k", "converged", "nonfinite"):
            setattr(s, k, int(v))
        elif k == "gramian":
            s.gramian = float(v)
        elif k == "similarity":
            pass  # computed on the device from the models
        else:
            raise KeyError(k)


class JointRRCG:
    """Joint gravity-magnetic inversion with L1 reweighting and the Gramian constraint.

    ops: (gravity operator, magnetic operator) with the same grids and dtype.
    dobs, wd: [sx][sy] tensors per data set (wd = 1/sigma); wdepth (and optional whard,
    mapr): [nz][nx][ny].  m0: starting models (default m_apr, or zeros).
    anchor: "apr" (alpha (m~ - W m_apr), the gradient of the objective) or "prev" (RRCG:4 as
    printed, alpha (m~ - W m_prev), m_prev the model at the start of the last CG step).
    """

    def __init__(self, ops: Sequence[Operator], dobs, wd, wdepth, whard=None, mapr=None, **kw):
        self._inv = _Inversion(ops, dobs, wd, wdepth, whard, mapr, **kw)
        inv = self._inv
        self.ops, self.dtype, self.device = inv.ops, inv.dtype, inv.device
        self.dobs, self.wd, self.wdepth, self.whard, self.mapr = inv.dobs, inv.wd, inv.wdepth, inv.whard, inv.mapr
        self.m, self.p, self.resid, self.mprev = inv.m, inv.p, inv.resid, inv.mprev
        self._h = C.c_void_p()
        L.check(L.lib().rrcg_create(C.byref(inv.desc), C.c_void_p(self._stream()), C.byref(self._h)),
                "rrcg_create")

    def _stream(self) -> int:
        return _stream(self.device)

    def prepare(self, n_inner: int) -> None:
        """Capture the graph of an outer step with n_inner CG steps ahead of its first use."""
        L.check(L.lib().rrcg_prepare(self._h, int(n_inner)), "rrcg_prepare")

    def autotune(self, reps: int = 3) -> dict:
        """Choose the launch shape of the solver's products by timing CG steps (plans that can
        join a product group); the solver state is restored afterwards."""
        from .operator import _tune_dict
        r = L.TuneResult()
        L.check(L.lib().rrcg_autotune(self._h, int(reps), C.c_void_p(self._stream()), C.byref(r)), "rrcg_autotune")
        return _tune_dict(r)

    def products(self) -> Optional[Group]:
        """The product group the solver runs on (plans that can join one), as a non-owning view
        valid while the solver is open; None for other plans."""
        g = C.c_void_p()
        if L.lib().rrcg_products(self._h, C.byref(g)) != L.BTTB_OK:
            return None
        return Group.view(g, self.ops)

    def step(self, n_inner: int = 1) -> None:
        """One outer step (asynchronous)."""
        L.check(L.lib().rrcg_step(self._h, int(n_inner), C.c_void_p(self._stream())), "rrcg_step")

    def scalars(self) -> dict:
        s = L.RrcgScalars()
        L.check(L.lib().rrcg_read_scalars(self._h, C.byref(s), C.c_void_p(self._stream())), "rrcg_read_scalars")
        return _scalars_dict(s)

    def set_scalars(self, **kw) -> None:
        s = L.RrcgScalars()
        L.check(L.lib().rrcg_read_scalars(self._h, C.byref(s), C.c_void_p(self._stream())), "rrcg_read_scalars")
        _apply_scalars(s, kw)
        L.check(L.lib().rrcg_write_scalars(self._h, C.byref(s), C.c_void_p(self._stream())), "rrcg_write_scalars")

    def refresh(self) -> None:
        L.check(L.lib().rrcg_refresh(self._h, C.c_void_p(self._stream())), "rrcg_refresh")

    def run(self, n_outer: int, n_inner: int = 1, stop_on_chi2: bool = False, log=None):
        """n_outer outer steps.  With stop_on_chi2 (or a log callback) the scalars are read
        once per outer step; otherwise the whole run is enqueued without host reads."""
        for _ in range(n_outer):
            self.step(n_inner)
            if stop_on_chi2 or log is not None:
                sc = self.scalars()
                if log is not None:
                    log(sc)
                if sc["nonfinite"]:
                    raise L.BTTBError(L.BTTB_ENAN, "JointRRCG.run", "non-finite value in a reduction")
                if stop_on_chi2 and sc["converged"]:
                    break
        return self.m

    def state_dict(self) -> dict:
        st = dict(m=[x.clone() for x in self.m], p=[x.clone() for x in self.p], scalars=self.scalars())
        if self.mprev is not None:
            st["mprev"] = [x.clone() for x in self.mprev]
        return st

    def load_state_dict(self, st: dict) -> None:
        if self.mprev is not None and "mprev" not in st:
            raise ValueError("the checkpoint has no m_prev: it comes from a solver with the prior-model anchor")
        keys = ("m", "p") + (("mprev",) if self.mprev is not None else ())
        for key in keys:
            for i in range(2):
                src, dst = st[key][i], getattr(self, key)[i]
                if tuple(src.shape) != tuple(dst.shape):  # copy_ would broadcast a smaller tensor
                    raise ValueError(f"checkpoint {key}[{i}] has shape {tuple(src.shape)}, expected {tuple(dst.shape)}")
        for i in range(2):
            self.m[i].copy_(st["m"][i])
            self.p[i].copy_(st["p"][i])
            if self.mprev is not None:
                self.mprev[i].copy_(st["mprev"][i])
        sc = dict(st["scalars"])
        sc.pop("threshold", None)
        self.set_scalars(**sc)
        self.refresh()
        # keep the recorded Phi / S_G of the checkpoint
        self.set_scalars(phi=st["scalars"]["phi"], gramian=st["scalars"]["gramian"])

    def close(self):
        if self._h:
            torch.cuda.synchronize(self.device)
            L.lib().rrcg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                L.lib().rrcg_destroy(self._h)
                self._h = C.c_void_p()
        except Exception:
            pass


class JointRRCGGroup:
    """Many joint inversions (up to 32, uneven sizes) stepped together: every phase of an
    outer step is one launch over all of them.  problems: sequence of dicts with the
    arguments of JointRRCG (ops, dobs, wd, wdepth and optionally whard, mapr and any solver
    parameter); `defaults` fills parameters a problem does not give.  The operators must be
    plans that can join a product group (see Group) of one dtype."""

    def __init__(self, problems, use_graph: bool = True, **defaults):
        self.inv = []
        for pr in problems:
            kw = dict(defaults)
            kw.update(pr)
            ops = kw.pop("ops")
            args = [kw.pop(k) for k in ("dobs", "wd", "wdepth")]
            whard, mapr = kw.pop("whard", None), kw.pop("mapr", None)
            kw["use_graph"] = use_graph
            self.inv.append(_Inversion(ops, *args, whard, mapr, **kw))
        if not self.inv:
            raise ValueError("no problems")
        self.device = self.inv[0].device
        arr = (L.RrcgDesc * len(self.inv))(*[v.desc for v in self.inv])
        self._h = C.c_void_p()
        L.check(L.lib().rrcg_group_create(arr, len(self.inv), C.c_void_p(self._stream()), C.byref(self._h)),
                "rrcg_group_create")

    def __len__(self):
        return len(self.inv)

    def _stream(self) -> int:
        return _stream(self.device)

    def m(self, i: int):
        return self.inv[i].m

    def prepare(self, n_inner: int) -> None:
        """Capture the graph of an outer step with n_inner CG steps ahead of its first use."""
        L.check(L.lib().rrcg_group_prepare(self._h, int(n_inner)), "rrcg_group_prepare")

    def step(self, n_inner: int = 1) -> None:
        """One outer step of every inversion (asynchronous)."""
        L.check(L.lib().rrcg_group_step(self._h, int(n_inner), C.c_void_p(self._stream())), "rrcg_group_step")

    def scalars(self, i: int) -> dict:
        s = L.RrcgScalars()
        L.check(L.lib().rrcg_group_read_scalars(self._h, int(i), C.byref(s), C.c_void_p(self._stream())),
                "rrcg_group_read_scalars")
        return _scalars_dict(s)

    def set_scalars(self, i: int, **kw) -> None:
        s = L.RrcgScalars()
        L.check(L.lib().rrcg_group_read_scalars(self._h, int(i), C.byref(s), C.c_void_p(self._stream())),
                "rrcg_group_read_scalars")
        _apply_scalars(s, kw)
        L.check(L.lib().rrcg_group_write_scalars(self._h, int(i), C.byref(s), C.c_void_p(self._stream())),
                "rrcg_group_write_scalars")

    def refresh(self) -> None:
        L.check(L.lib().rrcg_group_refresh(self._h, C.c_void_p(self._stream())), "rrcg_group_refresh")

    def set_launch(self, model_row_threads=0, data_row_threads=0, col_threads=0, layer_chunks=0) -> None:
        L.check(L.lib().rrcg_group_set_launch(self._h, int(model_row_threads), int(data_row_threads),
                                              int(col_threads), int(layer_chunks), C.c_void_p(self._stream())),
                "rrcg_group_set_launch")

    def autotune(self, reps: int = 3) -> dict:
        """Choose the launch shape of the group's products by timing CG steps; the solver
        state is restored afterwards and the graphs are recaptured."""
        from .operator import _tune_dict
        r = L.TuneResult()
        L.check(L.lib().rrcg_group_autotune(self._h, int(reps), C.c_void_p(self._stream()), C.byref(r)),
                "rrcg_group_autotune")
        return _tune_dict(r)

    def products(self) -> Group:
        """The solver's product group as a non-owning view (valid while the solver is open)."""
        g = C.c_void_p()
        L.check(L.lib().rrcg_group_products(self._h, C.byref(g)), "rrcg_group_products")
        return Group.view(g, [op for v in self.inv for op in v.ops])

    def launch_info(self) -> dict:
        return self.products().info()

    def close(self):
        if self._h:
            torch.cuda.synchronize(self.device)
            L.lib().rrcg_group_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
