"""GPU BTTB sensitivity operators (Sec. 2.7.1) behind the C ABI.

Every product runs in the HIP library; this module only checks tensors and passes
pointers and the current HIP stream.  Device memory comes from PyTorch.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L

GRAVITY = L.BTTB_GRAVITY
MAGNETIC = L.BTTB_MAGNETIC
_DT = {torch.float64: L.BTTB_F64, torch.float32: L.BTTB_F32}


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _geometry(g) -> L.Geometry:
    get = (lambda k, d=None: g.get(k, d) if d is not None else g[k]) if isinstance(g, dict) else \
        (lambda k, d=None: getattr(g, k, d) if d is not None else getattr(g, k))
    return L.Geometry(int(get("sx")), int(get("sy")), int(get("nx")), int(get("ny")), int(get("nz")),
                      float(get("dx")), float(get("dy")), float(get("dz")), float(get("h")),
                      float(get("top")), float(get("incl")), float(get("decl")), float(get("field")),
                      int(get("ox", 0)), int(get("oy", 0)))


def prism_kernels(kind: int, geometry, device="cuda") -> torch.Tensor:
    """Kernel array T [nz][sx+nx-1][sy+ny-1] (FP64) of the gravity or magnetic operator,
    evaluated on the GPU from the closed-form prism responses (Sec. 2.1).  `geometry`
    has sx, sy, nx, ny, nz, dx, dy, dz, h, top, incl, decl, field and optionally the
    station offset ox, oy (station (p, q) above prism column (p + ox, q + oy); default 0)."""
    g = _geometry(geometry)
    dev = torch.device(device)
    out = torch.empty((g.nz, g.sx + g.nx - 1, g.sy + g.ny - 1), dtype=torch.float64, device=dev)
    L.check(L.lib().bttb_prism_kernels(int(kind), C.byref(g), _ptr(out), C.c_void_p(_stream(dev))),
            "bttb_prism_kernels")
    return out


class Operator:
    """y = A x and z = A^T r for one data set (gravity or magnetic) on one GPU.

    kernels: FP64 tensor [nz][sx+nx-1][sy+ny-1] (host or device), T_(r) of Sec. 2.7.1.
    stations: (sx, sy); the prism grid follows from the kernel array's shape.
    dtype: torch.float64 (plain FP64 path) or torch.float32 (FFTs and products in FP32,
    eigenvalues computed in FP64 and rounded).
    pad: "smooth" (the smallest 5-smooth multiple of 8 >= sx+nx-1, sy+ny-1), "pow2" (powers of two,
    at least 32; also pad_pow2=True) or "auto" (per axis the power of two or 5-smooth size of least
    estimated cost in the group kernels).
    full_eig: keep the complex eigenvalues of a symmetric operator (by default a plan stores only
    the real, x-even half of them when the operator is symmetric; info()["eig_real_even"]).
    """

    def __init__(self, kernels: torch.Tensor, stations: Sequence[int], dtype=torch.float64,
                 max_batch: int = 1, device="cuda", pad_pow2: bool = False, full_eig: bool = False,
                 pad: str = "smooth"):
        if dtype not in _DT:
            raise TypeError("dtype must be torch.float32 or torch.float64")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        k = torch.as_tensor(kernels).to(device=self.device, dtype=torch.float64).contiguous()
        if k.dim() != 3:
            raise ValueError("kernels must be [nz][sx+nx-1][sy+ny-1]")
        sx, sy = int(stations[0]), int(stations[1])
        nz, Lx, Ly = k.shape
        nx, ny = Lx - sx + 1, Ly - sy + 1
        if nx < 1 or ny < 1:
            raise ValueError("kernel array smaller than the station grid")
        self.sx, self.sy, self.nx, self.ny, self.nz = sx, sy, nx, ny, nz
        self.dtype = dtype
        self.max_batch = int(max_batch)
        self._plan = C.c_void_p()
        if pad not in ("smooth", "pow2", "auto"):
            raise ValueError("pad must be 'smooth', 'pow2' or 'auto'")
        pad = "pow2" if pad_pow2 else pad
        flags = (_DT[dtype] | {"smooth": 0, "pow2": L.BTTB_PAD_POW2, "auto": L.BTTB_PAD_AUTO}[pad]
                 | (L.BTTB_EIG_FULL if full_eig else 0))
        L.check(L.lib().bttb_setup(_ptr(k), sx, sy, nx, ny, nz, flags, self.max_batch,
                                   C.c_void_p(_stream(self.device)), C.byref(self._plan)), "bttb_setup")

    @classmethod
    def from_geometry(cls, kind: int, geometry, dtype=torch.float64, max_batch: int = 1, device="cuda",
                      pad_pow2: bool = False, full_eig: bool = False, pad: str = "smooth"):
        T = prism_kernels(kind, geometry, device)
        g = _geometry(geometry)
        return cls(T, (g.sx, g.sy), dtype=dtype, max_batch=max_batch, device=device, pad_pow2=pad_pow2,
                   full_eig=full_eig, pad=pad)

    # ------------------------------------------------------------------------------
    @property
    def plan(self) -> C.c_void_p:
        if not self._plan:
            raise RuntimeError("operator is closed")
        return self._plan

    @property
    def model_shape(self):
        return (self.nz, self.nx, self.ny)

    @property
    def data_shape(self):
        return (self.sx, self.sy)

    def info(self) -> dict:
        d = L.PlanDesc()
        L.check(L.lib().bttb_plan_info(self.plan, C.byref(d)), "bttb_plan_info")
        return {f: getattr(d, f) for f, _ in L.PlanDesc._fields_}

    def set_launch(self, col_fft_per_block: int = 0, row_fft_per_block: int = 0, layer_chunks: int = 0):
        L.check(L.lib().bttb_set_launch(self.plan, col_fft_per_block, row_fft_per_block, layer_chunks),
                "bttb_set_launch")

    def autotune(self, reps: int = 5) -> dict:
        """Time the products under every valid launch shape and keep the fastest (run it
        before creating a solver on this operator)."""
        r = L.TuneResult()
        L.check(L.lib().bttb_autotune(self.plan, int(reps), C.c_void_p(_stream(self.device)), C.byref(r)),
                "bttb_autotune")
        return {"us_per_pair": r.us_per_pair, "col_fft_per_block": r.shape[0], "row_fft_per_block": r.shape[1],
                "layer_chunks": r.shape[2], "tried": r.tried}

    def timing_enable(self, max_launches: int, repeat: int = 1) -> None:
        """Record HIP events around each product kernel (max_launches kernels), each kernel
        launched `repeat` times back to back between its events."""
        L.check(L.lib().bttb_timing_enable(self.plan, int(max_launches), int(repeat)), "bttb_timing_enable")

    def timing_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the last read; synchronises."""
        tot = (C.c_double * L.NKERNELS)()
        cnt = (C.c_int * L.NKERNELS)()
        L.check(L.lib().bttb_timing_read(self.plan, tot, cnt), "bttb_timing_read")
        return {L.KERNEL_NAMES[k]: (tot[k], cnt[k]) for k in range(L.NKERNELS)}

    def eigenvalues(self) -> torch.Tensor:
        """Copy of the eigenvalues, complex [nz][Py/2+1][Px], scaled by 1/(Px Py) (a real-even
        store expanded)."""
        info = self.info()
        K2 = info["Py"] // 2 + 1
        out = torch.empty(self.nz * K2 * info["Px"] * 2, dtype=self.dtype, device=self.device)
        L.check(L.lib().bttb_plan_eigenvalues(self.plan, _ptr(out), C.c_void_p(_stream(self.device))),
                "bttb_plan_eigenvalues")
        cplx = torch.complex128 if self.dtype == torch.float64 else torch.complex64
        return out.view(cplx).view(self.nz, K2, info["Px"])

    # ------------------------------------------------------------------------------
    def _check_vec(self, t: torch.Tensor, tail, name: str) -> int:
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype:
            raise TypeError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if tuple(t.shape[-len(tail):]) != tuple(tail):
            raise ValueError(f"{name} must end with shape {tuple(tail)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        b = 1
        for s in t.shape[:-len(tail)]:
            b *= int(s)
        return b

    def apply(self, op: int, x: torch.Tensor, winv: Optional[torch.Tensor] = None,
              wd: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        tin, tout = ((self.model_shape, self.data_shape) if op == L.BTTB_OP_FORWARD
                     else (self.data_shape, self.model_shape))
        batch = self._check_vec(x, tin, "input")
        if winv is not None:
            self._check_vec(winv, self.model_shape, "winv")
        if wd is not None:
            self._check_vec(wd, self.data_shape, "wd")
        lead = tuple(x.shape[:-len(tin)])
        if out is None:
            out = torch.empty(lead + tuple(tout), dtype=self.dtype, device=self.device)
        elif self._check_vec(out, tout, "out") != batch:
            raise ValueError("out batch does not match the input batch")
        nin = 1
        for s in tin:
            nin *= s
        nout = 1
        for s in tout:
            nout *= s
        if batch > 0:
            L.check(L.lib().bttb_apply(self.plan, op, batch, _ptr(x), nin, _ptr(out), nout, _ptr(winv),
                                       _ptr(wd), C.c_void_p(_stream(self.device))), "bttb_apply")
        return out

    def matvec(self, x, winv=None, wd=None, out=None):
        """A x (or W_d A (winv . x)); x [..., nz, nx, ny] -> [..., sx, sy]."""
        return self.apply(L.BTTB_OP_FORWARD, x, winv, wd, out)

    def rmatvec(self, r, winv=None, wd=None, out=None):
        """A^T r (or winv . A^T (W_d . r)); r [..., sx, sy] -> [..., nz, nx, ny]."""
        return self.apply(L.BTTB_OP_ADJOINT, r, winv, wd, out)

    def close(self):
        if self._plan:
            torch.cuda.synchronize(self.device)
            L.lib().bttb_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            if getattr(self, "_plan", None):
                L.lib().bttb_destroy(self._plan)
                self._plan = C.c_void_p()
        except Exception:
            pass


def _tune_dict(r) -> dict:
    return {"us_per_pair": r.us_per_pair, "model_row_threads": r.shape[0], "data_row_threads": r.shape[1],
            "col_threads": r.shape[2], "layer_chunks": r.shape[3], "tried": r.tried}


def pointer_array(tensors, device) -> torch.Tensor:
    """Device array of the tensors' addresses (int64), for the group entry points."""
    return torch.tensor([0 if t is None else t.data_ptr() for t in tensors], dtype=torch.int64, device=device)


class Group:
    """The products of many operators (e.g. gravity and magnetic of many inversions of
    uneven sizes) in one kernel launch per stage per transform size.  Members share one dtype,
    and each transform size is a power of two from 32 (Operator(..., pad_pow2=True)) or a
    5-smooth size up to 640 whose rows and columns fill at most half of it (the default padding
    of stations over prism centres); the operators must stay open."""

    def __init__(self, ops: Sequence[Operator]):
        ops = list(ops)
        if not ops:
            raise ValueError("empty group")
        self.ops = ops
        self.dtype = ops[0].dtype
        self.device = ops[0].device
        arr = (C.c_void_p * len(ops))(*[op.plan.value for op in ops])
        self._g = C.c_void_p()
        self._owned = True
        L.check(L.lib().bttb_group_create(arr, len(ops), C.c_void_p(_stream(self.device)), C.byref(self._g)),
                "bttb_group_create")

    @classmethod
    def view(cls, handle: C.c_void_p, ops: Sequence[Operator]) -> "Group":
        """Non-owning view of a group that a solver owns (for timing and inspection)."""
        g = cls.__new__(cls)
        g.ops = list(ops)
        g.dtype = g.ops[0].dtype
        g.device = g.ops[0].device
        g._g = handle
        g._owned = False
        return g

    @property
    def handle(self) -> C.c_void_p:
        if not self._g:
            raise RuntimeError("group is closed")
        return self._g

    def info(self) -> dict:
        d = L.GroupDesc()
        L.check(L.lib().bttb_group_info(self.handle, C.byref(d)), "bttb_group_info")
        return {"count": d.count, "model_row_threads": d.model_row_threads,
                "data_row_threads": d.data_row_threads, "col_threads": d.col_threads,
                "layer_chunks": d.layer_chunks, "blocks": list(d.blocks)}

    def set_launch(self, model_row_threads: int = 0, data_row_threads: int = 0, col_threads: int = 0,
                   layer_chunks: int = 0):
        L.check(L.lib().bttb_group_set_launch(self.handle, int(model_row_threads), int(data_row_threads),
                                              int(col_threads), int(layer_chunks),
                                              C.c_void_p(_stream(self.device))), "bttb_group_set_launch")

    def timing_enable(self, max_launches: int, repeat: int = 1) -> None:
        """Record HIP events around each stage launch (all members), each launched `repeat`
        times back to back between its events."""
        L.check(L.lib().bttb_group_timing_enable(self.handle, int(max_launches), int(repeat)),
                "bttb_group_timing_enable")

    def timing_read(self) -> dict:
        tot = (C.c_double * L.NKERNELS)()
        cnt = (C.c_int * L.NKERNELS)()
        L.check(L.lib().bttb_group_timing_read(self.handle, tot, cnt), "bttb_group_timing_read")
        return {L.KERNEL_NAMES[k]: (tot[k], cnt[k]) for k in range(L.NKERNELS)}

    def timing_list(self, cap: int = 4096) -> list:
        """[(kernel name, ms of one launch)] of the timed launches since the last read, in
        launch order; synchronises."""
        kid = (C.c_int * cap)()
        ms = (C.c_double * cap)()
        n = C.c_int()
        L.check(L.lib().bttb_group_timing_list(self.handle, int(cap), kid, ms, C.byref(n)), "bttb_group_timing_list")
        return [(L.KERNEL_NAMES[kid[k]], ms[k]) for k in range(n.value)]

    def autotune(self, reps: int = 5) -> dict:
        """Tune the threads per block of each stage and the layer chunks by timing."""
        r = L.TuneResult()
        L.check(L.lib().bttb_group_autotune(self.handle, int(reps), C.c_void_p(_stream(self.device)), C.byref(r)),
                "bttb_group_autotune")
        return _tune_dict(r)

    def apply_ptrs(self, op: int, ins: torch.Tensor, outs: torch.Tensor, winv: Optional[torch.Tensor] = None,
                   wd: Optional[torch.Tensor] = None) -> None:
        """Products with device pointer arrays: int64 tensors on the group's device holding one
        address per member (winv and wd entries may be 0).  The arrays' form is checked here; the
        addresses are not -- each must point to a contiguous vector of that member's dtype and
        shape (what `apply` checks before it calls this)."""
        n = len(self.ops)
        if op not in (L.BTTB_OP_FORWARD, L.BTTB_OP_ADJOINT):
            raise ValueError("op must be BTTB_OP_FORWARD or BTTB_OP_ADJOINT")
        for name, a in (("ins", ins), ("outs", outs), ("winv", winv), ("wd", wd)):
            if a is None:
                if name in ("ins", "outs"):
                    raise ValueError(f"{name}: a pointer array is required")
                continue
            if a.dtype != torch.int64 or a.numel() != n or a.device != self.device or not a.is_contiguous():
                raise ValueError(f"{name}: expected a contiguous int64 tensor of {n} addresses on {self.device}")
        L.check(L.lib().bttb_group_apply(self.handle, int(op), _ptr(ins), _ptr(outs), _ptr(winv), _ptr(wd),
                                         C.c_void_p(_stream(self.device))), "bttb_group_apply")

    def apply(self, op: int, xs: Sequence[torch.Tensor], winv=None, wd=None, outs=None):
        """Products of every member; xs, outs (optional) and the optional diagonals winv (model
        shape) and wd (data shape) hold one tensor per member (winv and wd entries may be None).
        Every tensor is checked here: the library receives bare device pointers."""
        n = len(self.ops)
        if op not in (L.BTTB_OP_FORWARD, L.BTTB_OP_ADJOINT):
            raise ValueError("op must be BTTB_OP_FORWARD or BTTB_OP_ADJOINT")
        fwd = op == L.BTTB_OP_FORWARD

        def check(vs, what, shape_of, nullable):
            if vs is None:
                return
            if len(vs) != n:
                raise ValueError(f"{what}: one tensor per member ({n}), got {len(vs)}")
            for o, v in zip(self.ops, vs):
                if v is None and nullable:
                    continue
                if v is None or o._check_vec(v, shape_of(o), what) != 1 or v.dim() != len(shape_of(o)):
                    raise ValueError(f"{what}: one {shape_of(o)} tensor per member")
        check(xs, "input", (lambda o: o.model_shape) if fwd else (lambda o: o.data_shape), False)
        check(outs, "out", (lambda o: o.data_shape) if fwd else (lambda o: o.model_shape), False)
        check(winv, "winv", lambda o: o.model_shape, True)
        check(wd, "wd", lambda o: o.data_shape, True)
        if outs is None:
            outs = [torch.empty(o.data_shape if fwd else o.model_shape, dtype=self.dtype, device=self.device)
                    for o in self.ops]
        keep = [pointer_array(xs, self.device), pointer_array(outs, self.device),
                pointer_array(winv, self.device) if winv is not None else None,
                pointer_array(wd, self.device) if wd is not None else None]
        self.apply_ptrs(op, *keep)
        return outs

    def matvec(self, xs, winv=None, wd=None):
        return self.apply(L.BTTB_OP_FORWARD, xs, winv, wd)

    def rmatvec(self, rs, winv=None, wd=None):
        return self.apply(L.BTTB_OP_ADJOINT, rs, winv, wd)

    def close(self):
        if self._g:
            if self._owned:
                L.lib().bttb_group_destroy(self._g)
            self._g = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
