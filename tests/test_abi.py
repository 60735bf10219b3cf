"""The C ABI library loads and exports every declared symbol; host-side argument checks
(no GPU work is started by any call here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import __graft_entry__
    b = __graft_entry__._builder()
    if not b.is_built():
        b.build()
    from paper_2112_15562_amd import _lib
    return _lib


def declared_functions():
    with open(os.path.join(ROOT, "include", "bttb.h")) as f:
        text = f.read()
    return re.findall(r"BTTB_API\s+(?:int|const char\*)\s+(\w+)\s*\(", text)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    L = lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(lib.EXPORTED)


def test_strerror(lib):
    L = lib.lib()
    assert L.bttb_strerror(0) == b"ok"
    assert L.bttb_strerror(lib.BTTB_EINVAL) == b"invalid argument"
    assert L.bttb_strerror(lib.BTTB_ESIZE) == b"size out of range"
    assert L.bttb_strerror(12345) == b"unknown status"


def test_argument_checks_fail_before_any_gpu_work(lib):
    L = lib.lib()
    plan = C.c_void_p()
    # NULL kernels
    assert L.bttb_setup(None, 4, 4, 4, 4, 2, 0, 1, None, C.byref(plan)) == lib.BTTB_EINVAL
    assert b"kernels" in L.bttb_last_error()
    # NULL out
    assert L.bttb_setup(C.c_void_p(256), 4, 4, 4, 4, 2, 0, 1, None, None) == lib.BTTB_EINVAL
    # sizes < 1, bad precision, too large
    assert L.bttb_setup(C.c_void_p(256), 0, 4, 4, 4, 2, 0, 1, None, C.byref(plan)) == lib.BTTB_EINVAL
    assert L.bttb_setup(C.c_void_p(256), 4, 4, 4, 4, 2, 7, 1, None, C.byref(plan)) == lib.BTTB_EINVAL
    assert L.bttb_setup(C.c_void_p(256), 1500, 4, 1500, 4, 2, 0, 1, None, C.byref(plan)) == lib.BTTB_ESIZE
    # misaligned kernels pointer
    assert L.bttb_setup(C.c_void_p(257), 4, 4, 4, 4, 2, 0, 1, None, C.byref(plan)) == lib.BTTB_EINVAL
    # products on a NULL plan
    assert L.bttb_matvec(None, C.c_void_p(256), C.c_void_p(512), None) == lib.BTTB_EINVAL
    assert L.bttb_apply(None, 0, 1, C.c_void_p(256), 0, C.c_void_p(512), 0, None, None, None) == lib.BTTB_EINVAL
    assert L.bttb_set_launch(None, 1, 1, 1) == lib.BTTB_EINVAL
    # prism kernels: NULL geometry, bad kind, bad cell size
    g = lib.Geometry(4, 4, 4, 4, 2, 50.0, 50.0, 50.0, 1.0, 0.0, 65.0, 2.0, 5e4)
    assert L.bttb_prism_kernels(0, None, C.c_void_p(256), None) == lib.BTTB_EINVAL
    assert L.bttb_prism_kernels(5, C.byref(g), C.c_void_p(256), None) == lib.BTTB_EINVAL
    g.dz = 0.0
    assert L.bttb_prism_kernels(0, C.byref(g), C.c_void_p(256), None) == lib.BTTB_EINVAL
    # RRCG: NULL descriptor / plans
    h = C.c_void_p()
    assert L.rrcg_create(None, None, C.byref(h)) == lib.BTTB_EINVAL
    d = lib.RrcgDesc()
    assert L.rrcg_create(C.byref(d), None, C.byref(h)) == lib.BTTB_EINVAL
    assert L.rrcg_step(None, 1, None) == lib.BTTB_EINVAL
    assert L.bttb_destroy(None) == lib.BTTB_OK
    assert L.rrcg_destroy(None) == lib.BTTB_OK


def _c_layouts(structs):
    """sizeof and every field's offsetof of the header's structs, as gcc lays them out."""
    import json
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bttb.h"', 'int main(void) {', 'printf("{");']
    first = True
    for cname, fields in structs:
        for f in ["__size__"] + fields:
            expr = f"sizeof({cname})" if f == "__size__" else f"offsetof({cname}, {f})"
            sep = "" if first else ","
            lines.append(f'printf("{sep}\\"{cname}.{f}\\": %zu", (size_t)({expr}));')
            first = False
    lines += ['printf("}\\n");', 'return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "probe.c"), os.path.join(d, "probe")
        with open(src, "w") as fh:
            fh.write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        return json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)


def test_struct_layouts_match_header(lib):
    # every ctypes mirror has the size and field offsets the C compiler gives the header
    pairs = [("bttb_geometry", lib.Geometry), ("bttb_plan_desc", lib.PlanDesc), ("bttb_group_desc", lib.GroupDesc),
             ("bttb_tune_result", lib.TuneResult), ("rrcg_desc", lib.RrcgDesc), ("rrcg_scalars", lib.RrcgScalars)]
    cname = {"lambda_": "lambda"}
    structs = [(c, [cname.get(f, f) for f, _ in py._fields_]) for c, py in pairs]
    got = _c_layouts(structs)
    for c, py in pairs:
        assert C.sizeof(py) == got[f"{c}.__size__"], c
        for f, _ in py._fields_:
            assert getattr(py, f).offset == got[f"{c}.{cname.get(f, f)}"], (c, f)


def test_binding_rejects_unknown_solver_options(lib):
    # checked before any operator or device state is touched
    from paper_2112_15562_amd import rrcg
    for kw in ({"anchor": "previous"}, {"gramian": "weight"}):
        with pytest.raises(ValueError):
            rrcg._Inversion((None, None), [], [], [], **kw)


def test_checkpoint_shapes_are_checked_before_loading(lib):
    # a wrong-shaped or incomplete checkpoint is refused before any tensor is written
    import torch
    from paper_2112_15562_amd import rrcg
    s = rrcg.JointRRCG.__new__(rrcg.JointRRCG)
    s.m = [torch.zeros(2, 3, 4), torch.zeros(2, 3, 4)]
    s.p = [torch.zeros(2, 3, 4), torch.zeros(2, 3, 4)]
    s.mprev = None
    good = [torch.ones(2, 3, 4), torch.ones(2, 3, 4)]
    with pytest.raises(ValueError, match="shape"):
        s.load_state_dict(dict(m=good, p=[torch.ones(3, 4), torch.ones(2, 3, 4)], scalars={}))
    assert float(s.m[0].sum()) == 0.0
    s.mprev = [torch.zeros(2, 3, 4), torch.zeros(2, 3, 4)]
    with pytest.raises(ValueError, match="m_prev"):
        s.load_state_dict(dict(m=good, p=good, scalars={}))
