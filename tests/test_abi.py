"""The C-ABI library loads and exports every function include/gmacop.h
declares; argument checks that run before any device work return the
documented codes.  No GPU needed (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2010_14244_amd import gmacop
from workloads import grid8

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "gmacop.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(gmacop_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(gmacop.library_path()):
        pytest.fail("libgmacop.so is not built; run __graft_entry__.build()")
    return gmacop.lib()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("gmacop_graph_create", "gmacop_route_batch", "gmacop_release"):
        assert name in fns
    assert set(fns) == set(gmacop.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and offsets."""
    structs = {"gmacop_graph_desc": gmacop._Desc, "gmacop_od": gmacop._OD, "gmacop_params": gmacop._Params,
               "gmacop_result": gmacop._Result, "gmacop_stats": gmacop._Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gmacop.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_invalid_graph_rejected_before_device_work(L):
    w = grid8()
    g = w.graph
    bad_cols = g.col.copy()
    bad_cols[3] = g.n          # head out of range
    G = type(g)(**{**g.__dict__, "col": bad_cols})
    with pytest.raises(gmacop.GmacopError) as ei:
        gmacop.gmacop_graph_create(G)
    assert ei.value.code == gmacop.E_INVAL
    rp = g.row_ptr.copy()
    rp[-1] = g.m + 1
    G = type(g)(**{**g.__dict__, "row_ptr": rp})
    with pytest.raises(gmacop.GmacopError) as ei:
        gmacop.gmacop_graph_create(G)
    assert ei.value.code == gmacop.E_INVAL
    sp = g.speed_kmh.copy()
    sp[0] = 0
    G = type(g)(**{**g.__dict__, "speed_kmh": sp})
    with pytest.raises(gmacop.GmacopError) as ei:
        gmacop.gmacop_graph_create(G)
    assert ei.value.code == gmacop.E_INVAL
    assert b"speed" in L.gmacop_last_error()


def test_null_arguments(L):
    assert L.gmacop_graph_create(None, None) == gmacop.E_INVAL
    assert L.gmacop_route_batch(None, None, 0, None, None, None) == gmacop.E_INVAL
    L.gmacop_release(None)    # NULL-safe
    assert L.gmacop_state_get(None, None, None, None) == gmacop.E_INVAL


def test_kernel_machine_code_hash_of_the_built_library():
    """bench.py decides whether a profile's counters still hold from a hash
    of the kernel's gfx950 instructions in the built library: every walker
    kind is found, instantiations differ, and a missing kernel gives None."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    if not os.path.exists(os.path.join(bench.LLVM_BIN, "llvm-objdump")):
        pytest.skip("ROCm LLVM tools not installed")
    lib = gmacop.library_path()
    h42 = bench.kernel_isa_hash(lib, r"k_walk_glbILi4ELi2ELb0EE")
    h42t = bench.kernel_isa_hash(lib, r"k_walk_glbILi4ELi2ELb1EE")
    h41 = bench.kernel_isa_hash(lib, r"k_walk_glbILi4ELi1ELb0EE")
    hl = bench.kernel_isa_hash(lib, r"k_walk_ldsrILi4ELi1EEE")
    for h in (h42, h42t, h41, hl):
        assert h is not None and re.fullmatch(r"[0-9a-f]{16}", h)
    assert len({h42, h42t, h41, hl}) == 4
    assert bench.kernel_isa_hash(lib, r"no_such_kernel_name") is None
    assert bench.kernel_isa_hash(os.path.join(ROOT, "bench.py"), r"k_walk_glb") is None


def test_simulate_binding_checks_before_the_library():
    """gmacop_simulate's binding rejects malformed arrays itself (no device
    work, no graph needed)."""
    class NoGraph:
        handle = None
    p = grid8().params
    with pytest.raises(ValueError):
        gmacop.gmacop_simulate(NoGraph(), p, np.zeros(4, np.uint32), [1], [36])            # not [V, stride]
    with pytest.raises(ValueError):
        gmacop.gmacop_simulate(NoGraph(), p, np.zeros((2, 3), np.uint32), [1], [36, 36])   # lengths per vehicle
    with pytest.raises(ValueError):
        gmacop.gmacop_simulate(NoGraph(), p, np.zeros((2, 3), np.uint32), [1, 1], [36, 36], scen_off=[0, 1])
