"""The C-ABI library loads on the CPU and exports every entry point that
include/moto.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "moto.h")
LIB = os.path.join(ROOT, "paper_2509_26269_amd", "libmoto.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(moto_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = declared()
    for n in ["moto_energy_grad", "moto_tangent_hvp", "moto_min_modes", "moto_reflected_step", "moto_descend"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmoto.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmoto.so not built")
def test_host_only_entry_points_without_gpu():
    """Pure host logic: status strings and argument validation (no device)."""
    from paper_2509_26269_amd import moto as M

    L = M.lib()
    assert L.moto_status_string(0) == b"ok"
    assert b"workspace" in L.moto_status_string(-4)
    # a plan with no lattice is rejected before any device call
    h = M._Ham()
    h.Lx, h.Ly, h.n_shells = 0, 4, 1
    p = ctypes.c_void_p()
    assert L.moto_plan_create(ctypes.byref(h), ctypes.byref(p)) == -1
    # more shells than the table holds
    h.Lx, h.n_shells = 4, M.MAX_SHELLS + 1
    assert L.moto_plan_create(ctypes.byref(h), ctypes.byref(p)) == -1
    # DMI beyond the nearest-neighbour shell is outside the GPU scope
    h.n_shells = 2
    h.D[1] = 0.1
    assert L.moto_plan_create(ctypes.byref(h), ctypes.byref(p)) == -6
