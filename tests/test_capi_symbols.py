"""The C-ABI library loads without a GPU and exports every function include/tcmi.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "tcmi.h")
LIB = os.path.join(ROOT, "paper_2302_07420_amd", "libtcmi.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("tc_create", "tc_set_cell", "tc_set_kmesh", "tc_set_grid", "tc_set_basis", "tc_set_jastrow",
                 "tc_load_orbitals", "tc_apply_all", "tc_energy", "tc_orbital_energies", "tc_energy_backward",
                 "tc_apply", "tc_scf", "tc_set_nspin", "tc_load_orbitals_spin"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_without_device_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    st = lib.tc_create(0, None, ctypes.byref(h))
    assert st == -6 and not h.value
