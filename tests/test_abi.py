"""C-ABI contract checks that need no GPU: the library loads, exports every function
include/sapmi.h declares, and rejects bad geometry on the host (no HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sapmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_hot_path_calls():
    names = _declared_functions()
    for n in ["apply_M", "apply_W1_block", "solve_full", "solve_blocks",
              "schwarz_boundary_force", "hmc_trajectory", "block_pf_force", "sap_create"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_0710_0066_amd as sap
    lib = ctypes.CDLL(sap.lib_path())
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version():
    import paper_0710_0066_amd as sap
    assert sap.sap_version() == 102


@pytest.mark.parametrize("L,l0,l0_sub,kappa,max_rhs,ok", [
    ((4, 4, 4, 4), 2, 0, 0.155, 1, True),
    ((48, 24, 24, 24), 4, 2, 0.158, 12, True),
    ((32, 16, 16, 16), 4, 2, 0.1575, 1, True),
    ((4, 4, 4, 5), 2, 0, 0.155, 1, False),      # odd extent
    ((6, 4, 4, 4), 2, 0, 0.155, 1, False),      # L0 not a multiple of 2*l0
    ((8, 4, 4, 4), 1, 0, 0.155, 1, False),      # l0 < 2
    ((16, 4, 4, 4), 4, 3, 0.155, 1, False),     # l0 not a multiple of 2*l0_sub
    ((16, 4, 4, 4), 4, 1, 0.155, 1, False),     # l0_sub < 2
    ((8, 4, 4, 4), 2, 0, float("nan"), 1, False),
    ((8, 4, 4, 4), 2, 0, 0.155, 0, False),      # max_rhs < 1
])
def test_geometry_validation_on_host(L, l0, l0_sub, kappa, max_rhs, ok):
    import paper_0710_0066_amd as sap
    rc = sap.sap_check_geom(L, l0, l0_sub, kappa, max_rhs)
    assert (rc == sap.SAP_OK) == ok
    if not ok:
        assert rc == sap.SAP_E_ARG


def test_create_rejects_bad_geometry_before_any_hip_call():
    import paper_0710_0066_amd as sap
    with pytest.raises(sap.SapError) as e:
        sap.Context((4, 4, 4, 5), 2, 0.155)
    assert e.value.code == sap.SAP_E_ARG
