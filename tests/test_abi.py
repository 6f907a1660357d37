"""The C ABI library loads and exports every function include/lp.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lu_factor", "lu_solve", "residual_check", "lu_workspace_bytes",
                     "lu_solve_ir", "lp_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2202_13995_amd as lp
    lib = ctypes.CDLL(lp.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    import paper_2202_13995_amd as lp
    assert set(declared_functions()) <= set(lp.SIGNATURES)


def test_host_only_queries():
    import paper_2202_13995_amd as lp
    assert lp.lib.lu_workspace_bytes(1024, 64, 0) > 0
    assert lp.lib.lu_workspace_bytes(-1, 64, 0) == 0
    assert lp.lib.lu_workspace_bytes(1024, 0, 0) == 0
    assert lp.lib.lu_workspace_bytes(1024, 64, 9) == 0
    assert lp.strerror(0) == "success"
    assert "workspace" in lp.strerror(-900)
    assert lp.lib.lp_version() >= 100


def test_argument_checks_without_device():
    # illegal arguments are rejected before anything touches the device
    import paper_2202_13995_amd as lp
    L = lp.lib
    assert L.lu_factor(-1, 64, 0, None, 1, None, None, None, 0, None) == -1
    assert L.lu_factor(10, 0, 0, None, 10, None, None, None, 0, None) == -2
    assert L.lu_factor(10, 8, 7, None, 10, None, None, None, 0, None) == -3
    assert L.lu_factor(10, 8, 0, None, 10, None, None, None, 0, None) == -4
    assert L.lu_solve(-1, 0, None, 1, None, None, None, 1, 1, None, None) == -1
    assert L.lu_solve(4, 5, None, 4, None, None, None, 1, 1, None, None) == -2
    assert L.residual_check(-1, None, 1, None, 1, None, 1, 1, None, None) == -1
    assert L.lp_gemm_update(0, -1, 1, 1, None, 1, None, 1, None, 1, None) == -2
    # packed bfloat16 / half update: precision and size limits, workspace first
    assert L.lp_gemm_update_packed(0, 1, 1, 1, None, 1, None, 1, None, 1, None, 0, None) == -1
    assert L.lp_gemm_update_packed(2, 1, 1, 1025, None, 1025, None, 1, None, 1, None, 0, None) == -4
    assert L.lp_gemm_packed_workspace_bytes(100, 100, 2000) == 0
    # padded to 256-row tiles and a power-of-two multiple of 64 in k (2 bytes each)
    assert L.lp_gemm_packed_workspace_bytes(300, 10, 96) == 512 * 128 * 2 + 256 * 128 * 2
