"""CPU checks of the C ABI: the built library loads (no GPU needed to load
it) and exports every function that include/bemfmm.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bemfmm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(bem_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_calls():
    names = _declared()
    for need in ("bem_fmm_matvec", "bem_fmm_matvec_adjoint", "bem_gmres_solve",
                 "bem_plan_create", "bem_plan_destroy", "bem_last_error"):
        assert need in names


def test_library_loads_and_exports_every_declared_symbol():
    import torch  # noqa: F401  (HIP runtime first)
    from paper_1606_02383_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1606_02383_amd import build
        build.build()
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_1606_02383_amd as bem
    assert sorted(bem.EXPORTS) == _declared()
