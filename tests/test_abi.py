"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/wcl.h declares, and reports errors without a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1011_3318_amd", "libwcl.so")
HEADER = os.path.join(ROOT, "include", "wcl.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wcl_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1011_3318_amd import build
        build.build()
    import torch  # noqa: F401  (same HIP runtime as on the GPU path)
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["wcl_init", "wcl_create_lattice", "wcl_upload_gauge", "wcl_compute_clover", "wcl_upload_clover",
                 "wcl_apply_D", "wcl_ras_precondition", "wcl_solve_nested_bicgstab", "wcl_solve_bicgstab_f64"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_no_device_reports_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib.wcl_init.argtypes = [C.c_int, C.c_uint64, C.POINTER(C.c_void_p)]
    lib.wcl_last_error.restype = C.c_char_p
    h = C.c_void_p()
    rc = lib.wcl_init(0, 0, C.byref(h))
    assert rc < 0 and not h.value
    assert lib.wcl_last_error()


def test_null_arguments_rejected(lib):
    lib.wcl_create_lattice.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    assert lib.wcl_create_lattice(None, None, None, None) == -1
    lib.wcl_spinor_bytes.restype = C.c_uint64
    lib.wcl_spinor_bytes.argtypes = [C.c_void_p, C.c_int, C.c_int]
    assert lib.wcl_spinor_bytes(None, 1, 1) == 0


def test_no_dot_instruction_in_inline_asm():
    """Device code issues no instruction through inline asm: the only asm
    statements are empty ones that pin a value in a register.  The compiler
    inserts the wait states the hardware needs between dependent instructions
    (a DOT result read by a different instruction, for one) only around the
    instructions it generates itself; an inline-asm v_dot2 scheduled next to
    its reader has produced wrong link products."""
    csrc = os.path.join(ROOT, "paper_1011_3318_amd", "csrc")
    bad = []
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".hip", ".h", ".cpp")):
            continue
        src = open(os.path.join(csrc, name)).read()
        for m in re.finditer(r"\basm\b\s*(?:volatile\s*)?\(\s*\"([^\"]*)\"", src):
            if m.group(1).strip():
                bad.append((name, src.count("\n", 0, m.start()) + 1))
    assert not bad, bad
