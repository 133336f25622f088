"""The C ABI library loads on the CPU host and exports every entry point include/iga.h declares
(no compute calls: those need a GPU)."""
import ctypes
import os
import re

import paper_1305_4452_amd as iga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "iga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:iga|igann)_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["iga_create", "iga_destroy", "iga_assemble_residual", "iga_assemble_jacobian", "iga_apply",
              "iga_newton_solve", "iga_csr_pattern", "iga_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(iga.LIB_PATH):
        from paper_1305_4452_amd import build
        build.build()
    lib = ctypes.CDLL(iga.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(iga.exported_symbols()) == declared_functions()


def test_struct_layouts_match_header_sizes():
    # iga_desc: 4 + 12 + 12 (+4 pad) + 24 + 8 + 8 + 12 (+4) + 8 + 4 (+4) + 8 + 8 + 4 + 12 (+4) = 136 bytes
    assert ctypes.sizeof(iga.iga_desc) == 136
    assert ctypes.sizeof(iga.iga_newton_opts) == 48


def test_binding_constants_match_header_enums():
    """Every enumerator the header defines (status codes, precisions, kappa modes, Jacobian algorithms,
    options, preconditioners) has the same value in the Python binding."""
    src = open(os.path.join(ROOT, "include", "iga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    enums = re.findall(r"typedef enum\s*\{(.*?)\}", src, flags=re.S)
    values = {}
    for body in enums:
        for name, val in re.findall(r"\b(IGA_[A-Z0-9_]+)\s*=\s*(\d+)", body):
            values[name] = int(val)
    assert len(values) >= 30 and "IGA_OPT_FDM_KERNEL" in values and "IGA_OPT_RES_ZRUN" in values
    for name, val in values.items():
        assert getattr(iga, name) == val, name
