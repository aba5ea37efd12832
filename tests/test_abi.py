"""The C-ABI library loads and exports every symbol include/resolvent.h declares (CPU only, no compute calls)."""
import ctypes
import os
import re

from paper_2008_10904_amd import _lib

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "resolvent.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(resolvent_\w+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.SIGNATURES)


def test_library_loads_and_exports_every_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu():
    lib = _lib.load()
    assert lib.resolvent_strerror(_lib.RES_EGRID).decode().startswith("frequency grid")
    assert lib.resolvent_strerror(_lib.RES_OK).decode() == "success"


def test_struct_layouts_match_header_sizes():
    # offsets follow the C layout of the header (x86-64 SysV)
    assert ctypes.sizeof(_lib.Grid) == 24
    assert ctypes.sizeof(_lib.Run) == 32
    assert _lib.OpDesc.h.offset == 8 and _lib.OpDesc.inst_offsets.offset == 24
