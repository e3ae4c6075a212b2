"""The C-ABI library loads and exports every symbol include/femcg.h declares,
and the binding's argument lists have the header's parameter counts (no
compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "femcg.h")
LIB = os.path.join(ROOT, "paper_2201_05413_amd", "libfemcg.so")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["fem_assemble", "pcg_solve", "pcg_stats", "fem_rhs", "fem_free", "fem_last_error",
                 "pcg_solve_batch", "serve_submit"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2201_05413_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_export():
    from paper_2201_05413_amd import femcg
    assert sorted(femcg.EXPORTS) == declared_functions()


def test_last_error_is_empty_string_without_gpu_work():
    lib = ctypes.CDLL(LIB)
    lib.fem_last_error.restype = ctypes.c_char_p
    assert lib.fem_last_error() is not None


def declared_signatures():
    """name -> number of parameters, from the prototypes in the header."""
    txt = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(([^;{]*?)\)\s*;",
                         txt, flags=re.M | re.S):
        params = " ".join(m.group(2).split())
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argument_lists_match_the_header():
    from paper_2201_05413_amd import femcg
    L = femcg.lib()
    sigs = declared_signatures()
    assert sorted(sigs) == declared_functions()
    bad = {n: (k, len(getattr(L, n).argtypes or [])) for n, k in sigs.items()
           if len(getattr(L, n).argtypes or []) != k}
    assert not bad, bad  # name: (header, binding)
