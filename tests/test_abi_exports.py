"""The HIP library loads and exports every entry point include/flix.h declares.

No compute call is made (this runs without a GPU).
"""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "flix.h")


def _declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^(?:int|const char\s*\*)\s*(flix_\w+)\s*\(", src, flags=re.M)))


def _lib_path():
    from paper_2604_16725_amd import build_lib
    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    return build_lib.LIB


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["flix_create", "flix_bulk_load", "flix_insert", "flix_delete",
                     "flix_lookup", "flix_successor", "flix_range", "flix_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads_without_gpu():
    _lib_path()
    from paper_2604_16725_amd import flix
    lib = flix.load_library()
    assert lib.flix_create is not None
    # argument validation happens on the host before any device work
    h = ctypes.c_void_p()
    cfg = flix.FlixConfig(48, 128, 16, 8, 1024, 0, 0, 0)  # bad key width
    assert lib.flix_create(ctypes.byref(cfg), None, ctypes.byref(h)) == flix.FLIX_EINVAL
    cfg = flix.FlixConfig(32, 100, 16, 8, 1024, 0, 0, 0)  # capacity not a power of 2
    assert lib.flix_create(ctypes.byref(cfg), None, ctypes.byref(h)) == flix.FLIX_EINVAL
    cfg = flix.FlixConfig(32, 128, 8, 8, 1024, 0, 0, 0)   # lanes not in {16,32,64}
    assert lib.flix_create(ctypes.byref(cfg), None, ctypes.byref(h)) == flix.FLIX_EINVAL
    assert lib.flix_insert(None, None, None, 5, None) == flix.FLIX_ESTATE


def test_no_oracle_on_product_path():
    """The product package never imports, loads or names the oracle."""
    pkg = os.path.join(ROOT, "paper_2604_16725_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), os.path.join(dirpath, f)
