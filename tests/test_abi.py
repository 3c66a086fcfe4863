"""The C-ABI library loads and exports every symbol its header declares (CPU)."""
import ctypes
import os
import re

from paper_2603_28648_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(dmrg_[a-z_0-9]+)\s*\(", txt))
    return names


def test_header_declares_the_four_calls():
    names = declared_symbols()
    for n in ("dmrg_build_ops", "dmrg_sigma", "dmrg_create", "dmrg_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_binding.LIB_PATH)
    missing = [n for n in sorted(declared_symbols()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert declared_symbols() <= set(_binding.EXPORTS)


def test_no_device_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        return
    lib = _binding.load_library()
    h = ctypes.c_void_p()
    st = lib.dmrg_create(ctypes.byref(h), 0, None)
    assert st == -5  # DMRG_ERR_NO_DEVICE
    assert b"device" in lib.dmrg_last_error(None).lower()


def test_binding_calls_every_export():
    """Each exported call has a binding that uses it (argument marshalling
    for tests and the benchmark), so none is declared but unreachable."""
    import inspect
    src = inspect.getsource(_binding)
    unused = [n for n in _binding.EXPORTS if f"lib.{n}(" not in src]
    assert not unused, unused
