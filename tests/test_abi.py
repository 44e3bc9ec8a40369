"""The C-ABI library builds, loads without a GPU, and exports every symbol
declared in include/*.h (no compute calls here)."""
import ctypes
import glob
import os
import re

from paper_2509_22857_amd import ckks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(ckc_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(ckks.LIB_PATH), "run __graft_entry__.build() first"
    lib = ctypes.CDLL(ckks.LIB_PATH)
    declared = declared_functions()
    assert len(declared) >= 20
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    declared = declared_functions()
    assert declared <= set(ckks.exported_names()) | set(getattr(ckks, "EXTRA_NAMES", []))


def test_last_error_callable_without_gpu():
    lib = ckks.lib()
    assert lib.ckc_last_error() is not None


def test_test_fault_hook_argument_checks_without_gpu():
    """The fault hook only sets host-side state: a non-negative code or a
    negative index is refused, index 0 disarms."""
    import pytest
    with pytest.raises(ckks.CkcError, match="CKC_EINVAL"):
        ckks.set_test_fault(1, 5)
    with pytest.raises(ckks.CkcError, match="CKC_EINVAL"):
        ckks.set_test_fault(-1, -6)
    ckks.set_test_fault(0, 0)


def test_variant_counter_without_gpu():
    """The per-instantiation launch counter is host-side state: enabling it
    clears it, an unknown name counts zero, and the list parses."""
    ckks.variant_enable(True)
    try:
        assert ckks.variant_counts() == {}
        n = ctypes.c_int64(-1)
        assert ckks.lib().ckc_variant_count(b"conv_mac<8,4>+dbuf", ctypes.byref(n)) == 0
        assert n.value == 0
    finally:
        ckks.variant_enable(False)
