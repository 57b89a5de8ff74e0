"""The C ABI library loads on the CPU and exports every symbol the header
declares; argument validation happens before any GPU work."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "krr.h")


def header_symbols():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(krr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2304_12465_amd import binding
    L = binding.lib()
    syms = header_symbols()
    assert syms, "no declarations found"
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(binding.declared_symbols()) == syms


def test_validation_errors_without_gpu():
    from paper_2304_12465_amd import binding as B
    with pytest.raises(B.KrrError) as e:
        B.kernel_matvec_ws(B.FP64, 10, 10, 65, 1)
    assert e.value.code == -1
    with pytest.raises(B.KrrError):
        B.kernel_matvec_ws(B.FP64, -1, 10, 3, 1)
    with pytest.raises(B.KrrError):
        B.kernel_matvec_ws(B.FP64, 10, 10, 3, 0)
    assert B.kernel_matvec_ws(B.FP32, 1000, 1000, 20, 4) > 0


def test_krill_rejects_mixed_before_any_launch():
    """KRILL's sketch and restricted products have FP64 and FP32 tiles only:
    a MIXED request is refused by the size query and by the build, before
    anything touches the device (the build gets a dummy pointer it must not
    dereference)."""
    import ctypes
    from paper_2304_12465_amd import binding as B
    for kind in (B.GAUSSIAN, B.LAPLACE):
        with pytest.raises(B.KrrError) as e:
            B.krill_ws(kind, B.MIXED, 10000, 16, 100)
        assert e.value.code == -1
        assert B.krill_ws(kind, B.FP32, 10000, 16, 100) > 0
        out = ctypes.c_void_p(0)
        rc = B.lib().krr_krill_build(kind, 1.0, B.MIXED, ctypes.c_void_p(256), 10000, 16, 1.0,
                                     None, 100, 0, 0, 1, 1, ctypes.c_void_p(256), 1 << 30,
                                     ctypes.byref(out), None)
        assert rc == -1 and not out.value
        assert b"MIXED" in B.lib().krr_last_error()
