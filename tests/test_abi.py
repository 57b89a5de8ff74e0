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


def test_krill_mixed_workspace_adds_fp32_sketch_layouts():
    """A MIXED KRILL build runs the FP64 build's restricted products with the
    sketch on FP32 tiles: its workspace is the FP64 one plus FP32 copies of X
    and of the centres (at most 64 padded FP32 coordinates and a few scalars
    per point, plus alignment)."""
    from paper_2304_12465_amd import binding as B
    N, d, k = 10000, 16, 100
    for kind in (B.GAUSSIAN, B.LAPLACE):
        w64 = B.krill_ws(kind, B.FP64, N, d, k)
        wm = B.krill_ws(kind, B.MIXED, N, d, k)
        assert w64 < wm <= w64 + 4 * (N + k) * (64 + 4) + 65536, (w64, wm)
