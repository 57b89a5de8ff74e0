"""The allocation-free product entry point (krr_kernel_matvec_noalloc)
against the workspace entry point (krr_kernel_matvec): the same kernels on
the same tile decomposition, so the outputs must agree bit for bit; two calls
in a row with the second smaller (the fixed scratch keeps the first call's
contents, which the second must not read), every precision and kernel, and a
product too large for the fixed scratch refused before any launch."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def B():
    from paper_2304_12465_amd import binding
    return binding


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


@pytest.mark.parametrize("kind,prec", [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1)])
def test_noalloc_matches_workspace_entry_point_twice(kind, prec):
    b = B()
    g = np.random.default_rng(50 + 3 * kind + prec)
    shapes = [(9000, 7000, 20, 3, 0.0), (1300, 1300, 7, 1, 0.4)]   # second call smaller
    for nr, nc, d, m, shift in shapes:
        Xr = g.standard_normal((nr, d))
        Xc = Xr if shift else g.standard_normal((nc, d))
        V = g.standard_normal((nc, m))
        Xr_t = T(Xr)
        Xc_t = Xr_t if shift else T(Xc)
        sigma = np.sqrt(d) * (1.0 if kind == 0 else 1.5)
        W_ws = b.kernel_matvec(kind, sigma, prec, Xr_t, Xc_t, T(V), shift=shift)
        W_na = b.kernel_matvec_noalloc(kind, sigma, prec, Xr_t, Xc_t, T(V), shift=shift)
        torch.cuda.synchronize()
        assert torch.equal(W_ws, W_na), (nr, nc, d, m)
        # and a spot check against the oracle's direct differences
        from oracle import kernels as OK
        rows = np.arange(0, nr, max(1, nr // 16))
        ref = OK.matvec(Xr[rows], Xc, V, kind, sigma) + (shift * V[rows] if shift else 0.0)
        scale = np.abs(OK.block(Xr[rows], Xc, kind, sigma)) @ np.abs(V) + abs(shift) * np.abs(V[rows] if shift else 0)
        tol = {0: 1e-13, 1: 3e-5, 2: 1e-3}[prec]
        assert np.all(np.abs(W_na.cpu().numpy()[rows] - ref) <= tol * scale + 1e-300)


def test_noalloc_refusal_returns_eworkspace():
    # a product whose layouts exceed the fixed scratch is refused from its
    # shapes alone, before any pointer is read or kernel launched (the
    # one-row tensors below are never dereferenced)
    b = B()
    assert b.kernel_matvec_ws(b.FP64, 2_000_000, 2_000_000, 32, 16) > (256 << 20)
    X = torch.zeros((1, 32), dtype=torch.float64, device=DEV)
    rc = b.lib().krr_kernel_matvec_noalloc(0, 1.0, 0, b._ptr(X), 2_000_000, b._ptr(X), 2_000_000,
                                           32, b._ptr(X), 16, 0.0, b._ptr(X), b._stream(DEV))
    assert rc == -2
    assert b"fixed scratch" in b.lib().krr_last_error()
