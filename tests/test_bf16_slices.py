"""The three-slice bf16 split that the FP32 Gaussian tiles and the FP32 KRILL
sketch contract on the bf16 matrix cores, emulated bit by bit on the host:
x = h + m + l with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m), each
conversion rounding to nearest even.

Pinned here: the two remainders are exact in FP32 and the three slices hold
every normal FP32 value exactly; the three slice products the tiles drop
(m l, l m, l l) stay below 2^-24 |x||y|, and the six they keep are exact in
FP32 (at most 16 significant bits each).  Runs on the CPU.
"""
import numpy as np
import pytest


def bf16_rne(x):
    """FP32 array -> the nearest bf16 values (ties to even), as FP32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split3(x):
    x = np.asarray(x, dtype=np.float32)
    h = bf16_rne(x)
    r1 = (x - h).astype(np.float32)
    m = bf16_rne(r1)
    r2 = (r1 - m).astype(np.float32)
    l_ = bf16_rne(r2)
    return h, m, l_, r1, r2


def significant_bits(v):
    """Significand bits an FP64 value needs (0 for zero)."""
    v = np.abs(np.asarray(v, dtype=np.float64))
    out = np.zeros(v.shape, dtype=np.int64)
    nz = v > 0
    mant, _ = np.frexp(v[nz])
    bits = np.zeros(mant.shape, dtype=np.int64)
    m = mant.copy()
    for _ in range(60):
        frac = m != np.floor(m)
        bits += frac
        m = np.where(frac, m * 2, m)
    out[nz] = bits
    return out


def sample(n, lo=-60, hi=60, seed=0):
    g = np.random.default_rng(seed)
    mant = g.uniform(1.0, 2.0, n)
    exp = g.integers(lo, hi, n)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return (sign * mant * 2.0 ** exp).astype(np.float32)


def test_rne_matches_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even (1); 1 + 3 2^-8 rounds up
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0e38], dtype=np.float32)
    got = bf16_rne(x)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2.0 ** -6
    assert got[3] == -2.5
    assert np.isfinite(got[4])


def test_three_slices_hold_every_fp32_value_exactly():
    x = np.concatenate([sample(200_000), np.array([1.0, -1.0, 0.0, 1.0 + 2.0 ** -23],
                                                  dtype=np.float32)])
    h, m, l_, r1, r2 = split3(x)
    xd = x.astype(np.float64)
    # the remainders are exact: x - h and (x - h) - m computed in FP32 equal
    # the exact differences
    assert np.array_equal(r1.astype(np.float64), xd - h.astype(np.float64))
    assert np.array_equal(r2.astype(np.float64), r1.astype(np.float64) - m.astype(np.float64))
    # and the last slice takes the rest without rounding
    assert np.array_equal(h.astype(np.float64) + m.astype(np.float64) + l_.astype(np.float64), xd)
    # sizes: |m| <= 2^-8 |x|, |l| <= 2^-16 |x| (to within the halving of round to nearest)
    ax = np.abs(xd)
    assert np.all(np.abs(m.astype(np.float64)) <= 2.0 ** -8 * ax)
    assert np.all(np.abs(l_.astype(np.float64)) <= 2.0 ** -16 * ax)


@pytest.mark.parametrize("d", [8, 16, 32])
def test_dropped_products_below_fp32_rounding_and_kept_ones_exact(d):
    g = np.random.default_rng(d)
    n = 4000
    X = (g.standard_normal((n, d)) * np.exp(g.uniform(-3, 3, (n, 1)))).astype(np.float32)
    Y = (g.standard_normal((n, d)) * np.exp(g.uniform(-3, 3, (n, 1)))).astype(np.float32)
    hx, mx, lx, _, _ = split3(X)
    hy, my, ly, _, _ = split3(Y)
    f = lambda a: a.astype(np.float64)
    exact = np.sum(f(X) * f(Y), axis=1)
    kept = np.sum(f(hx) * f(hy) + f(hx) * f(my) + f(mx) * f(hy) + f(hx) * f(ly)
                  + f(lx) * f(hy) + f(mx) * f(my), axis=1)
    dropped_bound = np.sum(np.abs(f(X)) * np.abs(f(Y)), axis=1) * 2.0 ** -24
    assert np.all(np.abs(exact - kept) <= dropped_bound)
    # each kept product of two bf16 slices has at most 16 significant bits:
    # exact in FP32's 24
    for a, b in ((hx, hy), (hx, my), (mx, hy), (hx, ly), (lx, hy), (mx, my)):
        assert significant_bits(f(a) * f(b)).max() <= 16
