"""SplitMix64 as a counter-based generator (oracle side).

Randomness in the method (RPCholesky pivot draws, Alg. 3; uniform centres,
Sec. 2.2; sparse sign embedding, Sec. 2.2.1) cannot be handed in as data
through the library boundary, so both the oracle and the GPU library
implement this one published generator independently.

Definition (Steele, Lea & Flood 2014): a SplitMix64 generator seeded with
``s`` returns, as its n-th output (n = 0, 1, ...), ``mix64(s + (n+1)*GAMMA)``
modulo 2**64, where ``mix64`` is the variant-13 finaliser below.  Random
access to the n-th output is what makes it counter-based.

Streams used by the method (tags are this library's convention):

* ``key(seed, tag) = sm(seed, tag)``;
* pivot draw t of RPCholesky block b: ``sm(sm(key(seed,1), b), t)``;
* centre key of point i: ``sm(key(seed,2), i)``;
* sparse-sign row candidate t of column j: ``sm(sm(key(seed,3), j), t)``;
* sparse-sign sign of nonzero q of column j: top bit of
  ``sm(sm(key(seed,4), j), q)`` (0 -> +1, 1 -> -1).

Conversions: ``u53(x) = (x >> 11) * 2**-53`` (an exact double in [0,1));
``below(x, n) = (x * n) >> 64`` (an integer in [0, n)).
"""
MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
TAG_PIVOT = 1
TAG_CENTER = 2
TAG_SKETCH_ROW = 3
TAG_SKETCH_SIGN = 4


def mix64(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def sm(seed: int, n: int) -> int:
    """n-th output (0-based) of SplitMix64 seeded with ``seed``."""
    return mix64((seed + (n + 1) * GAMMA) & MASK)


def key(seed: int, tag: int) -> int:
    return sm(seed & MASK, tag)


def u53(x: int) -> float:
    return (x >> 11) * (2.0 ** -53)


def below(x: int, n: int) -> int:
    return (x * n) >> 64


# Vectorised forms over numpy uint64 arrays (wrapping arithmetic mod 2**64).
import numpy as _np

_U = _np.uint64


def mix64_vec(z):
    z = _np.asarray(z, dtype=_np.uint64)
    z = (z ^ (z >> _U(30))) * _U(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> _U(27))) * _U(0x94D049BB133111EB)
    return z ^ (z >> _U(31))


def sm_vec(seed, n):
    """sm(seed, n) for an array of counters n (or an array of seeds)."""
    with _np.errstate(over="ignore"):
        seed = _np.asarray(seed, dtype=_np.uint64)
        n = _np.asarray(n, dtype=_np.uint64)
        return mix64_vec(seed + (n + _U(1)) * _U(GAMMA))
