"""The exact float32 FMA emulation used to re-check GPU bins (CPU only)."""
from fractions import Fraction

import numpy as np

from _gpu_common import bins_fp32, fma32


def _exact(a, b, c):
    x = Fraction(float(np.float32(a))) * Fraction(float(np.float32(b))) + Fraction(float(np.float32(c)))
    lo = np.float32(float(x))
    best = None
    for cnd in (lo, np.nextafter(lo, np.float32(np.inf)), np.nextafter(lo, np.float32(-np.inf))):
        d = abs(Fraction(float(cnd)) - x)
        key = (d, int(np.asarray(cnd).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cnd)
    return best[1]


def test_fma32_matches_exact_rational_rounding():
    rng = np.random.default_rng(0)
    a = rng.normal(size=3000).astype(np.float32)
    b = rng.normal(size=3000).astype(np.float32)
    c = (-(a.astype(np.float64) * b) + rng.normal(size=3000) * 1e-6).astype(np.float32)  # heavy cancellation
    got = fma32(a, b, c)
    ref = np.array([_exact(x, y, z) for x, y, z in zip(a, b, c)], np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_fma32_differs_from_two_roundings_on_a_crafted_case():
    # a*b = 1 + 2^-24 + 2^-48 exactly; c = 0: single rounding goes up (above the tie),
    # while rounding a*b to float32 first and adding gives 1.0
    a = np.float32(1 + 2 ** -23)
    b = np.float32(1 + 2 ** -24) if np.float32(1 + 2 ** -24) != 1 else np.float32(1 + 2 ** -23)
    got = fma32([a], [b], [np.float32(0)])[0]
    assert got == _exact(a, b, 0.0)


def test_bins_rule_lowest_k_on_ties():
    dirs = np.array([[1, 0, 1], [0, 1, 0], [0, 0, 0]], np.float32)  # d0 == d2
    n = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]], np.float32)
    assert bins_fp32(n, dirs).tolist() == [0, 1]
