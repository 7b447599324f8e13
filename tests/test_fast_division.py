"""The FFT passes divide block-local indices by block-uniform divisors with
one 24-bit multiply and a shift (UDiv in paper_2203_02962_amd/csrc/fft.hip):
q = (x * M mod 2^32) >> 21 with M = ceil(2^21 / d).  The comment there
states it is exact whenever x d <= 2^21 and x M < 2^32; this checks that
claim for every divisor 1..1024 and every index below 4096 inside those
bounds (the passes use divisors up to 256 and indices below 4096), and that
the uses the passes make (index below 4096, divisor up to 256, quotient
below 32 beyond 2048) stay inside them."""
import numpy as np


def _udiv(x, d):
    M = ((1 << 21) + d - 1) // d
    return ((x * np.uint64(M)) & np.uint64(0xFFFFFFFF)) >> np.uint64(21), M


def test_exact_inside_the_stated_bounds():
    x = np.arange(4096, dtype=np.uint64)
    checked = 0
    for d in range(1, 1025):
        q, M = _udiv(x, d)
        ok = (x * np.uint64(d) <= (1 << 21)) & (x * np.uint64(M) < (1 << 32))
        assert np.array_equal(q[ok], (x // np.uint64(d))[ok]), d
        checked += int(ok.sum())
    assert checked > 3_000_000


def test_the_passes_stay_inside_the_bounds():
    for d in range(1, 257):
        M = ((1 << 21) + d - 1) // d
        # indices below 2048 for any divisor; up to 4096 only where the
        # quotient (rows of an x-pass block) stays below 32
        xmax = 2048 if 2048 // d >= 32 else min(4096, 32 * d)
        xs = np.arange(xmax, dtype=np.uint64)
        assert np.all(xs * np.uint64(d) <= (1 << 21))
        assert np.all(xs * np.uint64(M) < (1 << 32))
        q, _ = _udiv(xs, d)
        assert np.array_equal(q, xs // np.uint64(d))
