"""The generic template decodes linear indices with the round-up
multiply-shift division of Granlund and Montgomery: for a divisor d >= 1 with
l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, every x < 2^31 has
x // d == (umulhi(x, m) + x) >> l.  Checked here over divisors and dividends
that cover the kernels' extents and index ranges."""
import random


def _magic(d):
    if d <= 1:
        return 1, 0
    l = (d - 1).bit_length()
    return ((1 << 32) * ((1 << l) - d)) // d + 1, l


def _div(x, m, l):
    return (((x * m) >> 32) + x) >> l


def test_multiply_shift_division_matches_integer_division():
    rng = random.Random(2601_12220)
    divisors = list(range(1, 130)) + [255, 256, 257, 1000, 4095, 4096, 1 << 20, (1 << 21) - 1,
                                      (1 << 30) + 3]
    for d in divisors:
        m, l = _magic(d)
        assert 0 < m < (1 << 32)
        xs = [0, 1, d - 1, d, d + 1, 2 * d - 1, (1 << 31) - 1, (1 << 31) - d]
        xs += [rng.randrange(0, 1 << 31) for _ in range(2000)]
        for x in xs:
            if 0 <= x < (1 << 31):
                assert _div(x, m, l) == x // d, (x, d)
