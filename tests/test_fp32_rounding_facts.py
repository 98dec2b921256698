"""Facts about FP32 rounding of roots of unity that the FP32 transforms are designed
around (no GPU involved): rounded to FP32, the twiddles of the first twiddled FFT
stage (the 64th roots for radix 8 x 8, the 48th for 12 x 4) are biased low in squared
modulus by about a third of a unit roundoff on average, so every uncompensated
transform shrinks the energy and a long run drifts linearly; a second FP32 part
(the rounded remainder) represents each twiddle to about the square of the unit
roundoff, which removes the bias when the product is formed with both parts."""
import numpy as np

U32 = 2.0 ** -24


def roots(n):
    a = 2 * np.pi * np.arange(n) / n
    return np.cos(a), -np.sin(a)


def stage_pairs(n, r0, r1):
    # twiddle indices of the first twiddled stage of an r0 x r1 pass: exp(-2 pi i j r / n)
    # for j < r0, r < r1 (n = r0 r1)
    return [(j * r) % n for j in range(r0) for r in range(r1)]


def test_first_stage_twiddles_are_biased_low_in_fp32():
    for n, r0, r1 in ((64, 8, 8), (48, 12, 4)):
        c, s = roots(n)
        ch, sh = c.astype(np.float32).astype(float), s.astype(np.float32).astype(float)
        m = (ch ** 2 + sh ** 2 - 1.0)[stage_pairs(n, r0, r1)]
        assert m.mean() < -0.3 * U32, (n, m.mean() / U32)
        assert np.abs(m).max() < 2 * U32


def test_two_part_twiddles_are_exact_to_second_order():
    for n in (48, 64, 256, 384, 512):
        c, s = roots(n)
        ch, sh = c.astype(np.float32), s.astype(np.float32)
        cl = (c - ch.astype(float)).astype(np.float32)
        sl = (s - sh.astype(float)).astype(np.float32)
        cc = ch.astype(float) + cl.astype(float)
        ss = sh.astype(float) + sl.astype(float)
        assert np.abs(cc ** 2 + ss ** 2 - 1.0).max() < 4 * U32 ** 2, n
