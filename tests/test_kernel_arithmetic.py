"""Arithmetic the kernels rely on, checked on the host with every FMA
rounded once (emulated exactly):

* the cos(pi x) polynomial of the general Fourier velocity encoding
  (csrc/sl_device.h, cospi_poly): the coefficients in the header are the ones
  csrc/cospi_poly.py computes, both copies (constant-memory table and
  literals) agree, and the evaluation as the kernel performs it stays within
  3e-16 of cos(pi x);
* the trajectory quotient div_by (one Markstein correction of a * RN(1/b)) is
  the correctly rounded a / b for the spacings and magnitudes of the
  trajectory updates, and keeps whole-cell displacements exact."""
from fractions import Fraction
import os
import random
import re
import sys

import mpmath as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_2817_amd", "csrc")
sys.path.insert(0, CSRC)
import cospi_poly  # noqa: E402


def _header():
    with open(os.path.join(CSRC, "sl_device.h")) as fh:
        return fh.read()


def _table():
    m = re.search(r"kCosPiPoly\[8\] = \{([^}]*)\}", _header())
    return [float(v) for v in m.group(1).replace("\n", " ").split(",")]


def _literals():
    body = _header().split("__device__ __forceinline__ double cospi_poly(double x)")[1]
    body = body.split("} else {")[1].split("}")[0]
    vals = re.findall(r"p = (?:fma\(p, s, )?([-0-9.e+]+)\)?;", body)
    return [float(v) for v in vals][::-1]


def _fma(a, b, c):
    with mp.workdps(60):
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def _cospi_as_kernel(x, k):
    n = float(round(x))  # rint: ties to even, as round() does
    t = x - n
    s = t * t
    p = k[7]
    for i in range(6, -1, -1):
        p = _fma(p, s, k[i])
    p = _fma(p, s, 1.0)
    h = 0.5 * n
    return -p if h != float(round(h)) else p


def test_header_holds_the_generated_coefficients():
    want = cospi_poly.coefficients()
    assert _table() == want
    assert _literals() == want


def test_error_bound_over_the_reduced_range_and_beyond():
    k = _table()
    rnd = random.Random(5)
    pts = [rnd.uniform(-0.5, 0.5) for _ in range(1500)]
    pts += [rnd.uniform(-40.0, 40.0) for _ in range(1500)]
    pts += [0.0, 0.5, -0.5, 0.25, 1.0, 2.5, -3.5, 1e-12, 7.0 + 2 ** -30]
    worst = 0.0
    with mp.workdps(40):
        for x in pts:
            err = abs(mp.mpf(_cospi_as_kernel(x, k)) - mp.cos(mp.pi * mp.mpf(x)))
            worst = max(worst, float(err))
    assert worst <= 3e-16, worst
    assert _cospi_as_kernel(0.0, k) == 1.0
    assert _cospi_as_kernel(1.0, k) == -1.0


def _div_by(a, b, y):
    q = a * y
    r = float(Fraction(-q) * Fraction(b) + Fraction(a))
    return float(Fraction(r) * Fraction(y) + Fraction(q))


def test_corrected_quotient_is_the_rounded_division():
    rnd = random.Random(3)
    for n in (24, 28, 96, 100, 128, 255, 256, 300, 512, 1000, 1024, 4096, 3):
        for length in (1.0, 2.0, 0.7, 3.3):
            h = length / n
            for b in (6.0 * h, h):
                y = 1.0 / b
                for _ in range(400):
                    a = rnd.uniform(-1.0, 1.0) * 10.0 ** rnd.uniform(-12.0, 1.0)
                    assert _div_by(a, b, y) == a / b, (a, b)
                # whole cells: dt * 6 u = 6 k h gives exactly k
                for k in range(-8, 9):
                    assert _div_by(6.0 * k * h, 6.0 * h, 1.0 / (6.0 * h)) == (6.0 * k * h) / (6.0 * h)
