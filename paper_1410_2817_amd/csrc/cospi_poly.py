"""Coefficients of the cos(pi t) polynomial of the general Fourier velocity
encoding (sl_device.h, kCosPiPoly): cos(pi t) = 1 + s P(s) for |t| <= 1/2,
s = t^2, with P the degree-7 Chebyshev interpolant of (cos(pi sqrt(s)) - 1) / s
on [0, 1/4] (interpolation at the 8 Chebyshev points of the interval, solved in
60-digit arithmetic, then rounded to FP64).  Run it to print the C table."""
import mpmath as mp

DEGREE = 7


def coefficients(degree=DEGREE):
    """P's coefficients, constant term first, rounded to FP64."""
    with mp.workdps(60):
        a, b = mp.mpf(0), mp.mpf(1) / 4

        def h(s):
            if s == 0:
                return -mp.pi ** 2 / 2
            return (mp.cos(mp.pi * mp.sqrt(s)) - 1) / s

        nodes = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (2 * k + 1) / (2 * (degree + 1)))
                 for k in range(degree + 1)]
        m = mp.matrix([[x ** j for j in range(degree + 1)] for x in nodes])
        c = mp.lu_solve(m, mp.matrix([h(x) for x in nodes]))
        return [float(c[j]) for j in range(degree + 1)]


if __name__ == "__main__":
    c = coefficients()
    print("__constant__ double kCosPiPoly[%d] = {" % len(c))
    print(",\n".join("    %s" % repr(v) for v in c) + "};")
