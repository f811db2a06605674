"""Derivation of the codec's own log2 and exp2 polynomial coefficients.

The LOG domain of the codec (Section 4.3, Algorithm 2) quantizes log2|x|;
both the device codec and the CPU oracle evaluate log2 and 2^x with their own
polynomials instead of a math library, so that the two sides round
identically.  The coefficients are least-squares Chebyshev fits in float64
on 2000 Chebyshev nodes of the interval, converted to the monomial basis of
the interval's own variable and rounded to float32:

* log2(1 + t) / t on t in [sqrt(1/2) - 1, sqrt(2) - 1], degree 8 (the
  significand folded into [sqrt(1/2), sqrt(2)]; log2 x = e + t P(t));
* 2^f on f in [-1/2, 1/2], degree 6.

Run it to print both sets (lowest degree first); tests/test_oracle_codec.py
checks that the oracle and the device code both use exactly these values,
and the oracle's exhaustive error bounds pin their accuracy.
"""
import numpy as np
from numpy.polynomial import chebyshev as Ch
from numpy.polynomial import polynomial as P

NODES = 2000


def fit(fn, a: float, b: float, degree: int, nodes: int = NODES):
    """float32 monomial coefficients (lowest degree first) of the
    least-squares Chebyshev fit of fn on [a, b]."""
    x = np.cos(np.pi * (np.arange(nodes) + 0.5) / nodes)          # Chebyshev nodes of [-1, 1]
    c = Ch.chebfit(x, fn((x + 1) / 2 * (b - a) + a), degree)
    pc = Ch.cheb2poly(c)                                          # monomials in x
    lin = P.Polynomial([-(a + b) / (b - a), 2 / (b - a)])         # x as a function of the variable
    poly = P.Polynomial([0.0])
    for k, ck in enumerate(pc):
        poly = poly + ck * lin ** k
    return [float(v) for v in np.float32(poly.coef)]


def _log2_1p_over_t(t):
    t = np.asarray(t, dtype=np.float64)
    safe = np.where(t == 0, 1.0, t)
    return np.where(t == 0, 1 / np.log(2), np.log1p(t) / np.log(2) / safe)


def log2_coefficients():
    return fit(_log2_1p_over_t, np.sqrt(0.5) - 1, np.sqrt(2) - 1, 8)


def exp2_coefficients():
    return fit(lambda f: 2.0 ** f, -0.5, 0.5, 6)


if __name__ == "__main__":
    print("log2(1+t)/t:", log2_coefficients())
    print("2^f:", exp2_coefficients())
