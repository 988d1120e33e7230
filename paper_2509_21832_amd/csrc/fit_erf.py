"""Coefficients of the branch-free GELU of the closure network (mm_closure.hip).

With a = |z|, erfc(a / sqrt 2) = 2^(-a Q(a)), Q a polynomial in a: the function
g(a) = -log2(erfc(a / sqrt 2)) / a is smooth on [0, A], A = 4 sqrt 2
(g(0) = 2 / sqrt(2 pi) / ln 2), and beyond A erfc is below 2e-8.  Q is the least-squares
Chebyshev fit of g on [0, A], weighted by 1 / g (relative error), degree 5, converted to
powers of a and rounded to FP32.  Then, for either sign of z,
  GELU(z) = z Phi(z) = max(z, 0) - a 2^(-a Q(a) - 1),
  Phi(z) = 1 - 2^(-a Q(a) - 1) (z >= 0) or 2^(-a Q(a) - 1) (z < 0).
With the FP32 Horner evaluation the GELU is within 2e-6 absolute and Phi within 2e-6
of the exact values: far below the bf16 rounding of the activations (2^-9 relative).
Run: python3 fit_erf.py (prints the errors and the C initialiser)."""
import numpy as np
from scipy.special import erfc, ndtr

A, DEG = 4.0 * np.sqrt(2.0), 5


def fit():
    a = np.linspace(1e-6, A, 20001)
    g = -np.log2(erfc(a / np.sqrt(2.0))) / a
    c = np.polynomial.chebyshev.chebfit(2 * a / A - 1, g, DEG, w=1 / g)
    p = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))
    return p(np.polynomial.Polynomial([-1, 2 / A])).coef.astype(np.float32)


def errors(coef):
    """max |GELU - z Phi(z)| and max |Phi - Phi exact| over z in [-10, 10], FP32 steps"""
    z = np.linspace(-10, 10, 80001).astype(np.float32)
    a = np.abs(z)
    ac = np.minimum(a, np.float32(A))
    q = np.float32(coef[-1])
    for k in range(len(coef) - 2, -1, -1):
        q = (q * ac + coef[k]).astype(np.float32)
    he = np.exp2(-((a * q).astype(np.float32) + np.float32(1.0)).astype(np.float64)).astype(np.float32)
    g = (np.maximum(z, 0) - (a * he).astype(np.float32)).astype(np.float64)
    phi = np.where(z >= 0, np.float32(1) - he, he).astype(np.float64)
    zz = z.astype(np.float64)
    return float(np.max(np.abs(g - zz * ndtr(zz)))), float(np.max(np.abs(phi - ndtr(zz))))


if __name__ == "__main__":
    coef = fit()
    eg, ep = errors(coef)
    print(f"// GELU: max abs {eg:.2e}; Phi: max abs {ep:.2e}")
    print("{" + ", ".join(f"{float(c):.9e}f" for c in coef) + "}")
