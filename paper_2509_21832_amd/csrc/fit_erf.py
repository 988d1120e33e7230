"""Coefficients of the branch-free erf of the closure network's GELU (mm_closure.hip).

erf(t) = 1 - exp(-t P(t)) for t >= 0 (odd extension), P a polynomial in t: the function
g(t) = -log(erfc(t)) / t is smooth on [0, 4] (g(0) = 2 / sqrt(pi)), and beyond t = 4 erf
rounds to 1 in FP32.  P is the least-squares Chebyshev fit of g on [0, 4], weighted by
1 / g (relative error), degree 9, converted to powers of t and rounded to FP32.  With the
FP32 Horner evaluation the erf is within 4e-7 relative and 8e-8 absolute on [0, 4].
Run: python3 fit_erf.py (prints the C initialiser)."""
import numpy as np
from scipy.special import erf, erfc

T, DEG = 4.0, 9


def fit():
    t = np.linspace(1e-6, T, 20001)
    g = -np.log(erfc(t)) / t
    c = np.polynomial.chebyshev.chebfit(2 * t / T - 1, g, DEG, w=1 / g)
    p = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))
    coef = p(np.polynomial.Polynomial([-1, 2 / T])).coef.astype(np.float32)
    tf = t.astype(np.float32)
    acc = np.float32(coef[-1])
    for k in range(DEG - 1, -1, -1):
        acc = (acc * tf + coef[k]).astype(np.float32)
    approx = 1.0 - np.exp(-(tf * acc).astype(np.float64))
    return coef, float(np.max(np.abs(approx - erf(t)) / erf(t))), float(np.max(np.abs(approx - erf(t))))


if __name__ == "__main__":
    coef, rel, ab = fit()
    print(f"// max rel {rel:.2e}, max abs {ab:.2e}")
    print("{" + ", ".join(f"{float(c):.9e}f" for c in coef) + "}")
