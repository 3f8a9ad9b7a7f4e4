"""Write stencils.json: interior 1D mass/stiffness stencils in exact rational
arithmetic from the truncated-power formula of the cardinal B-spline
N_m(x) = 1/m! sum_{j=0}^{m+1} (-1)^j C(m+1, j) (x - j)_+^m.

Mass row (times 1/h):       M_k = N_{2p+1}(p+1+k),        k = -p..p
Stiffness row (times h):    K_k = -N_{2p+1}''(p+1+k)
"""
import json
import os
from fractions import Fraction
from math import comb, factorial


def cardinal(m, x, deriv=0):
    s = Fraction(0)
    for j in range(m + 2):
        t = Fraction(x) - j
        if t <= 0:
            continue
        # d^deriv/dx^deriv of t^m
        if deriv > m:
            continue
        c = Fraction(factorial(m), factorial(m - deriv))
        s += (-1) ** j * comb(m + 1, j) * c * t ** (m - deriv)
    return s / factorial(m)


def stencils(p):
    m = 2 * p + 1
    mass = [cardinal(m, p + 1 + k) for k in range(-p, p + 1)]
    stiff = [-cardinal(m, p + 1 + k, 2) for k in range(-p, p + 1)]
    return mass, stiff


if __name__ == "__main__":
    out = {"citation": "cardinal B-spline autocorrelation identity (see README.md)"}
    for p in (1, 2, 3, 4, 5):
        mass, stiff = stencils(p)
        out[f"p{p}"] = {"mass_over_h": [[f.numerator, f.denominator] for f in mass],
                        "stiffness_times_h": [[f.numerator, f.denominator] for f in stiff]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stencils.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)
