"""Exact closed forms of uniform (cardinal) B-splines, independent of the
Cox-de Boor recursion: the order-m cardinal B-spline on [0, m] is
  N_m(x) = 1/(m-1)! sum_{j=0}^{m} (-1)^j C(m, j) (x - j)_+^{m-1},
and autocorrelations of order-(p+1) B-splines are order-(2p+2) B-splines:
  int N(x) N(x - s) dx = N_{2p+2}(p + 1 + s).
Used by the tests to pin interior stencils of the 1D matrices and the interior
values of the SU coefficients tau_k.
"""
from fractions import Fraction
from math import comb, factorial


def cardinal(m: int, x, r: int = 0) -> Fraction:
    """r-th derivative of N_m at x (exact; valid where N_m^(r) is continuous)."""
    x = Fraction(x)
    tot = Fraction(0)
    e = m - 1 - r
    for j in range(m + 1):
        t = x - j
        if t > 0:
            tot += (-1) ** j * comb(m, j) * t ** e
    return tot / factorial(e)


def mass_stencil(p):
    """h-scaled interior mass row: M[i, i+k] / h for k = -p..p."""
    return [cardinal(2 * p + 2, p + 1 + k) for k in range(-p, p + 1)]


def stiff_stencil(p):
    """h^-1-scaled interior stiffness row: K[i, i+k] * h."""
    return [-cardinal(2 * p + 2, p + 1 + k, 2) for k in range(-p, p + 1)]


def adv_stencil(p):
    """Interior W[i, i+k] = int b_{i+k}' b_i (dimensionless)."""
    return [-cardinal(2 * p + 2, p + 1 + k, 1) for k in range(-p, p + 1)]


def interior_tau(p):
    """Constant interior solution (h = 1) of the tau equations: for l = 1..p,
    -N'(p+1+l) + sum_k tau_k (-1)^k N^(2k)(p+1+l) = 0 with N = N_{2p+2}."""
    m = 2 * p + 2
    A = [[(-1) ** k * cardinal(m, p + 1 + l, 2 * k) for k in range(1, p + 1)] for l in range(1, p + 1)]
    b = [cardinal(m, p + 1 + l, 1) for l in range(1, p + 1)]
    # exact Gaussian elimination
    n = p
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]
