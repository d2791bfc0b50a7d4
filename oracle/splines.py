"""Univariate B-splines (paper Section 2): knots, spans, values/derivatives,
Greville abscissae and Gauss rules.  Test infrastructure (see package doc).

Indices are 0-based in code; the paper's b_{i,p} with i = 1..n is
``basis index i-1`` here.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(nel: int, p: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Open knot vector with p+1 repeated end knots and nel equal elements (Section 2)."""
    inner = lo + (hi - lo) * np.arange(1, nel) / nel
    return np.concatenate([np.full(p + 1, lo), inner, np.full(p + 1, hi)])


def n_basis(knots: np.ndarray, p: int) -> int:
    """Number of B-splines n = len(knots) - p - 1."""
    return len(knots) - p - 1


def breakpoints(knots: np.ndarray) -> np.ndarray:
    """Knots without repetitions (the vector Z of Section 2)."""
    return np.unique(knots)


def find_span(knots: np.ndarray, p: int, x: float) -> int:
    """Largest i (0-based) with knots[i] <= x < knots[i+1], restricted to the
    non-degenerate range p..n-1; x equal to the right end maps to the last
    non-empty span."""
    n = n_basis(knots, p)
    if x >= knots[n]:
        i = n - 1
        while knots[i] == knots[i + 1]:
            i -= 1
        return i
    i = int(np.searchsorted(knots, x, side="right")) - 1
    return min(max(i, p), n - 1)


def _ratio(num, den):
    """num/den with the Cox-de Boor convention 0/0 = 0 (den == 0 -> 0)."""
    return np.where(den != 0.0, num / np.where(den != 0.0, den, 1.0), 0.0)


def bspline_all(knots: np.ndarray, p: int, x, der: int = 0) -> np.ndarray:
    """Matrix B[m, i] = d^der/dx^der b_{i,p}(x_m) for all basis functions.

    Straight Cox-de Boor recursion on the degree (Cottrell et al. 2009):
      b_{i,0}(x) = 1 on [xi_i, xi_{i+1}), with the last non-empty interval
      closed on the right;
      b_{i,q} = (x - xi_i)/(xi_{i+q} - xi_i) b_{i,q-1}
              + (xi_{i+q+1} - x)/(xi_{i+q+1} - xi_{i+1}) b_{i+1,q-1};
    and derivatives by the recursion
      b^{(k)}_{i,q} = q [ b^{(k-1)}_{i,q-1}/(xi_{i+q}-xi_i)
                        - b^{(k-1)}_{i+1,q-1}/(xi_{i+q+1}-xi_{i+1}) ].
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    kn = np.asarray(knots, dtype=np.float64)
    m = len(kn) - 1                       # number of degree-0 functions
    last = max(j for j in range(m) if kn[j] < kn[j + 1])

    def deg0():
        B = np.zeros((len(x), m))
        for j in range(m):
            if kn[j] < kn[j + 1]:
                inside = (x >= kn[j]) & (x < kn[j + 1])
                if j == last:
                    inside |= x == kn[j + 1]
                B[:, j] = inside
        return B

    def rec(q, k):
        """d^k/dx^k of all degree-q functions (len(kn)-q-1 columns)."""
        if k > q:
            return np.zeros((len(x), len(kn) - q - 1))
        if q == 0:
            return deg0()
        lower = rec(q - 1, k) if k == 0 else rec(q - 1, k - 1)
        cols = len(kn) - q - 1
        out = np.zeros((len(x), cols))
        for i in range(cols):
            d1 = kn[i + q] - kn[i]
            d2 = kn[i + q + 1] - kn[i + 1]
            if k == 0:
                out[:, i] = (_ratio(x - kn[i], d1) * lower[:, i]
                             + _ratio(kn[i + q + 1] - x, d2) * lower[:, i + 1])
            else:
                out[:, i] = q * (_ratio(lower[:, i], d1) - _ratio(lower[:, i + 1], d2))
        return out

    return rec(p, der)


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae gamma_i = (xi_{i+1} + ... + xi_{i+p}) / p (Section 2)."""
    n = n_basis(knots, p)
    return np.array([np.sum(knots[i + 1: i + p + 1]) / p for i in range(n)])


def gauss_rule(nq: int):
    """nq-point Gauss-Legendre nodes/weights on [0, 1]."""
    g, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (g + 1.0), 0.5 * w


def quadrature(knots: np.ndarray, nq: int):
    """Tensor-ready 1D rule: nq Gauss points in every non-empty element.

    Returns (points, weights, element_of_point); elements are numbered by the
    breakpoint intervals in increasing order.
    """
    z = breakpoints(knots)
    g, w = gauss_rule(nq)
    pts, wts, el = [], [], []
    for e in range(len(z) - 1):
        h = z[e + 1] - z[e]
        pts.append(z[e] + h * g)
        wts.append(h * w)
        el.append(np.full(nq, e))
    return np.concatenate(pts), np.concatenate(wts), np.concatenate(el)
