"""Univariate Galerkin matrices and the SU coefficients tau_k.
Test infrastructure (see package doc).

Matrices follow Section 3.1.1 of the paper on the *full* basis b_1..b_n
(0-based columns 0..n-1):
  M[i, j] = int b_i b_j,   K[i, j] = int b_i' b_j',   W[i, j] = int b_j' b_i,
evaluated with (p+1)-point Gauss quadrature per element (reading: the paper
does not name its rule; p+1 points integrate these polynomial products of
degree <= 2p exactly).

The tau_k of the SU term (eq. (3.5)) are splines of degree p_t - k with
maximal regularity on the time breakpoints.  Reading of the index set: the
equations are imposed for every pair (i, i + l) of the *full* time basis with
1 <= l <= min(p_t, n_t - i); this makes the linear system square (its
unknown count is sum_k (nel + p_t - k)) and the matrix W_t + sum_k S_k[tau_k]
exactly lower triangular.  Taken literally over the N_t = n_t - 1 functions
of X_t the system would have p_t fewer equations than unknowns.
"""
from __future__ import annotations

import numpy as np

from .splines import bspline_all, breakpoints, n_basis, quadrature


def gram(knots, p, d_test: int, d_trial: int, weight=None, nq=None) -> np.ndarray:
    """G[i, j] = int weight(x) b_i^(d_test)(x) b_j^(d_trial)(x) dx by Gauss quadrature."""
    xq, wq, _ = quadrature(knots, nq or p + 1)
    Bi = bspline_all(knots, p, xq, d_test)
    Bj = bspline_all(knots, p, xq, d_trial)
    w = wq if weight is None else wq * np.asarray(weight(xq), dtype=np.float64)
    return Bi.T @ (w[:, None] * Bj)


def mass(knots, p, weight=None, nq=None):
    """Mass matrix M (Section 3.1.1), optionally weighted."""
    return gram(knots, p, 0, 0, weight, nq)


def stiffness(knots, p, nq=None):
    """Stiffness matrix K with K[i, j] = int b_i' b_j'."""
    return gram(knots, p, 1, 1, None, nq)


def advection(knots, p, nq=None):
    """Time-derivative matrix W with W[i, j] = int b_j' b_i (Section 3.1.1)."""
    return gram(knots, p, 0, 1, None, nq)


def reduced_knots(knots, q: int) -> np.ndarray:
    """Open knot vector of degree q with maximal regularity on the breakpoints of knots."""
    z = breakpoints(knots)
    return np.concatenate([np.full(q + 1, z[0]), z[1:-1], np.full(q + 1, z[-1])])


def tau_splines(knots_t, p_t: int, nq=None):
    """Solve eq. (3.5) for tau_1..tau_{p_t}.

    Returns a list of (knots_k, degree_k, coefficients_k).  The square system
    has one row per full-basis pair (i, i+l) and one column per basis function
    of each tau_k; columns are equilibrated (scaled to unit max-norm) before a
    dense LU solve, which changes nothing in exact arithmetic.
    """
    nq = nq or p_t + 1
    n_t = n_basis(knots_t, p_t)
    W = advection(knots_t, p_t, nq)
    xq, wq, _ = quadrature(knots_t, nq)
    ders = [bspline_all(knots_t, p_t, xq, k) for k in range(p_t + 1)]
    spaces = []
    for k in range(1, p_t + 1):
        kk = reduced_knots(knots_t, p_t - k)
        spaces.append((kk, p_t - k, bspline_all(kk, p_t - k, xq, 0)))
    rows = [(i, l) for i in range(n_t - 1) for l in range(1, min(p_t, n_t - 1 - i) + 1)]
    ncols = sum(s[2].shape[1] for s in spaces)
    A = np.zeros((len(rows), ncols))
    rhs = np.zeros(len(rows))
    for r, (i, l) in enumerate(rows):
        rhs[r] = -W[i, i + l]
        c0 = 0
        for k, (_, _, beta) in enumerate(spaces, start=1):
            prod = wq * ders[k][:, i + l] * ders[k][:, i]
            A[r, c0: c0 + beta.shape[1]] = prod @ beta
            c0 += beta.shape[1]
    if A.shape[0] != A.shape[1]:
        raise ValueError("tau system is not square")
    scale = np.max(np.abs(A), axis=0)
    scale[scale == 0] = 1.0
    y = np.linalg.solve(A / scale, rhs)
    coef = y / scale
    out, c0 = [], 0
    for kk, q, beta in spaces:
        m = beta.shape[1]
        out.append((kk, q, coef[c0: c0 + m].copy()))
        c0 += m
    return out


def eval_spline(knots, q, coef, x, der=0):
    """Value (or derivative) of sum_i coef_i b_{i,q}(x)."""
    return bspline_all(knots, q, x, der) @ coef
