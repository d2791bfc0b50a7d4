"""Pins of the oracle's ionic model, fixed-point coefficient, theta numerator
and Newton Jacobian (no GPU).  Each check is fixed by the paper's definitions
or by calculus, not by retyping the oracle's formulas:

* the Rogers-McCulloch current of eq. (3.1) vanishes at its three resting
  roots u = 0, a, 1 when w = 0, and is linear in w with slope c2 u;
* dI_ion/du against a central difference of I_ion;
* C_r of eq. (3.8) splits the current, C_r(u, w) u = I_ion(u, w) (the
  fixed-point scheme of Section 3.1 moves exactly this factor to the
  unknown);
* the residual inside Theta of eq. (3.6) against SymPy's
  C_m u_t - sum_l sigma_l u_ll + I_ion(u, w) - f, for splines that reproduce
  polynomials exactly (coefficients from SciPy's independent B-spline
  interpolation at the Greville points);
* the linearised operator with the pointwise derivative against a central
  difference of the residual, and Newton's quadratic contraction.
"""
import numpy as np
import pytest
import sympy as sy
from scipy.interpolate import make_interp_spline

import st_workloads as W
from oracle.spacetime import SpaceTime, ionic_current, ionic_du, reaction_coefficient


def _params():
    return W.config(0)


def test_ionic_current_roots_and_w_slope():
    P = _params()
    for root in (0.0, P.a, 1.0):
        assert ionic_current(np.array([root]), np.array([0.0]), P)[0] == pytest.approx(0.0, abs=1e-15)
    rng = np.random.default_rng(1)
    u, w = rng.uniform(-0.5, 1.5, 50), rng.uniform(-0.2, 0.5, 50)
    lin = ionic_current(u, w, P) - ionic_current(u, np.zeros_like(w), P)
    np.testing.assert_allclose(lin, P.c2 * u * w, rtol=1e-12, atol=1e-14)
    # cubic in u with leading coefficient c1: third difference / h^3 = 6 c1
    h = 0.25
    x = rng.uniform(-1, 2, 20)
    third = (ionic_current(x + 3 * h, w[:20], P) - 3 * ionic_current(x + 2 * h, w[:20], P)
             + 3 * ionic_current(x + h, w[:20], P) - ionic_current(x, w[:20], P)) / h ** 3
    np.testing.assert_allclose(third, 6.0 * P.c1, rtol=1e-10)


def test_ionic_du_is_central_difference():
    P = _params()
    rng = np.random.default_rng(2)
    u, w = rng.uniform(-0.5, 1.5, 200), rng.uniform(-0.2, 0.5, 200)
    h = 1e-5
    fd = (ionic_current(u + h, w, P) - ionic_current(u - h, w, P)) / (2 * h)
    # central difference of a cubic: error exactly c1 h^2
    np.testing.assert_allclose(ionic_du(u, w, P), fd, rtol=0, atol=2 * P.c1 * h * h + 1e-9)


def test_reaction_coefficient_splits_current():
    P = _params()
    rng = np.random.default_rng(3)
    u, w = rng.uniform(-0.5, 1.5, 200), rng.uniform(-0.2, 0.5, 200)
    np.testing.assert_allclose(reaction_coefficient(u, w, P) * u, ionic_current(u, w, P), rtol=1e-12, atol=1e-14)


def _interp_coeffs(kn, p, f):
    """Spline coefficients interpolating f at the Greville points (SciPy)."""
    n = len(kn) - p - 1
    g = np.array([np.mean(kn[i + 1:i + p + 1]) for i in range(n)])
    return make_interp_spline(g, np.asarray(f(g), dtype=float) * np.ones_like(g), k=p, t=kn).c


def _poly_state(st, expr_u, expr_w, syms):
    """Full coefficient vectors of separable polynomials sum_k prod_l f_kl(x_l)
    given as lists of per-direction factor lists (time last)."""
    d = st.d
    out = []
    for terms in (expr_u, expr_w):
        X = np.zeros(st.shape)
        for factors in terms:
            # factors[l] for directions 0..d-1 (space) and d (time)
            vecs = [_interp_coeffs(st.kn[l], st.p[l], sy.lambdify(syms[l], factors[l], "numpy"))
                    for l in range(d + 1)]
            T = np.array([1.0])
            for a in range(d + 1):
                T = np.multiply.outer(T, vecs[st.dirs[a]])
            X += T.reshape(st.shape)
        out.append(X.reshape(-1))
    return out


@pytest.mark.parametrize("d,p,with_f", [(1, 2, False), (2, 2, True), (2, 3, False), (3, 2, True)])
def test_theta_numerator_against_sympy(d, p, with_f):
    """Theta of eq. (3.6) from the residual evaluated symbolically at the Gauss points."""
    # a short final time keeps the denominator of eq. (3.6) (which holds
    # ||u||/T) large, so that Theta stays below its cap of 1 and the numerator
    # is visible
    T = 0.02
    P = W.tiny(d, p, 3, nel_t=4, T=T)
    syms = sy.symbols("x1 x2 x3")[:d] + (sy.Symbol("t"),)
    x = syms
    t = syms[-1]
    s_ = t / T
    # u: separable terms of degree <= p per variable (exactly reproduced)
    u_terms = [[0.4 + 0.3 * x[0] - 0.5 * x[0] ** 2] + [1 + 0 * xx for xx in x[1:d]] + [1 - 0.2 * s_ + 0.05 * s_ ** 2],
               [0.3 * x[0]] + [0.2 + 0.6 * xx ** 2 for xx in x[1:d]] + [0.5 * s_]]
    w_terms = [[1 + 0 * x[0]] + [1 + 0 * xx for xx in x[1:d]] + [0.1 * s_]]
    f_expr = (0.7 * x[0] * s_ + 0.2) if with_f else 0
    f_fun = None
    if with_f:
        ff = sy.lambdify(syms, f_expr, "numpy")
        f_fun = lambda xs, tt: ff(*xs, tt) * np.ones_like(tt)
    st = SpaceTime(P, f=f_fun)
    uf, wf = _poly_state(st, u_terms, w_terms, syms)

    def total(terms):
        return sum(sy.prod(fs) for fs in terms)
    us, ws = total(u_terms), total(w_terms)
    R = P.Cm * sy.diff(us, t) - sum(P.sigma[l] * sy.diff(us, x[l], 2) for l in range(d)) \
        + P.c1 * us * (us - P.a) * (us - 1) + P.c2 * us * ws - f_expr
    Rf, Uf, Utf = (sy.lambdify(syms, e, "numpy") for e in (R, us, sy.diff(us, t)))
    grids = np.meshgrid(*([st.quad[d][0]] + [st.quad[l][0] for l in range(d - 1, -1, -1)]), indexing="ij")
    coords = {d: grids[0]}
    for l in range(d):
        coords[l] = grids[d - l]
    args = [coords[l] for l in range(d)] + [coords[d]]
    one = np.ones_like(grids[0])
    Rq, Uq, Utq = (np.asarray(F(*args)) * one for F in (Rf, Uf, Utf))
    # the splines reproduce u exactly at the Gauss points
    np.testing.assert_allclose(st.ev(uf, {}).reshape(Uq.shape), Uq, rtol=0, atol=1e-12)
    den = P.Cm * (np.abs(Uq).max() / P.T + np.abs(Utq).max())
    Th = st.theta_grid(uf, wf)

    def window(l, j):          # support extension of eq. (2.3), 1-based j, clamped
        kn, pp = st.kn[l], st.p[l]
        return kn[max(j - pp, 1) - 1], kn[min(j + pp + 1, len(kn)) - 1]

    rng = np.random.default_rng(d * 10 + p)
    below_cap = 0
    for _ in range(40):
        it = int(rng.integers(0, st.n[d] - 1))
        idx = [int(rng.integers(0, st.n[l])) for l in range(d)]
        m = np.ones(Rq.shape, dtype=bool)
        lo, hi = window(d, it + 2)
        m &= (coords[d] > lo) & (coords[d] < hi)
        for l in range(d):
            lo, hi = window(l, idx[l] + 1)
            m &= (coords[l] > lo) & (coords[l] < hi)
        want = min(np.abs(Rq[m]).max() / den, 1.0)
        below_cap += want < 1.0
        flat = 0
        for l in range(d - 1, -1, -1):
            flat = flat * st.n[l] + idx[l]
        assert Th[it, flat] == pytest.approx(want, rel=1e-11, abs=1e-13)
    assert below_cap >= 30


def _frozen_theta(st, u, w):
    return st.lowrank_at_quad(st.lowrank(st.theta_grid(u, w), 0.1))


def test_jacobian_is_derivative_of_residual():
    """(N(u + h v) - N(u - h v)) / 2h = J(u) v with J's reaction coefficient the
    pointwise dI_ion/du (w and theta fixed)."""
    P = W.tiny(2, 2, 4, nel_t=4)
    st = SpaceTime(P)
    u, w = W.smooth_state(P, 5, noise=0.05)
    thq = _frozen_theta(st, u, w)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(st.n[2] * st.n[1] * st.n[0] - st.n[1] * st.n[0])
    h = 1e-5
    N_p = st.residual(u + st.full(h * v), w, thq)
    N_m = st.residual(u - st.full(h * v), w, thq)
    fd = (N_p - N_m) / (2 * h)
    jq = ionic_du(st.ev(u, {}), st.ev(w, {}), P)
    Jv = st.apply_J(v, jq, thq)
    assert np.linalg.norm(Jv - fd) <= 1e-8 * np.linalg.norm(Jv)


def test_newton_quadratic_contraction():
    """Exact Newton on the frozen-theta, fixed-w system (config 0): the update
    norms contract quadratically, |delta_{k+1}| <= C |delta_k|^2."""
    import scipy.sparse.linalg as spla
    P = W.config(0)
    st = SpaceTime(P)
    u = np.tile(st.lift(), st.n[1])
    w = st.w_update_explicit(u)
    # a few damped steps bring the iterate into Newton's quadratic region
    thq = _frozen_theta(st, u, w)
    deltas = []
    for k in range(14):
        jq = ionic_du(st.ev(u, {}), st.ev(w, {}), P)
        J = st.assemble_J(jq, thq)
        delta = -spla.splu(J.tocsc()).solve(st.residual(u, w, thq))
        u = u + st.full(delta)
        deltas.append(float(np.max(np.abs(delta))))
        if deltas[-1] < 1e-12:
            break
    assert deltas[-1] < 1e-12, deltas
    # the last contractions are quadratic: ratios delta_{k+1} / delta_k^2 stay bounded
    tail = [(a, b) for a, b in zip(deltas[:-1], deltas[1:]) if a < 1e-2 and b > 1e-15]
    assert tail, deltas
    for a, b in tail:
        assert b <= 50.0 * a * a, deltas
