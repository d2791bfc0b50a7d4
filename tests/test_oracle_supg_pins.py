"""Pins of the oracle's SUPG + shock-capturing discretisation (Section 4.2.2),
no GPU.  Each check is fixed independently of the oracle's own formulas:

* the whole bilinear form (Galerkin + SUPG + shock capturing) and the load
  vector against a direct quadrature of their defining integrals with SciPy's
  B-spline evaluation (BSpline objects, a finer Gauss rule), on C^0 and on
  graded time knots, with coefficient functions for which both quadratures
  are exact;
* the shock-capturing coefficient against SymPy's residual of a state that
  the splines reproduce exactly;
* consistency: a manufactured solution in the spline space with zero normal
  flux, forced by f = C_m u_t - div(D grad u) + I_ion(u), makes the discrete
  residual (Galerkin + SUPG + shock capturing) vanish.
"""
import numpy as np
import pytest
import sympy as sy
from scipy.interpolate import BSpline, make_interp_spline

import st_workloads as W
from oracle.solver import solve_picard
from oracle.spacetime import SpaceTime, ionic_current, reaction_coefficient


def _graded_time_knots(nel, p):
    z = (np.arange(nel + 1) / nel) ** 1.5
    return np.concatenate([np.zeros(p + 1), z[1:-1], np.ones(p + 1)])


def _basis(kn, p, x, der):
    """All B-splines of the knot vector (SciPy) or their derivative at x: len(x) x n."""
    n = len(kn) - p - 1
    B = BSpline(kn, np.eye(n), p, extrapolate=False)
    if der:
        B = B.derivative(der)
    out = B(x)
    return np.nan_to_num(out)


def _fine_rule(kn, m):
    z = np.unique(kn)
    g, w = np.polynomial.legendre.leggauss(m)
    pts, wts, h = [], [], []
    for a, b in zip(z[:-1], z[1:]):
        pts.append(0.5 * (a + b) + 0.5 * (b - a) * g)
        wts.append(0.5 * (b - a) * w)
        h.append(np.full(m, b - a))
    return np.concatenate(pts), np.concatenate(wts), np.concatenate(h)


def _case(d, kind):
    p = 3 if d == 1 else 2
    P = W.tiny(d, p, 4, nel_t=4, T=2.0)
    kn = P.uniform_knots()
    kn[d] = W.c0_time_knots(4, p) if kind == "c0" else _graded_time_knots(4, p)
    return P, kn


def _direct_form(P, kn, u, coef, rho, f):
    """sum over Gauss points (SciPy basis, p + 3 points per element) of the
    Galerkin + SUPG + SC integrands for every full-basis test function."""
    d, p, pt = P.d, P.p_s, P.p_t
    Tk = P.T * np.asarray(kn[d])
    rules = [_fine_rule(kn[l], p + 3) for l in range(d)] + [_fine_rule(Tk, pt + 3)]
    B = [[_basis(kn[l], p, rules[l][0], k) for k in range(3)] for l in range(d)]
    B.append([_basis(Tk, pt, rules[d][0], k) for k in range(2)])
    # grids [t][x_d]..[x_1]
    axes = [d] + list(range(d - 1, -1, -1))

    def phi(ders):
        M = B[axes[0]][ders.get(axes[0], 0)]
        for a in axes[1:]:
            M = np.kron(M, B[a][ders.get(a, 0)])
        return M

    def grid(vals):
        out = vals[axes[0]]
        for a in axes[1:]:
            out = np.multiply.outer(out, vals[a])
        return out.reshape(-1)

    om = grid([rules[l][1] for l in range(d + 1)])
    tau = grid([np.ones_like(rules[l][0]) for l in range(d)] + [rules[d][2] / (2 * pt + 1)])
    sc = grid([np.ones_like(rules[l][0]) for l in range(d)] + [rules[d][2] ** 2 / 4.0])
    xs = [grid([rules[k][0] if k == l else np.ones_like(rules[k][0]) for k in range(d)] +
               [np.ones_like(rules[d][0])]) for l in range(d)]
    tt = grid([np.ones_like(rules[l][0]) for l in range(d)] + [rules[d][0]])
    C = coef(xs, tt)
    Rh = rho(xs, tt)
    P0, Pt = phi({}), phi({d: 1})
    uq, ut = P0 @ u, Pt @ u
    lap = sum(P.sigma[l] * (phi({l: 2}) @ u) for l in range(d))
    y = P0.T @ (om * (P.Cm * ut + C * uq))
    for l in range(d):
        y += P.sigma[l] * phi({l: 1}).T @ (om * (phi({l: 1}) @ u))
    y += Pt.T @ (om * tau * (P.Cm * ut - lap + C * uq))
    y += Pt.T @ (om * sc * Rh * ut)
    Fv = P0.T @ (om * f(xs, tt)) + Pt.T @ (om * tau * f(xs, tt))
    return y, Fv


@pytest.mark.parametrize("d,kind", [(1, "c0"), (1, "graded"), (2, "c0"), (2, "graded")])
def test_supg_form_and_load_against_scipy(d, kind):
    P, kn = _case(d, kind)
    coef = lambda xs, t: 1.0 + xs[0] * t                          # degree 1 in x_1 and t
    rho = lambda xs, t: 0.3 + 0.5 * xs[0]                          # degree 1 in x_1
    f = lambda xs, t: 0.7 * xs[0] * t + 0.2
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=1.0, f=f)
    rng = np.random.default_rng(d)
    u = rng.standard_normal(int(np.prod(st.shape)))
    grids = np.meshgrid(*([st.quad[d][0]] + [st.quad[l][0] for l in range(d - 1, -1, -1)]), indexing="ij")
    xs = [grids[d - l].reshape(-1) for l in range(d)]
    t = grids[0].reshape(-1)
    # the oracle's shock-capturing coefficient carries c h^2/4; the direct sum
    # multiplies by h^2/4 itself, so pass rho through the oracle's scale
    scale = np.repeat(st.sc_scale_t, int(np.prod(st.qshape[1:])))
    A = st.assemble_full(coef(xs, t), None, scale * rho(xs, t))
    y_dir, F_dir = _direct_form(P, kn, u, coef, rho, f)
    y = A @ u
    assert np.max(np.abs(y - y_dir)) <= 1e-12 * max(1.0, np.max(np.abs(y_dir)))
    F = st.load_vector()
    assert np.max(np.abs(F - F_dir)) <= 1e-12 * max(1.0, np.max(np.abs(F_dir)))


def _interp(kn, p, fun):
    n = len(kn) - p - 1
    g = np.array([np.mean(kn[i + 1:i + p + 1]) for i in range(n)])
    return make_interp_spline(g, np.asarray(fun(g), dtype=float) * np.ones_like(g), k=p, t=kn).c


def _separable(st, factors):
    T = np.array([1.0])
    for a in range(st.d + 1):
        l = st.dirs[a]
        T = np.multiply.outer(T, _interp(st.kn[l], st.p[l], factors[l]))
    return T.reshape(-1)


@pytest.mark.parametrize("d", [1, 2])
def test_sc_coefficient_against_sympy(d):
    p = 3 if d == 1 else 2
    Tf = 0.5
    P = W.tiny(d, p, 3, nel_t=3, T=Tf)
    kn = P.uniform_knots()
    kn[d] = W.c0_time_knots(3, p)
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=0.8)
    x = sy.symbols("x1 x2")[:d]
    t = sy.Symbol("t")
    fu = [0.4 + 0.3 * x[0] - 0.5 * x[0] ** 2] + [0.2 + 0.6 * xx ** 2 for xx in x[1:]] + [1 - 0.4 * t + 0.3 * t ** 2]
    fw = [1 + 0 * x[0]] + [1 + 0 * xx for xx in x[1:]] + [0.1 * t]
    lam = lambda e, v: sy.lambdify(v, e, "numpy")
    syms = list(x) + [t]
    u = _separable(st, [lam(fu[l], syms[l]) for l in range(d + 1)])
    w = _separable(st, [lam(fw[l], syms[l]) for l in range(d + 1)])
    us, ws = sy.prod(fu), sy.prod(fw)
    R = P.Cm * sy.diff(us, t) - sum(P.sigma[l] * sy.diff(us, x[l], 2) for l in range(d)) \
        + P.c1 * us * (us - P.a) * (us - 1) + P.c2 * us * ws
    grids = np.meshgrid(*([st.quad[d][0]] + [st.quad[l][0] for l in range(d - 1, -1, -1)]), indexing="ij")
    args = [grids[d - l] for l in range(d)] + [grids[0]]
    one = np.ones_like(grids[0])
    Rq, Uq, Utq = (np.asarray(lam(e, syms)(*args)) * one for e in (R, us, sy.diff(us, t)))
    den = P.Cm * (np.abs(Uq).max() / Tf + np.abs(Utq).max())
    h = Tf / 3
    want = 0.8 * h * h / 4.0 * np.abs(Rq) / den
    got = st.sc_coefficient(u, w).reshape(want.shape)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-14)
    # zero state: the coefficient is zero (reading for a vanishing denominator)
    assert not np.any(st.sc_coefficient(np.zeros_like(u), w))


@pytest.mark.parametrize("kind", ["c0", "graded"])
def test_supg_consistency_manufactured(kind):
    """N(u*) = A(u*) u* - F = 0 for u* in the spline space with zero normal flux
    and f making the residual vanish pointwise (then the SC coefficient is 0)."""
    p = 3
    P = W.tiny(2, p, 3, nel_t=3, T=1.5)
    kn = P.uniform_knots()
    kn[2] = W.c0_time_knots(3, p) if kind == "c0" else _graded_time_knots(3, p)
    x1, x2, t = sy.symbols("x1 x2 t")
    fx1 = x1 ** 2 * (3 - 2 * x1)               # zero derivative at 0 and 1
    fx2 = 0.5 + x2 ** 2 * (1.5 - x2)
    ft = 0.2 + 0.5 * t - 0.1 * t ** 2
    us = fx1 * fx2 * ft
    ws = 0.3 * t * fx2
    fs = P.Cm * sy.diff(us, t) - P.sigma[0] * sy.diff(us, x1, 2) - P.sigma[1] * sy.diff(us, x2, 2) \
        + P.c1 * us * (us - P.a) * (us - 1) + P.c2 * us * ws
    ff = sy.lambdify((x1, x2, t), fs, "numpy")
    f = lambda xs, tt: ff(xs[0], xs[1], tt) * np.ones_like(tt)
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=1.0, f=f)
    lam = lambda e, v: sy.lambdify(v, e, "numpy")
    u = _separable(st, [lam(fx1, x1), lam(fx2, x2), lam(ft, t)])
    w = _separable(st, [lambda z: np.ones_like(z), lam(fx2, x2), lam(0.3 * t, t)])
    sc = st.sc_coefficient(u, w)
    assert np.max(np.abs(sc)) < 1e-12
    A = st.assemble_full(st.reaction_at_quad(u, w), None, sc)
    N = st.rows(A @ u - st.load_vector())
    scale = np.max(np.abs(st.rows(st.load_vector())))
    assert np.max(np.abs(N)) <= 1e-11 * scale
    # a flipped sign of the SUPG diffusion term would add this, far above N
    tau = np.repeat(st.supg_tau_t, int(np.prod(st.qshape[1:])))
    extra = sum(2 * P.sigma[l] * st.phi({2: 1}).T @ (st.omega * tau * (st.phi({l: 2}) @ u)) for l in range(2))
    assert np.max(np.abs(st.rows(extra))) > 1e3 * np.max(np.abs(N))


def test_supg_picard_fixed_point():
    """The Section 3.1 iteration with SUPG + SC on C^0 time splines converges;
    at its limit the discrete equations hold to the size of the last change."""
    P = W.tiny(1, 3, 8, nel_t=4)
    kn = P.uniform_knots()
    kn[1] = W.c0_time_knots(4, 3)
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=0.5)
    u, w, log = solve_picard(st, tol=1e-10, max_outer=400)
    assert log.deltas[-1] <= 1e-10
    # u is the fixed point for the (u, w) it was built from
    N_s = st.n[0]
    sc = st.sc_coefficient(u, w)
    A = st.assemble_full(st.reaction_at_quad(u, w), None, sc)
    N = st.rows(A @ u - st.load_vector())
    assert np.max(np.abs(N)) <= 1e-7
    assert np.all(np.isfinite(u)) and u[:N_s].max() == pytest.approx(1.0)


def test_supg_preconditioner_reduces_to_fast_diagonalization_operator():
    """With tau = 0, cr = a c1 and sc = 0 the preconditioner's bilinear form is
    the operator A-hat of Section 3.2 (assembled independently)."""
    P, kn = _case(2, "c0")
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=1.0)
    st.supg_tau_t = np.zeros_like(st.supg_tau_t)
    Qt = st.qshape[0]
    A = st.assemble_precond_supg(np.full(Qt, P.a * P.c1), np.zeros(Qt))
    B = st.assemble_precond()
    assert abs(A - B).max() <= 1e-13 * abs(B).max()


@pytest.mark.parametrize("d", [1, 2])
def test_supg_preconditioner_is_kronecker(d):
    """The preconditioner is A_t (x) M_s + B_t (x) K_s with 1D matrices from
    SciPy's basis: B_t = M_t + W_tau, A_t = C_m (W_t + K_tau) + cr-terms + sc-term."""
    P, kn = _case(d, "graded")
    st = SpaceTime(P, knots=kn, su=False, supg=True, sc_c=1.0)
    Qt = st.qshape[0]
    rng = np.random.default_rng(5)
    cr_t, sc_t = rng.uniform(0.0, 0.5, Qt), rng.uniform(0.0, 2.0, Qt)
    A = st.assemble_precond_supg(cr_t, sc_t).toarray()
    # 1D matrices on a fine rule with SciPy's B-splines; the time coefficients
    # are given at the oracle's Gauss points, so integrate them on that rule
    Tk = P.T * np.asarray(kn[d])
    tq, tw, tel = st.quad[d]
    h = np.diff(np.unique(Tk))[tel]
    tau = h / (2 * P.p_t + 1)
    b0, b1 = _basis(Tk, P.p_t, tq, 0), _basis(Tk, P.p_t, tq, 1)
    g = lambda wt, X, Y: X.T @ (wt[:, None] * Y)
    At = P.Cm * (g(tw, b0, b1) + g(tw * tau, b1, b1)) + g(tw * cr_t, b0, b0) + g(tw * tau * cr_t, b1, b0) \
        + g(tw * sc_t, b1, b1)
    Bt = g(tw, b0, b0) + g(tw * tau, b1, b0)
    Ms, Ks = [], []
    for l in range(d):
        x, w, _ = _fine_rule(kn[l], P.p_s + 2)
        B0, B1 = _basis(kn[l], P.p_s, x, 0), _basis(kn[l], P.p_s, x, 1)
        Ms.append(g(w, B0, B0))
        Ks.append(g(w, B1, B1))
    if d == 1:
        M, K = Ms[0], P.sigma[0] * Ks[0]
    else:
        M = np.kron(Ms[1], Ms[0])
        K = P.sigma[0] * np.kron(Ms[1], Ks[0]) + P.sigma[1] * np.kron(Ks[1], Ms[0])
    want = np.kron(At[1:, 1:], M) + np.kron(Bt[1:, 1:], K)
    assert np.max(np.abs(A - want)) <= 1e-12 * np.max(np.abs(want))
