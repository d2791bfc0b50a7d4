"""Pins of the CPU oracle to facts fixed by the paper and by mathematics
(no GPU).  Each test names the passage or the closed form it relies on."""
import numpy as np
import pytest

import st_workloads as W
from oracle import solver
from oracle.operators1d import advection, mass, stiffness, tau_splines, eval_spline
from oracle.spacetime import SpaceTime, truncated_svd, hat_matrix, LowRank
from oracle.splines import (bspline_all, find_span, greville, open_uniform_knots, quadrature,
                            n_basis)
from tests.cardinal import adv_stencil, interior_tau, mass_stencil, stiff_stencil


def nonuniform_knots(p, rng):
    inner = np.sort(rng.uniform(0.05, 0.95, 7))
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


# ---------------------------------------------------------------- splines (Section 2)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_partition_of_unity(p):
    """sum_i b_i = 1 and sum_i b_i^(k) = 0 (B-spline partition of unity)."""
    rng = np.random.default_rng(p)
    for kn in (open_uniform_knots(7, p), nonuniform_knots(p, rng)):
        x = rng.uniform(0, 1, 200)
        assert np.allclose(bspline_all(kn, p, x, 0).sum(1), 1.0, atol=1e-14)
        for k in range(1, p + 1):
            s = bspline_all(kn, p, x, k).sum(1)
            assert np.max(np.abs(s)) < 1e-9 * (1 + np.max(np.abs(bspline_all(kn, p, x, k))))


def test_bspline_known_values():
    """Degree-1 B-splines are hat functions; derivative of a degree-2 spline
    equals the difference formula on the degree-1 basis (textbook identity)."""
    kn = open_uniform_knots(4, 1)
    x = np.linspace(0, 1, 41)
    B = bspline_all(kn, 1, x)
    for i, g in enumerate(greville(kn, 1)):
        assert np.allclose(B[:, i], np.maximum(0, 1 - np.abs(x - g) * 4), atol=1e-14)


def test_spans_bruteforce():
    """find_span is the largest i with xi_i <= x < xi_{i+1} (bit-exact)."""
    rng = np.random.default_rng(0)
    for p in (1, 2, 3):
        kn = nonuniform_knots(p, rng)
        n = n_basis(kn, p)
        for x in np.concatenate([rng.uniform(0, 1, 100), kn[p:n + 1]]):
            i = find_span(kn, p, x)
            if x < 1.0:
                assert kn[i] <= x < kn[i + 1]
            else:
                assert i == n - 1


def test_greville_uniform():
    """Uniform open knots: gamma ends at 0 and 1 and is strictly increasing."""
    for p in (1, 2, 3):
        g = greville(open_uniform_knots(8, p), p)
        assert g[0] == 0.0 and g[-1] == 1.0 and np.all(np.diff(g) > 0)
    # p = 2, h = 1/32: interior Greville points are element midpoints
    g = greville(open_uniform_knots(32, 2), 2)
    assert np.allclose(g[1:4], [1 / 64, 3 / 64, 5 / 64], atol=0)


# ---------------------------------------------------------------- 1D matrices
@pytest.mark.parametrize("p", [1, 2, 3])
def test_matrix_sums_and_kernels(p):
    """1^T M 1 = |interval|, K 1 = 0, W 1 = 0 and W + W^T = e_n e_n^T - e_1 e_1^T
    (fundamental theorem of calculus), for uniform and non-uniform knots, T-scaled."""
    rng = np.random.default_rng(10 + p)
    for kn in (open_uniform_knots(9, p), nonuniform_knots(p, rng), 3.5 * open_uniform_knots(5, p)):
        L = kn[-1] - kn[0]
        M, K, Wm = mass(kn, p), stiffness(kn, p), advection(kn, p)
        one = np.ones(M.shape[0])
        assert abs(one @ M @ one - L) < 1e-13 * L
        assert np.max(np.abs(K @ one)) < 1e-11
        assert np.max(np.abs(Wm @ one)) < 1e-12
        E = np.zeros_like(Wm)
        E[0, 0], E[-1, -1] = -1.0, 1.0
        assert np.max(np.abs(Wm + Wm.T - E)) < 1e-13
        assert np.allclose(M, M.T, atol=1e-15) and np.allclose(K, K.T, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_interior_stencils_closed_form(p):
    """Interior rows equal the cardinal B-spline autocorrelation closed forms
    (M/h = N_{2p+2}(p+1+k), K h = -N''_{2p+2}(p+1+k), W = -N'_{2p+2}(p+1+k))."""
    nel = 12
    h = 1.0 / nel
    kn = open_uniform_knots(nel, p)
    M, K, Wm = mass(kn, p), stiffness(kn, p), advection(kn, p)
    i = n_basis(kn, p) // 2
    sl = slice(i - p, i + p + 1)
    assert np.allclose(M[i, sl] / h, [float(v) for v in mass_stencil(p)], rtol=0, atol=1e-14)
    assert np.allclose(K[i, sl] * h, [float(v) for v in stiff_stencil(p)], rtol=0, atol=1e-12)
    assert np.allclose(Wm[i, sl], [float(v) for v in adv_stencil(p)], rtol=0, atol=1e-14)
    if p == 1:   # the textbook values
        assert np.allclose(M[i, sl] / h, [1 / 6, 4 / 6, 1 / 6])
        assert np.allclose(K[i, sl] * h, [-1, 2, -1])


# ---------------------------------------------------------------- tau (eq. 3.5)
def test_tau_p1_is_half_h():
    """p_t = 1: tau_1 = h/2 (closed form; with T-scaled time h is physical)."""
    for T in (1.0, 300.0):
        kn = T * open_uniform_knots(10, 1)
        (kk, q, c), = tau_splines(kn, 1)
        assert q == 0 and np.allclose(c, T / 20.0, rtol=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_tau_interior_closed_form(p):
    """Far from the ends the tau_k are constants fixed by the translation
    invariant interior equations, solved exactly with cardinal B-splines;
    tau_k scales like h^(2k-1)."""
    nel = 64
    h = 1.0 / nel
    taus = tau_splines(open_uniform_knots(nel, p), p)
    exact = interior_tau(p)
    for k, (kk, q, c) in enumerate(taus, start=1):
        mid = c[len(c) // 2 - 2: len(c) // 2 + 2] / h ** (2 * k - 1)
        assert np.allclose(mid, float(exact[k - 1]), rtol=1e-6), (k, mid, exact[k - 1])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tau_makes_time_block_triangular(p):
    """With theta = 1, W_t + sum_k S_k[tau_k] is lower triangular on the full
    time basis (the property the SU term is built for, end of Section 3.1)."""
    kn = 2.0 * open_uniform_knots(13, p)
    taus = tau_splines(kn, p)
    A = advection(kn, p)
    xq, wq, _ = quadrature(kn, p + 1)
    for k, (kk, q, c) in enumerate(taus, start=1):
        Bk = bspline_all(kn, p, xq, k)
        A = A + Bk.T @ ((wq * eval_spline(kk, q, c, xq))[:, None] * Bk)
    assert np.max(np.abs(np.triu(A, 1))) < 1e-11 * np.max(np.abs(A))
    assert np.min(np.diag(A)[1:]) > 0          # the X_t block is invertible


# ---------------------------------------------------------------- evaluators
@pytest.mark.parametrize("d,p,nel", [(1, 2, 5), (2, 3, 3), (3, 2, 2)])
def test_explicit_equals_tensor(d, p, nel):
    """The mode-product evaluator reproduces the explicit sparse Phi (kron of
    1D collocation matrices) for values and all derivative kinds."""
    P = W.tiny(d, p, nel)
    a = SpaceTime(P, mode="explicit")
    b = SpaceTime(P, mode="tensor")
    x = W.random_vector(int(np.prod(a.shape)), 1)
    g = W.random_vector(int(np.prod(a.qshape)), 2)
    for spec in ({}, {d: 1}, {d: p}, {0: 1}, {d - 1: 2}):
        assert np.allclose(a.ev(x, spec), b.ev(x, spec), rtol=1e-13, atol=1e-11)
        assert np.allclose(a.evT(g, spec), b.evT(g, spec), rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("d,p,nel", [(1, 3, 4), (2, 2, 3), (3, 1, 2)])
def test_spacetime_mass_is_measure(d, p, nel):
    """1^T (M_t (x) M_s) 1 = T |Omega| through the full space-time quadrature."""
    P = W.tiny(d, p, nel, T=2.5)
    st = SpaceTime(P)
    one = np.ones(int(np.prod(st.shape)))
    assert abs(one @ st.evT(st.omega * st.ev(one, {}), {}) - 2.5) < 1e-12


def test_assembly_symmetry():
    """M_t (x) K_s and the SU term are symmetric; the dt term is not (Section 3.1.1)."""
    P = W.tiny(2, 2, 3)
    st = SpaceTime(P)
    nq = len(st.omega)
    A0 = st.assemble_J(np.zeros(nq), None)
    Jsu = st.assemble_J(np.zeros(nq), np.full(nq, 0.7)) - A0
    assert abs(Jsu - Jsu.T).max() < 1e-13
    A1 = st.assemble_J(np.full(nq, 2.0), None) - A0          # reaction mass
    assert abs(A1 - A1.T).max() < 1e-14
    assert abs(A0 - A0.T).max() > 1e-3


def test_explicit_apply_matches_assembly():
    """apply_J (quadrature sums) equals the assembled sparse matrix times x."""
    P = W.tiny(2, 3, 3)
    st = SpaceTime(P)
    rng = np.random.default_rng(3)
    nq = len(st.omega)
    cq, tq = rng.uniform(-3, 10, nq), rng.uniform(0, 1, nq)
    x = W.random_vector(P.unknowns, 4)
    assert np.allclose(st.assemble_J(cq, tq) @ x, st.apply_J(x, cq, tq), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- low rank (eq. 3.9)
def test_truncated_svd_eckart_young():
    """||A - A_R||_F <= eps ||A||_F and R is the smallest rank achieving it."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 8)) @ np.diag(2.0 ** -np.arange(8)) @ rng.standard_normal((8, 200))
    for eps in (0.3, 0.1, 1e-2, 1e-4):
        R, U, s, V = truncated_svd(A, eps)
        err = np.linalg.norm(A - U @ np.diag(s) @ V.T)
        assert err <= eps * np.linalg.norm(A) * (1 + 1e-12)
        if R > 0:
            R2, U2, s2, V2 = R - 1, U[:, :-1], s[:-1], V[:, :-1]
            assert np.linalg.norm(A - U2 @ np.diag(s2) @ V2.T) > eps * np.linalg.norm(A)
    assert truncated_svd(np.zeros((3, 4)), 0.1)[0] == 0


def test_hat_interpolation():
    """Piecewise-linear interpolation reproduces linear functions and sums to 1;
    constant extension below the first node."""
    nodes = np.array([0.1, 0.3, 0.35, 0.8, 1.0])
    x = np.linspace(0, 1, 57)
    H = hat_matrix(nodes, x)
    assert np.allclose(H.sum(1), 1.0)
    f = 2.0 * nodes - 0.5
    inside = x >= 0.1
    assert np.allclose((H @ f)[inside], 2.0 * x[inside] - 0.5)
    assert np.allclose((H @ f)[~inside], f[0])


# ---------------------------------------------------------------- theta (eq. 3.6)
def test_theta_bruteforce_windows():
    """Theta entries recomputed by brute force: residual at the Gauss points whose
    coordinates lie inside the support extension (eq. (2.3)), max, normalised."""
    P = W.tiny(2, 2, 4)
    st = SpaceTime(P)
    u, w = W.smooth_state(P, 7)
    Th = st.theta_grid(u, w)
    d = st.d
    from oracle.spacetime import ionic_current
    uq, wq, utq = st.ev(u, {}), st.ev(w, {}), st.ev(u, {d: 1})
    R = P.Cm * utq + ionic_current(uq, wq, P)
    for l in range(d):
        R -= P.sigma[l] * st.ev(u, {l: 2})
    den = P.Cm * (np.abs(uq).max() / P.T + np.abs(utq).max())
    grids = np.meshgrid(st.quad[2][0], st.quad[1][0], st.quad[0][0], indexing="ij")
    coords = [g.reshape(-1) for g in grids]          # t, x2, x1

    def window(l, j):          # 1-based paper formula with j 1-based
        kn, p = st.kn[l], st.p[l]
        lo = kn[max(j - p, 1) - 1]
        hi = kn[min(j + p + 1, len(kn)) - 1]
        return lo, hi

    rng = np.random.default_rng(0)
    for _ in range(25):
        it = rng.integers(0, st.n[2] - 1)
        i2, i1 = rng.integers(0, st.n[1]), rng.integers(0, st.n[0])
        (t0, t1), (a0, a1), (b0, b1) = window(2, it + 2), window(1, i2 + 1), window(0, i1 + 1)
        m = ((coords[0] > t0) & (coords[0] < t1) & (coords[1] > a0) & (coords[1] < a1)
             & (coords[2] > b0) & (coords[2] < b1))
        want = min(np.abs(R[m]).max() / den, 1.0)
        assert Th[it, i2 * st.n[0] + i1] == pytest.approx(want, rel=1e-14)


def test_theta_zero_state():
    """u = w = 0, f = 0: residual vanishes, Theta = 0 (denominator 0 reading)."""
    P = W.tiny(1, 2, 6, u0_kind=0)
    st = SpaceTime(P)
    z = np.zeros(int(np.prod(st.shape)))
    assert np.all(st.theta_grid(z, z) == 0.0)


# ---------------------------------------------------------------- w update (Section 3.2)
@pytest.mark.parametrize("d,p", [(1, 2), (2, 3), (3, 1)])
def test_w_explicit_equals_kron(d, p):
    """Explicit sparse L-solve equals the Kronecker formula with M_s cancelled."""
    P = W.tiny(d, p, 3)
    st = SpaceTime(P)
    u, _ = W.smooth_state(P, 2)
    assert np.allclose(st.w_update_explicit(u), st.w_update_kron(u), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- whole solves
def test_zero_datum_gives_zero():
    """u0 = 0, f = 0: u = w = 0 exactly (I_ion(0, 0) = 0)."""
    P = W.tiny(2, 2, 3, u0_kind=0)
    st = SpaceTime(P)
    u, w, log = solver.solve(st, max_outer=3)
    assert np.all(u == 0.0) and np.all(w == 0.0)


def _rk4(P, u0, T, n):
    f = lambda y: np.array([-(P.c1 * y[0] * (y[0] - P.a) * (y[0] - 1) + P.c2 * y[0] * y[1]) / P.Cm,
                            P.b * (y[0] - P.de * y[1])])
    h = T / n
    ts, ys = [0.0], [np.array([u0, 0.0])]
    y = ys[0]
    for k in range(n):
        k1 = f(y); k2 = f(y + h / 2 * k1); k3 = f(y + h / 2 * k2); k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        ys.append(y)
    return np.array(ys)


@pytest.mark.parametrize("su", [False, True])
def test_constant_datum_is_rm_ode(su):
    """Spatially constant u0: u_h is constant in x (K_s 1 = 0) and follows the RM
    ODE of eq. (3.1); against RK4 (dt = 1e-5) the L2-in-time error of the
    space-time Galerkin solution decays at order p+1 without SU and still
    decays with SU."""
    p = 2
    errs = []
    ref = _rk4(W.tiny(1, p, 2), 0.5, 1.0, 100000)
    tref = np.linspace(0, 1, 100001)
    for nel_t in (8, 16, 32):
        P = W.tiny(1, p, 2, nel_t=nel_t, u0_kind=1, u0_center=(5.0, 0, 0), u0_value=0.5)
        st = SpaceTime(P, su=su)
        u, w, log = solver.solve(st, tol=1e-12, max_outer=40)
        U = u.reshape(st.shape)
        assert np.max(np.abs(U - U[:, :1])) < 1e-10
        tq, wq, _ = quadrature(st.kn[1], p + 3)
        uh = bspline_all(st.kn[1], p, tq) @ U[:, 0]
        ue = np.interp(tq, tref, ref[:, 0])
        errs.append(np.sqrt(np.sum(wq * (uh - ue) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    if su:
        assert errs[2] < errs[1] < errs[0]
    else:
        assert np.all(rates > p + 1 - 0.4), (errs, rates)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("su", [False, True])
def test_manufactured_solution_rate(p, su):
    """Section 4.1: u_ex = 10 sin(pi x) sin(pi t)(1-e^-x)(1-e^(x-1))(1-e^(t-1)),
    C_m = 1, D = 1e-4, linear heat variant (c1 = c2 = 0), h_1 = h_t: the L2
    error of the Galerkin solution decays at the optimal order p+1.  With SU,
    theta is evaluated once at the Galerkin solution (theta = O(h^p) there) and
    the SU solution keeps the optimal order."""
    import sympy as sy
    import scipy.sparse.linalg as spla
    X, Tt = sy.symbols("x t")
    ue = 10 * sy.sin(sy.pi * X) * sy.sin(sy.pi * Tt) * (1 - sy.exp(-X)) * (1 - sy.exp(X - 1)) * (1 - sy.exp(Tt - 1))
    D = 1e-4
    fe = sy.lambdify((X, Tt), sy.diff(ue, Tt) - D * sy.diff(ue, X, 2), "numpy")
    ul = sy.lambdify((X, Tt), ue, "numpy")
    errs = []
    for nel in (4, 8, 16):
        P = W.tiny(1, p, nel, u0_kind=0, c1=0.0, c2=0.0, sigma=(D,))
        f = lambda xs, t: fe(xs[0], t)
        u, w, log = solver.solve(SpaceTime(P, su=False, f=f), tol=1e-12, max_outer=30)
        if su:
            st = SpaceTime(P, su=True, f=f)
            thq = st.lowrank_at_quad(st.lowrank(st.theta_grid(u, w), 0.1))
            J = st.assemble_J(np.zeros_like(thq), thq)
            u = u + st.full(-spla.splu(J.tocsc()).solve(st.residual(u, w, thq)))
        xq, xw, _ = quadrature(open_uniform_knots(nel, p), p + 3)
        tq, tw, _ = quadrature(open_uniform_knots(nel, p), p + 3)
        uh = bspline_all(open_uniform_knots(nel, p), p, tq) @ u.reshape(nel + p, nel + p) @ \
            bspline_all(open_uniform_knots(nel, p), p, xq).T
        ex = ul(xq[None, :], tq[:, None])
        errs.append(np.sqrt(np.sum(np.outer(tw, xw) * (uh - ex) ** 2) / np.sum(np.outer(tw, xw) * ex ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.35, (errs, rates)


def test_newton_and_picard_same_fixed_point():
    """With theta fixed, the Newton (alpha = 1) and Picard (C_r, alpha = 0.5,
    Section 3.1) iterations converge to the same discrete solution."""
    P = W.config(0)
    st = SpaceTime(P)
    u0 = np.tile(st.lift(), st.n[1])
    w0 = st.w_update_explicit(u0)
    th = st.lowrank(st.theta_grid(u0, w0), 0.1)
    import oracle.solver as S
    orig = S.linearize

    def frozen(st_, u, w, eps_theta=0.1, eps_react=1e-2, newton=True, theta_lr=None):
        return orig(st_, u, w, eps_theta, eps_react, newton, th)
    S.linearize = frozen
    try:
        un, _, ln = S.solve(st, newton=True, tol=1e-12, max_outer=60)
        up, _, lp = S.solve(st, newton=False, tol=1e-12, max_outer=400)
    finally:
        S.linearize = orig
    assert ln.deltas[-1] <= 1e-12 and lp.deltas[-1] <= 1e-12
    assert np.max(np.abs(un - up)) < 1e-10


def test_stimulus_greville_counts():
    """Integer pin: spatial Greville points inside the stimulus, counted
    directly from the uniform-knot Greville formula (gamma_i = mean of p
    consecutive interior knots)."""
    def direct(nel, p, d, r):
        kn = [0.0] * (p + 1) + [k / nel for k in range(1, nel)] + [1.0] * (p + 1)
        g = np.array([sum(kn[i + 1: i + p + 1]) / p for i in range(nel + p)])
        if d == 1:
            return int(np.sum(g < 0.1))
        G = np.meshgrid(*([g] * d), indexing="ij")
        return int(np.sum(sum(x ** 2 for x in G) <= r * r))
    for idx, d, p, nel in ((0, 1, 2, 32), (1, 2, 3, 64), (2, 3, 2, 48)):
        P = W.config(idx)
        st = SpaceTime(P, mode="tensor")
        assert int(np.sum(st.lift() > 0)) == direct(nel, p, d, 0.1)


@pytest.mark.parametrize("d,p,nel", [(1, 2, 6), (2, 3, 4), (3, 2, 3)])
def test_rowsample_matches_full_apply(d, p, nel):
    """The row-sampled local-quadrature evaluator equals the full-grid one."""
    from oracle.rowsample import RowSampler
    P = W.tiny(d, p, nel)
    st = SpaceTime(P, mode="tensor")
    ft, fc = W.random_factors(P, 2, 1), W.random_factors(P, 3, 2, scale=4.0)
    x = W.random_vector(P.unknowns, 3)
    full = st.apply_J(x, st.lowrank_at_quad(LowRank(*fc)), st.lowrank_at_quad(LowRank(*ft)))
    rows = np.random.default_rng(0).choice(P.unknowns, 25, replace=False)
    rs = RowSampler(P)
    got = rs.apply_rows(x, rows, theta=ft, coef=fc)
    assert np.allclose(got, full[rows], rtol=1e-12, atol=1e-12 * np.abs(full).max())
    # constant reaction, no SU: the preconditioner operator
    Ahat = st.assemble_precond() @ x
    got = rs.apply_rows(x, rows, coef_const=P.a * P.c1)
    assert np.allclose(got, Ahat[rows], rtol=1e-12, atol=1e-12 * np.abs(Ahat).max())


@pytest.mark.parametrize("d,p,nel,with_f", [(1, 2, 6, False), (2, 3, 4, True), (3, 2, 3, False)])
def test_rowsample_residual_matches_full(d, p, nel, with_f):
    """Row-sampled residual N(u) (exact ionic current, optional source) equals
    the full-grid one."""
    from oracle.rowsample import RowSampler
    P = W.tiny(d, p, nel)
    f = (lambda xs, t: np.exp(-20.0 * sum((x - 0.3) ** 2 for x in xs)) * (t > 0.2)) if with_f else None
    st = SpaceTime(P, mode="tensor", f=f)
    ft = W.random_factors(P, 2, 1)
    u, w = W.smooth_state(P, 4)
    full = st.residual(u, w, st.lowrank_at_quad(LowRank(*ft)))
    rows = np.random.default_rng(0).choice(P.unknowns, 25, replace=False)
    got = RowSampler(P).residual_rows(u, w, rows, theta=ft, f=f)
    assert np.allclose(got, full[rows], rtol=1e-12, atol=1e-12 * np.abs(full).max())


# ---------------------------------------------------------------- source term (eq. (3.1), Section 4 stimuli)
def test_source_residual_total():
    """u = w = 0 and f = amp on the whole space-time domain: the residual
    -int f v summed over the test functions of X_h is -amp |Omega| (T -
    int b_1), with int b_1 = T h_t / (p + 1) for the first B-spline of an open
    uniform time knot vector (partition of unity, closed form)."""
    for d, p in ((1, 2), (2, 3), (3, 2)):
        P = W.tiny(d, p, 3, nel_t=5, T=2.0, u0_kind=0, f_kind=1, f_center=(0.5, 0.5, 0.5), f_radius=10.0,
                   f_t0=0.0, f_t1=2.0, f_amp=0.7)
        st = SpaceTime(P)
        z = np.zeros(int(np.prod(st.shape)))
        r = st.residual(z, z, None)
        want = -0.7 * 1.0 * (P.T - P.T * (1.0 / P.nel_t) / (P.p_t + 1))
        assert r.sum() == pytest.approx(want, rel=1e-13)


def test_source_theta_indicator():
    """u = w = 0 with a localized source: R = -f, the denominator of eq. (3.6)
    is 0, so Theta is 1 exactly on the windows that contain a Gauss point with
    f != 0 and 0 elsewhere (brute force over point coordinates)."""
    P = W.tiny(2, 2, 6, nel_t=6, u0_kind=0, f_kind=1, f_center=(0.2, 0.7, 0.0), f_radius=0.15,
               f_t0=0.3, f_t1=0.5, f_amp=1.0)
    st = SpaceTime(P)
    z = np.zeros(int(np.prod(st.shape)))
    Th = st.theta_grid(z, z)
    assert set(np.unique(Th)) <= {0.0, 1.0} and Th.max() == 1.0 and Th.min() == 0.0
    grids = np.meshgrid(st.quad[2][0], st.quad[1][0], st.quad[0][0], indexing="ij")
    fq = P.source([grids[2], grids[1]], grids[0])

    def window(l, j):
        kn, p = st.kn[l], st.p[l]
        return kn[max(j - p, 1) - 1], kn[min(j + p + 1, len(kn)) - 1]
    for it in range(st.n[2] - 1):
        for i2 in range(st.n[1]):
            for i1 in range(st.n[0]):
                (t0, t1), (a0, a1), (b0, b1) = window(2, it + 2), window(1, i2 + 1), window(0, i1 + 1)
                m = ((grids[0] > t0) & (grids[0] < t1) & (grids[1] > a0) & (grids[1] < a1)
                     & (grids[2] > b0) & (grids[2] < b1))
                assert Th[it, i2 * st.n[0] + i1] == (1.0 if np.any(fq[m] != 0) else 0.0)


def test_clustered_time_knots():
    """p+1 distinct knots around each event, the rest evenly spaced, open and
    of the requested element count (the graded partition of Section 4.2.1)."""
    for p in (2, 3):
        kn = W.clustered_time_knots(24, p, [0.3, 0.6], 0.01)
        assert len(kn) == 24 + 2 * p + 1
        inner = kn[p + 1:-p - 1]
        assert np.all(np.diff(inner) > 0)
        for te in (0.3, 0.6):
            assert np.sum(np.abs(inner - te) <= 0.5 * p * 0.01 + 1e-12) == p + 1


# ---------------------------------------------------------------- fixed-point scheme of Section 3.1
def test_picard_defect_identity():
    """A(u^k, w^k) u^k - F = N(u^k) on the test functions of X_h: with the exact
    C_r of eq. (3.8) in M_R, C_r(u, w) u = I_ion(u, w) at every Gauss point, so
    the fixed-point matrix applied to its own linearization point reproduces
    the residual (the defect form the library solves)."""
    P = W.tiny(2, 2, 4, nel_t=5, f_kind=1, f_center=(0.2, 0.3, 0.0), f_radius=0.3, f_t0=0.2, f_t1=0.6,
               f_amp=1.5)
    st = SpaceTime(P)
    u, w = W.smooth_state(P, 3)
    thq = st.lowrank_at_quad(st.lowrank(st.theta_grid(u, w), 0.1))
    A = st.assemble_full(st.reaction_at_quad(u, w), thq)
    N_s = P.N_s
    lhs = (A @ u - st.load_vector())[N_s:]
    r = st.residual(u, w, thq)
    assert np.max(np.abs(lhs - r)) <= 1e-13 * np.max(np.abs(r))


def test_paper_picard_reaches_newton_solution():
    """The literal fixed-point scheme (exact C_r, u and w relaxed with
    alpha = 0.5) and Newton with lagged w reach the same discrete solution
    when theta is held fixed (same fixed point, different iterations)."""
    P = W.config(0)
    st = SpaceTime(P)
    u0 = np.tile(st.lift(), st.n[1])
    th = st.lowrank(st.theta_grid(u0, st.w_update_explicit(u0)), 0.1)
    up, wp, lp = solver.solve_picard(st, tol=1e-12, max_outer=400, theta_lr=th)
    import oracle.solver as S
    orig = S.linearize

    def frozen(st_, u, w, eps_theta=0.1, eps_react=1e-2, newton=True, theta_lr=None):
        return orig(st_, u, w, eps_theta, eps_react, newton, th)
    S.linearize = frozen
    try:
        un, wn, ln = S.solve(st, newton=True, tol=1e-12, max_outer=60)
    finally:
        S.linearize = orig
    assert lp.deltas[-1] <= 1e-12 and ln.deltas[-1] <= 1e-12
    assert np.max(np.abs(un - up)) < 1e-10
    assert np.max(np.abs(wn - wp)) < 1e-10


# ---------------------------------------------------------------- separable geometry (Section 2, map G = (F, T tau))
MAPS = [(1, (0.2, 1.7, 0.0)), (2, (-0.5, 1.0, 2.5)), (2, (0.0, 2.0, -1.7))]


@pytest.mark.parametrize("kind,param", MAPS)
def test_geometry_derivatives_by_differences(kind, param):
    """Physical first and second derivatives of a spline at the mapped Gauss
    points against central differences in x through the inverse map
    (bisection), for random coefficients."""
    P = W.tiny(1, 3, 5, map_kind=(kind, 0, 0), map_param=(param,) * 3)
    st = SpaceTime(P)
    a, b, k = param
    rng = np.random.default_rng(kind)
    c = rng.standard_normal(st.n[0])
    kn = st.kn[0]

    def F(e):
        return a + (b - a) * e if kind == 1 else a + (b - a) * np.expm1(k * e) / np.expm1(k)

    def Finv(x):
        lo, hi = np.zeros_like(x), np.ones_like(x)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            go = F(mid) < x
            lo, hi = np.where(go, mid, lo), np.where(go, hi, mid)
        return 0.5 * (lo + hi)

    def g(x):
        return bspline_all(kn, 3, Finv(x)) @ c
    xq = st.quad[0][0]
    h1, h2 = 1e-6 * (b - a), 1e-4 * (b - a)
    d1 = (g(xq + h1) - g(xq - h1)) / (2 * h1)
    d2 = (g(xq + h2) - 2 * g(xq) + g(xq - h2)) / h2 ** 2
    assert np.max(np.abs(st.E[0][1] @ c - d1)) < 1e-6 * max(1.0, np.max(np.abs(d1)))
    assert np.max(np.abs(st.E[0][2] @ c - d2)) < 1e-3 * max(1.0, np.max(np.abs(d2)))
    # mapped Gauss points and Greville abscissae
    assert np.allclose(xq, F(quadrature(kn, 4)[0]), rtol=0, atol=1e-14)
    assert np.allclose(st.grev_phys[0], F(greville(kn, 3)), rtol=0, atol=1e-14)


def test_geometry_measure():
    """Space-time mass = |Omega| T with |Omega| the physical measure of the
    mapped box (exact for the affine direction; for the graded one the Gauss
    rule integrates F' = c e^{k eta} with an error that vanishes as the rule
    grows); K 1 = 0 in every direction."""
    mp = ((0.2, 1.7, 0.0), (-0.5, 1.0, 2.5), (0, 1, 0))
    for extra, tol in ((0, 1e-6), (4, 1e-13)):
        P = W.tiny(2, 2, 4, nel_t=3, T=1.5, map_kind=(1, 2, 0), map_param=mp)
        st = SpaceTime(P, nq_extra=extra)
        one = np.ones(int(np.prod(st.shape)))
        assert np.sum(st.evT(st.omega * st.ev(one, {}), {})) == pytest.approx(1.5 * 1.5 * 1.5, rel=tol)
    for l in range(2):
        assert np.max(np.abs(st.ev(one, {l: 1}))) < 1e-12
        assert np.max(np.abs(st.ev(one, {l: 2}))) < 1e-10


@pytest.mark.parametrize("p", [2, 3])
def test_geometry_manufactured_rate(p):
    """Linear heat equation on a graded interval x = F(eta) in [0.2, 1.7]
    (exponential grading, k = 2.5) with sigma = 0.05 and the manufactured
    u = cos(pi (x - a)/(b - a)) sin(pi t) (Neumann at both ends, zero at
    t = 0): the physical L2 error of the Galerkin solution decays at order
    p + 1 under uniform parametric refinement."""
    import sympy as sy
    a, b, k = 0.2, 1.7, 2.5
    X, Tt = sy.symbols("x t")
    ue = sy.cos(sy.pi * (X - a) / (b - a)) * sy.sin(sy.pi * Tt)
    D = 0.05
    fe = sy.lambdify((X, Tt), sy.diff(ue, Tt) - D * sy.diff(ue, X, 2), "numpy")
    ul = sy.lambdify((X, Tt), ue, "numpy")
    errs = []
    for nel in (4, 8, 16):
        P = W.tiny(1, p, nel, u0_kind=0, c1=0.0, c2=0.0, sigma=(D,), map_kind=(2, 0, 0),
                   map_param=((a, b, k),) * 3)
        f = lambda xs, t: fe(xs[0], t)
        st = SpaceTime(P, su=False, f=f, nq_extra=2)
        u, w, log = solver.solve(st, tol=1e-12, max_outer=30)
        uh = (st.E[1][0] @ u.reshape(st.n[1], st.n[0]) @ st.E[0][0].T)
        ex = ul(st.quad[0][0][None, :], st.quad[1][0][:, None])
        wt = np.outer(st.quad[1][1], st.quad[0][1])
        errs.append(np.sqrt(np.sum(wt * (uh - ex) ** 2) / np.sum(wt * ex ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.35, (errs, rates)


# ------------------------------------------------ banded preconditioner (not from the paper)
def test_banded_precond_reduces_to_fast_diagonalization_operator():
    """With c = a c1 and no theta the banded preconditioner's form is A-hat of
    Section 3.2 (assembled independently by assemble_precond)."""
    P = W.tiny(2, 2, 5, nel_t=5)
    st = SpaceTime(P)
    Qt = st.qshape[0]
    A = st.assemble_precond_profiles(np.full(Qt, P.a * P.c1), np.zeros(Qt))
    B = st.assemble_precond()
    assert abs(A - B).max() <= 1e-13 * abs(B).max()


@pytest.mark.parametrize("d", [1, 2])
def test_banded_precond_is_kronecker(d):
    """A_t (x) M_s + M_t (x) K_s with the time matrix built from SciPy's
    B-spline basis and the oracle's tau_k at the time Gauss points:
    A_t = C_m W_t + int c b b + C_m sum_k int tau_k th b^(k) b^(k)."""
    from scipy.interpolate import BSpline
    P = W.tiny(d, 3, 4, nel_t=5)
    kn = P.uniform_knots()
    st = SpaceTime(P, knots=kn)
    Qt = st.qshape[0]
    rng = np.random.default_rng(d + 7)
    c_t, th_t = rng.uniform(0.0, 2.0, Qt), rng.uniform(0.0, 0.8, Qt)
    A = st.assemble_precond_profiles(c_t, th_t).toarray()

    def basis(kv, p, x, der):
        n = len(kv) - p - 1
        B = BSpline(kv, np.eye(n), p, extrapolate=False)
        return np.nan_to_num((B.derivative(der) if der else B)(x))

    Tk = P.T * np.asarray(kn[d])
    tq, tw, _ = st.quad[d]
    g = lambda wt, X, Y: X.T @ (wt[:, None] * Y)
    b = [basis(Tk, P.p_t, tq, k) for k in range(P.p_t + 1)]
    At = P.Cm * g(tw, b[0], b[1]) + g(tw * c_t, b[0], b[0])
    for k in range(1, P.p_t + 1):
        At = At + g(tw * np.maximum(P.Cm * st.tau_q[k - 1] * th_t, 0.0), b[k], b[k])
    Mt = g(tw, b[0], b[0])
    Ms, Ks = [], []
    for l in range(d):
        z = np.unique(kn[l])
        gg, ww = np.polynomial.legendre.leggauss(P.p_s + 2)
        x = np.concatenate([0.5 * (a0 + a1) + 0.5 * (a1 - a0) * gg for a0, a1 in zip(z[:-1], z[1:])])
        w = np.concatenate([0.5 * (a1 - a0) * ww for a0, a1 in zip(z[:-1], z[1:])])
        B0, B1 = basis(kn[l], P.p_s, x, 0), basis(kn[l], P.p_s, x, 1)
        Ms.append(g(w, B0, B0))
        Ks.append(g(w, B1, B1))
    if d == 1:
        M, K = Ms[0], P.sigma[0] * Ks[0]
    else:
        M = np.kron(Ms[1], Ms[0])
        K = P.sigma[0] * np.kron(Ms[1], Ks[0]) + P.sigma[1] * np.kron(Ks[1], Ms[0])
    want = np.kron(At[1:, 1:], M) + np.kron(Mt[1:, 1:], K)
    assert np.max(np.abs(A - want)) <= 1e-12 * np.max(np.abs(want))
