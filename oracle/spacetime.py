"""Space-time Galerkin + Spline Upwind discretisation (paper Sections 2-3).
Test infrastructure (see package doc).

Layout: a space-time coefficient vector on the full basis has shape
(n_t, n_d, ..., n_1) in C order, i.e. x_1 fastest and time slowest (the
colexicographic order of Section 2).  Time layer 0 is the first B-spline in
time, the only one that is non-zero at t = 0; the unknowns are layers
1..n_t-1 (the space X_h with the initial condition, N_t = n_t - 1).

Every quantity is an integral evaluated by (p+1)-point Gauss quadrature on
each space-time element.  Two interchangeable evaluators are provided:
``explicit`` builds the sparse matrix Phi of basis values at all tensor Gauss
points (a Kronecker product of the 1D collocation matrices: a tensor-product
B-spline is the product of its univariate factors) and assembles the explicit
sparse space-time matrices Phi_i^T diag(omega * coef) Phi_j; ``tensor``
evaluates the same sums with 1D contractions along each axis (for sizes where
Phi would not fit).  Tests pin one against the other on small grids.

Readings taken here (the paper is silent or ambiguous):
* Initial datum (eq. (3.1) has u = 0 at t = 0 plus a source; the workloads
  use an indicator initial datum and no source): the datum is lifted into time
  layer 0 with coefficients u0(gamma_i) sampled at the spatial Greville points.
* theta (eq. (3.6)): the L-infinity norms are maxima of |.| over the Gauss
  points of the elements inside the window; the window of the full-basis
  function j (0-based) in a direction is (xi_{j-p}, xi_{j+p+1}) in the paper's
  1-based knot indexing (eq. (2.3)) with indices clamped to the knot vector;
  time functions of X_t are full indices 1..n_t-1.  If the denominator is 0,
  Theta = 1 where the numerator is positive, else 0.
* theta is min(..., 1) on the Greville grid, then low-ranked; the low-rank
  interpolant is not clipped again.  Interpolation in time uses the Greville
  points of X_t; below the first of them it is extended by a constant.
* The low rank (eq. (3.9)) is the truncated SVD with the smallest R such that
  the Frobenius tail is <= eps times the norm (a deterministic stand-in for a
  randomized sketch: the same tolerance, a unique answer).
* Outer loop: defect correction u <- u + alpha*delta with
  (A_lin + M[c~]) delta = -N(u), N the full residual with the exact ionic
  current at the Gauss points.  Newton: c = dI_ion/du, alpha = 1.  Picard
  (Section 3.1): c = C_r of eq. (3.8), alpha = 0.5.  c is sampled on the
  Greville grid and low-ranked like theta.  w is lagged: w^k solves the
  L-system of Section 3.1.1 with u^k.  theta is refreshed while
  ||delta||_inf > theta_freeze and then kept fixed.
* The FD preconditioner of Section 3.2 uses sigma-scaled stiffness matrices
  (the paper's parametric version has unit diffusion).
* SUPG + shock capturing (Section 4.2.2): h in h/(2p+1) and c h^2/4 is the
  length of the time element (the streamline direction of the space-time
  operator is time), in physical time units; the diffusion part of the SUPG
  term is the strong form -sum_l sigma_l u_ll at the Gauss points, as the
  residual is written; C_r and the residual ratio of S_SC are taken exactly at
  the Gauss points (the paper low-ranks both to make assembly cheaper); the
  ratio is not capped and is zero when its denominator vanishes (u = 0).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators1d import eval_spline, tau_splines
from .splines import bspline_all, breakpoints, greville, n_basis, quadrature


def ionic_current(u, w, P):
    """I_ion = c1 u (u-a)(u-1) + c2 u w (eq. (3.1))."""
    return P.c1 * u * (u - P.a) * (u - 1.0) + P.c2 * u * w


def ionic_du(u, w, P):
    """dI_ion/du = c1 (3u^2 - 2(1+a)u + a) + c2 w."""
    return P.c1 * (3.0 * u * u - 2.0 * (1.0 + P.a) * u + P.a) + P.c2 * w


def reaction_coefficient(u, w, P):
    """C_r = c1 (u-a)(u-1) + c2 w (eq. (3.8)), the fixed-point reaction coefficient."""
    return P.c1 * (u - P.a) * (u - 1.0) + P.c2 * w


def geometry_map(prob, l):
    """Spatial map x = F(eta) of direction l (Section 2: the spatial part of
    G = (F, T tau), here separable) as a function returning (F, F', F'')
    at parametric points, or None for the identity.  Kinds: 1 affine
    a + (b - a) eta; 2 exponential grading a + (b - a) (e^{k eta} - 1) / (e^k - 1)."""
    kind = getattr(prob, "map_kind", (0, 0, 0))[l]
    if kind == 0:
        return None
    a, b, k = prob.map_param[l]
    if kind == 1:
        return lambda e: (a + (b - a) * e, np.full_like(e, b - a), np.zeros_like(e))

    def graded(e):
        d1 = (b - a) * k * np.exp(k * e) / np.expm1(k)
        return a + (b - a) * np.expm1(k * e) / np.expm1(k), d1, k * d1
    return graded


def truncated_svd(A: np.ndarray, eps: float, max_rank: int = None):
    """Smallest-rank R with ||A - U S V^T||_F <= eps ||A||_F (eq. (3.9)).
    The tolerance alone fixes R; a caller that can only hold max_rank terms
    gets a ValueError when R exceeds it (the tolerance is never missed
    silently)."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    tot = float(np.sum(s * s))
    if tot == 0.0:
        return 0, U[:, :0], s[:0], Vt[:0].T
    tail = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])  # tail[R] = sum_{k>=R} s_k^2
    R = int(np.argmax(tail <= eps * eps * tot))
    if max_rank is not None and R > max_rank:
        raise ValueError(f"truncated SVD needs rank {R} > cap {max_rank} for eps = {eps}")
    return R, U[:, :R], s[:R], Vt[:R].T


def hat_matrix(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """H[q, g] = value at x_q of the piecewise-linear interpolant of e_g on nodes
    (constant extension outside the node range)."""
    return np.stack([np.interp(x, nodes, e) for e in np.eye(len(nodes))], axis=1)


@dataclasses.dataclass
class LowRank:
    """c(x, t) ~ sum_r s_r phi_r(t) psi_r(x): U (N_t x R), s (R), V (N_s x R) on the Greville grid."""
    U: np.ndarray
    s: np.ndarray
    V: np.ndarray

    @property
    def R(self):
        return len(self.s)


class SpaceTime:
    """Discrete space-time problem of one workload (see module doc)."""

    def __init__(self, prob, knots: Optional[List[np.ndarray]] = None, mode: str = "explicit",
                 nq_extra: int = 0, su: bool = True, f: Optional[Callable] = None, supg: bool = False,
                 sc_c: float = 0.0):
        self.P = prob
        d = prob.d
        self.d = d
        kn = knots if knots is not None else prob.uniform_knots()
        self.kn = [np.asarray(k, dtype=np.float64) for k in kn[:d]] + [prob.T * np.asarray(kn[d], dtype=np.float64)]
        self.p = [prob.p_s] * d + [prob.p_t]
        self.n = [n_basis(k, p) for k, p in zip(self.kn, self.p)]
        self.mode = mode
        if su and supg:
            raise ValueError("the Spline Upwind and the SUPG + shock-capturing terms are alternatives")
        self.su = su
        # SUPG + shock capturing (Section 4.2.2), for splines of any regularity in time
        self.supg = supg
        self.sc_c = float(sc_c)
        # the source of eq. (3.1): given explicitly, or the problem's own
        self.f = f if f is not None else (prob.source if getattr(prob, "f_kind", 0) else None)
        # axis a of an array (time first): a = 0 is time, a = 1 is x_d, ..., a = d is x_1
        self.dirs = [d] + list(range(d - 1, -1, -1))      # direction index of each axis
        self.quad = [quadrature(k, p + 1 + nq_extra) for k, p in zip(self.kn, self.p)]
        maxder = [2] * d + [prob.p_t]
        self.E = [[bspline_all(self.kn[l], self.p[l], self.quad[l][0], k) for k in range(maxder[l] + 1)]
                  for l in range(d + 1)]
        # separable geometry: physical Gauss points and weights (w F'), and
        # physical derivatives d/dx = (1/F') d/deta,
        # d2/dx2 = (1/F'^2) d2/deta2 - (F''/F'^3) d/deta
        self.maps = [geometry_map(prob, l) for l in range(d)]
        self.grev_phys = []
        for l in range(d):
            mp = self.maps[l]
            eta, w, el = self.quad[l]
            g = greville(self.kn[l], self.p[l])
            if mp is None:
                self.grev_phys.append(g)
                continue
            F, F1, F2 = mp(eta)
            E0, E1, E2 = self.E[l]
            self.E[l] = [E0, E1 / F1[:, None], E2 / (F1 ** 2)[:, None] - (F2 / F1 ** 3)[:, None] * E1]
            self.quad[l] = (F, w * F1, el)
            self.grev_phys.append(mp(g)[0])
        self.omega = self._outer([self.quad[l][1] for l in range(d + 1)])
        tq = self.quad[d][0]
        # the tau_k splines of the SU term need C^{p-1} time splines: built for SU only
        self.taus = tau_splines(self.kn[d], prob.p_t, prob.p_t + 1 + nq_extra) if su else None
        self.tau_q = [eval_spline(kk, q, c, tq) for kk, q, c in self.taus] if su else None
        # SUPG parameter h/(2 p_t + 1) and shock-capturing scale c h^2/4 at the
        # time Gauss points, h the length of the time element holding the point
        ht = np.diff(breakpoints(self.kn[d]))[self.quad[d][2]]
        self.supg_tau_t = ht / (2 * prob.p_t + 1)
        self.sc_scale_t = self.sc_c * ht * ht / 4.0
        self.grev_s = [greville(self.kn[l], self.p[l]) for l in range(d)]
        self.grev_t = greville(self.kn[d], self.p[d])[1:]          # X_t Greville points
        self.Ht = hat_matrix(self.grev_t, tq)
        # theta's interpolation at the Greville abscissae mapped to the physical domain
        self.Hs = [hat_matrix(self.grev_phys[l], self.quad[l][0]) for l in range(d)]
        self.shape = tuple([self.n[d]] + [self.n[l] for l in range(d - 1, -1, -1)])
        self.qshape = tuple([len(self.quad[d][0])] + [len(self.quad[l][0]) for l in range(d - 1, -1, -1)])
        self._phi = {}

    # ------------------------------------------------------------------ helpers
    def _outer(self, vecs_by_dir):
        """Tensor (outer) product arranged [time][x_d]...[x_1], flattened."""
        out = np.array([1.0])
        for a in range(self.d + 1):
            out = np.multiply.outer(out, vecs_by_dir[self.dirs[a]])
        return out.reshape(-1)

    def _ders(self, spec):
        """spec maps direction -> derivative order; returns per-direction matrices."""
        return [self.E[l][spec.get(l, 0)] for l in range(self.d + 1)]

    def phi(self, spec) -> sp.csr_matrix:
        """Sparse matrix of the requested derivative of every space-time basis
        function at every tensor Gauss point (Kronecker product of 1D ones)."""
        key = tuple(sorted(spec.items()))
        if key not in self._phi:
            mats = self._ders(spec)
            M = sp.csr_matrix(mats[self.dirs[0]])
            for a in range(1, self.d + 1):
                M = sp.kron(M, sp.csr_matrix(mats[self.dirs[a]]), format="csr")
            M.eliminate_zeros()
            self._phi[key] = M
        return self._phi[key]

    def ev(self, x_full: np.ndarray, spec) -> np.ndarray:
        """Values at all tensor Gauss points of the spline with coefficients x_full."""
        if self.mode == "explicit":
            return self.phi(spec) @ x_full
        X = x_full.reshape(self.shape)
        mats = self._ders(spec)
        for a in range(self.d + 1):
            X = np.moveaxis(np.tensordot(mats[self.dirs[a]], X, axes=([1], [a])), 0, a)
        return X.reshape(-1)

    def evT(self, g: np.ndarray, spec) -> np.ndarray:
        """Transpose of ev: sum over Gauss points of g times the basis derivative."""
        if self.mode == "explicit":
            return self.phi(spec).T @ g
        G = g.reshape(self.qshape)
        mats = self._ders(spec)
        for a in range(self.d + 1):
            G = np.moveaxis(np.tensordot(mats[self.dirs[a]].T, G, axes=([1], [a])), 0, a)
        return G.reshape(-1)

    def lowrank_at_quad(self, lr: LowRank) -> np.ndarray:
        """sum_r s_r phi_r(t) psi_r(x) at all tensor Gauss points."""
        out = np.zeros(int(np.prod(self.qshape)))
        for r in range(lr.R):
            tpart = self.Ht @ lr.U[:, r]
            V = lr.V[:, r].reshape(self.shape[1:])
            for a in range(1, self.d + 1):
                V = np.moveaxis(np.tensordot(self.Hs[self.dirs[a]], V, axes=([1], [a - 1])), 0, a - 1)
            out += lr.s[r] * np.multiply.outer(tpart, V).reshape(-1)
        return out

    def full(self, x_unk: np.ndarray, layer0: Optional[np.ndarray] = None) -> np.ndarray:
        """Unknown vector (N_t*N_s) -> full vector with time layer 0 prepended."""
        N_s = int(np.prod(self.n[: self.d]))
        l0 = np.zeros(N_s) if layer0 is None else layer0
        return np.concatenate([l0, x_unk])

    def rows(self, y_full: np.ndarray) -> np.ndarray:
        """Drop the test functions of time layer 0 (they are not in X_h)."""
        N_s = int(np.prod(self.n[: self.d]))
        return y_full[N_s:]

    # --------------------------------------------------------- initial datum
    def lift(self) -> np.ndarray:
        """Coefficients of the lifted initial datum: u0 at the (mapped) spatial Greville grid."""
        grids = np.meshgrid(*[self.grev_phys[l] for l in range(self.d - 1, -1, -1)], indexing="ij")
        pts = np.stack([grids[self.d - 1 - l].reshape(-1) for l in range(self.d)], axis=1)
        return self.P.u0(pts)

    # ------------------------------------------------------- bilinear forms
    def _lin_terms(self, x_full, theta_q):
        """C_m int dt u v + int grad u . D grad v + SU term, tested against all full functions."""
        P, d = self.P, self.d
        om = self.omega
        y = P.Cm * self.evT(om * self.ev(x_full, {d: 1}), {})
        for l in range(d):
            y += P.sigma[l] * self.evT(om * self.ev(x_full, {l: 1}), {l: 1})
        if self.su and theta_q is not None:
            for k in range(1, P.p_t + 1):
                tk = np.repeat(self.tau_q[k - 1], int(np.prod(self.qshape[1:])))
                y += P.Cm * self.evT(om * tk * theta_q * self.ev(x_full, {d: k}), {d: k})
        return y

    def apply_J(self, x_unk, coef_q, theta_q):
        """Linearised operator applied to an unknown vector (Section 3.1.1 form)."""
        xf = self.full(x_unk)
        y = self._lin_terms(xf, theta_q) + self.evT(self.omega * coef_q * self.ev(xf, {}), {})
        return self.rows(y)

    def residual(self, u_full, w_full, theta_q):
        """N(u) = A(u, w; v) + S(u; v) - F(v) for all v in X_h, exact I_ion at Gauss points."""
        uq = self.ev(u_full, {})
        wq = self.ev(w_full, {})
        y = self._lin_terms(u_full, theta_q) + self.evT(self.omega * ionic_current(uq, wq, self.P), {})
        if self.f is not None:
            y -= self.evT(self.omega * self.f_at_quad(), {})
        return self.rows(y)

    def f_at_quad(self):
        grids = np.meshgrid(*([self.quad[self.d][0]] + [self.quad[l][0] for l in range(self.d - 1, -1, -1)]),
                            indexing="ij")
        t = grids[0].reshape(-1)
        xs = [grids[self.d - l].reshape(-1) for l in range(self.d)]
        return self.f(xs, t)

    def _constant_part(self):
        """C_m int dt B_j B_i + sum_l sigma_l int dl B_j dl B_i on the full basis
        (the same every iteration: assembled once and kept)."""
        if getattr(self, "_Aconst", None) is None:
            P, d, om = self.P, self.d, self.omega
            Dg = sp.diags
            A = P.Cm * self.phi({}).T @ Dg(om) @ self.phi({d: 1})
            for l in range(d):
                A = A + P.sigma[l] * self.phi({l: 1}).T @ Dg(om) @ self.phi({l: 1})
            self._Aconst = sp.csr_matrix(A)
        return self._Aconst

    def assemble_J(self, coef_q, theta_q):
        """Explicit sparse matrix of apply_J (unknown rows x unknown columns)."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags
        A = self._constant_part() + self.phi({}).T @ Dg(om * coef_q) @ self.phi({})
        if self.su and theta_q is not None:
            for k in range(1, P.p_t + 1):
                tk = np.repeat(self.tau_q[k - 1], int(np.prod(self.qshape[1:])))
                A = A + P.Cm * self.phi({d: k}).T @ Dg(om * tk * theta_q) @ self.phi({d: k})
        N_s = int(np.prod(self.n[:d]))
        return sp.csr_matrix(A)[N_s:, N_s:]

    def assemble_full(self, coef_q, theta_q, sc_q=None):
        """The same bilinear form on the full basis (all n_t time layers, rows
        and columns), before the lifting split.  With SUPG (Section 4.2.2) the
        stabilization is S_SUPG + S_SC instead of the SU term:
          S_SUPG(u, v) = int tau (C_m u_t - sum_l sigma_l u_ll + coef u) v_t,
          S_SC(u, v)   = int sc_q u_t v_t,
        tau = h/(2p+1) per time element and sc_q the shock-capturing
        coefficient at the Gauss points (``sc_coefficient``; None: no term)."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags
        A = self._constant_part() + self.phi({}).T @ Dg(om * coef_q) @ self.phi({})
        if self.su and theta_q is not None:
            for k in range(1, P.p_t + 1):
                tk = np.repeat(self.tau_q[k - 1], int(np.prod(self.qshape[1:])))
                A = A + P.Cm * self.phi({d: k}).T @ Dg(om * tk * theta_q) @ self.phi({d: k})
        if self.supg:
            tau = np.repeat(self.supg_tau_t, int(np.prod(self.qshape[1:])))
            Pt = self.phi({d: 1})
            Lu = P.Cm * Pt + Dg(coef_q) @ self.phi({})
            for l in range(d):
                Lu = Lu - P.sigma[l] * self.phi({l: 2})
            A = A + Pt.T @ Dg(om * tau) @ Lu
            if sc_q is not None:
                A = A + Pt.T @ Dg(om * sc_q) @ Pt
        return sp.csr_matrix(A)

    def load_vector(self):
        """F(v) = int f v of eq. (3.3) for every full-basis test function; with
        SUPG the residual's source also meets the test function tau v_t."""
        if self.f is None:
            return np.zeros(int(np.prod(self.shape)))
        fq = self.omega * self.f_at_quad()
        F = self.evT(fq, {})
        if self.supg:
            F = F + self.evT(np.repeat(self.supg_tau_t, int(np.prod(self.qshape[1:]))) * fq, {self.d: 1})
        return F

    def reaction_at_quad(self, u_full, w_full):
        """C_r(u_h, w_h) of eq. (3.8) at every space-time Gauss point (the
        exact fixed-point reaction coefficient of the matrix M_R)."""
        return reaction_coefficient(self.ev(u_full, {}), self.ev(w_full, {}), self.P)

    def assemble_precond(self):
        """Explicit A-hat of Section 3.2 (sigma-scaled stiffness, shift a*c1, no SU)."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags(om)
        A = P.Cm * self.phi({}).T @ Dg @ self.phi({d: 1}) + P.a * P.c1 * self.phi({}).T @ Dg @ self.phi({})
        for l in range(d):
            A = A + P.sigma[l] * self.phi({l: 1}).T @ Dg @ self.phi({l: 1})
        N_s = int(np.prod(self.n[:d]))
        return sp.csr_matrix(A)[N_s:, N_s:]

    def precond_time_profiles(self, coef_q, theta_q):
        """Time profiles of the banded preconditioner (not from the paper): at
        each time Gauss point the spatial mean (Gauss-weighted) of the reaction
        coefficient coef_q, floored at the shift a c1 of the fast
        diagonalization, and of theta_q, floored at 0 (zero without SU)."""
        Qt = self.qshape[0]
        ws = np.array([1.0])
        for a in range(1, self.d + 1):
            ws = np.multiply.outer(ws, self.quad[self.dirs[a]][1])
        ws = ws.reshape(-1)
        c = np.maximum(np.asarray(coef_q).reshape(Qt, -1) @ ws / ws.sum(), self.P.a * self.P.c1)
        th = (np.asarray(theta_q).reshape(Qt, -1) @ ws / ws.sum()) if (self.su and theta_q is not None) else np.zeros(Qt)
        return c, np.maximum(th, 0.0)

    def assemble_precond_profiles(self, c_t, th_t):
        """Banded preconditioner of the Galerkin / SU system on X_h x X_h: the
        bilinear form
          int C_m u_t v + sum_l sigma_l int u_l v_l + int c(t) u v
          + C_m sum_k int tau_k th(t) d^k_t u d^k_t v
        with coefficients depending on time only (a Kronecker sum
        A_t (x) M_s + M_t (x) K_s); c_t, th_t at the time Gauss points, the
        weights tau_k th floored at 0."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags
        Qs = int(np.prod(self.qshape[1:]))
        cq, thq = np.repeat(c_t, Qs), np.repeat(th_t, Qs)
        P0 = self.phi({})
        A = P.Cm * P0.T @ Dg(om) @ self.phi({d: 1}) + P0.T @ Dg(om * cq) @ P0
        for l in range(d):
            Pl = self.phi({l: 1})
            A = A + P.sigma[l] * Pl.T @ Dg(om) @ Pl
        if self.su and np.any(th_t):
            for k in range(1, P.p_t + 1):
                tk = np.repeat(self.tau_q[k - 1], Qs)
                Pk = self.phi({d: k})
                A = A + Pk.T @ Dg(om * np.maximum(P.Cm * tk * thq, 0.0)) @ Pk
        N_s = int(np.prod(self.n[:d]))
        return sp.csr_matrix(A)[N_s:, N_s:]

    def precond_means(self, u_full, w_full):
        """Time profiles of the preconditioner of the SUPG system (not from the
        paper, which solves directly): at each time Gauss point the spatial
        mean (Gauss-weighted) of C_r(u, w), clipped at 0, and of the
        shock-capturing coefficient (zero when sc_c = 0)."""
        Qt = self.qshape[0]
        ws = np.array([1.0])
        for a in range(1, self.d + 1):
            ws = np.multiply.outer(ws, self.quad[self.dirs[a]][1])
        ws = ws.reshape(-1)
        cr = np.maximum(self.reaction_at_quad(u_full, w_full).reshape(Qt, -1) @ ws / ws.sum(), 0.0)
        if self.sc_c > 0.0:
            sc = self.sc_coefficient(u_full, w_full).reshape(Qt, -1) @ ws / ws.sum()
        else:
            sc = np.zeros(Qt)
        return cr, sc

    def assemble_precond_supg(self, cr_t, sc_t):
        """Preconditioner of the SUPG system on X_h x X_h: the bilinear form
          int C_m u_t (v + tau v_t) + sum_l sigma_l int u_l (v + tau v_t)_l
          + int cr(t) u (v + tau v_t) + int sc(t) u_t v_t
        with coefficients depending on time only (so that it is a Kronecker
        sum A_t (x) M_s + B_t (x) K_s); cr_t, sc_t at the time Gauss points."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags
        Qs = int(np.prod(self.qshape[1:]))
        tau, cr, sc = (np.repeat(v, Qs) for v in (self.supg_tau_t, cr_t, sc_t))
        P0, Pt = self.phi({}), self.phi({d: 1})
        A = P0.T @ Dg(om) @ (P.Cm * Pt) + Pt.T @ Dg(om * tau) @ (P.Cm * Pt)
        A = A + P0.T @ Dg(om * cr) @ P0 + Pt.T @ Dg(om * tau * cr) @ P0 + Pt.T @ Dg(om * sc) @ Pt
        for l in range(d):
            Pl = self.phi({l: 1})
            A = A + P.sigma[l] * (Pl.T @ Dg(om) @ Pl + self.phi({l: 1, d: 1}).T @ Dg(om * tau) @ Pl)
        N_s = int(np.prod(self.n[:d]))
        return sp.csr_matrix(A)[N_s:, N_s:]

    # --------------------------------------------------------- w update
    def w_update_explicit(self, u_full):
        """Solve L w = g of Section 3.1.1 as one explicit sparse system.
        L = int (dt w + b d_e w) z, g = int b u z over X_h; w has zero initial layer."""
        P, d, om = self.P, self.d, self.omega
        Dg = sp.diags(om)
        Lf = self.phi({}).T @ Dg @ self.phi({d: 1}) + P.b * P.de * self.phi({}).T @ Dg @ self.phi({})
        Gf = P.b * self.phi({}).T @ Dg @ self.phi({})
        N_s = int(np.prod(self.n[:d]))
        L = sp.csc_matrix(Lf)[N_s:, N_s:]
        g = (sp.csr_matrix(Gf) @ u_full)[N_s:]
        w = spla.splu(L).solve(g)
        return self.full(w)

    def w_update_kron(self, u_full):
        """Same system through the Kronecker structure L = (W_t + b d_e M_t) (x) M_s and
        g = b (M_t[X_t, :] (x) M_s) u: M_s cancels, leaving one N_t x N_t solve per
        spatial index (Section 3.2, last part)."""
        P, d = self.P, self.d
        tq, tw, _ = self.quad[d]
        B0, B1 = self.E[d][0], self.E[d][1]
        Wt = B0.T @ (tw[:, None] * B1)
        Mt = B0.T @ (tw[:, None] * B0)
        Lt = (Wt + P.b * P.de * Mt)[1:, 1:]
        G = P.b * Mt[1:, :]
        U = u_full.reshape(self.n[d], -1)
        w = np.linalg.solve(Lt, G @ U)
        return self.full(w.reshape(-1))

    # --------------------------------------------------------- theta (eq. 3.6)
    def element_windows(self, l: int, first: int):
        """For each full basis index j >= first in direction l, the element range
        [e0, e1) inside (xi_{j-p}, xi_{j+p+1}) (1-based paper indices, clamped)."""
        kn, p = self.kn[l], self.p[l]
        z = breakpoints(kn)
        out = []
        for j in range(first, self.n[l]):
            lo = kn[max(j - p, 0)]
            hi = kn[min(j + p + 1, len(kn) - 1)]
            es = [e for e in range(len(z) - 1) if z[e] >= lo and z[e + 1] <= hi]
            out.append((min(es), max(es) + 1))
        return out

    def residual_at_quad(self, u_full, w_full):
        """The residual R = C_m u_t - sum_l sigma_l u_ll + I_ion(u, w) - f at every
        Gauss point and the denominator C_m (||u||_inf / T + ||u_t||_inf) of
        eq. (3.6) (maxima over the Gauss points)."""
        P, d = self.P, self.d
        uq = self.ev(u_full, {})
        wq = self.ev(w_full, {})
        utq = self.ev(u_full, {d: 1})
        R = P.Cm * utq + ionic_current(uq, wq, P)
        for l in range(d):
            R -= P.sigma[l] * self.ev(u_full, {l: 2})
        if self.f is not None:
            R -= self.f_at_quad()
        den = P.Cm * (np.max(np.abs(uq)) / P.T + np.max(np.abs(utq)))
        return R, den

    def sc_coefficient(self, u_full, w_full):
        """Shock-capturing coefficient c h^2/4 |R| / (C_m (T^-1 ||u||_inf +
        ||u_t||_inf)) of Section 4.2.2 at every Gauss point; zero everywhere
        when the denominator vanishes (u = 0)."""
        R, den = self.residual_at_quad(u_full, w_full)
        if not den > 0:
            return np.zeros_like(R)
        return np.repeat(self.sc_scale_t, int(np.prod(self.qshape[1:]))) * np.abs(R) / den

    def theta_grid(self, u_full, w_full):
        """Theta of eq. (3.6) on the (X_t time) x (space) Greville grid: N_t x N_s."""
        P, d = self.P, self.d
        R, den = self.residual_at_quad(u_full, w_full)
        # element-wise maxima of |R|
        nq = [self.p[self.dirs[a]] + 1 for a in range(d + 1)]
        nel = [self.qshape[a] // nq[a] for a in range(d + 1)]
        E = np.abs(R).reshape([v for a in range(d + 1) for v in (nel[a], nq[a])])
        E = E.max(axis=tuple(2 * a + 1 for a in range(d + 1)))
        # box maxima over the support-extension windows, axis by axis
        for a in range(d + 1):
            l = self.dirs[a]
            wins = self.element_windows(l, 1 if l == d else 0)
            E = np.stack([np.take(E, range(e0, e1), axis=a).max(axis=a) for e0, e1 in wins], axis=a)
        num = E.reshape(self.n[d] - 1, -1)
        if den > 0:
            return np.minimum(num / den, 1.0)
        return np.where(num > 0, 1.0, 0.0)

    def greville_values(self, x_full):
        """Spline values on the (X_t time) x (space) Greville grid: N_t x N_s."""
        d = self.d
        mats = [bspline_all(self.kn[l], self.p[l], self.grev_s[l], 0) for l in range(d)]
        mats.append(bspline_all(self.kn[d], self.p[d], self.grev_t, 0))
        X = x_full.reshape(self.shape)
        for a in range(d + 1):
            X = np.moveaxis(np.tensordot(mats[self.dirs[a]], X, axes=([1], [a])), 0, a)
        return X.reshape(self.n[d] - 1, -1)

    def coefficient_grid(self, u_full, w_full, newton: bool):
        """dI_ion/du (Newton) or C_r (Picard) at the Greville grid: N_t x N_s."""
        ug = self.greville_values(u_full)
        wg = self.greville_values(w_full)
        return ionic_du(ug, wg, self.P) if newton else reaction_coefficient(ug, wg, self.P)

    def lowrank(self, grid: np.ndarray, eps: float, max_rank: Optional[int] = None) -> LowRank:
        R, U, s, V = truncated_svd(grid, eps, max_rank)
        return LowRank(U, s, V)
