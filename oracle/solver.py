"""Outer nonlinear loop and direct linear solves of the oracle.
Test infrastructure (see package doc).

One outer iteration at the iterate (u^k, w^k) (readings listed in
``spacetime``):
  1. w^k from the L-system of Section 3.1.1 (explicit sparse solve);
  2. theta of eq. (3.6) on the Greville grid, truncated SVD with eps_theta,
     interpolated to the Gauss points (refreshed until ||delta||_inf <=
     theta_freeze, frozen afterwards);
  3. reaction coefficient (dI/du for Newton, C_r of eq. (3.8) for Picard) on
     the Greville grid, truncated SVD with eps_react, interpolated;
  4. J = explicit sparse matrix of the linearised form, r = N(u^k);
  5. delta = -J^{-1} r by a sparse LU (scipy splu);
  6. u^{k+1} = u^k + alpha delta;  stop when ||delta||_inf <= tol
     (the stopping rule of Section 4 applied to the update).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse.linalg as spla

from .spacetime import SpaceTime


@dataclasses.dataclass
class OuterLog:
    deltas: List[float] = dataclasses.field(default_factory=list)
    ranks_theta: List[int] = dataclasses.field(default_factory=list)
    ranks_react: List[int] = dataclasses.field(default_factory=list)


@dataclasses.dataclass
class Linearization:
    theta_q: np.ndarray
    coef_q: np.ndarray
    theta_lr: object
    coef_lr: object


def linearize(st: SpaceTime, u_full, w_full, eps_theta=0.1, eps_react=1e-2, newton=True,
              theta_lr=None):
    """Steps 2-3 above; pass theta_lr to keep a frozen theta."""
    if st.su and theta_lr is None:
        theta_lr = st.lowrank(st.theta_grid(u_full, w_full), eps_theta)
    theta_q = st.lowrank_at_quad(theta_lr) if st.su else None
    coef_lr = st.lowrank(st.coefficient_grid(u_full, w_full, newton), eps_react)
    coef_q = st.lowrank_at_quad(coef_lr)
    return Linearization(theta_q, coef_q, theta_lr, coef_lr)


def solve(st: SpaceTime, newton=True, alpha=None, eps_theta=0.1, eps_react=1e-2, tol=1e-10,
          theta_freeze=1e-4, max_outer=60, u_init=None, picard_switch=0):
    """Full nonlinear solve; returns (u_full, w_full, log).  picard_switch > 0:
    a Newton solve whose ||alpha delta||_inf grows in that many consecutive
    iterations continues as the Picard iteration (C_r, alpha = 0.5); the
    iteration count at the switch is log.switched_at (-1: none)."""
    alpha = (1.0 if newton else 0.5) if alpha is None else alpha
    switch_armed = newton and picard_switch > 0
    growth, dprev = 0, -1.0
    c0 = st.lift()
    nt = st.n[st.d]
    u = np.tile(c0, nt) if u_init is None else u_init.copy()
    log = OuterLog()
    log.switched_at = -1
    theta_lr = None
    frozen = False
    for k in range(max_outer):
        w = st.w_update_explicit(u)
        lin = linearize(st, u, w, eps_theta, eps_react, newton, theta_lr if frozen else None)
        theta_lr = lin.theta_lr
        J = st.assemble_J(lin.coef_q, lin.theta_q)
        r = st.residual(u, w, lin.theta_q)
        delta = -spla.splu(J.tocsc()).solve(r)
        u = u + alpha * st.full(delta)
        # the stopping quantity is the change of the iterate, ||u^{k+1} - u^k||_inf
        # (Section 4), i.e. the relaxed update
        dinf = float(alpha * np.max(np.abs(delta)))
        log.deltas.append(dinf)
        log.ranks_theta.append(theta_lr.R if theta_lr is not None else 0)
        log.ranks_react.append(lin.coef_lr.R)
        if switch_armed and log.switched_at < 0:
            growth = growth + 1 if (dprev >= 0.0 and dinf > dprev) else 0
            if growth >= picard_switch:
                newton, alpha = False, 0.5
                log.switched_at = k + 1
        dprev = dinf
        if dinf <= theta_freeze:
            frozen = True
        if dinf <= tol:
            break
    w = st.w_update_explicit(u)
    return u, w, log


def solve_picard(st: SpaceTime, alpha=0.5, eps_theta=0.1, tol=1e-4, max_outer=200, theta_freeze=None,
                 theta_lr=None):
    """The fixed-point scheme of Section 3.1 as the paper states it, step by
    step.  From u^0 (the lifted datum in every time layer) and w^0 = 0, each
    iteration
      1. builds theta(u^k, w^k) (eq. (3.6)) and its truncated SVD (eq. (3.9)),
         refreshed every iteration (while the change exceeds theta_freeze,
         when given; a fixed theta_lr skips this step);
      2. assembles A of Section 3.1.1 with M_R weighted by the exact
         C_r(u^k, w^k) of eq. (3.8) at the Gauss points and the low-rank SU
         term (or, with SUPG, the SUPG and shock-capturing terms of Section
         4.2.2 with C_r and the residual ratio at (u^k, w^k) taken exactly at
         the Gauss points), and the load vector F;
      3. solves A u~ = F for the unknown layers, the initial layer held at the
         lifted datum (sparse LU);
      4. solves L w~ = G(u^k) (the decoupled w-equation);
      5. relaxes both: u^{k+1} = alpha u~ + (1 - alpha) u^k and
         w^{k+1} = alpha w~ + (1 - alpha) w^k;
    and stops when ||u^{k+1} - u^k||_inf <= tol (Section 4: 1e-4).
    Returns (u, w, log)."""
    c0 = st.lift()
    nt = st.n[st.d]
    N_s = len(c0)
    u = np.tile(c0, nt)
    w = np.zeros_like(u)
    log = OuterLog()
    frozen = theta_lr is not None
    F = st.load_vector()
    for _ in range(max_outer):
        if st.su and not frozen:
            theta_lr = st.lowrank(st.theta_grid(u, w), eps_theta)
        theta_q = st.lowrank_at_quad(theta_lr) if st.su else None
        # SUPG + shock capturing (Section 4.2.2): the coefficients at (u^k, w^k)
        sc_q = st.sc_coefficient(u, w) if (st.supg and st.sc_c > 0.0) else None
        A = st.assemble_full(st.reaction_at_quad(u, w), theta_q, sc_q)
        rhs = F[N_s:] - A[N_s:, :N_s] @ c0
        ut = np.concatenate([c0, spla.splu(sp_csc(A[N_s:, N_s:])).solve(rhs)])
        wt = st.w_update_explicit(u)
        u_new = alpha * ut + (1.0 - alpha) * u
        w = alpha * wt + (1.0 - alpha) * w
        dinf = float(np.max(np.abs(u_new - u)))
        u = u_new
        log.deltas.append(dinf)
        log.ranks_theta.append(theta_lr.R if (st.su and theta_lr is not None) else 0)
        log.ranks_react.append(0)
        if theta_freeze is not None and dinf <= theta_freeze:
            frozen = True
        if dinf <= tol:
            break
    return u, w, log


def sp_csc(A):
    return A.tocsc()


def precond_solve(st: SpaceTime, r):
    """z = A-hat^{-1} r with A-hat assembled explicitly (Section 3.2)."""
    return spla.splu(st.assemble_precond().tocsc()).solve(r)
