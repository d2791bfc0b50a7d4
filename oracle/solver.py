"""Outer nonlinear loop and direct linear solves of the oracle.
Test infrastructure (see package doc).

One outer iteration at the iterate (u^k, w^k) (readings listed in
``spacetime``):
  1. w^k from the L-system of Section 3.1.1 (explicit sparse solve);
  2. theta of eq. (3.4) on the Greville grid, truncated SVD with eps_theta,
     interpolated to the Gauss points (refreshed until ||delta||_inf <=
     theta_freeze, frozen afterwards);
  3. reaction coefficient (dI/du for Newton, C_r of eq. (3.6) for Picard) on
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
          theta_freeze=1e-4, max_outer=60, u_init=None):
    """Full nonlinear solve; returns (u_full, w_full, log)."""
    alpha = (1.0 if newton else 0.5) if alpha is None else alpha
    c0 = st.lift()
    nt = st.n[st.d]
    u = np.tile(c0, nt) if u_init is None else u_init.copy()
    log = OuterLog()
    theta_lr = None
    frozen = False
    for _ in range(max_outer):
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
        if dinf <= theta_freeze:
            frozen = True
        if dinf <= tol:
            break
    w = st.w_update_explicit(u)
    return u, w, log


def precond_solve(st: SpaceTime, r):
    """z = A-hat^{-1} r with A-hat assembled explicitly (Section 3.2)."""
    return spla.splu(st.assemble_precond().tocsc()).solve(r)
