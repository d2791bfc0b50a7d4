"""Seeded synthetic workloads shared by the CPU oracle and the GPU path.

This module holds problem *inputs* only: mesh sizes, degrees, diffusivities,
Rogers-McCulloch parameters, stimulus descriptions and seeded random vectors.
It contains none of the method's arithmetic (no splines, no quadrature, no
operators), so both the oracle and the HIP path can import it without sharing
any computation.

Rogers-McCulloch parameters are stored in the paper's notation (Section 3,
eq. (3.1)): I_ion = c1 u (u - a)(u - 1) + c2 u w and w_t = b (u - d_e w).  The
benchmark workloads are specified in the equivalent "G, v_th, v_p, eta" form;
with v_p = 1 the conversion is c1 = G / (v_th v_p), a = v_th, c2 = eta1,
b = eta2 / v_p, d_e = eta3 v_p.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

# Scaled Rogers-McCulloch set used by every synthetic workload:
# G = 1.5, v_th = 0.13, v_p = 1, eta1 = 4.4, eta2 = 0.012, eta3 = 1.
RM_G, RM_VTH, RM_VP, RM_ETA1, RM_ETA2, RM_ETA3 = 1.5, 0.13, 1.0, 4.4, 0.012, 1.0


def rm_paper_params(G=RM_G, v_th=RM_VTH, v_p=RM_VP, eta1=RM_ETA1, eta2=RM_ETA2,
                    eta3=RM_ETA3):
    """Return (a, b, c1, c2, d_e) in the paper's notation (requires v_p == 1)."""
    if v_p != 1.0:
        raise ValueError("the paper's cubic form needs v_p = 1")
    return dict(a=v_th, b=eta2 / v_p, c1=G / (v_th * v_p), c2=eta1, de=eta3 * v_p)


@dataclasses.dataclass
class Problem:
    """One space-time problem on (0,1)^d x (0,T) with uniform open knots."""
    d: int
    p_s: int
    p_t: int
    nel_s: Tuple[int, ...]          # elements per spatial direction
    nel_t: int                      # elements in time
    sigma: Tuple[float, ...]        # D = diag(sigma)
    T: float = 1.0
    Cm: float = 1.0
    a: float = 0.13
    b: float = 0.012
    c1: float = 1.5 / 0.13
    c2: float = 4.4
    de: float = 1.0
    # stimulus: initial datum u0 = u0_value on a region, 0 elsewhere
    u0_kind: int = 2                # 0 none, 1 half-space x_1 < c, 2 closed ball |x-c| <= r
    u0_center: Tuple[float, ...] = (0.0, 0.0, 0.0)
    u0_radius: float = 0.1
    u0_value: float = 1.0
    # source f of the monodomain equation (0: none; 1: f_amp on the closed ball
    # |x - f_center| <= f_radius for t in [f_t0, f_t1]; 2: moving Gaussian
    # f_amp exp(-f_kappa |x - f_center - f_velocity t|^2) for t in [f_t0, f_t1])
    f_kind: int = 0
    f_center: Tuple[float, ...] = (0.0, 0.0, 0.0)
    f_radius: float = 0.0
    f_t0: float = 0.0
    f_t1: float = 0.0
    f_amp: float = 0.0
    f_kappa: float = 0.0
    f_velocity: Tuple[float, ...] = (0.0, 0.0, 0.0)
    # separable geometry map of each spatial direction, x_l = F_l(eta_l):
    # 0 identity, 1 affine a + (b - a) eta, 2 exponential grading
    # a + (b - a) (exp(k eta) - 1) / (exp(k) - 1); map_param[l] = (a, b, k)
    map_kind: Tuple[int, ...] = (0, 0, 0)
    map_param: Tuple[Tuple[float, float, float], ...] = ((0.0, 1.0, 0.0),) * 3

    @property
    def n_s(self):
        return tuple(n + self.p_s for n in self.nel_s)

    @property
    def n_t(self):
        return self.nel_t + self.p_t

    @property
    def N_s(self):
        return int(np.prod(self.n_s))

    @property
    def N_t(self):
        return self.n_t - 1

    @property
    def unknowns(self):
        return self.N_s * self.N_t

    @property
    def dof(self):
        """Degrees of freedom counted with the initial time layer (N_s * n_t)."""
        return self.N_s * self.n_t

    def uniform_knots(self):
        """Open uniform knot vectors on [0,1]: list of d spatial + 1 time arrays."""
        def ok(nel, p):
            return np.concatenate([np.zeros(p + 1), np.arange(1, nel) / nel, np.ones(p + 1)])
        return [ok(n, self.p_s) for n in self.nel_s] + [ok(self.nel_t, self.p_t)]

    def u0(self, pts):
        """Initial datum at points pts (M x d array)."""
        pts = np.atleast_2d(pts)
        if self.u0_kind == 0:
            return np.zeros(len(pts))
        if self.u0_kind == 1:
            return np.where(pts[:, 0] < self.u0_center[0], self.u0_value, 0.0)
        c = np.asarray(self.u0_center[: self.d])
        r2 = np.sum((pts - c) ** 2, axis=1)
        return np.where(r2 <= self.u0_radius ** 2, self.u0_value, 0.0)


    def source(self, xs, t):
        """Source f at points: xs is a list of d coordinate arrays, t an array
        of the same shape (absolute times); None when there is no source."""
        t = np.asarray(t, dtype=np.float64)
        if self.f_kind == 0:
            return np.zeros_like(t)
        r2 = np.zeros_like(t)
        for l in range(self.d):
            dx = np.asarray(xs[l], dtype=np.float64) - self.f_center[l]
            if self.f_kind == 2:
                dx = dx - self.f_velocity[l] * t
            r2 = r2 + dx * dx
        on = (t >= self.f_t0) & (t <= self.f_t1)
        if self.f_kind == 1:
            val = np.where(r2 <= self.f_radius * self.f_radius, self.f_amp, 0.0)
        else:
            val = self.f_amp * np.exp(-self.f_kappa * r2)
        return np.where(on, val, 0.0)


def clustered_time_knots(nel_t: int, p: int, events, width: float):
    """Open knot vector on [0,1] with nel_t elements: p+1 interior knots
    clustered (spacing `width`) around each event time, the remaining interior
    knots evenly spaced, none coinciding (maximal regularity in time)."""
    cl = []
    for te in events:
        cl.extend(te + (np.arange(p + 1) - 0.5 * p) * width)
    m = nel_t - 1 - len(cl)
    if m < 0:
        raise ValueError("too few elements for the clusters")
    cl = np.array(cl)
    even = (np.arange(m) + 1.0) / (m + 1.0)
    # keep the even knots away from the clusters (at least one cluster width)
    for te in events:
        near = np.abs(even - te) < (0.5 * p + 1.0) * width
        even[near] = np.where(even[near] < te, te - (0.5 * p + 1.0) * width, te + (0.5 * p + 1.0) * width)
    inner = np.sort(np.concatenate([cl, even]))
    if np.any(np.diff(inner) <= 0.25 * width) or inner[0] <= 0 or inner[-1] >= 1:
        raise ValueError("knots too close")
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


_RM = rm_paper_params()


def config(idx: int) -> Problem:
    """The synthetic benchmark workloads on the unit square/cube, T = 1, C_m = 1.

    0: d=1, p=2, 32 x 32 elements, sigma=1e-3, u0 = 1 on x < 0.1
    1: d=2, p=3, 64^2 x 64, sigma=(1e-3, 2.5e-4), u0 = 1 on the disc r=0.1 at 0
    2: d=3, p=2, 48^3 x 48, sigma=(1e-3, 5e-4, 2.5e-4), ball r=0.1 at 0
    4: d=3, p=3, 96^3 x 128, sigma as in 2, ball r=0.1 at 0
    """
    if idx == 0:
        return Problem(d=1, p_s=2, p_t=2, nel_s=(32,), nel_t=32, sigma=(1e-3,),
                       u0_kind=1, u0_center=(0.1, 0.0, 0.0), **_RM)
    if idx == 1:
        return Problem(d=2, p_s=3, p_t=3, nel_s=(64, 64), nel_t=64, sigma=(1e-3, 2.5e-4), **_RM)
    if idx == 2:
        return Problem(d=3, p_s=2, p_t=2, nel_s=(48, 48, 48), nel_t=48,
                       sigma=(1e-3, 5e-4, 2.5e-4), **_RM)
    if idx == 4:
        return Problem(d=3, p_s=3, p_t=3, nel_s=(96, 96, 96), nel_t=128,
                       sigma=(1e-3, 5e-4, 2.5e-4), **_RM)
    raise ValueError(f"no single-solve workload {idx}")


def tiny(d: int, p: int, nel: int, nel_t: Optional[int] = None, **kw) -> Problem:
    """Small version of the workloads (same physics, fewer elements)."""
    sig = {1: (1e-3,), 2: (1e-3, 2.5e-4), 3: (1e-3, 5e-4, 2.5e-4)}[d]
    args = dict(d=d, p_s=p, p_t=p, nel_s=(nel,) * d, nel_t=nel_t or nel, sigma=sig, **_RM)
    if d == 1:
        args.update(u0_kind=1, u0_center=(0.1, 0.0, 0.0))
    else:
        args.update(u0_radius=0.3)       # big enough to cover Greville points on coarse meshes
    args.update(kw)
    return Problem(**args)


def serve_stream(n_requests: int = 512, seed: int = 0):
    """Seeded arrival stream of 2D solves (Poisson arrivals at 20 req/s).

    Per request, draws in this order: exponential inter-arrival (mean 1/20 s),
    space elements per side from {24,32,48,64,96}, time elements from
    {32,64,128}, degree from {2,3}, log10 sigma_x ~ U[-4,-2] (sigma_y =
    sigma_x / 4), disc centre ~ U[0,1]^2 (radius 0.1).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / 20.0)
        nel_s = int(rng.choice([24, 32, 48, 64, 96]))
        nel_t = int(rng.choice([32, 64, 128]))
        p = int(rng.choice([2, 3]))
        sx = 10.0 ** rng.uniform(-4.0, -2.0)
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        prob = Problem(d=2, p_s=p, p_t=p, nel_s=(nel_s, nel_s), nel_t=nel_t,
                       sigma=(sx, sx / 4.0), u0_center=(float(cx), float(cy), 0.0), **_RM)
        out.append((t, prob))
    return out


def random_vector(n: int, seed: int = 0) -> np.ndarray:
    """Standard-normal FP64 vector (numpy PCG64, fixed seed)."""
    return np.random.default_rng(seed).standard_normal(n)


def smooth_state(prob: Problem, seed: int = 0, noise: float = 0.01):
    """A smooth synthetic (u, w) coefficient state of length N_s * n_t each.

    Coefficients are samples of a moving tanh front plus a seeded perturbation
    of size `noise`, laid out [time][x_d]...[x_1] (x_1 fastest).  Used to exercise
    the linearisation at states that are not the initial guess.
    """
    rng = np.random.default_rng(seed)
    grids = [np.linspace(0.0, 1.0, n) for n in prob.n_s]
    tg = np.linspace(0.0, 1.0, prob.n_t)
    mesh = np.meshgrid(*([tg] + grids[::-1]), indexing="ij")
    tt = mesh[0]
    r = np.sqrt(sum(m ** 2 for m in mesh[1:]))
    u = 0.5 * (1.0 - np.tanh((r - 0.15 - 0.2 * tt) / 0.05))
    u = u + noise * rng.standard_normal(u.shape)
    w = 0.05 * tt * u
    return u.reshape(-1), w.reshape(-1)


def random_factors(prob: Problem, R: int, seed: int = 0, scale: float = 1.0):
    """Seeded low-rank factors (U: N_t x R, s: R, V: N_s x R) for a coefficient
    field given on the Greville grid; rows are smooth random walks so that the
    field resembles a sampled function.  Used to exercise the operator with
    the same coefficient on both sides."""
    rng = np.random.default_rng(seed)
    U = np.cumsum(rng.standard_normal((prob.N_t, R)), axis=0) / np.sqrt(prob.N_t)
    V = np.cumsum(rng.standard_normal((prob.N_s, R)), axis=0) / np.sqrt(prob.N_s)
    s = scale * 0.5 ** np.arange(R)
    return U, s, V


def coefficient_factors(prob: Problem, R: int, seed: int = 0, base: float = 1.5, spread: float = 0.3):
    """Low-rank factors of a coefficient field of the shape the linearization
    produces: a constant level `base` (rank one) plus R-1 smooth random-walk
    modes of relative size `spread`."""
    U, s, V = random_factors(prob, max(R - 1, 0), seed, scale=base * spread)
    U = np.concatenate([np.ones((prob.N_t, 1)), U], axis=1)
    V = np.concatenate([np.ones((prob.N_s, 1)), V], axis=1)
    s = np.concatenate([[base], s])
    return U[:, :R], s[:R], V[:, :R]


def c0_time_knots(nel_t: int, p: int):
    """Open knot vector on [0,1] with nel_t uniform elements and every interior
    knot repeated p times: C^0 splines in time (n_t = p nel_t + 1)."""
    inner = np.repeat(np.arange(1, nel_t) / nel_t, p)
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])
