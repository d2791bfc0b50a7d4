"""Parity at the full workload sizes, in the precisions the benchmark runs.

Config 1 (2D, p=3, 64^2 x 64): full vectors against the oracle's tensor
evaluator.  Config 2 (3D, p=2, 48^3 x 48): sampled rows against the oracle's
local-quadrature evaluator, the whole theta grid of a linearization against
the oracle's tensor evaluator, plus properties that hold at any size.
Config 4 (3D, p=3, 96^3 x 128, at most 16 terms per low rank): sampled rows
of the operator, the preconditioner and a Krylov solution."""
import gc

import numpy as np
import pytest

import st_workloads as W
from oracle import solver as osolver
from oracle.rowsample import RowSampler
from oracle.spacetime import LowRank, SpaceTime

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def make(prob, **kw):
    from paper_2311_17500_amd.binding import Solver
    return Solver(prob, **kw)


@pytest.fixture(scope="module")
def cfg1():
    prob = W.config(1)
    return prob, SpaceTime(prob, mode="tensor")


@pytest.fixture(scope="module")
def cfg2():
    prob = W.config(2)
    return prob, RowSampler(prob)


# ----------------------------------------------------------------- config 1
def test_cfg1_lift_count(gpu_lib, cfg1):
    prob, st = cfg1
    S = make(prob)
    c0, cnt = S.lift()
    assert cnt == 54 and np.array_equal(c0, st.lift())


def test_cfg1_theta_grid(gpu_lib, torch, cfg1):
    prob, st = cfg1
    S = make(prob)
    u, w = W.smooth_state(prob, 21)
    got = S.theta_grid(dev(torch, u), dev(torch, w)).cpu().numpy()
    assert np.max(np.abs(got - st.theta_grid(u, w).reshape(-1))) < 1e-12


def test_cfg1_apply_precond_krylov(gpu_lib, torch, cfg1):
    prob, st = cfg1
    S = make(prob, precond=0)   # the fast diagonalization of Section 3.2 (A-hat below)
    ft, fc = W.random_factors(prob, 3, 4), W.random_factors(prob, 4, 5, scale=5.0)
    S.set_factors(ft, fc)
    thq = st.lowrank_at_quad(LowRank(*ft))
    cq = st.lowrank_at_quad(LowRank(*fc))
    x = W.random_vector(prob.unknowns, 6)
    y = S.apply(dev(torch, x)).cpu().numpy()
    assert rel(y, st.apply_J(x, cq, thq)) < 1e-12
    # preconditioner: A-hat z = r (A-hat evaluated by the oracle's quadrature)
    r = W.random_vector(prob.unknowns, 7)
    z = S.precond(dev(torch, r)).cpu().numpy()
    Az = st.apply_J(z, np.full(len(st.omega), prob.a * prob.c1), None)
    assert rel(Az, r) < 1e-10
    # linear solve on a coefficient field shaped like a linearization: oracle true residual
    ft, fc = W.coefficient_factors(prob, 3, 4, base=0.3), W.coefficient_factors(prob, 4, 5)
    S.set_factors(ft, fc)
    thq = st.lowrank_at_quad(LowRank(*ft))
    cq = st.lowrank_at_quad(LowRank(*fc))
    b = W.random_vector(prob.unknowns, 8)
    xs, it, rr = S.krylov(dev(torch, b), tol=1e-10)
    xs = xs.cpu().numpy()
    assert rr <= 1e-10
    assert rel(st.apply_J(xs, cq, thq), b) < 1.05e-10


def test_cfg1_linearize_and_residual(gpu_lib, torch, cfg1):
    prob, st = cfg1
    S = make(prob)
    u, w = W.smooth_state(prob, 22, noise=0.0)   # per-coefficient noise would need rank > 48
    ud, wd = dev(torch, u), dev(torch, w)
    S.linearize(ud, wd)
    lin = osolver.linearize(st, u, w)
    gt, gc = S.get_factors()
    assert len(gt[1]) == lin.theta_lr.R and len(gc[1]) == lin.coef_lr.R
    r = S.residual(ud, wd).cpu().numpy()
    assert rel(r, st.residual(u, w, lin.theta_q)) < 1e-11


def test_cfg1_mixed_fp32_solve(gpu_lib, torch, cfg1):
    prob, st = cfg1
    from paper_2311_17500_amd.binding import MIXED_FP32
    S = make(prob, prec=MIXED_FP32)
    ft, fc = W.coefficient_factors(prob, 3, 4, base=0.3), W.coefficient_factors(prob, 4, 5)
    S.set_factors(ft, fc)
    b = W.random_vector(prob.unknowns, 9)
    xs, it, rr = S.krylov(dev(torch, b), tol=1e-8)
    res = rel(st.apply_J(xs.cpu().numpy(), st.lowrank_at_quad(LowRank(*fc)), st.lowrank_at_quad(LowRank(*ft))), b)
    assert rr <= 1e-8 and res <= 1.05e-8


# ----------------------------------------------------------------- config 2
ROWS = 200


def test_cfg2_lift_count(gpu_lib):
    S = make(W.config(2))
    assert S.lift()[1] == 133


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16"])
def test_cfg2_apply_sampled_rows(gpu_lib, torch, cfg2, prec):
    """FP64 apply agrees with the oracle to 1e-12 on sampled rows; the mixed
    runs' FP64 operator (used for true residuals) is the same kernel path."""
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32, MIXED_BF16
    prob, rs = cfg2
    code = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}[prec]
    S = make(prob, prec=code)
    ft, fc = W.random_factors(prob, 2, 11), W.random_factors(prob, 3, 12, scale=5.0)
    S.set_factors(ft, fc)
    x = W.random_vector(prob.unknowns, 13)
    y = S.apply(dev(torch, x)).cpu().numpy()
    rows = np.random.default_rng(1).choice(prob.unknowns, ROWS, replace=False)
    want = rs.apply_rows(x, rows, theta=ft, coef=fc)
    assert np.max(np.abs(y[rows] - want)) < 1e-12 * np.max(np.abs(y))
    del S
    gc.collect()
    torch.cuda.empty_cache()


def test_cfg2_precond_sampled_rows(gpu_lib, torch, cfg2):
    prob, rs = cfg2
    S = make(prob)
    r = W.random_vector(prob.unknowns, 14)
    z = S.precond(dev(torch, r)).cpu().numpy()
    rows = np.random.default_rng(2).choice(prob.unknowns, ROWS, replace=False)
    Az = rs.apply_rows(z, rows, coef_const=prob.a * prob.c1)
    assert np.max(np.abs(Az - r[rows])) < 1e-10 * np.max(np.abs(r))


@pytest.mark.parametrize("prec,tol", [("mixed_fp32", 1e-8), ("mixed_bf16", 1e-8), ("fp64", 1e-8)])
def test_cfg2_krylov(gpu_lib, torch, cfg2, prec, tol):
    """The reported FP64 true residual meets the tolerance, and sampled rows of
    b - J x from the oracle are consistent with it."""
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32, MIXED_BF16
    prob, rs = cfg2
    code = {"fp64": FP64, "mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}[prec]
    S = make(prob, prec=code)
    ft, fc = W.coefficient_factors(prob, 2, 11, base=0.3), W.coefficient_factors(prob, 3, 12)
    S.set_factors(ft, fc)
    b = W.random_vector(prob.unknowns, 15)
    xs, it, rr = S.krylov(dev(torch, b), tol=tol)
    assert rr <= tol
    rows = np.random.default_rng(3).choice(prob.unknowns, ROWS, replace=False)
    res_rows = b[rows] - rs.apply_rows(xs.cpu().numpy(), rows, theta=ft, coef=fc)
    # a sampled residual entry cannot exceed the full residual norm
    assert np.max(np.abs(res_rows)) <= 1.01 * tol * np.linalg.norm(b)
    del S
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,bound_a,bound_p", [("mixed_fp32", 1e-5, 1e-5), ("mixed_bf16", 1e-5, 5e-2)])
def test_cfg2_lowp_operator_error(gpu_lib, torch, prec, bound_a, bound_p):
    """Low-precision operator and preconditioner against FP64 on the same
    context: relative error of the order of the unit roundoff (FP32 6e-8,
    BF16 3.9e-3) times a modest constant from the chained contractions.  In
    BF16 mode only the preconditioner is BF16."""
    from paper_2311_17500_amd.binding import MIXED_FP32, MIXED_BF16
    prob = W.config(2)
    S = make(prob, prec={"mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}[prec])
    ft, fc = W.random_factors(prob, 2, 11), W.random_factors(prob, 3, 12, scale=5.0)
    S.set_factors(ft, fc)
    x = dev(torch, W.random_vector(prob.unknowns, 16))
    y64, ylp = S.apply(x), S.apply_lowp(x)
    z64, zlp = S.precond(x), S.precond_lowp(x)
    ea = float(torch.linalg.norm(ylp - y64) / torch.linalg.norm(y64))
    ep = float(torch.linalg.norm(zlp - z64) / torch.linalg.norm(z64))
    assert ea < bound_a and ep < bound_p, (ea, ep)
    del S
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_cfg2_linearization_full_theta(gpu_lib, torch):
    """A linearization at a front-shaped state: every theta entry of eq. (3.6)
    against the oracle's tensor evaluator, identical truncated-SVD ranks and
    products, and sampled rows of the residual N(u) (with the oracle's own
    theta factors)."""
    from oracle.spacetime import truncated_svd
    prob = W.config(2)
    u, w = W.smooth_state(prob, 23, noise=0.0)
    st = SpaceTime(prob, mode="tensor")
    th_o = st.theta_grid(u, w)
    del st
    gc.collect()
    S = make(prob)
    ud, wd = dev(torch, u), dev(torch, w)
    th_g = S.theta_grid(ud, wd).cpu().numpy().reshape(th_o.shape)
    assert np.max(np.abs(th_g - th_o)) < 1e-12
    S.linearize(ud, wd)
    (gt, gc_) = S.get_factors()
    Rt, Ut, st_, Vt = truncated_svd(th_o, 0.1)
    assert len(gt[1]) == Rt
    assert np.linalg.norm((gt[0] * gt[1]) @ gt[2].T - (Ut * st_) @ Vt.T) <= 1e-11 * np.linalg.norm(th_o)
    r = S.residual(ud, wd).cpu().numpy()
    rows = np.random.default_rng(4).choice(prob.unknowns, 64, replace=False)
    want = RowSampler(prob).residual_rows(u, w, rows, theta=(Ut, st_, Vt))
    assert np.max(np.abs(r[rows] - want)) < 1e-11 * np.max(np.abs(r))
    del S
    gc.collect()
    torch.cuda.empty_cache()


# ----------------------------------------------------------------- config 4
ROWS4 = 48


@pytest.fixture(scope="module")
def cfg4():
    prob = W.config(4)
    return prob, RowSampler(prob)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_cfg4_apply_precond_sampled_rows(gpu_lib, torch, cfg4, prec):
    """FP64 operator and preconditioner (A-hat z = r) on sampled rows; in the
    mixed context also the FP32 operator, within a modest multiple of the
    FP32 unit roundoff of the largest entry."""
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32
    prob, rs = cfg4
    S = make(prob, prec={"fp64": FP64, "mixed_fp32": MIXED_FP32}[prec], max_rank=16, precond=0)
    ft, fc = W.random_factors(prob, 2, 41), W.random_factors(prob, 3, 42, scale=5.0)
    S.set_factors(ft, fc)
    x = W.random_vector(prob.unknowns, 43)
    xd = dev(torch, x)
    rows = np.random.default_rng(5).choice(prob.unknowns, ROWS4, replace=False)
    want = rs.apply_rows(x, rows, theta=ft, coef=fc)
    y = S.apply(xd).cpu().numpy()
    ymax = np.max(np.abs(y))
    assert np.max(np.abs(y[rows] - want)) < 1e-12 * ymax
    if prec == "mixed_fp32":
        yl = S.apply_lowp(xd).cpu().numpy()
        assert np.max(np.abs(yl[rows] - want)) < 1e-5 * ymax
    del y
    z = S.precond(xd).cpu().numpy()
    Az = rs.apply_rows(z, rows, coef_const=prob.a * prob.c1)
    assert np.max(np.abs(Az - x[rows])) < 1e-10 * np.max(np.abs(x))
    del S, z, xd
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_cfg4_mixed_krylov(gpu_lib, torch, cfg4):
    """Mixed FP32 solve at full size: the reported FP64 true residual meets
    1e-8 and sampled rows of b - J x from the oracle are consistent with it."""
    from paper_2311_17500_amd.binding import MIXED_FP32
    prob, rs = cfg4
    S = make(prob, prec=MIXED_FP32, max_rank=16)
    ft, fc = W.coefficient_factors(prob, 2, 44, base=0.3), W.coefficient_factors(prob, 3, 45)
    S.set_factors(ft, fc)
    b = W.random_vector(prob.unknowns, 46)
    xs, it, rr = S.krylov(dev(torch, b), tol=1e-8)
    assert rr <= 1e-8
    rows = np.random.default_rng(6).choice(prob.unknowns, ROWS4, replace=False)
    res_rows = b[rows] - rs.apply_rows(xs.cpu().numpy(), rows, theta=ft, coef=fc)
    assert np.max(np.abs(res_rows)) <= 1.01e-8 * np.linalg.norm(b)
    del S, xs
    gc.collect()
    torch.cuda.empty_cache()
