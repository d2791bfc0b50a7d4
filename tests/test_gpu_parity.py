"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.  Tolerances: FP64 paths 1e-10
relative (operators agree to ~1e-13; solves are limited by the Krylov
tolerance), integer data bit-exact."""
import numpy as np
import pytest

import st_workloads as W
from oracle import solver
from oracle.spacetime import LowRank, SpaceTime

pytestmark = pytest.mark.gpu

SMALL = [("1d_p2", W.tiny(1, 2, 9, nel_t=7)),
         ("2d_p3", W.tiny(2, 3, 5, nel_t=6)),
         ("3d_p2", W.tiny(3, 2, 3, nel_t=5)),
         ("3d_p1", W.tiny(3, 1, 4, nel_t=4)),
         ("cfg0", W.config(0)),
         ("3d_p3", W.tiny(3, 3, 3, nel_t=4)),
         ("3d_p3_small", W.tiny(3, 3, 2, nel_t=3))]


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def solver_for(prob, **kw):
    from paper_2311_17500_amd.binding import Solver
    return Solver(prob, **kw)


def to_dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def lowrank_product(f):
    U, s, V = f
    return (U * s) @ V.T


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_lift_bit_exact(gpu_lib, name, prob):
    S = solver_for(prob)
    st = SpaceTime(prob)
    c0, cnt = S.lift()
    want = st.lift()
    assert np.array_equal(c0, want) and cnt == int(np.sum(want != 0))


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_theta_grid(gpu_lib, torch, name, prob):
    S = solver_for(prob)
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 3)
    got = S.theta_grid(to_dev(torch, u), to_dev(torch, w)).cpu().numpy()
    want = st.theta_grid(u, w).reshape(-1)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_linearize_apply(gpu_lib, torch, name, prob):
    """Linearization (theta, reaction coefficient, low ranks) and y = J x."""
    S = solver_for(prob)
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 5)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    lin = solver.linearize(st, u, w)
    (gt, gc) = S.get_factors()
    assert len(gt[1]) == lin.theta_lr.R and len(gc[1]) == lin.coef_lr.R
    for g, o in ((gt, lin.theta_lr), (gc, lin.coef_lr)):
        if o.R:
            assert rel(lowrank_product(g), lowrank_product((o.U, o.s, o.V))) < 1e-11
    x = W.random_vector(prob.unknowns, 11)
    y = S.apply(to_dev(torch, x)).cpu().numpy()
    assert rel(y, st.apply_J(x, lin.coef_q, lin.theta_q)) < 1e-11


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_apply_with_given_factors(gpu_lib, torch, name, prob):
    S = solver_for(prob)
    st = SpaceTime(prob)
    ft = W.random_factors(prob, 3, 1)
    fc = W.random_factors(prob, 4, 2, scale=5.0)
    S.set_factors(ft, fc)
    x = W.random_vector(prob.unknowns, 12)
    y = S.apply(to_dev(torch, x)).cpu().numpy()
    thq = st.lowrank_at_quad(LowRank(*ft))
    cq = st.lowrank_at_quad(LowRank(*fc))
    assert rel(y, st.apply_J(x, cq, thq)) < 1e-12


@pytest.mark.parametrize("precond", [0, 1], ids=["fd_sec32", "banded"])
@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_precond(gpu_lib, torch, name, prob, precond):
    """z = A-hat^{-1} r against the oracle's direct solve, for the fast
    diagonalization of Section 3.2 and for the banded time solve (before any
    linearization its time profiles are the shift a c1 and no theta, so it
    inverts the same A-hat).  Both are backward stable, so they differ by a
    few times cond(A-hat) times the unit roundoff (cond = 2.2e5 for the 3D
    p = 3 case, <= 1e4 for the others)."""
    S = solver_for(prob, precond=precond)
    st = SpaceTime(prob)
    r = W.random_vector(prob.unknowns, 13)
    z = S.precond(to_dev(torch, r)).cpu().numpy()
    kappa = np.linalg.cond(st.assemble_precond().toarray()) if prob.unknowns <= 2000 else 1e4
    assert rel(z, solver.precond_solve(st, r)) < max(1e-11, 20 * kappa * np.finfo(float).eps)


@pytest.mark.parametrize("nel_s", [(142, 4), (4, 142)], ids=["x1_144", "x2_144"])
def test_largest_spatial_extent(gpu_lib, torch, nel_s):
    """144 B-splines along one spatial axis, the most setup accepts (p = 2):
    the FD mode products then span nine 16-row tiles, along x1 (row-staged
    kernel) or along x2 (column-tile kernel).  Operator with given low-rank
    factors and both preconditioners against the oracle, in FP64 and FP32
    (cond(A-hat) = 814 and 267)."""
    from paper_2311_17500_amd.binding import MIXED_FP32
    prob = W.tiny(2, 2, 4, nel_t=3, nel_s=nel_s)
    st = SpaceTime(prob)
    assert max(st.n[:2]) == 144
    ft = W.random_factors(prob, 3, 1)
    fc = W.random_factors(prob, 4, 2, scale=5.0)
    x = W.random_vector(prob.unknowns, 12)
    want_y = st.apply_J(x, st.lowrank_at_quad(LowRank(*fc)), st.lowrank_at_quad(LowRank(*ft)))
    want_z = solver.precond_solve(st, x)
    xd = to_dev(torch, x)
    for precond in (0, 1):
        S = solver_for(prob, prec=MIXED_FP32, precond=precond)
        # before any coefficients are set both preconditioners invert A-hat
        assert rel(S.precond(xd).cpu().numpy(), want_z) < 1e-11
        assert rel(S.precond_lowp(xd).cpu().numpy(), want_z) < 1e-4
        S.set_factors(ft, fc)
        assert rel(S.apply(xd).cpu().numpy(), want_y) < 1e-12
        assert rel(S.apply_lowp(xd).cpu().numpy(), want_y) < 1e-5
        S.close()


@pytest.mark.parametrize("nel_t", [140, 141])
def test_w_update_time_extent(gpu_lib, torch, nel_t):
    """The w-update (one dense product along time on MFMA) at the largest
    time extents setup accepts: 142 and 143 time B-splines (p = 2), nine
    16-row tiles with a ragged last one, against the oracle.  Overlapping u
    and w are refused."""
    from paper_2311_17500_amd.binding import StIgaError
    prob = W.tiny(1, 2, 4, nel_t=nel_t)
    S = solver_for(prob)
    st = SpaceTime(prob)
    u, _ = W.smooth_state(prob, 7)
    assert st.n[-1] == nel_t + 2
    ud = to_dev(torch, u)
    assert rel(S.w_update(ud).cpu().numpy(), st.w_update_explicit(u)) < 1e-12
    with pytest.raises(StIgaError, match="EINVAL"):
        S._chk(S.lib.st_iga_w_update(S.ctx, S._p(ud), S._p(ud), S._s()))


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_residual_and_w(gpu_lib, torch, name, prob):
    S = solver_for(prob)
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 6)
    ud, wd = to_dev(torch, u), to_dev(torch, w)
    wg = S.w_update(ud).cpu().numpy()
    assert rel(wg, st.w_update_explicit(u)) < 1e-12
    S.linearize(ud, wd)
    lin = solver.linearize(st, u, w)
    r = S.residual(ud, wd).cpu().numpy()
    assert rel(r, st.residual(u, w, lin.theta_q)) < 1e-11


@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_krylov_solve(gpu_lib, torch, name, prob):
    import scipy.sparse.linalg as spla
    S = solver_for(prob)
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 8)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    lin = solver.linearize(st, u, w)
    b = W.random_vector(prob.unknowns, 14)
    x, it, rr = S.krylov(to_dev(torch, b), tol=1e-12)
    J = st.assemble_J(lin.coef_q, lin.theta_q)
    want = spla.splu(J.tocsc()).solve(b)
    assert rr <= 1e-12 and it > 0
    # forward error <= cond(J) x relative residual (cond(J) = 4.6e4 for the
    # 3D p = 3 case, <= 3e3 for the others)
    kappa = np.linalg.cond(J.toarray()) if prob.unknowns <= 2000 else 1e3
    assert rel(x.cpu().numpy(), want) < max(1e-9, kappa * 1e-12)


def test_nonlinear_steps_3d_p3(gpu_lib, torch):
    """The outer loop at d = 3, p = 3 (w-update, theta refreshed, both low
    ranks, residual, Krylov solve, update) for three iterations from the
    lifted datum, against the oracle's first three iterations (the oracle's
    explicit 3D p = 3 assembly is too slow for a converged solve here)."""
    prob = SMALL[6][1]
    st = SpaceTime(prob)
    uo, wo, log = solver.solve(st, tol=1e-11, max_outer=3)
    S = solver_for(prob, tol_lin=1e-12)
    c0, _ = S.lift()
    u = to_dev(torch, np.tile(c0, prob.n_t))
    w = S.vec(S.full)
    for k in range(3):
        it, rr, dinf = S.newton_step(u, u, w, refresh_theta=True, tol=1e-12)
        assert rr <= 1e-12 and dinf == pytest.approx(log.deltas[k], rel=1e-8)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(S.w_update(u).cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("name,prob", [SMALL[0], SMALL[1], SMALL[4]], ids=["1d_p2", "2d_p3", "cfg0"])
def test_full_nonlinear_solve(gpu_lib, name, prob):
    """Whole outer loop: Newton with lagged w, theta frozen below 1e-4."""
    S = solver_for(prob, tol_nonlin=1e-11, tol_lin=1e-12)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, tol=1e-11)
    assert rep.outer_iters == len(log.deltas)
    assert list(rep.rank_theta[: rep.outer_iters]) == log.ranks_theta
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("name,prob", [SMALL[1], SMALL[2], SMALL[3]], ids=["2d_p3", "3d_p2", "3d_p1"])
@pytest.mark.parametrize("slab", [1, 2, 3])
def test_apply_time_slabs(gpu_lib, torch, name, prob, slab):
    """The low-rank terms computed over time slabs (with their input halos)
    equal the oracle's operator, for the unknown and the full-vector forms."""
    S = solver_for(prob, coef_slab=slab)
    st = SpaceTime(prob)
    ft = W.random_factors(prob, 3, 1)
    fc = W.random_factors(prob, 4, 2, scale=5.0)
    S.set_factors(ft, fc)
    x = W.random_vector(prob.unknowns, 17)
    y = S.apply(to_dev(torch, x)).cpu().numpy()
    thq = st.lowrank_at_quad(LowRank(*ft))
    cq = st.lowrank_at_quad(LowRank(*fc))
    assert rel(y, st.apply_J(x, cq, thq)) < 1e-12
    u, w = W.smooth_state(prob, 4)
    r = S.residual(to_dev(torch, u), to_dev(torch, w)).cpu().numpy()
    assert rel(r, st.residual(u, w, thq)) < 1e-11


# Cases for the fused coefficient kernel along the slowest spatial axis: few
# columns, so the axis is split into B-spline ranges walked independently
# (with the elements at each range boundary walked by both neighbours).
CHUNKED = [("2d_p2_chunked", W.tiny(2, 2, 12, nel_t=5)),
           ("3d_p1_chunked", W.tiny(3, 1, 8, nel_t=3))]


@pytest.mark.parametrize("name,prob", CHUNKED, ids=[n for n, _ in CHUNKED])
def test_apply_chunked_axis(gpu_lib, torch, name, prob):
    from paper_2311_17500_amd.binding import MIXED_FP32
    st = SpaceTime(prob)
    ft = W.random_factors(prob, 2, 3)
    fc = W.random_factors(prob, 3, 4, scale=5.0)
    thq = st.lowrank_at_quad(LowRank(*ft))
    cq = st.lowrank_at_quad(LowRank(*fc))
    x = W.random_vector(prob.unknowns, 18)
    want = st.apply_J(x, cq, thq)
    S = solver_for(prob, prec=MIXED_FP32)
    S.set_factors(ft, fc)
    xd = to_dev(torch, x)
    assert rel(S.apply(xd).cpu().numpy(), want) < 1e-12
    # the FP32 operator: relative error a modest multiple of the unit roundoff
    assert rel(S.apply_lowp(xd).cpu().numpy(), want) < 1e-5
    # FP32 preconditioner (mode products along odd and even axis lengths)
    # against the FP64 one, which the oracle pins in test_precond
    z64 = S.precond(xd).cpu().numpy()
    assert rel(S.precond_lowp(xd).cpu().numpy(), z64) < 1e-5


def test_apply_nonuniform_knots(gpu_lib, torch):
    """Graded spatial knots with a double interior knot on the slowest axis:
    consecutive elements there start one or two B-splines apart."""
    prob = W.tiny(2, 2, 6, nel_t=4)
    kn = prob.uniform_knots()
    kn[0] = np.array([0, 0, 0, 0.2, 0.3, 0.55, 0.7, 0.9, 1, 1, 1], float)
    kn[1] = np.array([0, 0, 0, 0.1, 0.25, 0.25, 0.5, 0.8, 1, 1, 1], float)
    st = SpaceTime(prob, knots=kn)
    S = solver_for(prob, knots=kn)
    assert S.N_s == prob.N_s and S.unknowns == prob.unknowns
    ft = W.random_factors(prob, 2, 5)
    fc = W.random_factors(prob, 2, 6, scale=5.0)
    S.set_factors(ft, fc)
    x = W.random_vector(prob.unknowns, 19)
    y = S.apply(to_dev(torch, x)).cpu().numpy()
    want = st.apply_J(x, st.lowrank_at_quad(LowRank(*fc)), st.lowrank_at_quad(LowRank(*ft)))
    assert rel(y, want) < 1e-12


@pytest.mark.parametrize("reorth", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_krylov_gram_schmidt_modes(gpu_lib, torch, reorth, prec):
    """Every Gram-Schmidt mode (second pass only after heavy cancellation,
    always in the same step, or delayed into the next step) reaches the
    requested true residual against the oracle's assembled operator."""
    import scipy.sparse.linalg as spla
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32
    prob = SMALL[2][1]
    S = solver_for(prob, reorth=reorth, prec={"fp64": FP64, "mixed_fp32": MIXED_FP32}[prec])
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 9)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    lin = solver.linearize(st, u, w)
    J = st.assemble_J(lin.coef_q, lin.theta_q)
    b = W.random_vector(prob.unknowns, 15)
    tol = 1e-11 if prec == "fp64" else 1e-8
    x, it, rr = S.krylov(to_dev(torch, b), tol=tol)
    x = x.cpu().numpy()
    assert rr <= tol and it > 0
    assert rel(J @ x, b) <= 1.05 * tol
    assert rel(x, spla.splu(J.tocsc()).solve(b)) < 1e4 * tol


@pytest.mark.parametrize("reorth", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_krylov_graph_replay(gpu_lib, torch, prec, reorth):
    """Arnoldi steps replayed from HIP graphs give bit-identical solves to
    eager launches, on every replay, with eager work and synchronizations in
    between, and after a relinearization (graphs re-captured when the ranks
    change)."""
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32
    code = {"fp64": FP64, "mixed_fp32": MIXED_FP32}[prec]
    prob = SMALL[2][1]
    Sg = solver_for(prob, prec=code, graphs=1, reorth=reorth)
    Se = solver_for(prob, prec=code, graphs=0, reorth=reorth)
    tol = 1e-11 if prec == "fp64" else 1e-8
    for seed in (10, 11):
        u, w = W.smooth_state(prob, seed)
        ud, wd = to_dev(torch, u), to_dev(torch, w)
        Sg.linearize(ud, wd)
        Se.linearize(ud, wd)
        b = to_dev(torch, W.random_vector(prob.unknowns, seed + 20))
        xe, ite, rre = Se.krylov(b, tol=tol)
        xe = xe.cpu().numpy()
        for rep in range(3):
            xg, itg, rrg = Sg.krylov(b, tol=tol)
            torch.cuda.synchronize()
            assert itg == ite and rrg == rre
            assert np.array_equal(xg.cpu().numpy(), xe)
            Sg.apply(xg)                # eager work between the replays
            torch.cuda.synchronize()


@pytest.mark.parametrize("restart", [3, 30])
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_krylov_next_step_always_queued(gpu_lib, torch, prec, restart):
    """With the next Arnoldi step always queued before the host reads the
    current one (graphs = 2), every stop of a cycle happens with one more
    step already run on the device, which overwrites the provisional column
    of R and g that the back substitution needs; its per-step copies must
    give bit-identical solves to eager launches, over short (3) and long
    restart cycles."""
    from paper_2311_17500_amd.binding import FP64, MIXED_FP32
    code = {"fp64": FP64, "mixed_fp32": MIXED_FP32}[prec]
    prob = SMALL[2][1]
    Sq = solver_for(prob, prec=code, graphs=2, restart=restart)
    Se = solver_for(prob, prec=code, graphs=0, restart=restart)
    tol = 1e-11 if prec == "fp64" else 1e-8
    u, w = W.smooth_state(prob, 12)
    ud, wd = to_dev(torch, u), to_dev(torch, w)
    Sq.linearize(ud, wd)
    Se.linearize(ud, wd)
    b = to_dev(torch, W.random_vector(prob.unknowns, 32))
    xe, ite, rre = Se.krylov(b, tol=tol)
    xq, itq, rrq = Sq.krylov(b, tol=tol)
    assert rre <= tol
    assert itq == ite and rrq == rre
    assert np.array_equal(xq.cpu().numpy(), xe.cpu().numpy())


@pytest.mark.parametrize("name,prob", [SMALL[1], SMALL[2]], ids=["2d_p3", "3d_p2"])
def test_linearize_picard(gpu_lib, torch, name, prob):
    """Picard linearization (reaction coefficient C_r of eq. (3.8)): ranks,
    low-rank products and the operator against the oracle."""
    S = solver_for(prob, outer=1, alpha=0.5)
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 7)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    lin = solver.linearize(st, u, w, newton=False)
    (gt, gc) = S.get_factors()
    assert len(gt[1]) == lin.theta_lr.R and len(gc[1]) == lin.coef_lr.R
    for g, o in ((gt, lin.theta_lr), (gc, lin.coef_lr)):
        if o.R:
            assert rel(lowrank_product(g), lowrank_product((o.U, o.s, o.V))) < 1e-11
    x = W.random_vector(prob.unknowns, 21)
    y = S.apply(to_dev(torch, x)).cpu().numpy()
    assert rel(y, st.apply_J(x, lin.coef_q, lin.theta_q)) < 1e-11


def test_full_nonlinear_solve_picard(gpu_lib):
    """Whole outer loop in the Picard mode (C_r, relaxation 0.5) against the
    oracle's Picard loop: same iteration count and solution."""
    prob = SMALL[0][1]
    S = solver_for(prob, outer=1, alpha=0.5, tol_nonlin=1e-11, tol_lin=1e-12, max_outer=200)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, newton=False, tol=1e-11, max_outer=200)
    assert rep.outer_iters == len(log.deltas)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("prec", ["mixed_fp32", "mixed_bf16"])
def test_full_nonlinear_solve_mixed(gpu_lib, prec):
    """Whole outer loop with low-precision inner solves: the FP64 refinement
    makes each linear solve meet tol_lin in FP64, so the solution matches the
    oracle's FP64 loop to the nonlinear tolerance."""
    from paper_2311_17500_amd.binding import MIXED_FP32, MIXED_BF16
    prob = SMALL[2][1]
    S = solver_for(prob, prec={"mixed_fp32": MIXED_FP32, "mixed_bf16": MIXED_BF16}[prec],
                   tol_nonlin=1e-9, tol_lin=1e-10)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, tol=1e-9)
    assert abs(rep.outer_iters - len(log.deltas)) <= 1
    assert rel(u.cpu().numpy(), uo) < 1e-8
    assert rel(w.cpu().numpy(), wo) < 1e-8


def test_zero_datum_gives_zero(gpu_lib):
    """u0 = 0 and no source: I_ion(0, 0) = 0, so u = w = 0 exactly, theta's
    denominator is 0 (Theta = 0, rank 0) and one outer iteration suffices."""
    prob = W.tiny(2, 2, 5, nel_t=4, u0_kind=0)
    S = solver_for(prob)
    u, w, rep = S.solve()
    assert rep.outer_iters == 1 and rep.rank_theta[0] == 0
    assert not np.any(u.cpu().numpy()) and not np.any(w.cpu().numpy())


def test_zero_shift_preconditioner(gpu_lib, torch):
    """a c1 = 0: with an odd N_t - 1 the zero-frequency time block meets the
    constant Neumann mode (a zero pivot of the arrowhead), which setup rejects
    with EINVAL; with an even N_t - 1 every block is invertible and the
    preconditioner still equals the oracle's direct solve."""
    from paper_2311_17500_amd.binding import StIgaError, EINVAL
    odd = W.tiny(1, 2, 9, nel_t=7, c1=0.0)
    assert (odd.N_t - 1) % 2 == 1
    with pytest.raises(StIgaError) as e:
        solver_for(odd, precond=0)
    assert e.value.code == EINVAL
    even = W.tiny(1, 2, 9, nel_t=6, c1=0.0)
    assert (even.N_t - 1) % 2 == 0
    S = solver_for(even, precond=0)
    st = SpaceTime(even)
    r = W.random_vector(even.unknowns, 31)
    z = S.precond(to_dev(torch, r)).cpu().numpy()
    assert rel(z, solver.precond_solve(st, r)) < 1e-10
    # the banded time solve factorizes without pivoting and needs a c1 > 0
    with pytest.raises(StIgaError) as e:
        solver_for(even, precond=1)
    assert e.value.code == EINVAL


# Source-term stimuli of the paper's experiments (Section 4): a ball times a
# time window and a moving Gaussian times a time window, on time knots
# clustered around the source's on/off times (Section 4.2.1).
def _src_case(d, p, kind, nel=5, nel_t=12):
    kw = dict(u0_kind=0, f_kind=kind, f_t0=0.25, f_t1=0.45, f_amp=2.0)
    if kind == 1:
        kw.update(f_center=(0.3, 0.4, 0.5), f_radius=0.35)
    else:
        kw.update(f_center=(0.1, 0.5, 0.5), f_kappa=20.0, f_velocity=(0.8, 0.0, 0.2))
    prob = W.tiny(d, p, nel, nel_t=nel_t, **kw)
    kn = prob.uniform_knots()
    kn[d] = W.clustered_time_knots(nel_t, p, [0.25, 0.45], 0.01)
    return prob, kn


SRC = [("1d_ball", 1, 2, 1), ("2d_gauss", 2, 3, 2), ("3d_ball", 3, 2, 1), ("3d_gauss_p3", 3, 3, 2)]


@pytest.mark.parametrize("name,d,p,kind", SRC, ids=[c[0] for c in SRC])
def test_source_theta_and_residual(gpu_lib, torch, name, d, p, kind):
    """Theta (residual -f inside eq. (3.6)) and N(u) (with -int f v) against
    the oracle on clustered time knots, at a non-trivial state."""
    prob, kn = _src_case(d, p, kind, nel=4 if d == 3 else 6, nel_t=10)
    st = SpaceTime(prob, knots=kn)
    S = solver_for(prob, knots=kn)
    u, w = W.smooth_state(prob, 12)
    ud, wd = to_dev(torch, u), to_dev(torch, w)
    th = S.theta_grid(ud, wd).cpu().numpy()
    assert np.max(np.abs(th - st.theta_grid(u, w).reshape(-1))) < 1e-12
    S.linearize(ud, wd)
    lin = solver.linearize(st, u, w)
    assert len(S.get_factors()[0][1]) == lin.theta_lr.R
    r = S.residual(ud, wd).cpu().numpy()
    assert rel(r, st.residual(u, w, lin.theta_q)) < 1e-11


@pytest.mark.parametrize("name,d,p,kind", [("1d_ball", 1, 2, 1), ("2d_gauss_p2", 2, 2, 2)],
                         ids=["1d_ball", "2d_gauss_p2"])
def test_source_driven_solve(gpu_lib, name, d, p, kind):
    """The paper's setting: zero initial datum, the excitation comes from the
    source.  Whole nonlinear solve on clustered time knots against the
    oracle's loop."""
    prob, kn = _src_case(d, p, kind, nel=8 if d == 1 else 4, nel_t=12)
    S = solver_for(prob, knots=kn, tol_nonlin=1e-11, tol_lin=1e-12)
    st = SpaceTime(prob, knots=kn)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, tol=1e-11)
    assert np.max(np.abs(uo)) > 0.1          # the source excites the tissue
    assert rep.outer_iters == len(log.deltas)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


# The fixed-point scheme of Section 3.1 as the paper states it (outer = 2):
# M_R with the exact C_r(u^k, w^k) at every Gauss point, u and w relaxed.
@pytest.mark.parametrize("name,prob", [SMALL[0], SMALL[1], SMALL[2]], ids=["1d_p2", "2d_p3", "3d_p2"])
def test_linearize_exact_reaction(gpu_lib, torch, name, prob):
    """J with the exact C_r at the Gauss points (no low rank) and the low-rank
    theta, in FP64 and in the FP32 operator of a mixed context."""
    from paper_2311_17500_amd.binding import MIXED_FP32
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 7)
    th = st.lowrank(st.theta_grid(u, w), 0.1)
    want_x = W.random_vector(prob.unknowns, 22)
    want = st.apply_J(want_x, st.reaction_at_quad(u, w), st.lowrank_at_quad(th))
    S = solver_for(prob, outer=2, alpha=0.5, prec=MIXED_FP32)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    gt, gc = S.get_factors()
    assert len(gt[1]) == th.R and len(gc[1]) == 0
    xd = to_dev(torch, want_x)
    assert rel(S.apply(xd).cpu().numpy(), want) < 1e-11
    assert rel(S.apply_lowp(xd).cpu().numpy(), want) < 1e-5


@pytest.mark.parametrize("name,prob", [SMALL[0], SMALL[4]], ids=["1d_p2", "cfg0"])
def test_paper_picard_solve(gpu_lib, name, prob):
    """The whole fixed-point loop with the paper's stopping rule (change of
    the iterate <= 1e-4, theta refreshed every iteration): same number of
    iterations and the same final (u, w) as the oracle's literal scheme."""
    S = solver_for(prob, outer=2, alpha=0.5, tol_nonlin=1e-4, tol_lin=1e-12, max_outer=200)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve_picard(st, tol=1e-4, max_outer=200)
    assert rep.outer_iters == len(log.deltas)
    assert list(rep.rank_theta[: rep.outer_iters]) == log.ranks_theta[:64]
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


def test_paper_picard_tight(gpu_lib):
    """The same scheme run to 1e-11 with theta frozen below 1e-4 on both sides."""
    prob = SMALL[1][1]
    S = solver_for(prob, outer=2, alpha=0.5, tol_nonlin=1e-11, tol_lin=1e-12, max_outer=300)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve_picard(st, tol=1e-11, max_outer=300, theta_freeze=1e-4)
    assert rep.outer_iters == len(log.deltas)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("outer", [0, 2])
def test_galerkin_solve(gpu_lib, outer):
    """Plain Galerkin (su = 0, no stabilization term): Newton with lagged w,
    and the paper's fixed-point scheme, against the oracle without SU."""
    prob = SMALL[0][1]
    st = SpaceTime(prob, su=False)
    if outer == 0:
        S = solver_for(prob, su=0, tol_nonlin=1e-11, tol_lin=1e-12)
        uo, wo, log = solver.solve(st, tol=1e-11)
    else:
        S = solver_for(prob, su=0, outer=2, alpha=0.5, tol_nonlin=1e-11, tol_lin=1e-12, max_outer=300)
        uo, wo, log = solver.solve_picard(st, tol=1e-11, max_outer=300)
    u, w, rep = S.solve()
    assert rep.outer_iters == len(log.deltas)
    assert rep.rank_theta[0] == 0
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("outer", [0, 2])
@pytest.mark.parametrize("name,prob", [SMALL[0], SMALL[1], SMALL[2], SMALL[5]], ids=["1d_p2", "2d_p3", "3d_p2", "3d_p3"])
def test_banded_precond_after_linearization(gpu_lib, torch, name, prob, outer):
    """The banded preconditioner after a linearization: time profiles of
    theta and of the reaction coefficient (low rank for Newton, exact C_r for
    the Section 3.1 scheme) in the time matrices, against a sparse LU of the
    oracle's assembly of the same form; FP32 in a mixed context."""
    import scipy.sparse.linalg as spla
    from paper_2311_17500_amd.binding import MIXED_FP32
    st = SpaceTime(prob)
    u, w = W.smooth_state(prob, 44)
    if outer == 0:
        lin = solver.linearize(st, u, w)
        coef_q, theta_q = lin.coef_q, lin.theta_q
    else:
        coef_q = st.reaction_at_quad(u, w)
        theta_q = st.lowrank_at_quad(st.lowrank(st.theta_grid(u, w), 0.1))
    c_t, th_t = st.precond_time_profiles(coef_q, theta_q)
    assert np.max(th_t) > 0.0
    want_A = st.assemble_precond_profiles(c_t, th_t)
    S = solver_for(prob, prec=MIXED_FP32, outer=outer, alpha=1.0 if outer == 0 else 0.5, precond=1)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    r = W.random_vector(prob.unknowns, 45)
    want = spla.splu(want_A.tocsc()).solve(r)
    rd = to_dev(torch, r)
    assert rel(S.precond(rd).cpu().numpy(), want) < 1e-10
    assert rel(S.precond_lowp(rd).cpu().numpy(), want) < 1e-4


def test_galerkin_mixed_no_low_rank(gpu_lib, torch):
    """A mixed-precision context with no low-rank terms at all (Galerkin, exact
    C_r): the empty factor tables are skipped, the FP32 operator matches."""
    from paper_2311_17500_amd.binding import MIXED_FP32
    prob = SMALL[1][1]
    st = SpaceTime(prob, su=False)
    u, w = W.smooth_state(prob, 8)
    S = solver_for(prob, su=0, outer=2, alpha=0.5, prec=MIXED_FP32)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    x = W.random_vector(prob.unknowns, 23)
    want = st.apply_J(x, st.reaction_at_quad(u, w), None)
    assert rel(S.apply(to_dev(torch, x)).cpu().numpy(), want) < 1e-11
    assert rel(S.apply_lowp(to_dev(torch, x)).cpu().numpy(), want) < 1e-5


# Failure handling, forced from the host (every kernel still exits normally).
@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_krylov_stagnation_enoconv(gpu_lib, torch, prec):
    """A restart cycle must cut the true residual by 99.9999 % to count as
    progress (stall_reduction), one stalled cycle is allowed (stall_cycles):
    the solve ends with ENOCONV instead of running to max_krylov; the same
    context then solves normally once the options are back to defaults."""
    from paper_2311_17500_amd.binding import ENOCONV, FP64, MIXED_FP32, StIgaError
    prob = SMALL[2][1]
    code = {"fp64": FP64, "mixed_fp32": MIXED_FP32}[prec]
    S = solver_for(prob, prec=code, restart=2, stall_cycles=1, stall_reduction=0.999999, graphs=0)
    u, w = W.smooth_state(prob, 9)
    S.linearize(to_dev(torch, u), to_dev(torch, w))
    b = to_dev(torch, W.random_vector(prob.unknowns, 15))
    with pytest.raises(StIgaError) as e:
        S.krylov(b, tol=1e-10)
    assert e.value.code == ENOCONV and "stagnated" in str(e.value)
    S2 = solver_for(prob, prec=code, restart=2, graphs=0)
    S2.linearize(to_dev(torch, u), to_dev(torch, w))
    x, it, rr = S2.krylov(b, tol=1e-8)
    assert rr <= 1e-8


def test_newton_to_picard_switch(gpu_lib):
    """A source-driven case on which Newton with refreshed theta circles
    without converging (theta's rank flips): with picard_switch = 2 the solve
    continues as Picard after the update grows twice in a row and converges;
    the switch point, iteration count and solution match the oracle's loop
    with the same rule."""
    prob, kn = _src_case(2, 2, 2, nel=4, nel_t=9)
    S = solver_for(prob, knots=kn, tol_nonlin=1e-11, tol_lin=1e-12, max_outer=150, picard_switch=2)
    st = SpaceTime(prob, knots=kn)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, tol=1e-11, max_outer=150, picard_switch=2)
    assert log.switched_at > 0 and rep.switched_at == log.switched_at
    assert rep.outer_iters == len(log.deltas)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10


@pytest.mark.parametrize("precond", [0, 1], ids=["fd_sec32", "banded"])
@pytest.mark.parametrize("name,prob", SMALL[:6], ids=[n for n, _ in SMALL[:6]])
def test_precond_bf16_mfma(gpu_lib, torch, name, prob, precond):
    """BF16 mode: the eigenvector mode products run on the BF16 MFMA with
    FP32 accumulation (BF16 vectors and matrices).  Against the oracle's
    direct solve the error is a small multiple of the BF16 unit roundoff
    (3.9e-3) times the conditioning of the eigenvector bases."""
    from paper_2311_17500_amd.binding import MIXED_BF16
    S = solver_for(prob, prec=MIXED_BF16, precond=precond)
    st = SpaceTime(prob)
    r = W.random_vector(prob.unknowns, 33)
    z = S.precond_lowp(to_dev(torch, r)).cpu().numpy()
    want = solver.precond_solve(st, r)
    assert rel(z, want) < 5e-2


# Separable geometry maps x_l = F_l(eta_l) (Section 2; the spatial part of G).
GEO = [("1d_graded", W.tiny(1, 2, 9, nel_t=7, map_kind=(2, 0, 0), map_param=((0.0, 2.0, 2.0),) * 3,
                            u0_center=(0.3, 0.0, 0.0))),
       ("2d_graded", W.tiny(2, 3, 5, nel_t=6, map_kind=(2, 2, 0),
                            map_param=((0.0, 1.5, 2.5), (-0.5, 0.5, -1.5), (0, 1, 0)), u0_center=(0.0, 0.5, 0.0))),
       ("3d_mixed", W.tiny(3, 2, 3, nel_t=5, map_kind=(1, 2, 2),
                           map_param=((0.0, 1.2, 0.0), (0.0, 1.0, 1.5), (0.0, 0.8, -2.0)), u0_radius=0.5))]


@pytest.mark.parametrize("name,prob", GEO, ids=[n for n, _ in GEO])
def test_geometry_linearization_and_operators(gpu_lib, torch, name, prob):
    """On a mapped box: the lifted datum at the mapped Greville points (bit
    exact), theta (physical Laplacian, interpolation at mapped Greville
    points), the linearized operator, the FD preconditioner built from the
    mapped 1D pencils against the oracle's direct solve, and the residual."""
    st = SpaceTime(prob)
    S = solver_for(prob, precond=0)
    c0, cnt = S.lift()
    assert np.array_equal(c0, st.lift()) and cnt > 0
    u, w = W.smooth_state(prob, 14)
    ud, wd = to_dev(torch, u), to_dev(torch, w)
    th = S.theta_grid(ud, wd).cpu().numpy()
    assert np.max(np.abs(th - st.theta_grid(u, w).reshape(-1))) < 1e-12
    S.linearize(ud, wd)
    lin = solver.linearize(st, u, w)
    gt, gc = S.get_factors()
    assert len(gt[1]) == lin.theta_lr.R and len(gc[1]) == lin.coef_lr.R
    x = W.random_vector(prob.unknowns, 34)
    assert rel(S.apply(to_dev(torch, x)).cpu().numpy(), st.apply_J(x, lin.coef_q, lin.theta_q)) < 1e-11
    kappa = np.linalg.cond(st.assemble_precond().toarray())
    z = S.precond(to_dev(torch, x)).cpu().numpy()
    assert rel(z, solver.precond_solve(st, x)) < max(1e-11, 20 * kappa * np.finfo(float).eps)
    r = S.residual(ud, wd).cpu().numpy()
    assert rel(r, st.residual(u, w, lin.theta_q)) < 1e-11


@pytest.mark.parametrize("name,prob", GEO[:2], ids=[n for n, _ in GEO[:2]])
def test_geometry_full_solve(gpu_lib, name, prob):
    S = solver_for(prob, tol_nonlin=1e-11, tol_lin=1e-12)
    st = SpaceTime(prob)
    u, w, rep = S.solve()
    uo, wo, log = solver.solve(st, tol=1e-11)
    assert rep.outer_iters == len(log.deltas)
    assert rel(u.cpu().numpy(), uo) < 1e-10
    assert rel(w.cpu().numpy(), wo) < 1e-10
