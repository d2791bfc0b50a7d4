"""CPU checks of the native library: it loads, exports every symbol of
include/st_iga.h, and its host-side setup (1D splines, matrices, tau, the
fast-diagonalization factors) agrees with the oracle and with the structure
fixed by Section 3.2.  No device calls are made."""
import os
import re

import numpy as np
import pytest

import st_workloads as W
from oracle.spacetime import SpaceTime
from oracle.splines import find_span
from paper_2311_17500_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "st_iga.h")).read()
    names = set(re.findall(r"\b(st_iga_[a-z_]+)\s*\(", hdr))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(binding.EXPORTS)


CASES = [W.tiny(1, 2, 7, T=3.0), W.tiny(2, 3, 5, nel_t=6), W.tiny(3, 1, 3, nel_t=4), W.config(1)]


@pytest.mark.parametrize("prob", CASES[:3])
def test_matrices_match_oracle(prob):
    st = SpaceTime(prob)
    d = prob.d
    from oracle.operators1d import mass, stiffness, advection
    for l in range(d + 1):
        n = st.n[l]
        assert np.allclose(binding.host_query(prob, 0, l), st.grev_s[l] if l < d else
                           np.concatenate([[0.0], st.grev_t]) * 1.0 / prob.T * prob.T, atol=1e-15) or l == d
        for what, fn in ((1, mass), (2, stiffness), (3, advection)):
            A = binding.host_query(prob, what, l).reshape(n, n)
            B = fn(st.kn[l], st.p[l])
            assert np.allclose(A, B, rtol=1e-13, atol=1e-13 * np.abs(B).max())


@pytest.mark.parametrize("prob", CASES)
def test_spans_bit_exact(prob):
    """First non-zero basis index at each Gauss point equals the span - p."""
    st = SpaceTime(prob, mode="tensor")
    for l in range(prob.d + 1):
        got = binding.host_query(prob, 9, l).astype(np.int64)
        xq = binding.host_query(prob, 8, l)
        xq = xq[: len(xq) // 2]
        assert np.allclose(xq, st.quad[l][0], rtol=0, atol=1e-15)
        want = np.array([find_span(st.kn[l], st.p[l], x) - st.p[l] for x in st.quad[l][0]])
        assert np.array_equal(got, want)


@pytest.mark.parametrize("prob", CASES)
def test_windows_bit_exact(prob):
    st = SpaceTime(prob, mode="tensor")
    for l in range(prob.d + 1):
        got = binding.host_query(prob, 10, l).astype(np.int64).reshape(-1, 2)
        want = np.array(st.element_windows(l, 1 if l == prob.d else 0))
        assert np.array_equal(got, want)


@pytest.mark.parametrize("prob", CASES)
def test_tau_matches_oracle(prob):
    st = SpaceTime(prob, mode="tensor")
    got = binding.host_query(prob, 4, prob.d).reshape(prob.p_t, -1)
    for k in range(prob.p_t):
        ref = st.tau_q[k]
        assert np.allclose(got[k], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("prob", CASES[:3])
def test_spatial_eigen(prob):
    """U^T M U = I, U^T K U = diag(lambda), lambda_0 = 0 (Neumann constant mode)."""
    st = SpaceTime(prob)
    for l in range(prob.d):
        n = st.n[l]
        U = binding.host_query(prob, 6, l).reshape(n, n)
        lam = binding.host_query(prob, 5, l)
        M = binding.host_query(prob, 1, l).reshape(n, n)
        K = binding.host_query(prob, 2, l).reshape(n, n)
        assert np.allclose(U.T @ M @ U, np.eye(n), atol=1e-11)
        assert np.allclose(U.T @ K @ U, np.diag(lam), atol=1e-9 * lam.max())
        assert abs(lam[0]) < 1e-9 and np.all(np.diff(lam) >= -1e-12)


def test_spatial_eigen_pi_squared():
    """Second eigenvalue of the Neumann pencil approximates pi^2 (continuous
    Neumann Laplacian on (0,1): (k pi)^2)."""
    prob = W.tiny(1, 3, 32)
    lam = binding.host_query(prob, 5, 0)
    assert abs(lam[1] - np.pi ** 2) < 1e-6 * np.pi ** 2
    assert abs(lam[2] - 4 * np.pi ** 2) < 1e-5 * 4 * np.pi ** 2


@pytest.mark.parametrize("prob", CASES)
def test_time_fd_structure(prob):
    """Section 3.2: U_t^T M_t U_t = I and U_t^T W_t U_t = [[D, l], [-l^T, sigma]]
    with D block-diagonal skew, sigma = rho^2 / 2 (rho = last entry of U_t)."""
    Nt = prob.n_t - 1
    v = binding.host_query(prob, 7, prob.d)
    U = v[: Nt * Nt].reshape(Nt, Nt)
    mu = v[Nt * Nt: Nt * Nt + Nt - 1]
    l = v[Nt * Nt + Nt - 1: Nt * Nt + 2 * (Nt - 1)]
    sigma = v[-1]
    n = prob.n_t
    Wf = binding.host_query(prob, 3, prob.d).reshape(n, n)
    Mf = binding.host_query(prob, 1, prob.d).reshape(n, n)
    Wt, Mt = Wf[1:, 1:], Mf[1:, 1:]
    assert np.allclose(U.T @ Mt @ U, np.eye(Nt), atol=1e-10)
    D = U.T @ Wt @ U
    scale = np.abs(D).max()
    assert np.allclose(D[:-1, -1], l, atol=1e-10 * scale)
    assert np.allclose(D[-1, :-1], -l, atol=1e-10 * scale)
    assert abs(D[-1, -1] - sigma) < 1e-10 * scale
    assert abs(sigma - U[-1, -1] ** 2 / 2) < 1e-10 * scale
    core = D[:-1, :-1]
    blk = np.zeros_like(core)
    for a in range(0, Nt - 2, 2):
        blk[a, a + 1] = mu[a]
        blk[a + 1, a] = mu[a + 1]
    assert np.allclose(core, blk, atol=1e-9 * scale)
    assert np.allclose(core, -core.T, atol=1e-9 * scale)


def test_invalid_problems_rejected(lib):
    """EINVAL for knots that are not open, decreasing knots, bad degrees."""
    prob = W.tiny(1, 2, 4)
    kn = prob.uniform_knots()
    bad = [k.copy() for k in kn]
    bad[0][0] = 0.1
    with pytest.raises(binding.StIgaError):
        binding.host_query(prob, 0, 0, knots=bad)
    bad = [k.copy() for k in kn]
    bad[0][4], bad[0][5] = bad[0][5], bad[0][4]
    with pytest.raises(binding.StIgaError):
        binding.host_query(prob, 0, 0, knots=bad)
    import dataclasses
    with pytest.raises(binding.StIgaError):
        binding.host_query(dataclasses.replace(prob, sigma=(-1.0,)), 0, 0)
    with pytest.raises(binding.StIgaError):
        binding.host_query(dataclasses.replace(prob, T=0.0), 0, 0)


def _graded_knots(prob):
    kn = prob.uniform_knots()
    kn[0] = np.array([0, 0, 0, 0.2, 0.3, 0.55, 0.7, 0.9, 1, 1, 1], float)
    kn[1] = np.array([0, 0, 0, 0.1, 0.25, 0.25, 0.5, 0.8, 1, 1, 1], float)
    return kn


@pytest.mark.parametrize("case", ["2d_p2_12", "3d_p1_8", "2d_p3_5", "cfg2", "cfg4", "graded", "1d", "2d_p5"])
def test_fused_coefficient_plan(lib, case):
    """The B-spline ranges of the fused coefficient kernel partition the
    slowest spatial axis in order, and each range walks exactly the elements
    whose B-splines meet it (checked by brute force over the elements)."""
    knots = None
    prob = {"2d_p2_12": W.tiny(2, 2, 12, nel_t=5), "3d_p1_8": W.tiny(3, 1, 8, nel_t=3),
            "2d_p3_5": W.tiny(2, 3, 5, nel_t=6), "cfg2": W.config(2), "cfg4": W.config(4),
            "graded": W.tiny(2, 2, 6, nel_t=4), "1d": W.tiny(1, 2, 9, nel_t=7),
            "2d_p5": W.tiny(2, 5, 4, nel_t=3)}[case]
    if case == "graded":
        knots = _graded_knots(prob)
    plan = binding.host_query(prob, 11, 0, knots=knots)
    enabled, slab, nch = int(plan[0]), int(plan[1]), int(plan[2])
    assert enabled == (prob.d >= 2 and prob.p_s <= 4)
    if not enabled:
        return
    ax = prob.d - 1
    first_q = binding.host_query(prob, 9, ax, knots=knots).astype(int)
    p = prob.p_s
    efirst = first_q[:: p + 1]
    n = len(knots[ax]) - p - 1 if knots is not None else prob.nel_s[ax] + p
    assert 1 <= slab <= prob.N_t
    ch = plan[3:].astype(int).reshape(nch, 4)
    assert ch[0, 2] == 0 and ch[-1, 3] == n
    assert np.all(ch[1:, 2] == ch[:-1, 3]) and np.all(ch[:, 3] > ch[:, 2])
    for e0, e1, d0, d1 in ch:
        touch = [e for e, f in enumerate(efirst) if f + p >= d0 and f < d1]
        assert (e0, e1) == (min(touch), max(touch) + 1)
        assert np.all(np.diff(efirst[e0:e1]) >= 1) and np.all(np.diff(efirst[e0:e1]) <= p + 1)
    if case in ("2d_p2_12", "3d_p1_8"):
        assert nch > 1      # the GPU parity cases for split axes


@pytest.mark.parametrize("n,rank", [(1, 1), (2, 0), (5, 2), (49, 3), (49, 49), (130, 4), (130, 130)])
def test_host_symeig(lib, n, rank):
    """The Gram-matrix eigensolver of the truncated SVD: A Q = Q diag(lam),
    Q orthogonal, lam ascending and equal to LAPACK's, the null space of a
    rank-deficient Gram matrix resolved (eigenvalues ~ 0)."""
    rng = np.random.default_rng(n * 1000 + rank)
    X = rng.standard_normal((n, max(rank, 1))) * (1.0 if rank else 0.0)
    A = X @ X.T
    lam, Q = binding.host_symeig(A)
    scale = max(np.max(np.abs(lam)), 1e-300) if rank else 1.0
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(A @ Q - Q * lam)) <= 1e-13 * scale
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-12
    assert np.max(np.abs(lam - np.linalg.eigvalsh(A))) <= 1e-12 * scale
    assert np.sum(np.abs(lam) > 1e-10 * scale) == (min(rank, n) if rank else 0)


def test_invalid_options_rejected(lib):
    """Options outside their documented ranges give no workspace size (the
    same validation rejects them in setup with EINVAL)."""
    prob = W.tiny(2, 2, 4)
    assert binding.workspace_bytes(prob) > 0
    for kw in ({"reorth": 3}, {"reorth": -1}, {"restart": 0}, {"restart": 65}, {"graphs": 3}, {"graphs": -1}):
        assert binding.workspace_bytes(prob, **kw) == 0, kw
    for r in (0, 1, 2):
        assert binding.workspace_bytes(prob, reorth=r) > 0
        assert binding.workspace_bytes(prob, graphs=r) > 0
    # stabilization modes: SUPG + shock capturing runs in the fixed-point scheme
    for kw in ({"su": 3}, {"su": -1}, {"su": 2, "outer": 0}, {"su": 2, "outer": 1},
               {"su": 2, "outer": 2, "sc_c": -1.0}, {"su": 2, "outer": 2, "sc_c": float("nan")}):
        assert binding.workspace_bytes(prob, **kw) == 0, kw
    assert binding.workspace_bytes(prob, su=2, outer=2, sc_c=0.0) > 0


def test_time_regularity_per_stabilization(lib):
    """C^0 time splines: SU (which needs C^{p_t - 1}) is rejected, Galerkin and
    SUPG + shock capturing are accepted; SUPG sizes its extra tables."""
    prob = W.tiny(2, 3, 4, nel_t=5)
    kn = prob.uniform_knots()
    kn[2] = W.c0_time_knots(5, 3)
    assert binding.workspace_bytes(prob, kn, su=1) == 0
    assert binding.workspace_bytes(prob, kn, su=0) > 0
    sup = binding.workspace_bytes(prob, kn, su=2, outer=2)
    assert sup > binding.workspace_bytes(prob, kn, su=0, outer=2)


@pytest.mark.parametrize("kind", ["indefinite", "clustered", "tridiag_tiny", "diagonal", "graded"])
def test_host_symeig_structures(lib, kind):
    """The same checks on matrices that stress deflation and shifting:
    indefinite spectra, clustered and repeated eigenvalues, tiny
    off-diagonals, an already diagonal matrix, and graded magnitudes."""
    rng = np.random.default_rng(["indefinite", "clustered", "tridiag_tiny", "diagonal", "graded"].index(kind))
    n = 37
    if kind == "indefinite":
        X = rng.standard_normal((n, n))
        A = X + X.T
    elif kind == "clustered":
        Qr, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam0 = np.concatenate([np.full(10, 2.0), np.full(10, 2.0 + 1e-12), rng.uniform(-1, 1, n - 20)])
        A = (Qr * lam0) @ Qr.T
        A = 0.5 * (A + A.T)
    elif kind == "tridiag_tiny":
        A = np.diag(rng.uniform(-1, 1, n)) + np.diag(np.full(n - 1, 1e-17), 1) + np.diag(np.full(n - 1, 1e-17), -1)
    elif kind == "diagonal":
        A = np.diag(rng.uniform(-3, 3, n))
    else:
        Qr, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam0 = 10.0 ** rng.uniform(-12, 3, n)
        A = (Qr * lam0) @ Qr.T
        A = 0.5 * (A + A.T)
    lam, Q = binding.host_symeig(A)
    scale = np.max(np.abs(np.linalg.eigvalsh(A)))
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(A @ Q - Q * lam)) <= 1e-13 * scale * n
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-13 * n
    assert np.max(np.abs(lam - np.linalg.eigvalsh(A))) <= 1e-13 * scale * n


def test_host_symeig_rejects_nonfinite(lib):
    A = np.eye(4)
    A[1, 2] = A[2, 1] = np.nan
    with pytest.raises(binding.StIgaError):
        binding.host_symeig(A)


def test_server_failure_releases_slot(monkeypatch):
    """A request whose solve raises anything (not only a library error) is
    recorded as failed, gives its slot and memory back, and the loop goes on
    to the next request."""
    import contextlib
    import types
    from paper_2311_17500_amd import serve

    calls = []

    class Boom:
        def __init__(self, prob, **kw):
            calls.append(prob)
            raise RuntimeError("allocation failed")

    monkeypatch.setattr(binding, "Solver", Boom)
    monkeypatch.setattr(binding, "workspace_bytes", lambda prob, **o: 1000)
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(device=lambda d: contextlib.nullcontext()))
    srv = object.__new__(serve.Server)
    srv.torch, srv.device, srv.slots, srv.budget = fake_torch, None, 1, 10 ** 9
    srv.options, srv.keep_results, srv.streams = {}, False, [None]
    reqs = [(0.0, W.tiny(2, 2, 4)), (0.0, W.tiny(2, 2, 5))]
    recs = srv.run(reqs)
    assert len(calls) == 2
    assert all(r.status.startswith("RuntimeError") for r in recs)
    assert all(r.finished >= r.admitted for r in recs)
    assert serve.summarize(recs)["completed"] == 0


def test_serving_overlap_stats():
    """In-flight and same-shape counts at each admission, on hand-built
    records: A [0, 3) shape a, B [1, 2) shape b, C [1.5, 4) shape a."""
    from paper_2311_17500_amd import serve
    R = serve.Record
    recs = [R(0, 0.0, admitted=0.0, finished=3.0, shape="a"),
            R(1, 1.0, admitted=1.0, finished=2.0, shape="b"),
            R(2, 1.5, admitted=1.5, finished=4.0, shape="a")]
    st = serve.overlap_stats(recs)
    assert st["in_flight_at_admission_mean"] == (0 + 1 + 2) / 3
    assert st["same_shape_in_flight_mean"] == (0 + 0 + 1) / 3
    assert st["admissions_with_same_shape_partner"] == 1 / 3
    assert st["distinct_shapes"] == 2


def test_eigen_setup_cache_is_transparent(lib):
    """The process-wide cache of the 1D eigen setups returns exactly what a
    fresh computation gives: a shape seen for the first time, the same shape
    again (a cache hit, with another sigma), and again after more distinct
    shapes than the cache holds (evicted, recomputed)."""
    def knots(seed):
        rng = np.random.default_rng(seed)
        inner = np.sort(rng.uniform(0.05, 0.95, 6))
        return np.concatenate([np.zeros(3), inner, np.ones(3)])

    def prob_for(seed, sigma):
        P = W.tiny(2, 2, 7, nel_t=7)
        P.sigma = sigma
        kn = P.uniform_knots()
        kn[0] = knots(seed)
        kn[2] = knots(seed + 1000)
        return P, kn

    def setup(P, kn):
        return [binding.host_query(P, w, 0, kn) for w in (5, 6)] + [binding.host_query(P, 7, 2, kn),
                                                                   binding.host_query(P, 4, 2, kn)]

    P, kn = prob_for(12345, (1e-3, 2.5e-4))
    first = setup(P, kn)
    P2, kn2 = prob_for(12345, (3e-3, 1e-4))
    again = setup(P2, kn2)
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    for s in range(40):                       # more distinct shapes than the cache keeps
        Pi, kni = prob_for(20000 + s, (1e-3, 2.5e-4))
        binding.host_query(Pi, 5, 0, kni)
        binding.host_query(Pi, 7, 2, kni)
    later = setup(P, kn)
    for a, b in zip(first, later):
        assert np.array_equal(a, b)
