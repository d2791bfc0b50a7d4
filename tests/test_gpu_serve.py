"""Serving: continuous batching gives each request the same result it gets
alone (contexts are independent, reductions deterministic), and served
results match the oracle's nonlinear solve."""
import numpy as np
import pytest

import st_workloads as W

pytestmark = pytest.mark.gpu


def small_stream():
    out = []
    for k, (nel, nel_t, p, sx, cx) in enumerate([(8, 8, 2, 1e-3, 0.2), (10, 6, 3, 3e-4, 0.7), (6, 8, 2, 5e-3, 0.5),
                                                 (12, 8, 3, 1e-4, 0.1), (8, 10, 2, 2e-3, 0.9), (6, 6, 3, 1e-3, 0.4)]):
        prob = W.Problem(d=2, p_s=p, p_t=p, nel_s=(nel, nel), nel_t=nel_t, sigma=(sx, sx / 4),
                         u0_center=(cx, 0.5, 0.0), u0_radius=0.3, **W._RM)
        out.append((0.0, prob))
    return out


@pytest.mark.parametrize("precond", [0, 1])
def test_solo_equals_mix(gpu_lib, precond):
    from paper_2311_17500_amd.binding import MIXED_FP32
    from paper_2311_17500_amd.serve import Server
    reqs = small_stream()
    opts = dict(prec=MIXED_FP32, tol_lin=1e-8, tol_nonlin=1e-8, precond=precond)
    solo = Server(slots=1, keep_results=True, **opts).run(reqs)
    mix = Server(slots=len(reqs), keep_results=True, **opts).run(reqs)
    for a, b in zip(solo, mix):
        assert a.status == "ok" and b.status == "ok", (a.status, b.status)
        assert np.max(np.abs(a.u - b.u)) <= 1e-12 * np.max(np.abs(a.u))


@pytest.mark.parametrize("precond", [0, 1])
def test_served_matches_oracle(gpu_lib, precond):
    from oracle import solver as osolver
    from oracle.spacetime import SpaceTime
    from paper_2311_17500_amd.binding import MIXED_FP32
    from paper_2311_17500_amd.serve import Server
    reqs = small_stream()[:2]
    recs = Server(slots=2, keep_results=True, prec=MIXED_FP32, tol_lin=1e-10, tol_nonlin=1e-10,
                  precond=precond).run(reqs)
    for (t, prob), r in zip(reqs, recs):
        uo, wo, log = osolver.solve(SpaceTime(prob), tol=1e-10)
        assert r.status == "ok"
        assert np.linalg.norm(r.u - uo) / np.linalg.norm(uo) < 1e-8


@pytest.mark.parametrize("precond", [0, 1])
def test_stream_prefix_completes(gpu_lib, precond):
    """The first 128 requests of the seeded serving stream (2D, up to 130
    time layers, several hundred Krylov iterations per request) all converge
    with the default Arnoldi options (long restart cycles keep the basis
    vectors of order one), with either preconditioner."""
    from paper_2311_17500_amd.binding import MIXED_FP32
    from paper_2311_17500_amd.serve import Server
    reqs = W.serve_stream(512, 0)[:128]
    recs = Server(slots=8, prec=MIXED_FP32, tol_lin=1e-8, tol_nonlin=1e-8, lin_forcing=0.1,
                  precond=precond).run(reqs)
    bad = [(i, r.status) for i, r in enumerate(recs) if r.status != "ok"]
    assert not bad, bad[:5]
