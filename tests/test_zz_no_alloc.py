"""The allocation-free preconditioner entry point (st_iga_precond_noalloc)
against st_iga_precond, through the C ABI: the same kernels on the same
inputs, so the outputs must be bit-identical.  Two calls in a row on one GPU
(the second with a smaller problem, so the shared scratch holds the first
call's larger contents), each also checked against the oracle's direct solve
of A-hat; sizes beyond the scratch are rejected with EINVAL."""
import numpy as np
import pytest

import st_workloads as W
from oracle import solver
from oracle.spacetime import SpaceTime

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def test_precond_noalloc_matches_precond(gpu_lib):
    import torch
    from paper_2311_17500_amd.binding import Solver
    big = W.tiny(2, 3, 12, nel_t=10)     # 15^2 x 12 = 2700 unknowns
    small = W.tiny(1, 2, 9, nel_t=6)     # 11 x 7 = 77 unknowns
    assert big.unknowns > small.unknowns
    for seed, prob, precond in ((41, big, 1), (42, small, 1), (43, big, 0), (44, small, 0)):
        S = Solver(prob, precond=precond)
        r = _dev(torch, W.random_vector(prob.unknowns, seed))
        z_ref = S.precond(r)
        z = S.vec()
        S.precond_noalloc(r, z)
        torch.cuda.synchronize()
        zr, zn = z_ref.cpu().numpy(), z.cpu().numpy()
        assert np.array_equal(zn, zr), f"seed {seed}: max diff {np.max(np.abs(zn - zr))}"
        want = solver.precond_solve(SpaceTime(prob), r.cpu().numpy())
        assert np.linalg.norm(zn - want) <= 1e-10 * np.linalg.norm(want)
        S.close()


def test_precond_noalloc_rejects_oversize(gpu_lib):
    import torch
    from paper_2311_17500_amd.binding import EINVAL, Solver, StIgaError
    prob = W.tiny(3, 2, 40, nel_t=30)   # 42^3 x 31 = 2,296,728 unknowns > 2^21
    assert prob.unknowns > (1 << 21)
    S = Solver(prob)
    r = S.vec()
    z = S.vec()
    with pytest.raises(StIgaError) as e:
        S.precond_noalloc(r, z)
    assert e.value.code == EINVAL
    torch.cuda.synchronize()
    S.close()
