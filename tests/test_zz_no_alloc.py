"""The allocation-free solve entry point (fds_solve_system_noalloc) against
fds_solve_system on the same factored operators, through the C ABI: two calls
in a row, the second with a smaller input. Inside the allocation-free call every
device allocation raises an error, so a call that succeeds made none."""
import numpy as np
import pytest
import torch

from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _relerr(a, b):
    return (torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)).max().item()


def _factored(ctx, nodes, k, form, n_modes, rank_cap, oversample, power_iters, tol):
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    ne = B.fds_filter(op, form, 1.0, n_modes)
    r = B.fds_compress(op, rank_cap, oversample, power_iters, tol, seed=7)
    B.fds_factor(op)
    return op, ne, r


def _rhs(ctx, op, form, nrhs, seed):
    ang, _ = wl.planewaves(seed, nrhs)
    amps = wl.random_amplitudes(seed + 1, nrhs)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang).cuda(), torch.from_numpy(amps).cuda())
    return B.fds_rhs_system(op, form, 1.0, f, h)


def test_noalloc_solve_matches_solve_system():
    ctx = B.fds_ctx_create(0)
    try:
        # 1) star N = 4096, 255 modes, exact skeleton, 600 right-hand sides: the
        # right-hand sides do not fit one block of the scratch (361 columns each)
        print("case: no-alloc star N=4096 EFIE n_modes=255 r=256 nrhs=600 sweeps=2", flush=True)
        op1, ne1, r1 = _factored(ctx, wl.star(4096), 10.0, "efie", 255, 256, 10, 2, 0.0)
        w1 = _rhs(ctx, op1, "efie", 600, 31)
        j1 = torch.full_like(w1, float("nan"))
        B.fds_solve_system_noalloc(op1, w1, j1, 2)
        ref1, _, _ = B.fds_solve_system(op1, w1, max_iters=2, tol=0.0, stats=False)
        torch.cuda.synchronize()
        e1 = _relerr(j1, ref1)
        print(f"  vs fds_solve_system: {e1:.2e}", flush=True)
        assert torch.isfinite(torch.view_as_real(j1)).all()
        assert e1 <= 1e-12
        # 2) a smaller input right after: ellipse N = 1200, truncating skeleton
        # (rank 40 < 81 kept modes), 7 right-hand sides, 3 sweeps; then 0 sweeps
        print("case: no-alloc ellipse N=1200 CFIE n_modes=81 r=40 nrhs=7 sweeps=3,0", flush=True)
        op2, ne2, r2 = _factored(ctx, wl.ellipse(1200), 5.0, "cfie", 81, 40, 6, 2, 0.0)
        assert r2 < ne2
        w2 = _rhs(ctx, op2, "cfie", 7, 41)
        for sweeps in (3, 0):
            j2 = torch.full_like(w2, float("nan"))
            B.fds_solve_system_noalloc(op2, w2, j2, sweeps)
            ref2, _, _ = B.fds_solve_system(op2, w2, max_iters=sweeps, tol=0.0, stats=False)
            torch.cuda.synchronize()
            e2 = _relerr(j2, ref2)
            print(f"  sweeps={sweeps}: vs fds_solve_system {e2:.2e}", flush=True)
            assert e2 <= 1e-12
        # the first operator again: the scratch holds the second call's contents
        j3 = torch.full_like(w1[:5], float("nan"))
        B.fds_solve_system_noalloc(op1, w1[:5].contiguous(), j3, 2)
        torch.cuda.synchronize()
        assert _relerr(j3, ref1[:5]) <= 1e-12
        # argument errors
        with pytest.raises(B.FdsError) as e:
            B.fds_solve_system_noalloc(op2, w2, torch.empty_like(w2), -1)
        assert e.value.name == "FDS_ERR_ARG"
        op3 = B.fds_assemble(ctx, torch.from_numpy(wl.circle(64)).cuda(), 1.0)
        with pytest.raises(B.FdsError) as e:
            B.fds_solve_system_noalloc(op3, torch.zeros((1, 64), dtype=torch.complex128, device="cuda"),
                                       torch.empty((1, 64), dtype=torch.complex128, device="cuda"), 1)
        assert e.value.name == "FDS_ERR_STATE"
        for o in (op1, op2, op3):
            o.close()
    finally:
        ctx.close()
