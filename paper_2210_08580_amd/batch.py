"""Many geometries at once: batched assembly and filter, and the solves of all
operators captured in one HIP graph and replayed for new right-hand sides.

Only orchestration lives here: the batched kernels are behind
fds_assemble_batch / fds_filter_batch (one persistent far-field launch, grouped
GEMMs), and the graph records the library's own solve launches on the context's
stream (torch.cuda.graph supplies the capture and a private memory pool).
"""
from __future__ import annotations

import torch

from . import binding as B


class BatchPipeline:
    """Operators for several curves of uneven size, factored for the filtered fast solve.

    problems: list of dicts with keys nodes (n, 2) float64 tensor, k, n_modes.
    The context must own a dedicated stream (Ctx(stream=torch.cuda.Stream())) for
    graph capture."""

    def __init__(self, ctx: B.Ctx, problems, form="cfie", alpha=1.0, rank_cap=None, oversample=10,
                 power_iters=2, seed=1):
        self.ctx = ctx
        self.problems = problems
        with torch.cuda.stream(ctx.stream):
            self.ops = B.fds_assemble_batch(ctx, [p["nodes"] for p in problems], [p["k"] for p in problems])
            self.n_eff = B.fds_filter_batch(self.ops, form, alpha, [p["n_modes"] for p in problems])
            self.rank = []
            for op, ne in zip(self.ops, self.n_eff):
                r = B.fds_compress(op, rank_cap if rank_cap is not None else ne, oversample, power_iters,
                                   seed=seed)
                B.fds_factor(op)
                self.rank.append(r)
        self.form = form
        self.graph = None

    def close(self):
        for op in self.ops:
            op.close()
        self.ops = []

    def solve_eager(self, angles_list, amps_list, sweeps=2):
        """Plane-wave right-hand sides and fixed-sweep solves, launched directly."""
        out = []
        with torch.cuda.stream(self.ctx.stream):
            for op, ang, amp in zip(self.ops, angles_list, amps_list):
                f, h = B.fds_rhs_planewave(op, ang, amp)
                j, _, _ = B.fds_solve(op, f, h, max_iters=sweeps, tol=0.0, stats=False)
                out.append(j)
        return out

    def capture(self, angles_list, amps_list, sweeps=2):
        """Records right-hand sides and solves of every operator in one graph.

        angles_list / amps_list become the graph's static inputs: later calls to
        replay() read their current contents."""
        self.angles = [a.to(device="cuda", dtype=torch.float64).contiguous() for a in angles_list]
        self.amps = [a.to(device="cuda", dtype=torch.complex128).contiguous() for a in amps_list]
        self.solve_eager(self.angles, self.amps, sweeps)   # warm caches outside the capture
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.ctx.stream):
            self.outputs = self.solve_eager(self.angles, self.amps, sweeps)
        return self.outputs

    def replay(self, angles_list=None, amps_list=None):
        """Replays the graph on the context's stream (after updating the inputs there)."""
        with torch.cuda.stream(self.ctx.stream):
            if angles_list is not None:
                for dst, src in zip(self.angles, angles_list):
                    dst.copy_(src)
            if amps_list is not None:
                for dst, src in zip(self.amps, amps_list):
                    dst.copy_(src)
            self.graph.replay()
        return self.outputs
