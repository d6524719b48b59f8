"""GPU tests of the batched path: persistent batched assembly, grouped-GEMM
filter, split-K autotuner and the graph-captured solves of several operators."""
import numpy as np
import pytest
import torch

from oracle import assembly, formulation, geometry, solver
from paper_2210_08580_amd import batch
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu

# uneven sizes, including ragged tiles, and spread wave numbers
SHAPES = [("random", 100, 0.7), ("star", 257, 12.0), ("random", 64, 5.0), ("ellipse", 513, 3.0),
          ("random", 130, 19.0)]


@pytest.fixture(scope="module")
def sctx():
    c = B.Ctx(0, stream=torch.cuda.Stream())
    yield c
    c.close()


def _nodes(kind, n, seed):
    return wl.curve_nodes(kind, n, seed=seed) if kind == "random" else wl.curve_nodes(kind, n)


def test_assemble_batch_matches_single(sctx):
    print("case: batched assembly of 5 uneven operators", flush=True)
    nodes = [torch.from_numpy(_nodes(kd, n, 1000 + i)).cuda() for i, (kd, n, k) in enumerate(SHAPES)]
    ks = [k for _, _, k in SHAPES]
    with torch.cuda.stream(sctx.stream):
        ops = B.fds_assemble_batch(sctx, nodes, ks)
        for x, k, op in zip(nodes, ks, ops):
            ref = B.fds_assemble(sctx, x, k)
            for a, b in zip(B.fds_op_matrices(op), B.fds_op_matrices(ref)):
                assert torch.equal(a, b)
            ref.close()
    torch.cuda.synchronize()
    # and against the oracle for one of them
    S, N, D = [t.cpu().numpy() for t in B.fds_op_matrices(ops[1])]
    So, No, Do = assembly.assemble(geometry.mesh(nodes[1].cpu().numpy()), ks[1])
    for g, r in ((S, So), (N, No), (D, Do)):
        assert np.abs(g - r).max() <= 1e-12 * np.abs(r).max()
    for op in ops:
        op.close()


def test_filter_batch_matches_single(sctx):
    print("case: batched filter (grouped GEMM) of 5 uneven operators", flush=True)
    nodes = [torch.from_numpy(_nodes(kd, n, 1000 + i)).cuda() for i, (kd, n, k) in enumerate(SHAPES)]
    ks = [k for _, _, k in SHAPES]
    nms = [21, 63, 15, 81, 31]
    for form in ("cfie", "efie", "mfie"):
        with torch.cuda.stream(sctx.stream):
            ops = B.fds_assemble_batch(sctx, nodes, ks)
            ne = B.fds_filter_batch(ops, form, 1.0, nms)
            for x, k, op, nm, e in zip(nodes, ks, ops, nms, ne):
                ref = B.fds_assemble(sctx, x, k)
                assert B.fds_filter(ref, form, 1.0, nm) == e
                B.fds_compress(op, rank_cap=e, oversample=0, power_iters=0)
                B.fds_compress(ref, rank_cap=e, oversample=0, power_iters=0)
                _, W = B.fds_op_factors(op)
                _, Wr = B.fds_op_factors(ref)
                assert (W - Wr).abs().max().item() <= 1e-12 * Wr.abs().max().item()
                ref.close()
            for op in ops:
                op.close()


def test_autotuned_gemm(sctx):
    print("case: split-K autotuner", flush=True)
    rs = np.random.default_rng(4)
    B.fds_autotune(sctx, True)
    try:
        for (m, n, k) in ((64, 48, 4000), (130, 70, 257), (300, 20, 9000)):
            A = rs.standard_normal((m, k)) + 1j * rs.standard_normal((m, k))
            Bm = rs.standard_normal((k, n)) + 1j * rs.standard_normal((k, n))
            ref = A @ Bm
            for rep in range(2):
                with torch.cuda.stream(sctx.stream):
                    tA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
                    tB = torch.from_numpy(np.ascontiguousarray(Bm.T)).cuda()
                    tC = torch.zeros((n, m), dtype=torch.complex128, device="cuda")
                    B.fds_zgemm(sctx, 0, 0, tA, tB, tC)
                sctx.stream.synchronize()
                got = tC.cpu().numpy().T
                assert np.abs(got - ref).max() <= 8 * 2.2e-16 * np.abs(A).max() * np.abs(Bm).max() * k
        cache = B.fds_autotune_read(sctx)
        assert len(cache) >= 3 and all(v >= 1 for v in cache.values())
    finally:
        B.fds_autotune(sctx, False)


def test_graph_captured_solves(sctx):
    print("case: graph-captured solves of 4 operators", flush=True)
    probs = []
    for i, (kd, n, k) in enumerate(SHAPES[:4]):
        probs.append({"nodes": torch.from_numpy(_nodes(kd, n, 1000 + i)).cuda(), "k": k,
                      "n_modes": min(63, n // 4 * 2 + 1)})
    pipe = batch.BatchPipeline(sctx, probs, form="cfie")
    rs = np.random.default_rng(7)
    nr = [3, 5, 2, 4]
    ang = [torch.from_numpy(rs.uniform(0, 2 * np.pi, r)) for r in nr]
    amp = [torch.from_numpy(wl.random_amplitudes(i, r)) for i, r in enumerate(nr)]
    with torch.cuda.stream(sctx.stream):   # the clones must follow the solves on the same stream
        eager = [j.clone() for j in pipe.solve_eager(ang, amp)]
    pipe.capture(ang, amp)
    for rep in range(3):
        # eager work between replays
        with torch.cuda.stream(sctx.stream):
            ang2 = [a + 0.1 * (rep + 1) for a in ang]
            eager2 = [j.clone() for j in pipe.solve_eager(ang2, amp)]
        outs = pipe.replay(ang2, amp)
        sctx.stream.synchronize()
        for a, b in zip(outs, eager2):
            assert (a - b).abs().max().item() <= 1e-13 * b.abs().max().item()
    outs = pipe.replay(ang, amp)
    sctx.stream.synchronize()
    for a, b in zip(outs, eager):
        assert (a - b).abs().max().item() <= 1e-13 * b.abs().max().item()
    # every replayed solution against the oracle's filtered solution j = G^{-1/2} y_fil
    for i, (pr, out) in enumerate(zip(probs, outs)):
        nodes = pr["nodes"].cpu().numpy()
        pb = solver.Problem(nodes, pr["k"], form="cfie", n_modes=pr["n_modes"])
        ops = solver.build_operators(pb)
        assert ops.n_eff == pipe.n_eff[i]
        fo, ho = assembly.rhs_planewave(ops.mesh, pr["k"], ang[i].numpy(), amp[i].numpy())
        v = formulation.rhs_vector("cfie", ops.S, ops.Gmh, ops.Gi, fo.T, ho.T)
        jf = ops.Gmh @ solver.y_filtered(ops, v)
        err = solver.relerr(out.cpu().numpy().T, jf)
        print(f"  replayed solve {i} (N={nodes.shape[0]}) vs the oracle: {err:.2e}", flush=True)
        assert err <= 1e-10
    pipe.close()
