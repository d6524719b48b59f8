"""GPU tests of the batch entry points (fds_batch_create / fds_batch_replay /
fds_batch_run) through the C ABI: operators of curves of uneven size built by
one persistent assembly launch, filtered, compressed and factored, and the
right-hand sides and solves of every problem replayed from one HIP graph.
Every solution is compared with the oracle's filtered solution
j = G^{-1/2} y_fil (paper, Inversion of the structured matrices: the Woodbury
identity with the exact skeleton reproduces the filtered system's solution),
on every replay, with eager library work and host synchronisations between
the replays."""
import numpy as np
import pytest
import torch

from oracle import assembly, formulation, solver
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu

# kind, n, k, n_modes, nrhs: uneven sizes (ragged tiles), spread wave numbers
PROBLEMS = [("random", 100, 0.7, 21, 3), ("star", 257, 12.0, 63, 5), ("random", 64, 5.0, 15, 2),
            ("ellipse", 513, 3.0, 81, 4)]


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = B.fds_ctx_create(0)
    yield c
    c.close()


def _nodes(kind, n, seed):
    return wl.curve_nodes(kind, n, seed=seed) if kind == "random" else wl.curve_nodes(kind, n)


def _problems(spec, seed0=0):
    out = []
    for i, (kd, n, k, nm, nr) in enumerate(spec):
        rs = np.random.default_rng(seed0 + 31 * i)
        out.append({"nodes": torch.from_numpy(_nodes(kd, n, 1000 + i)).cuda(), "k": k, "n_modes": nm,
                    "angles": torch.from_numpy(rs.uniform(0, 2 * np.pi, nr)).cuda(),
                    "amps": torch.from_numpy(wl.random_amplitudes(seed0 + i, nr)).cuda(),
                    "j_out": torch.zeros((nr, n), dtype=torch.complex128, device="cuda")})
    return out


_ORACLE = {}


def _oracle_ops(nodes, k, form, nm, alpha):
    key = (nodes.tobytes(), k, form, nm, alpha)
    if key not in _ORACLE:
        _ORACLE[key] = solver.build_operators(solver.Problem(nodes, k, form=form, alpha=alpha, n_modes=nm))
    return _ORACLE[key]


def _oracle_j(p, form, alpha):
    nodes = p["nodes"].cpu().numpy()
    ops = _oracle_ops(nodes, p["k"], form, p["n_modes"], alpha)
    fo, ho = assembly.rhs_planewave(ops.mesh, p["k"], p["angles"].cpu().numpy(), p["amps"].cpu().numpy())
    v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, fo.T, ho.T, alpha,
                               ops.Sy if form == "ycfie" else None)
    return ops, ops.Gmh @ solver.y_filtered(ops, v)


def _check_all(probs, form, alpha, bound, tag, batch=None):
    for i, p in enumerate(probs):
        ops, jf = _oracle_j(p, form, alpha)
        if batch is not None:
            assert batch.op(i).info()[1] == ops.n_eff
        err = solver.relerr(p["j_out"].cpu().numpy().T, jf)
        _say(f"  {tag} problem {i} (N={p['nodes'].shape[0]}): j vs oracle {err:.2e} (bound {bound:g})")
        assert err <= bound


@pytest.mark.parametrize("prec,form", [("fp64", "cfie"), ("fp32", "cfie"), ("fp64", "efie"), ("fp32", "mfie")])
def test_batch_replays_match_oracle(ctx, prec, form):
    _say(f"case: batch of {len(PROBLEMS)} problems {prec} {form}, graph replays vs oracle")
    probs = _problems(PROBLEMS)
    bound = 1e-10 if prec == "fp64" else 1e-6
    b = B.Batch(ctx, probs, precision=prec, form=form, alpha=1.0, rank_cap=0, sweeps=0)
    for rep in range(3):
        # new incidence directions in place, eager library work in between
        for p in probs:
            p["angles"].add_(0.37 * (rep + 1))
        eager = B.fds_assemble(ctx, probs[2]["nodes"], 2.0)
        B.fds_filter(eager, "efie", 1.0, 9)
        eager.close()
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        _check_all(probs, form, 1.0, bound, f"replay {rep}", batch=b)
    b.close()


def test_batch_run_one_call(ctx):
    _say("case: fds_batch_run, 3 problems, mixed CFIE alpha 0.5")
    probs = _problems(PROBLEMS[:3], seed0=50)
    B.fds_batch_run(ctx, probs, precision="fp32", form="cfie", alpha=0.5)
    _check_all(probs, "cfie", 0.5, 1e-6, "one call")


def test_batch_ycfie(ctx):
    _say("case: batch of 2 problems, Yukawa-Calderon CFIE (per-problem filter)")
    probs = _problems([("star", 300, 10.0, 41, 3), ("ellipse", 257, 5.0, 31, 2)], seed0=70)
    b = B.Batch(ctx, probs, precision="fp64", form="ycfie", alpha=1.0)
    b.replay()
    torch.cuda.synchronize()
    _check_all(probs, "ycfie", 1.0, 1e-10, "ycfie")
    b.close()


def test_batch_truncating_matches_single_pipeline(ctx):
    """Truncating skeletons (rank below n_eff) with three refinement sweeps: each
    replayed solution equals the single-operator pipeline with the same sketch
    seed and sweep count, and the oracle's same-sketch skeleton followed by the
    same three sweeps (paper, Inversion of the structured matrices)."""
    _say("case: truncating batch (rank cap 12) with 3 sweeps vs the single-operator path and the oracle")
    spec = [("star", 257, 12.0, 63, 3), ("ellipse", 300, 3.0, 41, 2)]
    probs = _problems(spec, seed0=90)
    b = B.Batch(ctx, probs, precision="fp64", form="cfie", rank_cap=12, oversample=6, power_iters=2, sweeps=3,
                seed=5)
    b.replay()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        assert b.op(i).info()[2] == 12
        op = B.fds_assemble(ctx, p["nodes"], p["k"])
        B.fds_filter(op, "cfie", 1.0, p["n_modes"])
        B.fds_compress(op, 12, 6, 2, 0.0, seed=5)
        B.fds_factor(op)
        f, h = B.fds_rhs_planewave(op, p["angles"], p["amps"])
        w = B.fds_rhs_system(op, "cfie", 1.0, f, h)
        j = torch.zeros_like(w)
        B.fds_solve_system_noalloc(op, w, j, sweeps=3)
        torch.cuda.synchronize()
        d = ((p["j_out"] - j).abs().max() / j.abs().max()).item()
        nodes = p["nodes"].cpu().numpy()
        pb = solver.Problem(nodes, p["k"], form="cfie", n_modes=p["n_modes"], rank_cap=12, oversample=6,
                            power_iters=2, seed=5, refine_tol=0.0, max_refine=3)
        ops = _oracle_ops(nodes, p["k"], "cfie", p["n_modes"], 1.0)
        sol = solver.solve(pb, ops, p["angles"].cpu().numpy(), p["amps"].cpu().numpy())
        assert len(sol.history) == 4
        e = solver.relerr(p["j_out"].cpu().numpy().T, sol.j)
        _say(f"  problem {i}: batch vs single {d:.2e}; vs the oracle's same-sketch 3-sweep solution {e:.2e}")
        assert d <= 1e-12
        assert e <= 1e-10
        op.close()
    b.close()


def test_batch_errors(ctx):
    _say("case: batch argument errors")
    good = _problems(PROBLEMS[:2], seed0=3)
    bad = [dict(good[0]), dict(good[1])]
    bad[1]["n_modes"] = bad[1]["nodes"].shape[0] + 1
    with pytest.raises(B.FdsError) as e:
        B.Batch(ctx, bad)
    assert e.value.name == "FDS_ERR_ARG"
    with pytest.raises(B.FdsError) as e:
        B.Batch(ctx, good, form="cfie", alpha=-0.5)    # beta = 0
    assert e.value.name == "FDS_ERR_ARG"
    with pytest.raises(B.FdsError) as e:
        B.Batch(ctx, good, sweeps=-1)
    assert e.value.name == "FDS_ERR_ARG"
    # a failed creation leaves the context usable
    b = B.Batch(ctx, good)
    b.replay()
    torch.cuda.synchronize()
    _check_all(good, "cfie", 1.0, 1e-10, "after errors")
    b.close()
