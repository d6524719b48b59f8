"""Pins of the oracle's Yukawa-Calderon TE-CFIE (paper, Filters Based Fast Direct
Solver, 2D case: the filtered CFIE with the localised Calderon preconditioner,
single layer at the imaginary wavenumber i k, kernel (1/2 pi) K0(k R)) against
facts fixed outside it. No GPU involved."""
import mpmath as mp
import numpy as np
import pytest
from scipy import special as sp

from oracle import assembly, formulation, geometry, solver, special
from paper_2210_08580_amd import workloads as wl

from test_oracle_pins import circulant_eigs
from test_oracle_solver import exact_circle_u


def test_yukawa_kernel_against_mpmath():
    mp.mp.dps = 30
    for kappa in (0.5, 3.0, 10.0):
        for R in (1e-5, 0.03, 0.4, 1.7, 6.0):
            ref = float(mp.besselk(0, mp.mpf(kappa) * mp.mpf(R)) / (2 * mp.pi))
            got = float(special.yukawa(kappa, np.array([R]))[0])
            assert abs(got - ref) <= 2e-15 * abs(ref), (kappa, R, got, ref)


def test_yukawa_regular_part_limit():
    kappa = 2.3
    g0 = special.yukawa_reg_at_zero(kappa)
    for R in (1e-6, 1e-8):
        assert abs(special.yukawa_reg(kappa, np.array([R]))[0] - g0) < 1e-10
    mp.mp.dps = 30
    ref = float(-(mp.log(mp.mpf(kappa) / 2) + mp.euler) / (2 * mp.pi))
    assert abs(g0 - ref) < 1e-15


def yukawa_circle_eigs(m, kappa, a=1.0):
    """Fourier-mode eigenvalues of the Yukawa single layer on the circle of radius a
    (Graf's addition theorem for K0): lam = a I_m(kappa a) K_m(kappa a)."""
    return a * sp.iv(m, kappa * a) * sp.kv(m, kappa * a)


@pytest.mark.parametrize("kappa", [1.0, 5.0])
def test_yukawa_circle_eigenvalues_second_order(kappa):
    ms = np.arange(0, 6)
    errs = []
    for n in (64, 128, 256):
        m = geometry.mesh(wl.circle(n))
        Sy = assembly.assemble_yukawa(m, kappa)
        G = assembly.periodic_dense(*assembly.gram(m))
        lam = yukawa_circle_eigs(ms, kappa)
        errs.append(np.max(np.abs(circulant_eigs(Sy, G, ms) - lam) / np.abs(lam)))
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 1.8), (errs, order)
    assert errs[-1] < 2e-3


def test_yukawa_operator_symmetric_positive():
    """S_y is symmetric (symmetric kernel, Galerkin) and positive definite (the
    symbols a I_m K_m are positive)."""
    m = geometry.mesh(wl.curve_nodes("star", 96))
    Sy = assembly.assemble_yukawa(m, 3.0)
    assert np.abs(Sy - Sy.T).max() <= 1e-14 * np.abs(Sy).max()
    assert np.linalg.eigvalsh(Sy).min() > 0.0


def test_yukawa_sampled_entries_match_assembly():
    m = geometry.mesh(wl.curve_nodes("ellipse", 40))
    Sy = assembly.assemble_yukawa(m, 2.0)
    rs = np.random.default_rng(3)
    I = rs.integers(0, 40, 50)
    J = rs.integers(0, 40, 50)
    v = assembly.entries_yukawa(m, 2.0, I, J)
    assert np.abs(v - Sy[I, J]).max() <= 1e-15 * np.abs(Sy).max()


def test_yukawa_calderon_circle_modes():
    """Discrete Z_e of the Yukawa-Calderon form -> lam_Sy lam_N, and the
    continuous symbols tend to 1/4 (the preconditioned EFIE is I/4 + compact)."""
    k = 1.0
    ms = np.arange(0, 9)
    lSy = yukawa_circle_eigs(ms, k)
    lN = -0.5j * np.pi * k * k * sp.jvp(ms, k) * sp.h1vp(ms, k)
    errs = []
    for n in (64, 128):
        pb = solver.Problem(wl.circle(n), k, form="ycfie", alpha=0.0, n_modes=n, rank_cap=n)
        ops = solver.build_operators(pb)
        Z = ops.C + 0.25 * np.eye(n)          # alpha = 0: the EFIE part alone
        th = 2 * np.pi * np.arange(n) / n
        E = np.exp(1j * np.outer(th, ms)) / np.sqrt(n)
        z = np.einsum("im,ij,jm->m", E.conj(), Z, E)
        errs.append(np.abs(z - lSy * lN).max())
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 3.3, errs
    d = np.abs(lSy * lN - 0.25)
    assert d[8] < 5e-3 and np.all(np.diff(d[2:]) < 0), d


def test_yukawa_cfie_exact_circle_solution():
    """The preconditioner changes the system, not its solution: the unfiltered
    Yukawa-Calderon CFIE reproduces the exact sound-hard circle field."""
    k = 1.0
    ang = np.array([0.3, 2.0])
    amp = np.array([1.0, 0.5 - 0.2j])
    errs = []
    for n in (64, 128):
        pb = solver.Problem(wl.circle(n), k, form="ycfie", n_modes=n, rank_cap=n)
        ops = solver.build_operators(pb)
        f, h = assembly.rhs_planewave(ops.mesh, k, ang, amp)
        v = formulation.rhs_vector("ycfie", ops.S, ops.Gmh, ops.Gi, f.T, h.T, 1.0, ops.Sy)
        j = ops.Gmh @ solver.y_unfiltered(ops, v)
        th = 2 * np.pi * np.arange(n) / n
        ue = np.stack([a * exact_circle_u(k, 1.0, th, p) for p, a in zip(ang, amp)], 1)
        errs.append(np.abs(j + ue).max() / np.abs(ue).max())
    assert errs[1] < 3e-4 and errs[0] / errs[1] > 3.5, errs


def test_yukawa_cfie_agrees_with_cfie_on_star():
    """Same scattering problem, two preconditioners: the solutions agree to the
    discretisation's consistency (both are Galerkin solutions of N j = -f mixed
    with the MFIE)."""
    nodes = wl.curve_nodes("star", 128)
    k = 4.0
    ang = np.array([0.7])
    amp = np.array([1.0 + 0.0j])
    js = []
    for form in ("cfie", "ycfie"):
        pb = solver.Problem(nodes, k, form=form, n_modes=128, rank_cap=128)
        ops = solver.build_operators(pb)
        f, h = assembly.rhs_planewave(ops.mesh, k, ang, amp)
        v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, f.T, h.T, 1.0, ops.Sy)
        js.append(ops.Gmh @ solver.y_unfiltered(ops, v))
    assert np.abs(js[0] - js[1]).max() <= 2e-2 * np.abs(js[0]).max()
