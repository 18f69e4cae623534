"""Pins of the oracle's shifted solves (section "The Sternheimer formulation
of linear-response", eq. (sternheimer)), against what linear algebra fixes:

- on a small sphere with wells and projectors, H is built densely column by
  column and (H + sigma) x = b solved directly; QMR (complex shifts, several
  per batch) and CG (a real shift that makes H + sigma positive definite)
  reach that solution;
- an eigenvector right-hand side lies in a one-dimensional Krylov space: both
  methods stop after one iteration with x = b / (lambda + sigma) exactly, and
  a sum of two eigenvectors takes two;
- b = 0 and an exact initial guess stop before the first iteration;
- H is real symmetric, the property that lets QMR use A in place of A^T."""
import numpy as np
import pytest

import oracle
import synth
from oracle import shifted as sv


@pytest.fixture(scope="module")
def small():
    g = oracle.Grid(0.5, R=2.6)
    pos = g.positions()
    wells = synth.gaussian_wells(5, 2, ball=1.0)
    V = synth.well_potential(pos, wells)
    proj = synth.kb_projectors(5, pos, wells.centres, rcut=1.2)
    ham = oracle.Ham(g, V=V, kin=-0.5, projectors=proj)
    Hd = oracle.hpsi(ham, np.eye(g.np, dtype=np.complex128))
    return g, ham, Hd


def test_dense_h_is_real_symmetric(small):
    g, ham, Hd = small
    assert np.abs(Hd.imag).max() == 0.0
    np.testing.assert_allclose(Hd, Hd.T, rtol=0, atol=1e-12 * np.abs(Hd).max())


def test_qmr_reaches_the_direct_solution(small):
    g, ham, Hd = small
    rng = np.random.default_rng(1)
    nst = 3
    b = rng.standard_normal((g.np, nst)) + 1j * rng.standard_normal((g.np, nst))
    shifts = np.array([0.3 + 0.1j, -0.2 + 0.05j, 1.0 + 0.5j])
    x, its, res, st = sv.solve_batch(ham, b, shifts, "qmr", tol=1e-12, maxiter=2000)
    assert np.all(st == 0)
    for n in range(nst):
        ref = np.linalg.solve(Hd + shifts[n] * np.eye(g.np), b[:, n])
        assert np.linalg.norm(x[:, n] - ref) <= 1e-9 * np.linalg.norm(ref), n
        assert res[n] <= 1e-12
        assert 1 < its[n] < 2000


def test_cg_reaches_the_direct_solution(small):
    g, ham, Hd = small
    lam = np.linalg.eigvalsh(Hd.real)
    sigma = -lam[0] + 0.5  # H + sigma positive definite
    rng = np.random.default_rng(2)
    b = rng.standard_normal((g.np, 2)) + 1j * rng.standard_normal((g.np, 2))
    x, its, res, st = sv.solve_batch(ham, b, sigma, "cg", tol=1e-12, maxiter=2000)
    assert np.all(st == 0)
    ref = np.linalg.solve(Hd + sigma * np.eye(g.np), b)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("method,sigma", [("qmr", 0.7 + 0.2j), ("cg", 3.0)])
def test_krylov_dimension_one_and_two(small, method, sigma):
    g, ham, Hd = small
    lam, U = np.linalg.eigh(Hd.real)
    k, j = 3, 11
    b1 = U[:, k].astype(np.complex128) * (0.5 - 2.0j)
    x, its, res, st = sv.solve_batch(ham, b1[:, None], sigma, method, tol=1e-12, maxiter=10)
    assert its[0] == 1 and st[0] == 0
    np.testing.assert_allclose(x[:, 0], b1 / (lam[k] + sigma), rtol=0, atol=1e-12 * np.abs(b1).max())
    b2 = U[:, k] + 2.0 * U[:, j]
    x, its, res, st = sv.solve_batch(ham, b2[:, None], sigma, method, tol=1e-12, maxiter=10)
    assert its[0] == 2 and st[0] == 0
    ref = U[:, k] / (lam[k] + sigma) + 2.0 * U[:, j] / (lam[j] + sigma)
    np.testing.assert_allclose(x[:, 0], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("method", ["qmr", "cg"])
def test_trivial_starts(small, method):
    g, ham, Hd = small
    b = np.zeros((g.np, 1), dtype=np.complex128)
    x, its, res, st = sv.solve_batch(ham, b, 2.0, method)
    assert its[0] == 0 and st[0] == 0 and not np.any(x)
    rng = np.random.default_rng(3)
    xe = rng.standard_normal(g.np) + 0j
    b = (Hd + 2.0 * np.eye(g.np)) @ xe
    x, its, res, st = sv.solve_batch(ham, b[:, None], 2.0, method, x0=xe[:, None], tol=1e-10)
    assert its[0] == 0 and st[0] == 0


def test_isotropic_rhs_is_a_qmr_breakdown(small):
    """b = u + i w with u orthogonal to w and |u| = |w| has b^T b = 0: the
    bilinear form QMR runs on vanishes at the start, so QMR must stop at
    once with status 2 (breakdown) and x untouched; CG, which uses the
    Hermitian product, solves the same system with a real shift."""
    g, ham, Hd = small
    rng = np.random.default_rng(9)
    u = rng.standard_normal(g.np)
    w = rng.standard_normal(g.np)
    w -= (w @ u) / (u @ u) * u
    w *= np.linalg.norm(u) / np.linalg.norm(w)
    b = (u + 1j * w)[:, None]
    assert abs(b[:, 0] @ b[:, 0]) < 1e-12 * np.linalg.norm(b) ** 2
    x, its, res, st = sv.solve_batch(ham, b, 0.5 + 0.2j, "qmr", tol=1e-10)
    assert st[0] == 2 and its[0] == 0 and not np.any(x)
    lam0 = np.linalg.eigvalsh(Hd.real)[0]
    x, its, res, st = sv.solve_batch(ham, b, -lam0 + 1.0, "cg", tol=1e-10, maxiter=2000)
    assert st[0] == 0
