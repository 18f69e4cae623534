"""Pins for the oracle's grid integrals, its control target and its control
field, fixed by mathematics rather than by restating the oracle's formulas
(CPU only).

- weight: a continuum-normalised Gaussian sampled on the grid integrates to 1
  (the Poisson-summation aliasing, of order exp(-pi^2/h^2), and the box
  truncation are far below rounding at h = 0.3 on a 48^3 cube);
- conjugation side: the discrete plane waves of an n^3 cube are orthogonal
  over the grid, and a phase factor on the right operand comes out with its
  own sign only when the left operand is the conjugated one;
- dipole target: a normalised Gaussian centred at a has first moment a;
- field: the sine series vanishes at both ends of the interval and its
  coefficients are recovered exactly by the discrete sine orthogonality of
  the step midpoints.
Sections "Introduction" (integrals as grid sums) and "Quantum optimal
control" (the field given by its Fourier coefficients, the dipole target).
"""
import math

import numpy as np
import pytest

import oracle
from tests import fdmath

H = 0.3
N = 48


@pytest.fixture(scope="module")
def cube():
    g = oracle.Grid(H, n=N)
    pos = fdmath.positions(g.ijk, g.dims, H)
    return g, pos


def _gauss(pos, centre):
    """pi^(-3/4) exp(-|r - c|^2 / 2): unit norm in the continuum."""
    d2 = ((pos - np.asarray(centre)) ** 2).sum(axis=1)
    return np.pi ** -0.75 * np.exp(-0.5 * d2)


def test_norm_weight_is_h_cubed(cube):
    """h^3 sum |g|^2 = 1 for the continuum-normalised Gaussian: a wrong power
    of h (or none) misses by a factor 0.3^k."""
    g, pos = cube
    psi = np.stack([_gauss(pos, (0, 0, 0)), 1j * _gauss(pos, (0.45, -0.3, 0.15))], axis=1)
    n2 = oracle.norm2(g, psi)
    np.testing.assert_allclose(n2, 1.0, rtol=0, atol=1e-13)
    d = oracle.dot(g, psi, psi)
    np.testing.assert_allclose(d.real, 1.0, rtol=0, atol=1e-13)
    assert np.abs(d.imag).max() < 1e-15


def test_overlap_of_two_gaussians(cube):
    """<g_a|g_b> = exp(-|a - b|^2 / 4) for unit Gaussians (continuum)."""
    g, pos = cube
    a, b = np.array([0.6, 0.0, -0.3]), np.array([-0.9, 0.3, 0.6])
    ga = _gauss(pos, a).astype(np.complex128)[:, None]
    gb = _gauss(pos, b).astype(np.complex128)[:, None]
    ref = math.exp(-((a - b) ** 2).sum() / 4.0)
    assert oracle.dot(g, ga, gb)[0] == pytest.approx(ref, rel=1e-13, abs=0)


def test_dot_conjugates_the_left_operand(cube):
    """Discrete plane waves e_m(r) = exp(i k_m . r), k_m = 2 pi m / (n h):
    <e_m | e^{i phi} e_m'> = e^{i phi} h^3 n^3 delta_{m m'}.  Conjugating the
    right operand instead would return e^{-i phi}."""
    g, pos = cube
    ms = [(1, 0, 0), (0, 2, -1), (3, -1, 2), (-2, 5, 1)]
    k = 2 * np.pi / (N * H) * np.asarray(ms, dtype=np.float64)
    waves = np.exp(1j * pos @ k.T)                       # [np][4]
    phis = np.array([0.7, -1.3, 2.1, 0.25])
    vol = H ** 3 * N ** 3
    for j in range(len(ms)):
        right = np.exp(1j * phis)[None, :] * waves[:, [j] * len(ms)]
        d = oracle.dot(g, waves, right)
        for i in range(len(ms)):
            if i == j:
                assert d[i] == pytest.approx(np.exp(1j * phis[i]) * vol, rel=1e-11, abs=0)
            else:
                assert abs(d[i]) < 1e-9 * vol
    np.testing.assert_allclose(oracle.norm2(g, waves), vol, rtol=1e-11)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dipole_target_is_first_moment(cube, axis):
    """J = sum_n <psi_n|x_axis|psi_n> for Gaussians centred at a_n: J = sum_n
    a_n along the axis, with its sign (centres +3h and -2h give J = +h)."""
    g, pos = cube
    ham = oracle.Ham(g, dipole_axis=axis)
    c1 = np.zeros(3)
    c2 = np.zeros(3)
    c1[axis] = 3 * H
    c2[axis] = -2 * H
    c2[(axis + 1) % 3] = 4 * H   # an offset across the axis changes nothing
    psi = np.stack([_gauss(pos, c1), np.exp(0.4j) * _gauss(pos, c2)], axis=1).astype(np.complex128)
    assert oracle.dipole_target(ham, psi) == pytest.approx(H, rel=1e-12, abs=0)
    assert oracle.dipole_target(ham, psi[:, :1]) == pytest.approx(3 * H, rel=1e-12, abs=0)
    assert oracle.dipole_target(ham, psi[:, 1:]) == pytest.approx(-2 * H, rel=1e-12, abs=0)


def test_laser_field_vanishes_at_both_ends():
    c = np.random.default_rng(5).normal(0.0, 0.01, 64)
    T = 20.0
    scale = np.abs(c).sum()
    assert abs(oracle.laser_field(c, T, 0.0)) <= 1e-15 * scale
    assert abs(oracle.laser_field(c, T, T)) <= 1e-13 * scale


@pytest.mark.parametrize("nsteps,ncoef", [(100, 64), (2000, 64), (65, 64)])
def test_laser_field_discrete_sine_orthogonality(nsteps, ncoef):
    """At the step midpoints tau_n = (n + 1/2) T / N,
    (2/N) sum_n sin(k pi tau_n / T) sin(j pi tau_n / T) = delta_kj for
    1 <= k, j < N, so (2/N) sum_n E(tau_n) sin(k pi tau_n / T) = c_k: a wrong
    harmonic index, period or normalisation breaks the recovery."""
    c = np.random.default_rng(nsteps).normal(0.0, 0.005, ncoef)
    dt = 0.01
    T = dt * nsteps
    tau = (np.arange(nsteps) + 0.5) * dt
    E = np.array([oracle.laser_field(c, T, t) for t in tau])
    k = np.arange(1, ncoef + 1)
    rec = 2.0 / nsteps * (np.sin(np.pi * np.outer(k, tau) / T) @ E)
    np.testing.assert_allclose(rec, c, rtol=0, atol=1e-14)
