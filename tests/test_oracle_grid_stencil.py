"""Pins for the oracle's grid and kinetic stencil (CPU only).

Grid: the sphere/cube point sets and compact order against brute force.
Stencil: exactness on polynomials up to degree 9 (which fixes all five
weights), the textbook truncation constant on x^10, the plane-wave symbol
and the harmonic-oscillator Rayleigh quotient and eigenvalue convergence.
"""
import math

import numpy as np
import pytest

import oracle
from tests import fdmath


# ---------------------------------------------------------------- grid ---

@pytest.mark.parametrize("R,h", [(2.0, 0.5), (3.3, 0.3), (4.0, 0.25), (18.0, 0.2)])
def test_sphere_points_match_brute_force(R, h):
    g = oracle.Grid(h, R=R)
    q = math.floor((R / h) ** 2 + 1e-9)
    m = int(math.isqrt(q))
    ax = np.arange(-m, m + 1)
    K, J, I = np.meshgrid(ax, ax, ax, indexing="ij")
    inside = (I * I + J * J + K * K) <= q
    ref = np.stack([I[inside] + m, J[inside] + m, K[inside] + m], axis=1)  # z-major, y, x
    assert g.np == ref.shape[0]
    assert tuple(g.dims) == (2 * m + 1,) * 3
    np.testing.assert_array_equal(g.ijk, ref.astype(np.int32))


def test_sphere_c2_point_count():
    # R = 18 bohr at h = 0.2: R/h = 90 grid spacings.
    g = oracle.Grid(0.2, R=18.0)
    assert g.np == 3053617
    assert tuple(g.dims) == (181, 181, 181)


def test_cube_order_and_positions():
    g = oracle.Grid(0.3, n=6)
    assert g.np == 216
    key = g.ijk[:, 2] * 36 + g.ijk[:, 1] * 6 + g.ijk[:, 0]
    np.testing.assert_array_equal(key, np.arange(216))
    pos = g.positions()
    np.testing.assert_allclose(pos, fdmath.positions(g.ijk, g.dims, 0.3), rtol=0, atol=0)
    np.testing.assert_allclose(pos.sum(axis=0), 0.0, atol=1e-12)  # symmetric box


# ------------------------------------------------------------- stencil ---

def test_golden_weights_satisfy_moment_conditions():
    assert fdmath.fd8_weights_from_moments() == fdmath.fd8_weights_golden()


def _lap(g, f, h):
    ham = oracle.Ham(g, V=None, kin=1.0)
    return oracle.hpsi(ham, f.astype(np.complex128)[:, None])[:, 0]


@pytest.mark.parametrize("a,b,c", [(0, 0, 0), (2, 0, 0), (0, 3, 1), (4, 4, 0), (2, 3, 4),
                                   (8, 0, 0), (0, 9, 0), (1, 0, 8), (3, 3, 3)])
def test_polynomials_exact_at_interior(a, b, c):
    """The 8th-order star is exact for degree <= 9 in each variable pair sum;
    five moment conditions determine c0..c4, so a wrong weight, sign, axis
    or h-scaling fails here."""
    h = 0.3
    g = oracle.Grid(h, n=14)
    x, y, z = fdmath.positions(g.ijk, g.dims, h).T
    f = x ** a * y ** b * z ** c
    lap = _lap(g, f, h)

    def d2(p, t):
        return p * (p - 1) * t ** (p - 2) if p >= 2 else 0.0 * t

    exact = d2(a, x) * y ** b * z ** c + x ** a * d2(b, y) * z ** c + x ** a * y ** b * d2(c, z)
    m = fdmath.interior_mask(g.ijk, g.dims, 4)
    scale = max(1.0, np.abs(exact[m]).max(), np.abs(f[m]).max() / h ** 2)
    np.testing.assert_allclose(lap[m].real, exact[m], rtol=0, atol=1e-12 * scale)
    assert np.abs(lap.imag).max() == 0.0


def test_x10_truncation_constant():
    """D2_h x^10 - 90 x^8 = -(h^8/3150) * 10! exactly (Fornberg's constant)."""
    h = 0.25
    g = oracle.Grid(h, n=14)
    x = fdmath.positions(g.ijk, g.dims, h)[:, 0]
    lap = _lap(g, x ** 10, h).real
    m = fdmath.interior_mask(g.ijk, g.dims, 4)
    err = lap[m] - 90.0 * x[m] ** 8
    expect = -(h ** 8) * math.factorial(10) / 3150.0
    np.testing.assert_allclose(err, expect, rtol=1e-6)


def test_dirichlet_boundary():
    """Outside the box the orbital is zero: at a corner of a cube only the
    in-box taps contribute."""
    h = 0.3
    g = oracle.Grid(h, n=10)
    f = np.ones(g.np)
    lap = _lap(g, f, h).real
    c = [float(w) for w in fdmath.fd8_weights_from_moments()]
    # corner point (0,0,0): on each axis taps m = 0..4 are in the box
    corner = c[0] + sum(c[1:])
    assert lap[0] == pytest.approx(3 * corner / h ** 2, rel=1e-14)
    centre = (g.ijk == 5).all(axis=1)
    assert abs(lap[centre][0]) < 1e-10


@pytest.mark.parametrize("kvec", [(1, 2, 3), (16, 16, 16), (5, 0, 11)])
def test_plane_wave_symbol(kvec):
    """For V = 0 and psi = exp(i k.r), (H psi)(r) = lambda(k) psi(r) at every
    point at least 4 from the box edge, lambda the stencil symbol."""
    n, h = 32, 0.3
    g = oracle.Grid(h, n=n)
    k = 2.0 * math.pi * np.array(kvec) / (n * h)
    pos = fdmath.positions(g.ijk, g.dims, h)
    psi = np.exp(1j * pos @ k)[:, None]
    out = oracle.hpsi(oracle.Ham(g, V=None, kin=-0.5), psi)[:, 0]
    lam = fdmath.plane_wave_eigenvalue(k, h)
    m = fdmath.interior_mask(g.ijk, g.dims, 4)
    np.testing.assert_allclose(out[m], lam * psi[m, 0], rtol=1e-13, atol=1e-13 * abs(lam))
    # and the symbol approaches the continuum k^2/2 with the h^8 truncation error
    cont = 0.5 * float(k @ k)
    bound = 0.5 * sum(ka ** 10 for ka in k) * h ** 8 / 3150.0
    assert abs(lam - cont) <= 1.01 * bound + 1e-12


def test_ho_rayleigh_quotient_closed_form():
    """<g|H g>/<g|g> for the sampled Gaussian g = exp(-r^2/2) on a 48^3 cube
    at h = 0.3 (box truncation ~ exp(-49)) equals the closed form."""
    n, h = 48, 0.3
    g = oracle.Grid(h, n=n)
    pos = fdmath.positions(g.ijk, g.dims, h)
    V = 0.5 * (pos ** 2).sum(axis=1)
    ham = oracle.Ham(g, V=V, kin=-0.5)
    gs = np.exp(-0.5 * (pos ** 2).sum(axis=1))[:, None].astype(np.complex128)
    e, per = oracle.energy(ham, gs)
    rq = e / oracle.norm2(g, gs)[0]
    assert rq == pytest.approx(fdmath.ho_rayleigh_closed_form(h), rel=1e-13, abs=1e-13)
    assert abs(per[0].imag) < 1e-14 * abs(per[0].real)
    # leading term 1.5 - E = (9/640) h^8 from the x^10 moment; the next
    # (h^10) term has the opposite sign, so the ratio sits just below 1.
    assert 0.85 < (1.5 - rq) / (9.0 / 640.0 * h ** 8) < 1.0


def test_ho_eigenvalue_convergence_order8():
    """Lowest eigenvalues of -1/2 Lap_h + r^2/2 (box half-width 6 bohr) for
    h = 0.5, 0.4, 0.3: converge to 1.5 from below the Rayleigh bound with
    order ~8, and the 2.5 level is threefold degenerate."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    errs = []
    for h, n in [(0.5, 25), (0.4, 31), (0.3, 41)]:
        g = oracle.Grid(h, n=n)
        pos = fdmath.positions(g.ijk, g.dims, h)
        V = 0.5 * (pos ** 2).sum(axis=1)
        ham = oracle.Ham(g, V=V, kin=-0.5)

        def mv(v, ham=ham):
            return oracle.hpsi(ham, np.asarray(v, dtype=np.complex128).reshape(-1, 1))[:, 0].real

        op = LinearOperator((g.np, g.np), matvec=mv, dtype=np.float64)
        v0 = np.exp(-0.5 * (pos ** 2).sum(axis=1))
        w = np.sort(eigsh(op, k=4, which="SA", v0=v0, tol=1e-13)[0])
        assert w[0] <= fdmath.ho_rayleigh_closed_form(h) + 1e-12
        np.testing.assert_allclose(w[1:], w[1], rtol=1e-9)
        assert abs(w[1] - 2.5) < 1e-2
        errs.append(abs(w[0] - 1.5))
    order_a = math.log(errs[0] / errs[1]) / math.log(0.5 / 0.4)
    order_b = math.log(errs[1] / errs[2]) / math.log(0.4 / 0.3)
    assert 7.0 < order_a < 9.5, errs
    assert 7.0 < order_b < 9.5, errs
