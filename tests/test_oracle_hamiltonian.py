"""Pins for the oracle's full Hamiltonian, Taylor(4) step, reductions and
discrete adjoint (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import fdmath


def _small_system(R=2.6, h=0.3, nst=3, natoms=3, seed=11, dipole=2):
    g = oracle.Grid(h, R=R)
    pos = fdmath.positions(g.ijk, g.dims, h)
    wells = synth.gaussian_wells(seed, natoms, ball=1.0)   # close atoms: overlapping supports
    V = synth.well_potential(pos, wells)
    proj = synth.kb_projectors(seed, pos, wells.centres, rcut=1.5)
    ham = oracle.Ham(g, V=V, kin=-0.5, dipole_axis=dipole, projectors=proj)
    psi = synth.white_noise(seed, g.np, nst, h)
    return g, pos, ham, proj, psi


def _vdot_h3(h, a, b):
    return h ** 3 * np.einsum("pn,pn->n", a.conj(), b)


# -------------------------------------------------------- Hamiltonian ---

def test_projector_supports_overlap():
    g, pos, ham, proj, psi = _small_system()
    sets = [set(i.tolist()) for i in proj.idx]
    assert len(sets[0] & sets[1]) > 0 or len(sets[1] & sets[2]) > 0


def test_hermiticity_full_hamiltonian():
    """<phi|H psi> = <H phi|psi> with stencil, wells, overlapping projectors
    and dipole field all on."""
    g, pos, ham, proj, psi = _small_system()
    phi = synth.white_noise(99, g.np, 3, g.h)
    f = 0.37
    lhs = _vdot_h3(g.h, phi, oracle.hpsi(ham, psi, field=f))
    rhs = _vdot_h3(g.h, oracle.hpsi(ham, phi, field=f), psi)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13 * np.abs(lhs).max())


def test_single_projector_closed_form():
    """One atom, kinetic and local potential off, psi = p_i on its support:
    V_nl p_i = sum_j p_j E_j h^3 <p_j|p_i>; for the s channel, whose
    overlap with the p channels vanishes by symmetry when the atom sits on a
    grid point, V_nl p_s = E_s h^3 (sum p_s^2) p_s."""
    h = 0.25
    g = oracle.Grid(h, n=21)
    pos = fdmath.positions(g.ijk, g.dims, h)
    proj = synth.kb_projectors(3, pos, np.zeros((1, 3)), rcut=2.0)
    ham = oracle.Ham(g, V=None, kin=0.0, projectors=proj)
    idx, p, E = proj.idx[0], proj.p[0], proj.E[0]
    psi = np.zeros((g.np, 1), dtype=np.complex128)
    psi[idx, 0] = p[:, 0]
    out = oracle.hpsi(ham, psi)[:, 0]
    expect = np.zeros(g.np)
    expect[idx] = E[0] * h ** 3 * (p[:, 0] ** 2).sum() * p[:, 0]
    np.testing.assert_allclose(out.real, expect, rtol=0, atol=1e-14 * np.abs(expect).max())
    assert np.abs(out.imag).max() == 0.0


def test_nonlocal_rank():
    """With kinetic and local terms off, H has rank <= 4 * natoms."""
    g, pos, _, proj, _ = _small_system(R=1.6, h=0.3, natoms=2)
    ham = oracle.Ham(g, V=None, kin=0.0, projectors=proj)
    M = oracle.hpsi(ham, np.eye(g.np, dtype=np.complex128))
    s = np.linalg.svd(M, compute_uv=False)
    assert (s > 1e-12 * s[0]).sum() <= 4 * proj.natoms
    assert (s > 1e-12 * s[0]).sum() >= 4


def test_local_and_dipole_terms_pointwise():
    """Kinetic off, no projectors: (H psi)(r) = (V(r) + F x_axis(r)) psi(r)."""
    g = oracle.Grid(0.3, R=2.0)
    pos = fdmath.positions(g.ijk, g.dims, 0.3)
    V = synth.harmonic_potential(pos)
    for axis in range(3):
        ham = oracle.Ham(g, V=V, kin=0.0, dipole_axis=axis)
        psi = synth.white_noise(5, g.np, 2, g.h)
        out = oracle.hpsi(ham, psi, field=-0.8)
        np.testing.assert_allclose(out, (V - 0.8 * pos[:, axis])[:, None] * psi, rtol=1e-15, atol=1e-15)


def test_orbitals_independent_and_padding_untouched():
    g, pos, ham, proj, psi = _small_system(nst=3)
    full = oracle.hpsi(ham, psi, field=0.2)
    for n in range(3):
        one = oracle.hpsi(ham, psi[:, n:n + 1].copy(), field=0.2)
        np.testing.assert_array_equal(one[:, 0], full[:, n])
    padded = np.zeros((g.np, 5), dtype=np.complex128)
    padded[:, :3] = psi
    padded[:, 3:] = 7.0
    out = oracle.hpsi(ham, padded, field=0.2, nst=3)
    np.testing.assert_array_equal(out[:, :3], full)
    assert np.all(out[:, 3:] == 0.0)  # output columns beyond nst are not written


# ------------------------------------------------------------ Taylor ---

def test_taylor_pure_potential_pointwise():
    """Kinetic off: one step multiplies pointwise by T4(-i dt V(r)), whose
    distance to exp(-i dt V) is bounded by (dt V)^5 / 120, and whose squared
    modulus is 1 - x^6/72 + x^8/576."""
    g = oracle.Grid(0.3, R=2.5)
    pos = fdmath.positions(g.ijk, g.dims, 0.3)
    V = 3.0 * synth.harmonic_potential(pos) - 2.0
    ham = oracle.Ham(g, V=V, kin=0.0)
    psi = synth.white_noise(8, g.np, 2, g.h)
    dt = 0.05
    out = oracle.taylor_step(ham, psi, dt)
    x = dt * V
    t4 = fdmath.taylor4_scalar(-1j * x)
    np.testing.assert_allclose(out, t4[:, None] * psi, rtol=1e-14, atol=1e-15)
    assert np.all(np.abs(t4 - np.exp(-1j * x)) <= np.abs(x) ** 5 / 120 + 1e-15)
    amp = 1.0 - x ** 6 / 72.0 + x ** 8 / 576.0
    np.testing.assert_allclose(np.abs(out) ** 2, amp[:, None] * np.abs(psi) ** 2, rtol=1e-13)


def test_taylor_plane_wave_interior():
    """Plane wave on a 48^3 cube: after one step, every point at least 16
    from the edge (4 applications x 4-point reach) equals T4(-i dt lambda) psi."""
    n, h, dt = 48, 0.3, 0.01
    g = oracle.Grid(h, n=n)
    pos = fdmath.positions(g.ijk, g.dims, h)
    k = 2.0 * math.pi * np.array([3, -2, 5]) / (n * h)
    psi = np.exp(1j * pos @ k)[:, None]
    out = oracle.taylor_step(oracle.Ham(g, V=None, kin=-0.5), psi, dt)
    lam = fdmath.plane_wave_eigenvalue(k, h)
    m = fdmath.interior_mask(g.ijk, g.dims, 16)
    np.testing.assert_allclose(out[m, 0], fdmath.taylor4_scalar(-1j * dt * lam) * psi[m, 0],
                               rtol=1e-13, atol=1e-13)


def test_taylor_ho_norm_and_energy_drift():
    """HO ground state over 20 steps at dt = 0.01: norm and energy move by
    no more than the Taylor(4) amplification error of the lowest mode."""
    n, h, dt = 32, 0.3, 0.01
    g = oracle.Grid(h, n=n)
    pos = fdmath.positions(g.ijk, g.dims, h)
    ham = oracle.Ham(g, V=synth.harmonic_potential(pos), kin=-0.5)
    psi = synth.ho_ground_state(pos)[:, None].astype(np.complex128)
    n0 = oracle.norm2(g, psi)[0]
    e0 = oracle.energy(ham, psi)[0]
    out = oracle.propagate(ham, psi, dt, 20)
    n1 = oracle.norm2(g, out)[0]
    e1 = oracle.energy(ham, out)[0]
    assert abs(n1 - n0) < 1e-10
    assert abs(e1 - e0) < 1e-9
    # the lowest mode only picks up a phase: |<psi0|psi(t)>| ~ |T4(-i dt E0)|^20
    ov = abs(oracle.dot(g, psi, out)[0]) / n0
    assert ov == pytest.approx(abs(fdmath.taylor4_scalar(-1j * dt * e0 / n0)) ** 20, abs=1e-9)


# -------------------------------------------------------- reductions ---

def test_reductions_against_numpy():
    g, pos, ham, proj, psi = _small_system(nst=4)
    phi = synth.white_noise(12, g.np, 4, g.h)
    np.testing.assert_allclose(oracle.dot(g, phi, psi), _vdot_h3(g.h, phi, psi), rtol=1e-13)
    np.testing.assert_allclose(oracle.norm2(g, psi), 1.0, rtol=1e-13)  # synth normalises
    e, per = oracle.energy(ham, psi, field=0.1)
    assert np.abs(per.imag).max() < 1e-12 * np.abs(per.real).max()
    assert e == pytest.approx(per.real.sum(), rel=1e-15)


# ----------------------------------------------------------- adjoint ---

def test_adjoint_step_dot_product():
    """<u| T4(-i dt H) v> = <T4(+i dt H) u | v> for the oracle's forward step
    and the lambda-update of its adjoint step."""
    g, pos, ham, proj, psi = _small_system(nst=2)
    u = synth.white_noise(21, g.np, 2, g.h)
    dt, f = 0.02, 0.3
    fwd = oracle.taylor_step(ham, psi, dt, field=f)
    lam, _ = oracle.adjoint_step(ham, psi, u, dt, f)
    lhs = _vdot_h3(g.h, u, fwd)
    rhs = _vdot_h3(g.h, lam, psi)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-14, atol=1e-15)


def test_laser_field_sine_series():
    c = np.array([0.3, -0.2, 0.05])
    T = 2.0
    for t in [0.0, 0.31, 1.0, 1.7]:
        ref = sum(c[k - 1] * math.sin(k * math.pi * t / T) for k in (1, 2, 3))
        assert oracle.laser_field(c, T, t) == pytest.approx(ref, rel=1e-15, abs=1e-16)


def _control_system():
    h, n = 0.4, 14
    g = oracle.Grid(h, n=n)
    pos = fdmath.positions(g.ijk, g.dims, h)
    wells = synth.gaussian_wells(5, 2, box=1.5)
    ham = oracle.Ham(g, V=synth.well_potential(pos, wells), kin=-0.5, dipole_axis=2)
    psi0 = synth.gaussian_packets(5, pos, 2, h, centre_box=1.0)
    return g, ham, psi0


def test_control_gradient_matches_central_differences():
    """Discrete adjoint dJ/dc against central finite differences of the
    forward propagation, for every coefficient, at two step sizes
    (Richardson consistency)."""
    g, ham, psi0 = _control_system()
    dt, nsteps = 0.05, 30
    coef = synth.laser_coefficients(5, 6, sigma=0.3)
    J, grad, gsteps = oracle.control_gradient(ham, psi0, dt, nsteps, coef)
    J0, _ = oracle.control_forward(ham, psi0, dt, nsteps, coef)
    assert J == pytest.approx(J0, rel=1e-14)
    fd = {}
    for eps in (1e-3, 1e-4):
        d = np.zeros_like(coef)
        for k in range(coef.size):
            e = np.zeros_like(coef)
            e[k] = eps
            jp, _ = oracle.control_forward(ham, psi0, dt, nsteps, coef + e)
            jm, _ = oracle.control_forward(ham, psi0, dt, nsteps, coef - e)
            d[k] = (jp - jm) / (2 * eps)
        fd[eps] = d
    scale = np.abs(grad).max()
    assert scale > 1e-3
    assert np.abs(fd[1e-4] - grad).max() <= 1e-6 * scale
    # the FD error falls by ~100x between the two step sizes (O(eps^2))
    assert np.abs(fd[1e-4] - grad).max() < 0.05 * np.abs(fd[1e-3] - grad).max() + 1e-12 * scale


def test_step_gradient_matches_field_perturbation():
    """g_n = dJ/dE_n against a central difference of the field at one step."""
    g, ham, psi0 = _control_system()
    dt, nsteps = 0.05, 12
    coef = synth.laser_coefficients(6, 4, sigma=0.3)
    T = dt * nsteps
    fields = np.array([oracle.laser_field(coef, T, (n + 0.5) * dt) for n in range(nsteps)])
    _, _, gsteps = oracle.control_gradient(ham, psi0, dt, nsteps, coef)
    eps = 1e-4
    for n in (0, 5, 11):
        fp = fields.copy()
        fp[n] += eps
        fm = fields.copy()
        fm[n] -= eps
        jp = oracle.dipole_target(ham, oracle.propagate(ham, psi0, dt, nsteps, fp))
        jm = oracle.dipole_target(ham, oracle.propagate(ham, psi0, dt, nsteps, fm))
        assert gsteps[n] == pytest.approx((jp - jm) / (2 * eps), rel=1e-6, abs=1e-9)
