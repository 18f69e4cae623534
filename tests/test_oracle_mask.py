"""Pins of the oracle's mask boundary absorber (section "Photoemission",
eq. (mask_split)): psi <- M(r) U(dt) psi after every step, with the charge
that leaves the box accumulated per orbital."""
import numpy as np

import oracle
import synth
from tests.fdmath import taylor4_scalar


def _system(kin=-0.5, natoms=2, nst=3, seed=4):
    g = oracle.Grid(0.3, R=3.2)
    pos = g.positions()
    wells = synth.gaussian_wells(seed, max(natoms, 1), ball=1.0)
    V = synth.well_potential(pos, wells)
    proj = synth.kb_projectors(seed, pos, wells.centres[:natoms], rcut=1.2) if natoms else None
    H = oracle.Ham(g, V=V, kin=kin, dipole_axis=2, projectors=proj)
    psi = synth.white_noise(seed, g.np, nst, 0.3, ld=nst + 1)
    return g, pos, V, H, psi


def test_unit_mask_is_the_plain_propagation():
    g, pos, V, H, psi = _system()
    fields = np.array([0.1, -0.2, 0.05])
    plain = oracle.propagate(H, psi, 0.01, 3, fields=fields, nst=3)
    masked, removed = oracle.propagate_masked(H, psi, 0.01, 3, np.ones(g.np), fields=fields, nst=3)
    np.testing.assert_array_equal(masked, plain)
    np.testing.assert_array_equal(removed, np.zeros(3))


def test_pointwise_hamiltonian_closed_form():
    """kin = 0, no projectors, no field: H is V(r) pointwise, so one masked
    step is M(r) T4(-i dt V(r)) psi(r) at every point."""
    g, pos, V, H, psi = _system(kin=0.0, natoms=0)
    M = synth.radial_mask(pos, 3.2, 1.5)
    dt = 0.02
    got, removed = oracle.propagate_masked(H, psi, dt, 1, M, nst=3)
    u = taylor4_scalar(-1j * dt * V)[:, None] * psi[:, :3]
    ref = M[:, None] * u
    np.testing.assert_allclose(got[:, :3], ref, rtol=0, atol=1e-15 * np.abs(ref).max())
    np.testing.assert_array_equal(got[:, 3], psi[:, 3])  # spare column untouched
    # the charge that leaves: h^3 sum (1 - M^2) |U psi|^2 per orbital
    lost = g.h ** 3 * np.sum((1 - M[:, None] ** 2) * np.abs(u) ** 2, axis=0)
    np.testing.assert_allclose(removed, lost, rtol=1e-13)


def test_removed_charge_is_the_norm_loss_and_zero_mask_points_vanish():
    g, pos, V, H, psi = _system()
    M = synth.radial_mask(pos, 2.7, 1.2)  # zero on the outer shell of the box
    assert np.any(M == 0.0) and np.any(M == 1.0)
    n0 = oracle.norm2(g, psi, nst=3)
    plain = oracle.propagate(H, psi, 0.01, 1, nst=3)
    got, removed = oracle.propagate_masked(H, psi, 0.01, 1, M, nst=3)
    # one step: removed = |U psi|^2 - |M U psi|^2 with U psi the unmasked step
    np.testing.assert_allclose(removed, oracle.norm2(g, plain, nst=3) - oracle.norm2(g, got, nst=3),
                               rtol=1e-12)
    assert np.all(removed > 0)
    assert np.all(got[M == 0.0, :3] == 0)
    np.testing.assert_array_equal(got[M == 1.0, :3], plain[M == 1.0, :3])
    # several steps: the norm only decreases, by at least the removed charge minus Taylor damping
    got5, removed5 = oracle.propagate_masked(H, psi, 0.01, 5, M, nst=3)
    n5 = oracle.norm2(g, got5, nst=3)
    assert np.all(n5 < n0)
    assert np.all(n5 + removed5 <= n0 * (1 + 1e-12))
