"""Pins of the oracle's complex-scaled Hamiltonian (section "Complex scaling
and resonances": H_theta = -1/2 e^{-2 i theta} Lap + v(r e^{i theta}),
matrix elements without conjugation), against facts the section states:

- the free-particle continuum rotates by -2 theta about the origin: with
  V = 0 the spectrum of H_theta is e^{-2 i theta} times that of the kinetic
  term, exactly on the grid;
- H_theta is symmetric (not Hermitian), so the unconjugated Rayleigh quotient
  x^T H x / x^T x returns its eigenvalues;
- bound-state energies are unchanged: the harmonic oscillator v = r^2/2,
  continued to e^{2 i theta} r^2/2, keeps its lowest levels (1.5, 2.5) on
  the real axis, equal to the unscaled ones on the same grid to the box and
  discretisation error, while a wrong sign of the rotation would move them
  by 1.5 sin(2 theta) off the axis."""
import numpy as np

import oracle


def _dense(ham, npts):
    return oracle.hpsi(ham, np.eye(npts, dtype=np.complex128))


def test_free_continuum_rotates_by_minus_two_theta():
    g = oracle.Grid(0.4, n=7)
    theta = 0.3
    T = _dense(oracle.Ham(g, kin=-0.5), g.np)
    Ht = _dense(oracle.Ham(g, kin=-0.5, theta=theta), g.np)
    ev_t = np.sort(np.linalg.eigvalsh(T.real))
    ev = np.linalg.eigvals(Ht) * np.exp(2j * theta)  # undo the rotation
    assert np.abs(ev.imag).max() <= 1e-10 * np.abs(ev).max()
    np.testing.assert_allclose(np.sort(ev.real), ev_t, rtol=0, atol=1e-10 * np.abs(ev_t).max())


def test_scaled_operator_is_symmetric_and_rayleigh_quotient():
    g = oracle.Grid(0.5, R=2.0)
    x = g.positions()
    theta = 0.25
    r2 = (x ** 2).sum(axis=1)
    H = _dense(oracle.Ham(g, V=np.cos(2 * theta) * r2 / 2, V_im=np.sin(2 * theta) * r2 / 2,
                          kin=-0.5, theta=theta, dipole_axis=2), g.np)
    assert np.abs(H.imag).max() > 0.1  # genuinely complex
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
    assert np.abs(H - H.conj().T).max() > 0.1  # not Hermitian
    lam, U = np.linalg.eig(H)
    for k in np.argsort(lam.real)[:5]:
        u = U[:, k]
        rq = (u @ (H @ u)) / (u @ u)
        assert abs(rq - lam[k]) <= 1e-10 * abs(lam[k])


def test_bound_states_stay_on_the_real_axis():
    g = oracle.Grid(0.5, n=12)
    x = g.positions()
    r2 = (x ** 2).sum(axis=1)
    H0 = _dense(oracle.Ham(g, V=r2 / 2, kin=-0.5), g.np)
    ev0 = np.sort(np.linalg.eigvalsh(H0.real))
    # the grid resolves the lowest levels of the oscillator
    assert abs(ev0[0] - 1.5) < 2e-2 and np.all(np.abs(ev0[1:4] - 2.5) < 5e-2)
    for theta in (0.1, 0.3):
        Ht = _dense(oracle.Ham(g, V=np.cos(2 * theta) * r2 / 2, V_im=np.sin(2 * theta) * r2 / 2,
                               kin=-0.5, theta=theta), g.np)
        ev = np.linalg.eigvals(Ht)
        low = ev[np.argsort(np.abs(ev - 1.5))[:1]]
        nxt = ev[np.argsort(np.abs(ev - 2.5))[:3]]
        for got, ref in ((low, ev0[:1]), (nxt, ev0[1:4])):
            assert np.all(np.abs(got.imag) < 2e-2 * 1.5 * np.sin(2 * theta) + 2e-3), (theta, got)
            np.testing.assert_allclose(np.sort(got.real), ref, rtol=0, atol=5e-3)
