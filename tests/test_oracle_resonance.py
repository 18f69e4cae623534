"""Pin of the oracle's complex scaling by the paper's own resonance example
(section "Complex scaling and resonances", Figs. cs-spectrum and
cs-potential-wfs): the one-dimensional potential v(x) = 3 (x^2 - 2)
e^{-x^2/4} scaled with theta = 0.5.  The figures show two bound states and a
lowest resonance close to the origin of the complex plane whose imaginary
part is of order -10^-5.

The one-dimensional problem runs on a rectangular box one point thick in y
and z: the y and z taps of the star stencil then fall outside the box, so
the box's H_theta is the one-dimensional operator plus the constant
2 kin e^{-2 i theta} c_0 / h^2, which is subtracted.  Grid (the paper gives
none): h = 0.1 bohr, 801 points, |x| <= 40 bohr.  Checked here:
- exactly two eigenvalues with negative real part, both on the real axis and
  equal to the unscaled (Hermitian) problem's two bound levels;
- an isolated eigenvalue with real part between 0 and the barrier top
  (2.68 Ha) and imaginary part between -10^-4 and -10^-5;
- the resonance does not move with the scaling angle (theta = 0.4 gives the
  same value), while the rotated continuum does;
- the box constant is right: with v = 0 every eigenvalue of the shifted
  operator lies on the ray of angle -2 theta."""
import numpy as np
import pytest

import oracle
import synth

C0 = -205.0 / 72.0
N, H = 801, 0.1


def _spectrum(theta, potential=True):
    g = oracle.Grid(H, box=(N, 1, 1))
    x = g.positions()[:, 0]
    v = synth.resonance_potential_1d(x, theta) if potential else np.zeros(N, dtype=np.complex128)
    ham = oracle.Ham(g, V=v.real.copy(), V_im=v.imag.copy(), kin=-0.5, theta=theta)
    Hd = oracle.hpsi(ham, np.eye(N, dtype=np.complex128))
    shift = 2 * (-0.5) * np.exp(-2j * theta) * C0 / H ** 2
    return np.linalg.eigvals(Hd) - shift


@pytest.fixture(scope="module")
def spectra():
    return {th: _spectrum(th) for th in (0.0, 0.4, 0.5)}


def _resonance(ev):
    cand = ev[(ev.real > 0.0) & (ev.real < 2.68) & (np.abs(ev.imag) < 1e-3)]
    assert cand.size == 1, cand
    return cand[0]


def test_two_bound_states_unchanged_by_scaling(spectra):
    e0 = np.sort(spectra[0.0].real[spectra[0.0].real < 0])
    assert e0.size == 2 and np.abs(spectra[0.0].imag).max() < 1e-9
    for th in (0.4, 0.5):
        ev = spectra[th]
        b = ev[ev.real < 0]
        assert b.size == 2, (th, b)
        assert np.abs(b.imag).max() < 1e-6
        np.testing.assert_allclose(np.sort(b.real), e0, rtol=0, atol=1e-6)
    assert -6.0 < e0[0] < e0[1] < 0.0


def test_lowest_resonance_near_origin_with_small_width(spectra):
    r5 = _resonance(spectra[0.5])
    assert 0.0 < r5.real < 1.0
    assert -1e-4 < r5.imag < -1e-5
    # not a continuum eigenvalue: those near it sit far off the real axis
    near = spectra[0.5][np.abs(spectra[0.5] - r5) < 0.5]
    assert np.sort(np.abs(near.imag))[1] > 50 * abs(r5.imag)


def test_resonance_independent_of_angle_continuum_not(spectra):
    r4, r5 = _resonance(spectra[0.4]), _resonance(spectra[0.5])
    assert abs(r4.real - r5.real) < 1e-6
    assert abs(r4.imag - r5.imag) < 0.02 * abs(r5.imag)
    # the continuum just above zero energy turns with the angle
    c4 = spectra[0.4][(spectra[0.4].imag < -1e-3) & (np.abs(spectra[0.4]) < 0.05)]
    c5 = spectra[0.5][(spectra[0.5].imag < -1e-3) & (np.abs(spectra[0.5]) < 0.05)]
    assert c4.size and c5.size
    assert np.median(np.angle(c5)) < np.median(np.angle(c4)) - 0.1


def test_box_constant_free_particle_on_the_rotated_ray():
    ev = _spectrum(0.5, potential=False)
    np.testing.assert_allclose(np.angle(ev), -1.0, rtol=0, atol=1e-9)
