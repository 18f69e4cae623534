"""Complex scaling on the GPU (section "Complex scaling and resonances").

- H_theta psi (kinetic prefactor kin e^{-2 i theta}, potential V + i V_im,
  a dipole field) matches the oracle to the FP64 bar for every tile shape
  the library maps it to, with spare orbitals and padding points; one
  Taylor(4) step of the non-unitary propagator does too.
- theta = 0 without V_im gives back the Hermitian operator bit for bit.
- The bilinear form is h^3 sum a b without conjugation.
- Inverse iteration finds the eigenvalues of the scaled oscillator nearest
  the targets, equal to the dense eigenvalues of the oracle's H_theta, and
  the bound levels stay on the real axis.
- Entry points that need a Hermitian H, projectors, masks and the mixed path
  reject a complex-scaled handle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

THETA = 0.3


@pytest.fixture(scope="module")
def sys_():
    s = System(0.3, R=3.1, potential="wells", natoms=0, nst=5, ld=6, seed=51, dipole_axis=2, pad=4,
               well_ball=1.2)
    rng = np.random.default_rng(52)
    vim = -0.3 * rng.random(s.og.np)
    oh = oracle.Ham(s.og, V=s.V, kin=-0.5, dipole_axis=2, theta=THETA, V_im=vim)
    return s, vim, oh


def test_scaled_hpsi_and_step_match_oracle(sys_):
    R = rsg()
    s, vim, oh = sys_
    field, dt = 0.05, 0.01
    psi = s.to_gpu(s.psi)
    plain = s.from_gpu(R.hpsi(s.gh, psi, field=field, nst=s.nst))
    s.gh.set_complex_scaling(THETA, torch.from_numpy(vim).cuda())
    try:
        ref_h = oracle.hpsi(oh, s.psi, field=field, nst=s.nst)
        ref_s = oracle.taylor_step(oh, s.psi, dt, field=field, nst=s.nst)
        for tile in [(1, 32, 16, 0, 1, 0, 1, 0), (1, 16, 8, 0, 1, 0, 0, 0), (1, 8, 8, 4, 1, 1, 1, 1),
                     (1, 32, 16, 0, 2, 0, 2, 0), (1, 64, 8, 0, 1, 0, 1, 0)]:
            R.set_tile(s.gh, s.nst, *tile)
            y = s.from_gpu(R.hpsi(s.gh, psi, field=field, nst=s.nst))
            assert orbital_rel_err(y, ref_h, s.nst) <= 1e-12, tile
            assert not np.any(y[:, s.nst:])
            x = psi.clone()
            R.propagate_step(s.gh, x, dt, field=field, nst=s.nst)
            assert s.pad_untouched(x), tile
            xs = s.from_gpu(x)
            assert orbital_rel_err(xs, ref_s, s.nst) <= 1e-12, tile
            np.testing.assert_array_equal(xs[:, s.nst:], s.psi[:, s.nst:])
        # the step is not unitary any more: the norm changes
        n0 = R.norm2(s.gh.grid, psi, nst=s.nst).cpu().numpy()
        n1 = R.norm2(s.gh.grid, x, nst=s.nst).cpu().numpy()
        assert np.abs(n1 - n0).max() > 1e-6
    finally:
        s.gh.set_complex_scaling(0.0, None)
    back = s.from_gpu(R.hpsi(s.gh, psi, field=field, nst=s.nst))
    np.testing.assert_array_equal(back, plain)


def test_bilinear_form(sys_):
    R = rsg()
    s, vim, oh = sys_
    rng = np.random.default_rng(53)
    a = rng.standard_normal((s.og.np, s.ld)) + 1j * rng.standard_normal((s.og.np, s.ld))
    b = rng.standard_normal((s.og.np, s.ld)) + 1j * rng.standard_normal((s.og.np, s.ld))
    got = R.bilinear(s.gh.grid, s.to_gpu(a), s.to_gpu(b), nst=s.nst).cpu().numpy()
    h3 = s.og.h ** 3
    for n in range(s.nst):
        ref = h3 * np.sum(a[:, n] * b[:, n])
        assert abs(got[n] - ref) <= 1e-12 * np.sum(np.abs(a[:, n] * b[:, n])) * h3
    # symmetric, and different from the Hermitian product
    sym = R.bilinear(s.gh.grid, s.to_gpu(b), s.to_gpu(a), nst=s.nst).cpu().numpy()
    np.testing.assert_allclose(sym, got, rtol=1e-13)
    herm = R.dot(s.gh.grid, s.to_gpu(a), s.to_gpu(b), nst=s.nst).cpu().numpy()
    assert np.abs(herm - got).min() > 1e-3


def test_inverse_iteration_scaled_oscillator():
    """Cube 12^3 at h = 0.5, v = r^2/2 continued to e^{2 i theta} r^2/2,
    theta = 0.2: the eigenvalues nearest 1.45 and 2.4 equal the dense
    eigenvalues of the oracle's H_theta and lie next to 1.5 and 2.5."""
    R = rsg()
    theta = 0.2
    og, gg = oracle.Grid(0.5, n=12), R.Grid(0.5, n=12)
    x = og.positions()
    r2 = (x ** 2).sum(axis=1)
    vre, vim = np.cos(2 * theta) * r2 / 2, np.sin(2 * theta) * r2 / 2
    gh = R.Hamiltonian(gg, V=torch.from_numpy(vre).cuda(), kin=-0.5)
    gh.set_complex_scaling(theta, torch.from_numpy(vim).cuda())
    Hd = oracle.hpsi(oracle.Ham(og, V=vre, V_im=vim, kin=-0.5, theta=theta), np.eye(og.np, dtype=np.complex128))
    ev = np.linalg.eigvals(Hd)
    targets = np.array([1.45, 2.4 + 0.01j])
    start = synth.ho_low_states(x, 2)
    psi = torch.from_numpy(start.T.copy()).cuda()
    lam, its = R.cs_eigs(gh, psi, targets, max_outer=40, tol=1e-13, qmr_tol=1e-12, qmr_maxiter=4000)
    for k, z in enumerate(targets):
        ref = ev[np.argmin(np.abs(ev - z))]
        assert abs(lam[k] - ref) <= 1e-9 * abs(ref), (k, lam[k], ref)
    assert abs(lam[0] - 1.5) < 5e-3 and abs(lam[1] - 2.5) < 2e-2
    # the returned vectors are eigenvectors: H psi = lambda psi
    hp = R.hpsi(gh, psi).cpu().numpy()
    p = psi.cpu().numpy()
    for k in range(2):
        res = np.linalg.norm(hp[k] - lam[k] * p[k]) / np.linalg.norm(lam[k] * p[k])
        assert res < 1e-8, (k, res)


def test_scaled_handle_rejections(sys_):
    R = rsg()
    s, vim, oh = sys_
    psi = s.to_gpu(s.psi)
    # projectors cannot be complex-scaled
    p = System(0.3, R=3.1, potential="wells", natoms=2, nst=2, seed=54, rcut=1.0, well_ball=1.2)
    with pytest.raises(R.RSGError) as ei:
        p.gh.set_complex_scaling(0.2)
    assert ei.value.code == -6
    s.gh.set_complex_scaling(THETA, torch.from_numpy(vim).cuda())
    try:
        with pytest.raises(R.RSGError) as ei:
            R.propagate_step(s.gh, psi.clone(), 0.01, dtype="mixed", nst=s.nst)
        assert ei.value.code == -6
        with pytest.raises(R.RSGError) as ei:
            s.gh.set_mask(torch.ones(s.og.np, dtype=torch.float64, device="cuda"))
        assert ei.value.code == -6
        with pytest.raises(R.RSGError) as ei:
            R.adjoint_step(s.gh, psi, psi.clone(), 0.01, 0.0)
        assert ei.value.code == -6
        with pytest.raises(R.RSGError) as ei:
            R.shifted_solve(s.gh, psi, 3.0, method="cg", nst=s.nst)
        assert ei.value.code == -1
        # QMR is fine with the complex symmetric operator
        x, info = R.shifted_solve(s.gh, psi, 2.0 + 0.5j, method="qmr", tol=1e-10, nst=s.nst)
        assert np.all(info["status"] == 0)
    finally:
        s.gh.set_complex_scaling(0.0, None)


def test_paper_resonance_through_the_library():
    """The resonance example of the complex-scaling section (Figs.
    cs-spectrum, cs-potential-wfs): v(x) = 3 (x^2 - 2) e^{-x^2/4}, theta =
    0.5, on an 801 x 1 x 1 box at h = 0.1 (the one-dimensional Hamiltonian
    plus the box constant 2 kin e^{-2 i theta} c_0 / h^2).  Inverse iteration
    in the library finds the two bound states and the lowest resonance (real
    part in (0, 1), imaginary part between -1e-4 and -1e-5), each equal to the
    oracle's dense eigenvalue to 1e-9 relative."""
    R = rsg()
    theta, n, h = 0.5, 801, 0.1
    og, gg = oracle.Grid(h, box=(n, 1, 1)), R.Grid(h, box=(n, 1, 1))
    assert gg.np == og.np == n and gg.dims == (n, 1, 1)
    x = og.positions()[:, 0]
    v = synth.resonance_potential_1d(x, theta)
    vre, vim = v.real.copy(), v.imag.copy()
    gh = R.Hamiltonian(gg, V=torch.from_numpy(vre).cuda(), kin=-0.5)
    gh.set_complex_scaling(theta, torch.from_numpy(vim).cuda())
    shift = 2 * (-0.5) * np.exp(-2j * theta) * (-205.0 / 72.0) / h ** 2
    Hd = oracle.hpsi(oracle.Ham(og, V=vre, V_im=vim, kin=-0.5, theta=theta), np.eye(n, dtype=np.complex128))
    ev = np.linalg.eigvals(Hd)
    res = ev - shift
    cand = res[(res.real > 0) & (res.real < 2.68) & (np.abs(res.imag) < 1e-3)]
    assert cand.size == 1
    bound = np.sort_complex(res[res.real < 0])
    assert bound.size == 2
    targets = np.array([bound[0] + 0.05, bound[1] + 0.05, cand[0] + 0.02]) + shift
    start = synth.white_noise(61, n, 3, h)
    psi = torch.from_numpy(start.T.copy()).cuda()
    lam, its = R.cs_eigs(gh, psi, targets, max_outer=60, tol=1e-13, qmr_tol=1e-12, qmr_maxiter=20000)
    for k, z in enumerate(targets):
        ref = ev[np.argmin(np.abs(ev - z))]
        assert abs(lam[k] - ref) <= 1e-9 * abs(ref), (k, lam[k], ref)
    r = lam[2] - shift
    assert 0 < r.real < 1 and -1e-4 < r.imag < -1e-5, r
    np.testing.assert_allclose((lam[:2] - shift).real, bound.real, rtol=0, atol=1e-8)


def test_scaled_propagate_in_a_graph_matches_eager():
    """A complex-scaled handle whose tile is remapped at launch (64 x 8 and
    32 x 8 have no complex-scaled kernel; 32 x 16 runs at depth 1) captures
    its steps into a HIP graph, and every replay gives the eager steps'
    bits."""
    R = rsg()
    s = System(0.3, R=3.6, potential="wells", natoms=0, nst=3, seed=53, well_ball=1.2)
    rng = np.random.default_rng(54)
    vim = -0.2 * rng.random(s.og.np)
    s.gh.set_complex_scaling(0.25, torch.from_numpy(vim).cuda())
    stream = torch.cuda.Stream()
    for tile in [(1, 64, 8, 0, 2, 0, 1, 0), (1, 32, 8, 0, 2, 0, 1, 0), (1, 32, 16, 0, 2, 0, 2, 0)]:
        R.set_tile(s.gh, s.nst, *tile)
        with torch.cuda.stream(stream):
            eager = s.to_gpu(s.psi)
            R.propagate(s.gh, eager, 0.01, 4)
            g = s.to_gpu(s.psi)
            R.propagate(s.gh, g, 0.01, 4, graph=True)  # capture and first replay
            torch.cuda.synchronize()
            assert torch.equal(g, eager), tile
            for _ in range(2):  # later replays, with eager work in between
                h = s.to_gpu(s.psi)
                R.propagate(s.gh, h, 0.01, 4, graph=True)
                torch.cuda.synchronize()
                assert torch.equal(h, eager), tile
