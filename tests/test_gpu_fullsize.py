"""Full-size parity on the benchmark workload: the 3,053,617-point sphere
(R = 18 bohr, h = 0.2) with 64 orbitals, 16 wells and 4 projectors each,
stored with row-aligned rows (align 8, the benchmark's storage) and with
compact rows.  The GPU runs all 64 orbitals in the launch configuration the
benchmark times (the autotuner's tile, chosen the same way); the oracle
recomputes a sample of orbitals, which is exact because orbitals are
independent under H (pinned in the oracle tests)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

SAMPLE = [0, 29, 63]


@pytest.fixture(scope="module", params=[8, 1], ids=["align8", "compact"])
def sphere18(request):
    cfg = synth.WORKLOADS["sphere18_wells"]
    R = rsg()
    og = oracle.Grid(cfg["h"], R=cfg["R"])
    gg = R.Grid(cfg["h"], R=cfg["R"], align=request.param)
    assert gg.npoints == og.np == 3053617
    live = gg.live()
    np.testing.assert_array_equal(gg.coords()[live], og.ijk)
    pos = og.positions()
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], ball=cfg["well_ball"])
    V = synth.well_potential(pos, wells)
    proj = synth.kb_projectors(cfg["seed"], pos, wells.centres)
    psi = synth.white_noise(cfg["seed"], og.np, cfg["nst"], cfg["h"])
    # the library's orbital-major layout over the grid's slots (dead slots zero)
    psi_om = np.zeros((cfg["nst"], gg.np), dtype=np.complex128)
    psi_om[:, live] = psi.T
    Vs = np.zeros(gg.np)
    Vs[live] = V
    oh = oracle.Ham(og, V=V, kin=-0.5, projectors=proj)
    dev = torch.device("cuda")
    gh = R.Hamiltonian(gg, V=torch.from_numpy(Vs).to(dev), kin=-0.5,
                       projectors=[(torch.from_numpy(live[i].astype(np.int32)).to(dev),
                                    torch.from_numpy(p).to(dev), E)
                                   for i, p, E in zip(proj.idx, proj.p, proj.E)])
    # the launch configuration the benchmark times: the autotuner's tile
    tile, _ = R.autotune(gh, torch.from_numpy(psi_om).to(dev), reps=1)
    return dict(cfg=cfg, og=og, oh=oh, gg=gg, gh=gh, psi=psi, psi_om=psi_om, tile=tile, live=live,
                V=V, Vs=Vs)


def _sample(t, s):
    """Sampled orbitals of a GPU batch in the oracle's point order, and
    the largest magnitude in their dead slots."""
    a = t[SAMPLE, :].cpu().numpy()
    dead = np.delete(a, s["live"], axis=1)
    return np.ascontiguousarray(a[:, s["live"]].T), (float(np.abs(dead).max()) if dead.size else 0.0)


def test_sphere18_hpsi_sampled_orbitals(sphere18):
    s = sphere18
    psi = torch.from_numpy(s["psi_om"]).cuda()
    out = torch.full_like(psi, 2.0 - 1.0j)
    rsg().hpsi(s["gh"], psi, out=out)
    got, dead = _sample(out, s)
    ref = oracle.hpsi(s["oh"], np.ascontiguousarray(s["psi"][:, SAMPLE]))
    assert orbital_rel_err(got, ref, len(SAMPLE)) <= 1e-12
    assert dead == 0.0


def test_sphere18_taylor_step_sampled_orbitals(sphere18):
    s = sphere18
    psi = torch.from_numpy(s["psi_om"]).cuda()
    rsg().propagate_step(s["gh"], psi, s["cfg"]["dt"])
    got, dead = _sample(psi, s)
    ref = oracle.taylor_step(s["oh"], np.ascontiguousarray(s["psi"][:, SAMPLE]), s["cfg"]["dt"])
    assert orbital_rel_err(got, ref, len(SAMPLE)) <= 1e-12
    assert dead == 0.0


def test_sphere18_norm_conserved_over_steps(sphere18):
    """Property at full size: 5 steps change each orbital's norm only by the
    Taylor(4) amplification of its highest modes (|T4(ix)|^2 <= 1)."""
    s = sphere18
    R = rsg()
    psi = torch.from_numpy(s["psi_om"]).cuda()
    n0 = R.norm2(s["gg"], psi).cpu().numpy()
    R.propagate(s["gh"], psi, s["cfg"]["dt"], 5)
    n1 = R.norm2(s["gg"], psi).cpu().numpy()
    assert np.all(n1 <= n0 * (1 + 1e-12))
    assert np.all(n1 > 0.5 * n0)


def test_sphere18_complex_scaled_sampled_orbitals(sphere18):
    """The complex-scaling workload at full size: the 16 wells continued to
    r e^{i theta} (theta = 0.3, no projectors), 64 orbitals in one launch;
    H_theta psi and one step on sampled orbitals against the oracle."""
    s = sphere18
    R = rsg()
    cfg = synth.WORKLOADS["sphere18_cs"]
    th = cfg["theta"]
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], ball=cfg["well_ball"])
    vz = synth.well_potential_scaled(s["og"].positions(), wells, th)
    oh = oracle.Ham(s["og"], V=vz.real.copy(), V_im=vz.imag.copy(), kin=-0.5, theta=th)
    vre, vim = np.zeros(s["gg"].np), np.zeros(s["gg"].np)
    vre[s["live"]], vim[s["live"]] = vz.real, vz.imag
    gh = R.Hamiltonian(s["gg"], V=torch.from_numpy(vre).cuda(), kin=-0.5)
    gh.set_complex_scaling(th, torch.from_numpy(vim).cuda())
    psi = torch.from_numpy(s["psi_om"]).cuda()
    sub = np.ascontiguousarray(s["psi"][:, SAMPLE])
    got, dead = _sample(R.hpsi(gh, psi), s)
    assert orbital_rel_err(got, oracle.hpsi(oh, sub), len(SAMPLE)) <= 1e-12
    assert dead == 0.0
    R.propagate_step(gh, psi, 0.005)
    got, dead = _sample(psi, s)
    assert orbital_rel_err(got, oracle.taylor_step(oh, sub, 0.005), len(SAMPLE)) <= 1e-12
    assert dead == 0.0


def test_sphere18_reductions_sampled_orbitals(sphere18):
    """The reductions at full size, where every orbital's sum is split over
    the capped number of partial-sum workgroups: <a|b>, |a|^2, the energy
    and the dipole moment of all 64 orbitals in one call, against the
    oracle's serial sums on the sampled orbitals.  Sums with cancellation
    (the overlap of independent white-noise orbitals, the dipole moment of
    one) are held to 1e-12 of the sum of the magnitudes of their terms, the
    others to 1e-12 relative."""
    s = sphere18
    R = rsg()
    psi = torch.from_numpy(s["psi_om"]).cuda()
    phi_h = synth.white_noise(s["cfg"]["seed"] + 7, s["og"].np, s["cfg"]["nst"], s["cfg"]["h"])
    phi = torch.zeros_like(psi)
    phi[:, torch.from_numpy(s["live"]).cuda()] = torch.from_numpy(phi_h).cuda().t()
    sub = np.ascontiguousarray(s["psi"][:, SAMPLE])
    subp = np.ascontiguousarray(phi_h[:, SAMPLE])
    h3 = s["cfg"]["h"] ** 3
    d = R.dot(s["gg"], phi, psi).cpu().numpy()[SAMPLE]
    mag = h3 * np.sum(np.abs(subp) * np.abs(sub), axis=0)
    assert np.all(np.abs(d - oracle.dot(s["og"], subp, sub)) <= 1e-12 * mag)
    n2 = R.norm2(s["gg"], psi).cpu().numpy()[SAMPLE]
    np.testing.assert_allclose(n2, oracle.norm2(s["og"], sub), rtol=1e-12, atol=0)
    e = R.energy(s["gh"], psi).cpu().numpy()[SAMPLE]
    _, e_ref = oracle.energy(s["oh"], sub)
    np.testing.assert_allclose(e.real, e_ref.real, rtol=1e-12, atol=0)
    assert np.abs(e.imag - e_ref.imag).max() <= 1e-12 * np.abs(e_ref.real).max()
    # the dipole expectation along z, with a handle that has a dipole axis
    gz = R.Hamiltonian(s["gg"], V=torch.from_numpy(s["Vs"]).cuda(), kin=-0.5, dipole_axis=2)
    dz = R.dipole_expectation(gz, psi).cpu().numpy()[SAMPLE]
    oz = oracle.Ham(s["og"], V=s["V"], kin=-0.5, dipole_axis=2)
    ref = np.array([oracle.dipole_target(oz, sub[:, [k]]) for k in range(len(SAMPLE))])
    zabs = np.abs(s["og"].positions()[:, 2])
    mag = h3 * np.sum(zabs[:, None] * np.abs(sub) ** 2, axis=0)
    assert np.all(np.abs(dz - ref) <= 1e-12 * mag), (dz, ref, mag)
