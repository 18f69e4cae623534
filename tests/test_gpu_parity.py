"""GPU parity: every C-ABI entry point against the FP64 oracle on the same
seeded inputs.  FP64 results must agree to 1e-12 relative per orbital
(||gpu_n - oracle_n||_2 / ||oracle_n||_2, max over orbitals).  GPU batches
are orbital-major; several cases pad every orbital beyond np points and
check the padding is never written."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("kind,h,size", [("cube", 0.3, 32), ("cube", 0.4, 5), ("cube", 0.3, 1),
                                         ("sphere", 0.25, 4.0), ("sphere", 0.2, 18.0),
                                         ("sphere", 0.3, 0.2), ("sphere", 0.3, 3.33)])
def test_grid_matches_oracle(kind, h, size):
    R = rsg()
    if kind == "cube":
        g, o = R.Grid(h, n=size), oracle.Grid(h, n=size)
    else:
        g, o = R.Grid(h, R=size), oracle.Grid(h, R=size)
    assert g.np == o.np and g.dims == tuple(o.dims)
    np.testing.assert_array_equal(g.coords(), o.ijk)
    np.testing.assert_array_equal(g.positions(), o.positions())


def test_hpsi_cube32_harmonic_ten_calls():
    """32^3 cube, V = r^2/2, 4 white-noise orbitals: 10 hpsi calls on the
    same input, parity on every output."""
    s = System(0.3, n=32, potential="harmonic", nst=4, seed=1)
    ref = oracle.hpsi(s.oh, s.psi)
    psi = s.to_gpu(s.psi)
    for _ in range(10):
        out = s.from_gpu(rsg().hpsi(s.gh, psi))
        assert orbital_rel_err(out, ref, 4) <= TOL


@pytest.mark.parametrize("nst,ld", [(1, 1), (3, 4), (5, 8), (8, 8), (13, 16), (33, 40)])
def test_hpsi_sphere_projectors_dipole(nst, ld):
    """Sphere with wells, overlapping projector supports and a dipole field;
    ragged orbital counts with spare orbitals and padding points that must
    stay untouched."""
    s = System(0.3, R=4.1, potential="wells", natoms=5, nst=nst, ld=ld, seed=7, dipole_axis=2,
               well_ball=1.5, pad=ld % 5)
    ref = oracle.hpsi(s.oh, s.psi, field=0.23, nst=nst)
    psi = s.to_gpu(s.psi)
    out = torch.full_like(psi, 3.0 + 1.0j)
    rsg().hpsi(s.gh, psi, field=0.23, out=out, nst=nst)
    got = s.from_gpu(out)
    assert orbital_rel_err(got, ref, nst) <= TOL
    assert np.all(got[:, nst:] == 3.0 + 1.0j)
    assert np.all(out[:, s.og.np:].cpu().numpy() == 3.0 + 1.0j)
    assert s.pad_untouched(psi)


@pytest.mark.parametrize("axis", [0, 1])
def test_hpsi_dipole_axes(axis):
    s = System(0.35, R=3.0, potential="harmonic", nst=2, seed=3, dipole_axis=axis)
    ref = oracle.hpsi(s.oh, s.psi, field=-0.7)
    got = s.from_gpu(rsg().hpsi(s.gh, s.to_gpu(s.psi), field=-0.7))
    assert orbital_rel_err(got, ref, 2) <= TOL


def test_hpsi_tiny_boxes():
    """Boxes smaller than the stencil reach: a 1-point sphere, a 3^3 cube."""
    for kw in (dict(R=0.2), dict(n=3), dict(n=2)):
        s = System(0.3, potential="harmonic", nst=2, seed=5, **kw)
        ref = oracle.hpsi(s.oh, s.psi)
        got = s.from_gpu(rsg().hpsi(s.gh, s.to_gpu(s.psi)))
        assert orbital_rel_err(got, ref, 2) <= TOL


def test_taylor_steps_cube32():
    """10 Taylor(4) steps at dt = 0.01 on the 32^3 harmonic system."""
    s = System(0.3, n=32, potential="harmonic", nst=4, seed=1)
    ref = oracle.propagate(s.oh, s.psi, 0.01, 10)
    psi = s.to_gpu(s.psi)
    for _ in range(10):
        rsg().propagate_step(s.gh, psi, 0.01)
    assert orbital_rel_err(s.from_gpu(psi), ref, 4) <= TOL


def test_taylor_steps_at_the_stability_edge():
    """Steps with dt |lambda| up to 2.79, just inside the Taylor(4)
    stability limit 2 sqrt 2 (white noise holds the Nyquist modes: kinetic
    108.4 at h = 0.3 plus V <= 7.6 on the 16^3 cube, dt = 0.024): the
    product-form stages, whose factors reach their largest moduli there,
    still equal the oracle's power series, for the plain step, the masked
    step and in FP32 (mixed) to its own bar."""
    s = System(0.3, n=16, potential="harmonic", nst=3, seed=17)
    dt = 0.024
    ref = oracle.propagate(s.oh, s.psi, dt, 3)
    psi = s.to_gpu(s.psi)
    for _ in range(3):
        rsg().propagate_step(s.gh, psi, dt)
    assert orbital_rel_err(s.from_gpu(psi), ref, 3) <= TOL
    mixed = s.to_gpu(s.psi)
    for _ in range(3):
        rsg().propagate_step(s.gh, mixed, dt, dtype="mixed")
    assert orbital_rel_err(s.from_gpu(mixed), ref, 3) <= 1e-5
    # a mask of ones leaves the step unchanged, through the masked step form
    s.gh.set_mask(torch.ones(s.og.np, dtype=torch.float64, device="cuda"))
    try:
        x = s.to_gpu(s.psi)
        for _ in range(3):
            rsg().propagate_step(s.gh, x, dt)
        assert orbital_rel_err(s.from_gpu(x), ref, 3) <= TOL
    finally:
        s.gh.set_mask(None)


def test_cube32_sequence_autotuned_in_graph():
    """The 32^3 harmonic system as the benchmark runs it: the autotuner's
    tile, 10 hpsi calls and 10 Taylor(4) steps captured in one graph.  Two
    replays, with eager checks between them: each replay's last hpsi output
    and its final orbitals match the oracle (10 and 20 steps)."""
    s = System(0.3, n=32, potential="harmonic", nst=4, seed=1)
    R = rsg()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        psi = s.to_gpu(s.psi)
        hp = torch.zeros_like(psi)
        ws = torch.empty(s.gh.workspace_bytes("step", 4, psi.shape[1]), dtype=torch.uint8, device="cuda")
        R.autotune(s.gh, psi, reps=1)

        def seq():
            for _ in range(10):
                R.hpsi(s.gh, psi, out=hp)
            for _ in range(10):
                R.propagate_step(s.gh, psi, 0.01, ws=ws)

        # plans exist before capture; the warm-up run is undone
        seq()
        psi.copy_(s.to_gpu(s.psi))
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            seq()
    start = s.psi
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert orbital_rel_err(s.from_gpu(hp), oracle.hpsi(s.oh, start), 4) <= TOL, rep
        start = oracle.propagate(s.oh, start, 0.01, 10)
        assert orbital_rel_err(s.from_gpu(psi), start, 4) <= TOL, rep


def test_propagate_fields_sphere_projectors():
    """Steps with a per-step field array, projectors, spare orbitals and
    padding points."""
    s = System(0.3, R=4.0, potential="wells", natoms=4, nst=6, ld=8, seed=9, dipole_axis=1,
               well_ball=1.2, pad=37)
    fields = np.linspace(-0.3, 0.4, 6)
    ref = oracle.propagate(s.oh, s.psi, 0.005, 6, fields=fields, nst=6)
    psi = s.to_gpu(s.psi)
    rsg().propagate(s.gh, psi, 0.005, 6, fields=torch.from_numpy(fields).cuda(), nst=6)
    got = s.from_gpu(psi)
    assert orbital_rel_err(got, ref, 6) <= TOL
    np.testing.assert_array_equal(got[:, 6:], s.psi[:, 6:])
    assert s.pad_untouched(psi)


def test_propagate_graph_replays_match_eager():
    """A captured step sequence, replayed several times with eager work and
    synchronisations in between, matches the eager sequence every time."""
    s = System(0.3, n=24, potential="harmonic", nst=4, seed=2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = s.to_gpu(s.psi)
        graphed = s.to_gpu(s.psi)
        ws = torch.empty(s.gh.workspace_bytes("step", 4, eager.shape[1]), dtype=torch.uint8,
                         device="cuda")
        for rep in range(3):
            rsg().propagate(s.gh, eager, 0.01, 5, ws=ws)
            rsg().propagate(s.gh, graphed, 0.01, 5, graph=True, ws=ws)
            torch.cuda.synchronize()
            _ = (eager.abs() ** 2).sum().item()  # eager library work between replays
            np.testing.assert_array_equal(graphed.cpu().numpy(), eager.cpu().numpy())
    ref = oracle.propagate(s.oh, s.psi, 0.01, 15)
    assert orbital_rel_err(s.from_gpu(graphed), ref, 4) <= TOL


def test_reductions_and_energy():
    s = System(0.3, R=4.5, potential="wells", natoms=3, nst=5, ld=6, seed=4, dipole_axis=0,
               well_ball=1.0, pad=3)
    phi = synth.white_noise(77, s.og.np, 5, s.og.h, ld=6)
    R = rsg()
    a, b = s.to_gpu(phi), s.to_gpu(s.psi)
    d = R.dot(s.gg, a, b, nst=5).cpu().numpy()
    np.testing.assert_allclose(d, oracle.dot(s.og, phi, s.psi, nst=5), rtol=TOL, atol=TOL * np.abs(d).max())
    n2 = R.norm2(s.gg, b, nst=5).cpu().numpy()
    np.testing.assert_allclose(n2, oracle.norm2(s.og, s.psi, nst=5), rtol=TOL)
    e = R.energy(s.gh, b, field=0.1, nst=5).cpu().numpy()
    np.testing.assert_allclose(e, oracle.energy(s.oh, s.psi, field=0.1, nst=5)[1], rtol=TOL,
                               atol=TOL * np.abs(e).max())
    x = R.dipole_expectation(s.gh, b, nst=5).cpu().numpy()
    ref = np.array([s.og.h ** 3 * np.sum(s.pos[:, 0] * np.abs(s.psi[:, k]) ** 2) for k in range(5)])
    np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-13)


def test_reductions_deterministic():
    s = System(0.2, R=6.0, potential="harmonic", nst=16, seed=6)
    R = rsg()
    b = s.to_gpu(s.psi)
    d1 = R.dot(s.gg, b, b).cpu().numpy()
    d2 = R.dot(s.gg, b, b).cpu().numpy()
    np.testing.assert_array_equal(d1, d2)
    h1 = R.hpsi(s.gh, b).cpu().numpy()
    h2 = R.hpsi(s.gh, b).cpu().numpy()
    np.testing.assert_array_equal(h1, h2)


def test_adjoint_step_matches_oracle():
    s = System(0.3, R=3.6, potential="wells", natoms=3, nst=3, ld=4, seed=12, dipole_axis=2,
               well_ball=1.0, pad=2)
    lam0 = synth.white_noise(31, s.og.np, 3, s.og.h, ld=4)
    lam_ref, g_ref = oracle.adjoint_step(s.oh, s.psi, lam0, 0.02, 0.15, nst=3)
    lam = s.to_gpu(lam0)
    g = rsg().adjoint_step(s.gh, s.to_gpu(s.psi), lam, 0.02, 0.15, nst=3).item()
    assert orbital_rel_err(s.from_gpu(lam), lam_ref, 3) <= TOL
    assert g == pytest.approx(g_ref, rel=1e-11, abs=1e-14)


def test_control_gradient_matches_oracle():
    """Checkpointed discrete adjoint (ragged last segment) against the
    oracle's store-everything adjoint."""
    s = System(0.4, n=14, potential="wells", natoms=0, nst=2, seed=5, dipole_axis=2,
               well_box=1.5, orbitals="packets", packet_box=1.0)
    coef = synth.laser_coefficients(5, 6, sigma=0.3)
    dt, nsteps, ck = 0.05, 23, 5
    J_ref, g_ref, gs_ref = oracle.control_gradient(s.oh, s.psi, dt, nsteps, coef)
    R = rsg()
    psi = s.to_gpu(s.psi)
    c = torch.from_numpy(coef).cuda()
    J, store = R.control_forward(s.gh, psi, dt, nsteps, c, ck)
    grad, gs = R.control_backward(s.gh, psi, dt, nsteps, c, ck, store)
    assert J.item() == pytest.approx(J_ref, rel=1e-12)
    np.testing.assert_allclose(gs.cpu().numpy(), gs_ref, rtol=1e-10, atol=1e-12 * np.abs(gs_ref).max())
    np.testing.assert_allclose(grad.cpu().numpy(), g_ref, rtol=1e-10, atol=1e-12 * np.abs(g_ref).max())


def test_control_gradient_minimum_workspace():
    """With the minimum workspace the backward pass recomputes each step's
    stage outputs instead of keeping them: the same kernels on the same
    inputs, so the gradient is bit for bit the full-workspace one (and the
    oracle's to 1e-10)."""
    s = System(0.4, n=14, potential="wells", natoms=0, nst=2, seed=5, dipole_axis=2,
               well_box=1.5, orbitals="packets", packet_box=1.0)
    coef = synth.laser_coefficients(5, 6, sigma=0.3)
    dt, nsteps, ck = 0.05, 23, 5
    _, g_ref, gs_ref = oracle.control_gradient(s.oh, s.psi, dt, nsteps, coef)
    R = rsg()
    c = torch.from_numpy(coef).cuda()
    out = {}
    for mode in ("full", "min"):
        psi = s.to_gpu(s.psi)
        J, store = R.control_forward(s.gh, psi, dt, nsteps, c, ck, workspace=mode)
        out[mode] = R.control_backward(s.gh, psi, dt, nsteps, c, ck, store, workspace=mode)
    np.testing.assert_array_equal(out["min"][0].cpu().numpy(), out["full"][0].cpu().numpy())
    np.testing.assert_array_equal(out["min"][1].cpu().numpy(), out["full"][1].cpu().numpy())
    np.testing.assert_allclose(out["min"][0].cpu().numpy(), g_ref, rtol=1e-10, atol=1e-12 * np.abs(g_ref).max())
    assert R._lib.rsg_control_workspace_bytes_min(s.gh._h, 2, s.gg.np, nsteps, ck) < \
        R._lib.rsg_control_workspace_bytes(s.gh._h, 2, s.gg.np, nsteps, ck)


def test_optimal_control_autograd_matches_central_differences():
    s = System(0.4, n=14, potential="wells", natoms=0, nst=2, seed=8, dipole_axis=2,
               well_box=1.5, orbitals="packets", packet_box=1.0)
    R = rsg()
    dt, nsteps, ck = 0.05, 20, 4
    coef = torch.from_numpy(synth.laser_coefficients(8, 5, sigma=0.3)).cuda().requires_grad_(True)
    psi0 = s.to_gpu(s.psi)
    J = R.OptimalControlJ.apply(coef, s.gh, psi0, dt, nsteps, ck)
    J.backward()
    grad = coef.grad.cpu().numpy()
    eps = 1e-4
    fd = np.zeros_like(grad)
    for k in range(grad.size):
        e = torch.zeros_like(coef)
        e[k] = eps
        jp = R.OptimalControlJ.apply((coef + e).detach(), s.gh, psi0, dt, nsteps, ck).item()
        jm = R.OptimalControlJ.apply((coef - e).detach(), s.gh, psi0, dt, nsteps, ck).item()
        fd[k] = (jp - jm) / (2 * eps)
    assert np.abs(fd - grad).max() <= 1e-6 * np.abs(grad).max()


def test_mixed_precision_step_error():
    """FP32 Hamiltonian / FP64 accumulation: error vs the FP64 oracle stays
    at the FP32 rounding level after 10 steps."""
    s = System(0.3, n=32, potential="harmonic", nst=4, seed=4)
    ref = oracle.propagate(s.oh, s.psi, 0.01, 10)
    psi = s.to_gpu(s.psi)
    for _ in range(10):
        rsg().propagate_step(s.gh, psi, 0.01, dtype="mixed")
    err = orbital_rel_err(s.from_gpu(psi), ref, 4)
    assert err < 1e-5, err
    assert err > 1e-13  # really ran in FP32


def test_mixed_precision_thousand_steps_vs_oracle():
    """The mixed-precision workload as specified: the 32^3 harmonic system,
    1000 Taylor(4) steps at dt = 0.01 with the FP32 Hamiltonian, against
    the FP64 oracle's 1000 steps.  White-noise orbitals and smooth low
    oscillator states: orbital error, norm and energy stay at the FP32
    rounding level accumulated over 1000 steps (the benchmark reports
    4.7e-6 orbital error against the FP64 GPU path).

    The norm bound comes from the rounding, not from one observed run.  An
    FP32 H application sums terms of total size about
    (|kin|/h^2 sum|c| + max V) |psi| = (0.5/0.09 * 19.5 + 35) |psi| ~ 140 |psi|,
    so its error per point is about sqrt(25) u32 140 |psi| ~ 4e-5 |psi|
    (u32 = 6e-8), and a step adds dt times that to psi.  The norm moves by
    2 Re<psi|e>; with rounding signs independent over the few thousand
    points where the states live that is ~1e-8 per step, ~3e-7 as a random
    walk over 1000 steps (and 1e-5 if every step added with one sign).  Two
    builds that differ only in where the compiler fused a multiply-add gave
    0.9e-7 and 1.6e-7; the bound is 1e-6."""
    s = System(0.3, n=32, potential="harmonic", nst=4, seed=4)
    h3 = s.og.h ** 3
    for name, psi0 in (("white", s.psi), ("ho", synth.ho_low_states(s.og.positions(), 4))):
        ref = oracle.propagate(s.oh, psi0, 0.01, 1000)
        psi = s.to_gpu(psi0)
        rsg().propagate(s.gh, psi, 0.01, 1000, dtype="mixed")
        got = s.from_gpu(psi)
        err = orbital_rel_err(got, ref, 4)
        assert 1e-12 < err < 2e-5, (name, err)
        n_got = h3 * np.sum(np.abs(got) ** 2, axis=0)
        n_ref = h3 * np.sum(np.abs(ref) ** 2, axis=0)
        assert np.abs(n_got - n_ref).max() < 1e-6, name
        e_got = h3 * np.sum(np.conj(got) * oracle.hpsi(s.oh, got), axis=0).real
        e_ref = h3 * np.sum(np.conj(ref) * oracle.hpsi(s.oh, ref), axis=0).real
        assert np.abs(e_got - e_ref).max() < 1e-6 * np.abs(e_ref).max(), name


def test_mixed_precision_projectors():
    s = System(0.3, R=4.0, potential="wells", natoms=4, nst=5, ld=8, seed=10, well_ball=1.2, pad=9)
    ref = oracle.propagate(s.oh, s.psi, 0.005, 3, nst=5)
    psi = s.to_gpu(s.psi)
    rsg().propagate(s.gh, psi, 0.005, 3, dtype="mixed", nst=5)
    got = s.from_gpu(psi)
    assert orbital_rel_err(got, ref, 5) < 1e-5
    np.testing.assert_array_equal(got[:, 5:], s.psi[:, 5:])
    assert s.pad_untouched(psi)


def test_error_codes():
    import ctypes as C
    R = rsg()
    s = System(0.3, n=8, potential="harmonic", nst=2, seed=1)
    psi = s.to_gpu(s.psi)
    with pytest.raises(ValueError):
        R.hpsi(s.gh, psi, nst=3)  # more orbitals than the tensor holds
    with pytest.raises(R.RSGError) as ei:
        R.adjoint_step(s.gh, psi, psi.clone(), 0.01, 0.0)  # no dipole axis
    assert ei.value.code == -1
    p = C.c_void_p(psi.data_ptr())
    ldp = psi.shape[1]
    out = torch.zeros_like(psi)
    # stride shorter than the grid
    rc = R._lib.rsg_hpsi(s.gh._h, p, C.c_void_p(out.data_ptr()), 2, s.og.np - 1, 0, 0.0, None, 0, None)
    assert rc == -2
    # the C call rejects a too-small workspace before enqueuing anything
    rc = R._lib.rsg_propagate_step(s.gh._h, p, 2, ldp, 0, 0.01, 0.0, p, 16, None)
    assert rc == -5
    rc = R._lib.rsg_hpsi(s.gh._h, p, p, 2, ldp, 0, 0.0, None, 0, None)
    assert rc == -1  # psi and hpsi overlap


def test_mask_absorber_matches_oracle():
    """psi <- M U(dt) psi after every step (mask boundary absorber): FP64 parity
    with projectors, a per-step field, spare orbitals and padding points;
    graph replay equal to eager; the FP32 path within its rounding; removing
    the mask restores the plain step; the adjoint rejects a masked H."""
    R = rsg()
    s = System(0.3, R=4.0, potential="wells", natoms=4, nst=5, ld=6, seed=21, dipole_axis=2,
               well_ball=1.2, pad=7)
    M = synth.radial_mask(s.pos, 3.6, 1.4)
    assert np.any(M == 0.0) and np.any((M > 0) & (M < 1))
    fields = np.linspace(0.2, -0.1, 4)
    ref, removed = oracle.propagate_masked(s.oh, s.psi, 0.005, 4, M, fields=fields, nst=5)
    s.gh.set_mask(torch.from_numpy(M).cuda())
    f = torch.from_numpy(fields).cuda()
    psi = s.to_gpu(s.psi)
    n0 = R.norm2(s.gg, psi, nst=5).cpu().numpy()
    R.propagate(s.gh, psi, 0.005, 4, fields=f, nst=5)
    got = s.from_gpu(psi)
    assert orbital_rel_err(got, ref, 5) <= TOL
    np.testing.assert_array_equal(got[:, 5:], s.psi[:, 5:])
    assert s.pad_untouched(psi)
    assert np.all(got[M == 0.0, :5] == 0)
    n1 = R.norm2(s.gg, psi, nst=5).cpu().numpy()
    np.testing.assert_allclose(n0 - n1, oracle.norm2(s.og, s.psi, nst=5) - oracle.norm2(s.og, ref, nst=5),
                               rtol=1e-10)
    assert np.all(removed > 0)
    # graph capture of the masked steps
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = s.to_gpu(s.psi)
        for _ in range(2):
            g.copy_(s.to_gpu(s.psi))
            R.propagate(s.gh, g, 0.005, 4, fields=f, nst=5, graph=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(g.cpu().numpy(), psi.cpu().numpy())
    # mixed precision with the mask
    m = s.to_gpu(s.psi)
    R.propagate(s.gh, m, 0.005, 4, fields=f, nst=5, dtype="mixed")
    assert orbital_rel_err(s.from_gpu(m), ref, 5) < 1e-5
    with pytest.raises(R.RSGError) as ei:
        R.adjoint_step(s.gh, psi, psi.clone(), 0.01, 0.0, nst=5)
    assert ei.value.code == -6
    # removing the mask restores the plain step
    s.gh.set_mask(None)
    p = s.to_gpu(s.psi)
    R.propagate_step(s.gh, p, 0.005, field=0.2, nst=5)
    plain = oracle.taylor_step(s.oh, s.psi, 0.005, field=0.2, nst=5)
    assert orbital_rel_err(s.from_gpu(p), plain, 5) <= TOL
