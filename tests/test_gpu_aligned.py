"""Row-aligned grids (rsg_grid_create_aligned): the points keep their order,
every non-empty row's slots are its x-range widened to multiples of the
alignment, and the extra slots hold no point.

- Layout: the live slots carry the oracle's points in the oracle's order,
  every row starts at a multiple of the alignment, dead slots read
  coordinates -1 and position 0, for spheres and cubes and several
  alignments.
- H psi and a Taylor(4) step (wells, projectors, dipole field, spare
  orbitals, padding points) equal the oracle on the live slots to the FP64
  bar for every compiled tile, z-chunk and block order; every stencil output
  holds exact zeros in the dead slots even when the output buffer held
  other values; spare orbitals and padding stay untouched.
- The mixed path (alignments 8 and 16), the batched path (bit for bit
  against single systems), complex scaling, the reductions and the energy,
  the adjoint step and control gradient, and the QMR / CG shifted solves
  work on aligned grids.
- A bad alignment and a grid-to-memory map on an aligned grid are
  rejected; boxes smaller than the stencil reach work with mostly dead
  rows."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("shape,size,align", [("sphere", 3.1, 8), ("sphere", 4.4, 4), ("sphere", 2.0, 16),
                                              ("cube", 13, 8), ("cube", 16, 8), ("sphere", 0.2, 8)])
def test_aligned_layout(shape, size, align):
    R = rsg()
    h = 0.3
    kw = dict(R=size) if shape == "sphere" else dict(n=size)
    og = oracle.Grid(h, **kw)
    gg = R.Grid(h, align=align, **kw)
    assert gg.align == align and gg.npoints == og.np and gg.np >= og.np
    assert gg.np % align == 0
    ijk = gg.coords()
    live = gg.live()
    np.testing.assert_array_equal(ijk[live], og.ijk)
    dead = np.setdiff1d(np.arange(gg.np), live)
    assert np.all(ijk[dead] == -1)
    pos = gg.positions()
    np.testing.assert_array_equal(pos[live], og.positions())
    assert np.all(pos[dead] == 0)
    # the slot of x = 0 of every row is a multiple of the alignment
    assert np.all((live - ijk[live, 0]) % align == 0)
    # each row's slots are its x-range widened to multiples of align
    rows = {}
    for p, (x, y, z) in zip(live, ijk[live]):
        rows.setdefault((y, z), []).append((x, p))
    total = 0
    for v in rows.values():
        x0, x1 = v[0][0], v[-1][0] + 1
        total += ((x1 + align - 1) // align - x0 // align) * align
    assert total == gg.np


@pytest.fixture(scope="module")
def asys():
    return System(0.3, R=3.1, potential="wells", natoms=2, nst=13, ld=16, seed=71, dipole_axis=2,
                  rcut=1.2, pad=5, align=8)


def test_aligned_every_tile_matches_oracle(asys):
    R = rsg()
    s = asys
    assert s.gg.np > s.og.np  # there are dead slots
    field, dt = 0.07, 0.01
    ref_h = oracle.hpsi(s.oh, s.psi, field=field, nst=s.nst)
    ref_s = oracle.taylor_step(s.oh, s.psi, dt, field=field, nst=s.nst)
    psi = s.to_gpu(s.psi)
    n = 0
    for t in R.tile_candidates("c128"):
        for zc in (0, 4, 1):
            for bo in (0, 1):
                R.set_tile(s.gh, s.nst, t["B"], t["TX"], t["TY"], zc, t["PD"], 0, bo, 0)
                out = torch.full_like(psi, 3.0 + 1.0j)
                R.hpsi(s.gh, psi, field=field, out=out, nst=s.nst)
                y = s.from_gpu(out)
                assert orbital_rel_err(y, ref_h, s.nst) <= TOL, (t, zc, bo)
                d = s.dead_values(out)
                assert np.all(d[:s.nst] == 0), (t, zc, bo)
                assert np.all(d[s.nst:] == 3.0 + 1.0j) and np.all(y[:, s.nst:] == 3.0 + 1.0j)
                x = psi.clone()
                R.propagate_step(s.gh, x, dt, field=field, nst=s.nst)
                xs = s.from_gpu(x)
                assert orbital_rel_err(xs, ref_s, s.nst) <= TOL, (t, zc, bo)
                assert np.all(s.dead_values(x) == 0)
                np.testing.assert_array_equal(xs[:, s.nst:], s.psi[:, s.nst:])
                assert s.pad_untouched(x)
                n += 1
    assert n >= 60


def test_aligned_step_clears_dead_slots(asys):
    """Nonzero values left in dead slots of psi are never read: the live
    result is unchanged and the step leaves zeros there."""
    R = rsg()
    s = asys
    R.set_tile(s.gh, s.nst, 1, 32, 16, 0, 1, 0, 1, 0)
    ref_s = oracle.taylor_step(s.oh, s.psi, 0.01, nst=s.nst)
    x = s.to_gpu(s.psi)
    mask = torch.ones(s.gg.np, dtype=torch.bool, device="cuda")
    mask[torch.from_numpy(s.live).cuda()] = False
    x[:, :s.gg.np][:, mask] = 5.0 - 2.0j
    R.propagate_step(s.gh, x, 0.01, nst=s.nst)
    assert orbital_rel_err(s.from_gpu(x), ref_s, s.nst) <= TOL
    d = s.dead_values(x)
    assert np.all(d[:s.nst] == 0) and np.all(d[s.nst:] == 5.0 - 2.0j)


def test_aligned_reductions_energy_and_mixed(asys):
    R = rsg()
    s = asys
    R.set_tile(s.gh, s.nst, 1, 32, 16, 0, 1, 0, 1, 0)
    psi = s.to_gpu(s.psi)
    h3 = s.og.h ** 3
    n2 = R.norm2(s.gg, psi, nst=s.nst).cpu().numpy()
    ref = h3 * np.sum(np.abs(s.psi[:, :s.nst]) ** 2, axis=0)
    np.testing.assert_allclose(n2, ref, rtol=1e-13)
    e = R.energy(s.gh, psi, field=0.07, nst=s.nst).cpu().numpy()
    hp = oracle.hpsi(s.oh, s.psi, field=0.07, nst=s.nst)
    e_ref = h3 * np.sum(np.conj(s.psi[:, :s.nst]) * hp[:, :s.nst], axis=0)
    np.testing.assert_allclose(e, e_ref, rtol=0, atol=1e-12 * np.abs(e_ref).max())
    # mixed path: FP32 H on complex64 work buffers, against the FP64 step
    x64, x32 = psi.clone(), psi.clone()
    R.propagate_step(s.gh, x64, 0.01, nst=s.nst)
    R.propagate_step(s.gh, x32, 0.01, dtype="mixed", nst=s.nst)
    assert orbital_rel_err(s.from_gpu(x32), s.from_gpu(x64), s.nst) <= 1e-5
    assert np.all(s.dead_values(x32)[:s.nst] == 0)


def test_aligned_batch_matches_single_systems():
    """Two aligned systems (different radii and orbital counts) and one
    compact one in a batch: every system's steps equal its single-system
    steps bit for bit."""
    R = rsg()
    systems = [System(0.3, R=3.4, potential="wells", natoms=2, nst=5, seed=81, rcut=1.2, align=8),
               System(0.3, R=2.6, potential="wells", natoms=1, nst=3, ld=4, seed=82, rcut=1.2, align=8),
               System(0.3, R=2.9, potential="wells", natoms=1, nst=2, seed=83, rcut=1.2)]
    tile = (1, 16, 8, 0, 1, 0, 1, 0)
    singles, batched = [], []
    for s in systems:
        R.set_tile(s.gh, s.nst, *tile)
        x = s.to_gpu(s.psi)
        for _ in range(2):
            R.propagate_step(s.gh, x, 0.01, nst=s.nst)
        singles.append(x)
        batched.append(s.to_gpu(s.psi))
    b = R.Batch([(s.gh, x, s.nst) for s, x in zip(systems, batched)])
    b.set_tile(1, 16, 8, 0, 1)
    b.propagate(0.01, 2)
    torch.cuda.synchronize()
    for s, x, y in zip(systems, singles, batched):
        np.testing.assert_array_equal(y.cpu().numpy(), x.cpu().numpy())
        assert np.all(s.dead_values(y)[:s.nst] == 0)


def test_aligned_complex_scaling():
    R = rsg()
    s = System(0.3, R=3.1, potential="wells", natoms=0, nst=5, ld=6, seed=51, dipole_axis=2, pad=4,
               well_ball=1.2, align=8)
    rng = np.random.default_rng(52)
    vim = -0.3 * rng.random(s.og.np)
    oh = oracle.Ham(s.og, V=s.V, kin=-0.5, dipole_axis=2, theta=0.3, V_im=vim)
    s.gh.set_complex_scaling(0.3, torch.from_numpy(s.slots(vim)).cuda())
    psi = s.to_gpu(s.psi)
    out = torch.full_like(psi, 1.0 + 1.0j)
    R.hpsi(s.gh, psi, field=0.05, out=out, nst=s.nst)
    assert orbital_rel_err(s.from_gpu(out), oracle.hpsi(oh, s.psi, field=0.05, nst=s.nst), s.nst) <= TOL
    assert np.all(s.dead_values(out)[:s.nst] == 0)


def test_aligned_rejections():
    R = rsg()
    for bad in (0, 3, 128):
        with pytest.raises(R.RSGError) as ei:
            R.Grid(0.3, R=2.0, align=bad)
        assert ei.value.code == -1
    with pytest.raises(R.RSGError) as ei:
        R.GridMap(R.Grid(0.3, R=2.0, align=8), R.MAP_STANDARD)
    assert ei.value.code == -6


def test_align16_fp64_and_mixed_steps():
    """Alignment 16 (the mixed benchmark's storage: 16 complex64 slots per
    128-byte line): the FP64 step equals the oracle, the mixed step agrees
    with it to FP32 rounding, and both leave zeros in the dead slots."""
    R = rsg()
    s = System(0.3, R=3.6, potential="wells", natoms=3, nst=6, ld=8, seed=91, rcut=1.2, pad=3, align=16)
    assert s.gg.np % 16 == 0 and s.gg.np > s.og.np
    ref = oracle.taylor_step(s.oh, s.psi, 0.01, nst=s.nst)
    for tile in [(1, 32, 16, 0, 1, 0, 1, 0), (1, 32, 8, 4, 2, 0, 0, 1)]:
        R.set_tile(s.gh, s.nst, *tile)
        R.set_tile(s.gh, s.nst, *tile, dtype="mixed")
        x64, x32 = s.to_gpu(s.psi), s.to_gpu(s.psi)
        R.propagate_step(s.gh, x64, 0.01, nst=s.nst)
        R.propagate_step(s.gh, x32, 0.01, dtype="mixed", nst=s.nst)
        assert orbital_rel_err(s.from_gpu(x64), ref, s.nst) <= TOL, tile
        assert orbital_rel_err(s.from_gpu(x32), ref, s.nst) <= 1e-5, tile
        for x in (x64, x32):
            assert np.all(s.dead_values(x) == 0) and s.pad_untouched(x)


def test_aligned_adjoint_and_control_gradient():
    """The discrete adjoint step and the checkpointed control gradient on an
    aligned grid equal the oracle's (dipole operator and laser field act on
    the live slots only)."""
    import synth
    R = rsg()
    s = System(0.3, R=3.6, potential="wells", natoms=3, nst=3, ld=4, seed=12, dipole_axis=2,
               well_ball=1.0, pad=2, align=8)
    lam0 = synth.white_noise(31, s.og.np, 3, s.og.h, ld=4)
    lam_ref, g_ref = oracle.adjoint_step(s.oh, s.psi, lam0, 0.02, 0.15, nst=3)
    lam = s.to_gpu(lam0)
    g = R.adjoint_step(s.gh, s.to_gpu(s.psi), lam, 0.02, 0.15, nst=3).item()
    assert orbital_rel_err(s.from_gpu(lam), lam_ref, 3) <= TOL
    assert g == pytest.approx(g_ref, rel=1e-11, abs=1e-14)
    assert np.all(s.dead_values(lam)[:3] == 0)
    c = System(0.4, n=14, potential="wells", natoms=0, nst=2, seed=5, dipole_axis=2, well_box=1.5,
               orbitals="packets", packet_box=1.0, align=8)
    assert c.gg.np > c.og.np
    coef = synth.laser_coefficients(5, 6, sigma=0.3)
    dt, nsteps, ck = 0.05, 23, 5
    J_ref, gr_ref, gs_ref = oracle.control_gradient(c.oh, c.psi, dt, nsteps, coef)
    psi = c.to_gpu(c.psi)
    cc = torch.from_numpy(coef).cuda()
    J, store = R.control_forward(c.gh, psi, dt, nsteps, cc, ck)
    grad, gs = R.control_backward(c.gh, psi, dt, nsteps, cc, ck, store)
    assert J.item() == pytest.approx(J_ref, rel=1e-12)
    np.testing.assert_allclose(gs.cpu().numpy(), gs_ref, rtol=1e-10, atol=1e-12 * np.abs(gs_ref).max())
    np.testing.assert_allclose(grad.cpu().numpy(), gr_ref, rtol=1e-10, atol=1e-12 * np.abs(gr_ref).max())


@pytest.mark.parametrize("method", ["qmr", "cg"])
def test_aligned_shifted_solves(method):
    """QMR and CG on an aligned grid: the iterates after 1, 2 and 6
    iterations equal the oracle's, and a converged solve meets its residual
    with zeros left in the dead slots."""
    from oracle import shifted as sv
    R = rsg()
    s = System(0.5, R=2.9, potential="wells", natoms=2, nst=5, ld=6, seed=41, rcut=1.2, well_ball=1.0,
               pad=3, align=8)
    shifts = (np.array([0.3 + 0.1j, -0.2 + 0.05j, 1.0 + 0.5j, 0.05 + 0.02j, 2.0 - 0.3j]) if method == "qmr"
              else np.array([4.0, 5.0, 6.0, 7.0, 8.0]))
    rng = np.random.default_rng(8)
    b = np.zeros((s.og.np, s.ld), dtype=np.complex128)
    b[:, :s.nst] = rng.standard_normal((s.og.np, s.nst)) + 1j * rng.standard_normal((s.og.np, s.nst))
    for k in (1, 2, 6):
        xg, info = R.shifted_solve(s.gh, s.to_gpu(b), shifts, method=method, tol=0.0, maxiter=k, nst=s.nst)
        ref, _, _, _ = sv.solve_batch(s.oh, b, shifts, method, tol=0.0, maxiter=k, nst=s.nst)
        x = s.from_gpu(xg)
        for n in range(s.nst):
            assert np.linalg.norm(x[:, n] - ref[:, n]) <= 1e-10 * np.linalg.norm(ref[:, n]), (method, k, n)
    xg, info = R.shifted_solve(s.gh, s.to_gpu(b), shifts, method=method, tol=1e-10, maxiter=3000, nst=s.nst)
    assert np.all(info["status"] == 0)
    x = s.from_gpu(xg)
    Hx = oracle.hpsi(s.oh, x, nst=s.nst)
    for n in range(s.nst):
        r = b[:, n] - Hx[:, n] - shifts[n] * x[:, n]
        assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b[:, n]), (method, n)
    assert np.all(s.dead_values(xg)[:s.nst] == 0)


def test_aligned_tiny_boxes():
    """Boxes smaller than the stencil reach, stored row-aligned (every row
    mostly dead slots): a 1-point sphere and 2^3, 3^3 cubes; H psi and a
    step equal the oracle and leave zeros in the dead slots."""
    R = rsg()
    for kw in (dict(R=0.2), dict(n=3), dict(n=2)):
        s = System(0.3, potential="harmonic", nst=2, seed=5, align=8, **kw)
        assert s.gg.np > s.og.np
        psi = s.to_gpu(s.psi)
        out = torch.full_like(psi, 9.0)
        R.hpsi(s.gh, psi, out=out)
        assert orbital_rel_err(s.from_gpu(out), oracle.hpsi(s.oh, s.psi), 2) <= TOL, kw
        assert np.all(s.dead_values(out) == 0), kw
        R.propagate_step(s.gh, psi, 0.01)
        assert orbital_rel_err(s.from_gpu(psi), oracle.taylor_step(s.oh, s.psi, 0.01), 2) <= TOL, kw
        assert np.all(s.dead_values(psi) == 0), kw


@pytest.mark.parametrize("align,tile", [(16, (1, 8, 8, 0, 1, 0, 1, 0)), (16, (1, 8, 8, 3, 2, 1, 0, 1)),
                                        (32, (1, 16, 8, 0, 1, 0, 2, 0)), (64, (1, 32, 16, 0, 2, 0, 1, 0))])
def test_tiles_narrower_than_alignment(align, tile):
    """Tiles narrower than the row alignment: the launch plan covers each
    row's widened x-range (which may pass the box's last column), so every
    output zeroes every dead slot, and H psi, a step and an adjoint step
    still equal the oracle on the live slots."""
    import synth
    R = rsg()
    s = System(0.3, R=3.6, potential="wells", natoms=3, nst=3, ld=4, seed=17, dipole_axis=1,
               well_ball=1.0, rcut=1.2, pad=2, align=align)
    assert s.gg.np % align == 0 and s.gg.np > s.og.np
    R.set_tile(s.gh, s.nst, *tile)
    psi = s.to_gpu(s.psi)
    out = torch.full_like(psi, 4.0 - 1.0j)
    R.hpsi(s.gh, psi, field=0.05, out=out, nst=s.nst)
    assert orbital_rel_err(s.from_gpu(out), oracle.hpsi(s.oh, s.psi, field=0.05, nst=s.nst), s.nst) <= TOL
    assert np.all(s.dead_values(out)[:s.nst] == 0)
    x = psi.clone()
    R.propagate_step(s.gh, x, 0.01, field=0.05, nst=s.nst)
    assert orbital_rel_err(s.from_gpu(x), oracle.taylor_step(s.oh, s.psi, 0.01, field=0.05, nst=s.nst),
                           s.nst) <= TOL
    assert np.all(s.dead_values(x) == 0) and s.pad_untouched(x)
    lam0 = synth.white_noise(33, s.og.np, 3, s.og.h, ld=4)
    lam_ref, g_ref = oracle.adjoint_step(s.oh, s.psi, lam0, 0.02, 0.15, nst=3)
    lam = s.to_gpu(lam0)
    g = R.adjoint_step(s.gh, psi, lam, 0.02, 0.15, nst=3).item()
    assert orbital_rel_err(s.from_gpu(lam), lam_ref, 3) <= TOL
    assert g == pytest.approx(g_ref, rel=1e-11, abs=1e-14)
    assert np.all(s.dead_values(lam)[:3] == 0)


@pytest.mark.parametrize("box,align,axis", [((40, 24, 17), 1, 0), ((40, 24, 17), 8, 1), ((7, 33, 20), 8, 2),
                                            ((45, 9, 30), 16, 0)])
def test_rectangular_boxes_hpsi_step_and_adjoint(box, align, axis):
    """Rectangular boxes (every width, including ones that are not multiples
    of the tile or of the row alignment), with wells, overlapping projectors
    and a dipole field: H psi, a Taylor(4) step and an adjoint step equal the
    oracle's to 1e-12, and the dead slots of aligned rows stay zero."""
    s = System(0.3, box=box, potential="wells", natoms=3, nst=5, seed=21, dipole_axis=axis, well_box=1.5,
               align=align)
    R = rsg()
    psi = s.to_gpu(s.psi)
    ref = oracle.hpsi(s.oh, s.psi, field=0.17)
    out = R.hpsi(s.gh, psi, field=0.17)
    assert orbital_rel_err(s.from_gpu(out), ref, s.nst) <= 1e-12
    if align > 1:
        assert np.all(s.dead_values(out) == 0)
    ref = oracle.taylor_step(s.oh, s.psi, 0.01, field=0.17)
    R.propagate_step(s.gh, psi, 0.01, field=0.17)
    assert orbital_rel_err(s.from_gpu(psi), ref, s.nst) <= 1e-12
    if align > 1:
        assert np.all(s.dead_values(psi) == 0)
    lam0 = synth.white_noise(77, s.og.np, s.nst, s.og.h)
    lam_ref, g_ref = oracle.adjoint_step(s.oh, s.psi, lam0, 0.01, 0.17)
    lam = s.to_gpu(lam0)
    g = R.adjoint_step(s.gh, s.to_gpu(s.psi), lam, 0.01, 0.17).item()
    assert orbital_rel_err(s.from_gpu(lam), lam_ref, s.nst) <= 1e-12
    assert g == pytest.approx(g_ref, rel=1e-10, abs=1e-12)
    if align > 1:
        assert np.all(s.dead_values(lam) == 0)
