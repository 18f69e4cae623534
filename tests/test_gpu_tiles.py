"""Every compiled stencil tile the autotuner may pick, with every z-chunking,
tile order (row, Morton, patches), block order and z-march direction (upward,
or outward from the centre plane), gives the oracle's
H psi and Taylor(4) step to the FP64 bar; the mixed-precision tiles agree
with each other to FP32 rounding of the same arithmetic.

The grid is a small sphere with ragged rows, 13 of 16 orbitals in use and
padding points after every orbital, so partial tiles in x, y and z occur
for every shape and spare orbitals and padding must stay untouched."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import System, orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

ZCS = (0, 4, 1)     # whole z-range, chunks of 4 planes (several per tile), single planes
PTS = (0, 1, 2)     # row order, Morton order, 2 x 2 patches
BOS = (0, 1, 3)     # orbital fastest / slowest / groups of 3 (13 = 4 x 3 + 1)
ZMS = (0, 1, 2)     # upward from each tile's lowest plane / outward from the centre plane /
                    # chunks aligned in z for all tiles


@pytest.fixture(scope="module")
def sys_():
    return System(0.3, R=3.1, potential="wells", natoms=2, nst=13, ld=16, seed=71,
                  dipole_axis=2, rcut=1.2, pad=5)


def _variants(dtype):
    R = rsg()
    for t in R.tile_candidates(dtype):
        for zc in ZCS:
            for pt in PTS:
                for bo in BOS:
                    for zm in ZMS:
                        if zm >= 1 and pt >= 2:
                            continue  # patches apply to the upward march only
                        if zm == 2 and zc == 0:
                            continue  # aligned chunks need chunks
                        if zc == 1 and pt != 0:
                            continue  # single planes: row order suffices
                        yield dict(t, ZC=zc, PT=pt, BO=bo, ZM=zm)


def _set(R, s, t, dtype):
    R.set_tile(s.gh, s.nst, t["B"], t["TX"], t["TY"], t["ZC"], t["PD"], t["PT"], t["BO"],
               t["ZM"], dtype=dtype)


def test_every_fp64_tile_matches_oracle(sys_):
    R = rsg()
    s = sys_
    field, dt = 0.07, 0.01
    ref_h = oracle.hpsi(s.oh, s.psi, field=field, nst=s.nst)
    ref_s = oracle.taylor_step(s.oh, s.psi, dt, field=field, nst=s.nst)
    psi = s.to_gpu(s.psi)
    n = 0
    for t in _variants("c128"):
        _set(R, s, t, "c128")
        assert R.get_tile(s.gh, s.nst) == t
        y = s.from_gpu(R.hpsi(s.gh, psi, field=field, nst=s.nst))
        e = orbital_rel_err(y, ref_h, s.nst)
        assert e <= 1e-12, (t, e)
        assert not np.any(y[:, s.nst:]), t
        x = psi.clone()
        R.propagate_step(s.gh, x, dt, field=field, nst=s.nst)
        xs = s.from_gpu(x)
        assert s.pad_untouched(x), t
        e = orbital_rel_err(xs, ref_s, s.nst)
        assert e <= 1e-12, (t, e)
        np.testing.assert_array_equal(xs[:, s.nst:], s.psi[:, s.nst:])
        n += 1
    assert n >= 150


def test_every_mixed_tile_agrees(sys_):
    R = rsg()
    s = sys_
    dt = 0.01
    ref_s = oracle.taylor_step(s.oh, s.psi, dt, nst=s.nst)
    psi = s.to_gpu(s.psi)
    first = None
    for t in _variants("mixed"):
        _set(R, s, t, "mixed")
        x = psi.clone()
        R.propagate_step(s.gh, x, dt, dtype="mixed", nst=s.nst)
        xs = s.from_gpu(x)
        # FP32 Hamiltonian: error of FP32 rounding of a step of size dt |H|
        assert orbital_rel_err(xs, ref_s, s.nst) <= 2e-6, t
        if first is None:
            first = xs
        else:
            # each point's arithmetic does not depend on the tile
            np.testing.assert_allclose(xs, first, rtol=0, atol=1e-6 * np.abs(first).max())


def test_autotune_cache_second_handle_launches_nothing(tmp_path):
    """rsg_autotune_cache: the first handle times the candidates and appends
    its choice to the cache file; a second handle on a grid of the same shape
    finds the key and takes the same tile without launching a stencil, and
    its step still equals the oracle.  A different orbital count is a
    different key and is timed again."""
    R = rsg()
    path = str(tmp_path / "tiles.txt")
    a = System(0.3, R=2.8, potential="wells", natoms=1, nst=3, seed=21, rcut=1.2)
    psi = a.to_gpu(a.psi)
    with R.kernel_timing() as k1:
        t1, ms1, hit1 = R.autotune_cached(a.gh, psi, path, reps=1)
    assert not hit1 and k1.count > 0 and ms1 > 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "nst=3" in lines[0]
    b = System(0.3, R=2.8, potential="wells", natoms=1, nst=3, seed=22, rcut=1.2)
    psib = b.to_gpu(b.psi)
    with R.kernel_timing() as k2:
        t2, ms2, hit2 = R.autotune_cached(b.gh, psib, path, reps=1)
    assert hit2 and k2.count == 0 and t2 == t1 and ms2 == pytest.approx(ms1, rel=1e-6)
    assert R.get_tile(b.gh, 3) == t1
    R.propagate_step(b.gh, psib, 0.01)
    assert orbital_rel_err(b.from_gpu(psib), oracle.taylor_step(b.oh, b.psi, 0.01), 3) <= 1e-12
    _, _, hit3 = R.autotune_cached(b.gh, psib[:2], path, reps=1, nst=2)
    assert not hit3 and len(open(path).read().splitlines()) == 2
