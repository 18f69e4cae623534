"""Grid-to-memory maps on the GPU (section "Parallelization, optimizations and
graphics processing units", figures gridmaps and gpu_laplacian).

- The library's order is the oracle's order, bit for bit, for the standard,
  brick and Hilbert maps of spheres and cubes.
- The gather Laplacian in map order matches the oracle's kinetic term
  (applied in compact order, then permuted) to the FP64 bar (1e-12 relative
  per orbital) for 1, 5 and 64 orbitals with spare columns, which stay
  untouched; the one-point grid reduces to the centre tap.
- On the 500 k-point sphere of the mapping benchmark with 64 orbitals,
  sampled outputs agree with the stencil sum written out point by point.
- Bad arguments are rejected before anything is launched."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from oracle import gridmap as gm
from tests.gpu_common import orbital_rel_err, rsg

pytestmark = pytest.mark.gpu

SENT = 5.0 + 2.0j  # written into the spare columns of out


def _oracle_order(og, kind, param):
    if kind == 0:
        return gm.standard_order(og.ijk)
    if kind == 1:
        return gm.brick_order(og.ijk, param)
    return gm.hilbert_order(og.ijk, og.dims)


def _grids(h, **kw):
    R = rsg()
    og = oracle.Grid(h, **kw)
    gg = R.Grid(h, **kw)
    assert gg.np == og.np
    np.testing.assert_array_equal(gg.coords(), og.ijk)
    return og, gg


MAPS = [(0, 0), (1, 2), (1, 4), (1, 5), (2, 0)]


@pytest.mark.parametrize("shape", [dict(R=3.1), dict(n=11)])
@pytest.mark.parametrize("kind,param", MAPS)
def test_map_order_and_laplacian_match_oracle(shape, kind, param):
    R = rsg()
    og, gg = _grids(0.3, **shape)
    m = R.GridMap(gg, kind, param)
    order = m.order()
    np.testing.assert_array_equal(order, _oracle_order(og, kind, param))
    rng = np.random.default_rng(10 * kind + param)
    scale = -0.5 / og.h ** 2
    for nst, ld in ((1, 1), (5, 7), (64, 64)):
        psi = rng.standard_normal((og.np, ld)) + 1j * rng.standard_normal((og.np, ld))
        psi_map = psi[order]
        ref = gm.mapped_laplacian(og, psi_map, order, scale, nst=nst)
        x = torch.from_numpy(psi_map).to("cuda")
        out = torch.full_like(x, SENT)
        m.laplacian(x, out, nst=nst, scale=scale)
        got = out.cpu().numpy()
        e = orbital_rel_err(got, ref, nst)
        assert e <= 1e-12, (kind, param, nst, e)
        assert np.all(got[:, nst:] == SENT)


def test_one_point_grid_is_the_centre_tap():
    R = rsg()
    og, gg = _grids(1.0, R=0.5)
    assert og.np == 1
    for kind, param in MAPS:
        m = R.GridMap(gg, kind, param)
        assert list(m.order()) == [0]
        x = torch.tensor([[1.5 - 0.25j, 2.0 + 1.0j]], dtype=torch.complex128, device="cuda")
        out = m.laplacian(x, scale=2.0).cpu().numpy()
        c0 = -205.0 / 72.0
        np.testing.assert_allclose(out, 2.0 * 3.0 * c0 * x.cpu().numpy(), rtol=1e-15)


def test_full_size_sphere_sampled():
    """R = 9.85 bohr, h = 0.2 (np ~ 5.0e5), 64 orbitals, Hilbert and brick
    maps: 400 sampled (point, orbital) outputs against the stencil sum of
    the definition, evaluated one by one from the oracle grid."""
    R = rsg()
    og, gg = _grids(0.2, R=9.85)
    assert 490_000 < og.np < 510_000
    nst = 64
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    dense = og.map.reshape(tuple(int(d) for d in og.dims[::-1]))
    w = [-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]
    rng = np.random.default_rng(78)
    for kind, param in ((2, 0), (1, 4)):
        m = R.GridMap(gg, kind, param)
        order = m.order()
        np.testing.assert_array_equal(order, _oracle_order(og, kind, param))
        pos = np.empty(og.np, dtype=np.int64)
        pos[order] = np.arange(og.np)
        x = torch.randn(og.np, nst, dtype=torch.complex128, device="cuda", generator=g)
        out = m.laplacian(x, scale=1.0)
        xs, got = x.cpu().numpy(), out.cpu().numpy()
        for i, n in zip(rng.integers(0, og.np, 400), rng.integers(0, nst, 400)):
            c = order[i]
            ijk = og.ijk[c]
            acc = 3 * w[0] * xs[i, n]
            for ax in range(3):
                for s in (-4, -3, -2, -1, 1, 2, 3, 4):
                    q = ijk.copy()
                    q[ax] += s
                    if np.all(q >= 0) and np.all(q < og.dims):
                        cc = dense[q[2], q[1], q[0]]
                        if cc >= 0:
                            acc += w[abs(s)] * xs[pos[cc], n]
            assert abs(got[i, n] - acc) <= 1e-12 * max(1.0, abs(acc)), (kind, i, n)


def test_map_errors():
    R = rsg()
    og, gg = _grids(0.3, n=6)
    h = C.c_void_p()
    assert R._lib.rsg_map_create(gg._h, 3, 0, C.byref(h)) == -1
    assert R._lib.rsg_map_create(gg._h, 1, 0, C.byref(h)) == -1
    assert R._lib.rsg_map_create(gg._h, 1, 65, C.byref(h)) == -1
    m = R.GridMap(gg, 2)
    x = torch.zeros(og.np, 4, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    px, py = C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())
    assert R._lib.rsg_map_laplacian(m._h, px, py, 0, 4, 1.0, None) == -2
    assert R._lib.rsg_map_laplacian(m._h, px, py, 5, 4, 1.0, None) == -2
    assert R._lib.rsg_map_laplacian(m._h, px, px, 4, 4, 1.0, None) == -1
    assert R._lib.rsg_map_laplacian(m._h, None, py, 4, 4, 1.0, None) == -1
    with pytest.raises(ValueError):
        m.laplacian(x[:-1].contiguous())
