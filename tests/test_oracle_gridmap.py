"""Pins of the oracle's grid-to-memory maps and mapped Laplacian (section
"Parallelization, optimizations and graphics processing units", figure
gridmaps), against properties the definitions fix:

- every order is a permutation of the points;
- Hilbert: on a full 2^b cube the curve starts at the origin, every step
  moves to a face neighbour, and every aligned run of 8^j consecutive
  indices fills an aligned 2^j cube (the recursive structure of the curve);
- bricks: edge 1 and an edge covering the whole box reduce to the standard
  order; each brick is one contiguous run, in compact order inside;
- the mapped Laplacian reduces to the kinetic term for the standard map, is
  exact (up to rounding) for quadratic polynomials at interior points in
  every map, and commutes with the permutation."""
import numpy as np
import pytest

import oracle
from oracle import gridmap as gm


def _cube_coords(b):
    n = 1 << b
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


@pytest.mark.parametrize("b", [1, 2, 3, 4])
def test_hilbert_full_cube_is_a_face_connected_recursive_curve(b):
    ijk = _cube_coords(b)
    h = gm.hilbert_index(ijk[:, 0], ijk[:, 1], ijk[:, 2], b)
    n3 = 1 << (3 * b)
    # a bijection onto 0 .. 8^b - 1
    assert np.array_equal(np.sort(h), np.arange(n3, dtype=np.uint64))
    path = ijk[np.argsort(h)]
    assert np.array_equal(path[0], [0, 0, 0])
    steps = np.abs(np.diff(path, axis=0)).sum(axis=1)
    assert np.all(steps == 1)
    for j in range(1, b):
        run = 1 << (3 * j)
        for s in range(0, n3, run):
            blk = path[s:s + run]
            lo = blk.min(axis=0)
            assert np.all(blk.max(axis=0) - lo == (1 << j) - 1)
            assert np.all(lo % (1 << j) == 0)


def test_hilbert_first_cells():
    # the 2 x 2 x 2 cube: a face-connected tour of the 8 corners from the origin
    ijk = _cube_coords(1)
    path = ijk[np.argsort(gm.hilbert_index(ijk[:, 0], ijk[:, 1], ijk[:, 2], 1))]
    assert len({tuple(p) for p in path}) == 8
    # each step flips exactly one coordinate (a Gray-code walk)
    assert np.all(np.abs(np.diff(path, axis=0)).sum(axis=1) == 1)


@pytest.fixture(scope="module")
def sphere():
    return oracle.Grid(0.5, R=3.3)


def test_orders_are_permutations(sphere):
    for order in (gm.standard_order(sphere.ijk), gm.brick_order(sphere.ijk, 2),
                  gm.brick_order(sphere.ijk, 3), gm.hilbert_order(sphere.ijk, sphere.dims)):
        assert np.array_equal(np.sort(order), np.arange(sphere.np))


def test_brick_special_cases_and_contiguity(sphere):
    ijk = sphere.ijk
    assert np.array_equal(gm.brick_order(ijk, 1), np.arange(sphere.np))
    assert np.array_equal(gm.brick_order(ijk, int(max(sphere.dims))), np.arange(sphere.np))
    b = 3
    order = gm.brick_order(ijk, b)
    bid = [tuple(v) for v in (ijk[order] // b)[:, ::-1]]
    # each brick id appears in one contiguous run, runs in increasing id order
    runs = [bid[0]]
    for k in range(1, len(bid)):
        if bid[k] != bid[k - 1]:
            runs.append(bid[k])
    assert len(runs) == len(set(runs))
    assert runs == sorted(runs)
    # inside a brick: increasing compact index
    for k in range(1, len(bid)):
        if bid[k] == bid[k - 1]:
            assert order[k] > order[k - 1]


def test_standard_map_laplacian_is_the_kinetic_term(sphere):
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((sphere.np, 3)) + 1j * rng.standard_normal((sphere.np, 3))
    ref = oracle.hpsi(oracle.Ham(sphere, kin=-0.5), psi)
    got = gm.mapped_laplacian(sphere, psi, gm.standard_order(sphere.ijk), -0.5 / sphere.h ** 2)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("kind", ["standard", "bricks2", "hilbert"])
def test_mapped_laplacian_exact_for_quadratics(kind):
    g = oracle.Grid(0.25, R=2.6)
    ijk = g.ijk
    order = {"standard": gm.standard_order(ijk), "bricks2": gm.brick_order(ijk, 2),
             "hilbert": gm.hilbert_order(ijk, g.dims)}[kind]
    x = g.positions()
    # f = x^2 + 2 y^2 - z^2 + i (x y + 3 z): Laplacian 2 + 4 - 2 = 4 (the
    # imaginary part is harmonic); the 8th-order stencil is exact on quadratics
    f = x[:, 0] ** 2 + 2 * x[:, 1] ** 2 - x[:, 2] ** 2 + 1j * (x[:, 0] * x[:, 1] + 3 * x[:, 2])
    psi_map = f[order][:, None]
    lap = gm.mapped_laplacian(g, psi_map, order, 1.0 / g.h ** 2)[:, 0]
    # interior in map order: every stencil neighbour inside the sphere
    m = g.map.reshape(tuple(int(d) for d in g.dims[::-1]))
    inner = np.ones(g.np, dtype=bool)
    for ax in range(3):
        for s in (-4, -3, -2, -1, 1, 2, 3, 4):
            c = ijk.copy()
            c[:, ax] += s
            ok = np.all((c >= 0) & (c < g.dims), axis=1)
            idx = np.full(g.np, -1)
            idx[ok] = m[c[ok, 2], c[ok, 1], c[ok, 0]]
            inner &= idx >= 0
    inner_map = inner[order]
    assert inner_map.sum() > 100
    np.testing.assert_allclose(lap[inner_map], 4.0 + 0j, rtol=0, atol=1e-9)


def test_mapped_laplacian_commutes_with_the_permutation(sphere):
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((sphere.np, 2)) + 1j * rng.standard_normal((sphere.np, 2))
    ref = oracle.hpsi(oracle.Ham(sphere, kin=1.0), psi)
    order = gm.hilbert_order(sphere.ijk, sphere.dims)
    got = gm.mapped_laplacian(sphere, psi[order], order, 1.0 / sphere.h ** 2)
    np.testing.assert_allclose(got, ref[order], rtol=0, atol=1e-13 * np.abs(ref).max())
