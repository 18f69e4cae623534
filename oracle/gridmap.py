"""Grid-to-memory maps: plain numpy definitions.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it, and it never imports the GPU library.

Section "Parallelization, optimizations and graphics processing units"
(figures gridmaps and gpu_laplacian): a grid function is a linear array over
the grid points and the order of the points in it is free.  Three orders
are defined here on the box coordinates (x, y, z) of the oracle's grid
(``Grid.ijk``, compact order z-major, then y, then x):

- standard: the compact order itself;
- bricks of edge b: points sorted by (brick z, brick y, brick x, z, y, x),
  with brick coordinates floor(coordinate / b);
- Hilbert: points sorted by their 3D Hilbert index on the enclosing 2^bits
  cube, bits the smallest with 2^bits >= every box extent.  The index follows
  J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004):
  the axes-to-transpose transform, read level by level with x first.

An order is returned as ``order`` with ``order[i]`` = compact index of the
i-th point; a compact-order array f becomes ``f[order]``.  The mapped
Laplacian is the oracle's kinetic term applied in compact order and then
permuted: the stencil does not depend on how points are stored.
"""
from __future__ import annotations

import numpy as np

from . import Ham, hpsi


def standard_order(ijk: np.ndarray) -> np.ndarray:
    """The compact order: the identity permutation."""
    return np.arange(len(ijk), dtype=np.int64)


def brick_order(ijk: np.ndarray, b: int) -> np.ndarray:
    """Bricks of edge b in compact order of their corners, points inside a
    brick in compact order."""
    x, y, z = (ijk[:, k].astype(np.int64) for k in range(3))
    # lexsort: last key is the primary one
    return np.lexsort((x % b, y % b, z % b, x // b, y // b, z // b)).astype(np.int64)


def hilbert_index(x, y, z, bits: int) -> np.ndarray:
    """3D Hilbert index of integer coordinates below 2^bits (Skilling 2004).

    From the top level down to the second lowest: at level Q, every axis
    whose bit Q is set inverts the lower bits of axis 0; every axis whose
    bit is clear exchanges its lower bits with those of axis 0.  Then the
    axes are Gray-coded (each xor-ed with the one before), every axis is
    xor-ed with the lower-bit mask of each level where the last axis has its
    bit set, and the transposed bits are read level by level, axis 0 first.
    """
    X = [np.asarray(v, dtype=np.uint64).copy() for v in (x, y, z)]
    n = 3
    Q = 1 << (bits - 1)
    while Q > 1:
        P = np.uint64(Q - 1)
        q = np.uint64(Q)
        for i in range(n):
            has = (X[i] & q) != 0
            # invert: X0 ^= P where bit set
            inv = np.where(has, X[0] ^ P, X[0])
            # exchange low bits of X0 and Xi where bit clear
            t = (X[0] ^ X[i]) & P
            X0_ex = X[0] ^ t
            Xi_ex = X[i] ^ t
            if i == 0:
                # exchanging axis 0 with itself changes nothing
                X[0] = inv
            else:
                X[i] = np.where(has, X[i], Xi_ex)
                X[0] = np.where(has, inv, X0_ex)
        Q >>= 1
    for i in range(1, n):
        X[i] = X[i] ^ X[i - 1]
    t = np.zeros_like(X[0])
    Q = 1 << (bits - 1)
    while Q > 1:
        t = np.where((X[n - 1] & np.uint64(Q)) != 0, t ^ np.uint64(Q - 1), t)
        Q >>= 1
    for i in range(n):
        X[i] = X[i] ^ t
    h = np.zeros_like(X[0])
    for lev in range(bits - 1, -1, -1):
        for i in range(n):
            h = (h << np.uint64(1)) | ((X[i] >> np.uint64(lev)) & np.uint64(1))
    return h


def hilbert_bits(dims) -> int:
    bits = 1
    while (1 << bits) < max(int(d) for d in dims):
        bits += 1
    return bits


def hilbert_order(ijk: np.ndarray, dims) -> np.ndarray:
    """Points by ascending Hilbert index of (x, y, z)."""
    h = hilbert_index(ijk[:, 0], ijk[:, 1], ijk[:, 2], hilbert_bits(dims))
    return np.argsort(h, kind="stable").astype(np.int64)


def mapped_laplacian(grid, psi_map: np.ndarray, order: np.ndarray, scale: float,
                     nst: int | None = None) -> np.ndarray:
    """scale * (star stencil sum) of a point-major batch stored in map order:
    back to compact order, the oracle's kinetic term with kin = scale h^2,
    then into map order again."""
    psi_map = np.ascontiguousarray(psi_map, dtype=np.complex128)
    std = np.empty_like(psi_map)
    std[order] = psi_map
    ham = Ham(grid, V=None, kin=scale * grid.h * grid.h)
    out = hpsi(ham, std, nst=nst)
    return out[order]
