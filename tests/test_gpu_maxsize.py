"""Largest grids the stencil serves: one orbital field must stay below 2^27
points (its loads use 32-bit byte offsets into each orbital).

- A 511^3 cube (133,432,831 points, one orbital, 2.1 GB per field) runs H psi
  and one Taylor(4) step; 300 sampled outputs equal the stencil written out
  from the neighbouring values, gathered on the device.
- A 512^3 cube (exactly 2^27 points) is rejected (RSG_EUNSUPPORTED) before
  any stencil launch.
Inputs are drawn on the device from a seeded generator (the oracle's C loops
would take minutes at this size; the sampled check uses the definition)."""
import numpy as np
import pytest
import torch

from tests.gpu_common import rsg

pytestmark = pytest.mark.gpu

W = [-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0]


def test_largest_cube_sampled():
    R = rsg()
    n, h = 511, 0.1
    gg = R.Grid(h, n=n)
    assert gg.np == n ** 3 < 2 ** 27
    x = np.arange(n) - 0.5 * (n - 1)
    # V = 0.3 x^2 - 0.2 z: cheap to evaluate at any point from its index
    idx = torch.arange(gg.np, device="cuda", dtype=torch.int64)
    xs = (idx % n).to(torch.float64) - 0.5 * (n - 1)
    zs = (idx // (n * n)).to(torch.float64) - 0.5 * (n - 1)
    V = 0.3 * (h * xs) ** 2 - 0.2 * (h * zs)
    del idx, xs, zs
    gh = R.Hamiltonian(gg, V=V, kin=-0.5)
    g = torch.Generator(device="cuda")
    g.manual_seed(91)
    psi = torch.randn(1, gg.np, dtype=torch.complex128, device="cuda", generator=g)
    out = R.hpsi(gh, psi)
    rng = np.random.default_rng(92)
    pts = np.stack([rng.integers(0, n, 300) for _ in range(3)], axis=1)  # (i, j, k)
    pts[:8] = [[0, 0, 0], [n - 1, n - 1, n - 1], [3, 250, 0], [n - 4, 7, n - 1],
               [255, 255, 255], [1, 2, 3], [n - 2, 0, 200], [100, n - 1, 4]]
    offs = []
    for a in range(3):
        for m in (-4, -3, -2, -1, 1, 2, 3, 4):
            d = [0, 0, 0]
            d[a] = m
            offs.append((d, abs(m)))
    lin = lambda q: (q[:, 2] * n + q[:, 1]) * n + q[:, 0]
    nb_idx, nb_ok, nb_w = [], [], []
    for d, am in offs:
        q = pts + np.array(d)
        ok = np.all((q >= 0) & (q < n), axis=1)
        nb_idx.append(np.where(ok, lin(np.clip(q, 0, n - 1)), 0))
        nb_ok.append(ok)
        nb_w.append(W[am])
    nb = torch.from_numpy(np.stack(nb_idx)).cuda()
    vals = psi[0][nb].cpu().numpy() * np.stack(nb_ok)
    centre = psi[0][torch.from_numpy(lin(pts)).cuda()].cpu().numpy()
    lap = 3 * W[0] * centre + (np.array(nb_w)[:, None] * vals).sum(axis=0)
    Vp = 0.3 * (h * x[pts[:, 0]]) ** 2 - 0.2 * (h * x[pts[:, 2]])
    ref = -0.5 / h ** 2 * lap + Vp * centre
    got = out[0][torch.from_numpy(lin(pts)).cuda()].cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    del out
    # one Taylor(4) step runs at this size too (three fields of 2.1 GB)
    n0 = R.norm2(gg, psi).item()
    R.propagate_step(gh, psi, 2e-5)
    n1 = R.norm2(gg, psi).item()
    assert abs(n1 - n0) <= 1e-9 * n0


def test_grid_of_2_27_points_is_rejected():
    R = rsg()
    gg = R.Grid(0.1, n=512)
    assert gg.np == 2 ** 27
    gh = R.Hamiltonian(gg, V=None, kin=-0.5)
    psi = torch.zeros(1, gg.np, dtype=torch.complex128, device="cuda")
    with pytest.raises(R.RSGError) as ei:
        R.hpsi(gh, psi)
    assert ei.value.code == -6
