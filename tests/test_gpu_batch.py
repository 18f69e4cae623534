"""Batched propagation of many independent, uneven systems: parity with the
oracle for every system, bitwise equality with propagating each system on
its own with the same tile, and HIP-graph replays equal to eager runs."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import from_om, orbital_rel_err, pad_untouched, rsg, to_om

pytestmark = pytest.mark.gpu


def _systems(n=7, seed=33):
    """Uneven spheres (radii 2.2..4.6 bohr at h = 0.3), 1..9 orbitals with
    spare orbitals and padding points, 0..3 atoms with projectors."""
    R_ = rsg()
    g = synth.rng(seed, 9)
    out = []
    for k in range(n):
        R = float(g.uniform(2.2, 4.6))
        nst = int(g.integers(1, 10))
        ld = nst + int(g.integers(0, 3))
        na = int(g.integers(0, 4))
        og = oracle.Grid(0.3, R=R)
        gg = R_.Grid(0.3, R=R)
        assert gg.np == og.np
        pos = og.positions()
        wells = synth.gaussian_wells(seed + k, max(na, 1), ball=max(R - 1.5, 0.5))
        V = synth.well_potential(pos, wells)
        proj = synth.kb_projectors(seed + k, pos, wells.centres[:na], rcut=1.5) if na else None
        oh = oracle.Ham(og, V=V, kin=-0.5, projectors=proj)
        projs = []
        if proj is not None:
            projs = [(torch.from_numpy(i).cuda(), torch.from_numpy(p).cuda(), E)
                     for i, p, E in zip(proj.idx, proj.p, proj.E)]
        gh = R_.Hamiltonian(gg, V=torch.from_numpy(V).cuda(), kin=-0.5, projectors=projs)
        psi = synth.white_noise(seed * 100 + k, og.np, nst, 0.3, ld=ld)
        out.append(dict(og=og, oh=oh, gg=gg, gh=gh, psi=psi, nst=nst, ld=ld, pad=k % 3))
    return out


def test_batch_matches_oracle_and_single_system_bitwise():
    R = rsg()
    systems = _systems()
    dt, nsteps = 0.005, 3
    tens = [to_om(s["psi"], s["pad"]) for s in systems]
    b = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, tens)])
    tile = b.get_tile()
    b.propagate(dt, nsteps)
    torch.cuda.synchronize()
    for s, t in zip(systems, tens):
        got = from_om(t, s["og"].np)
        ref = oracle.propagate(s["oh"], s["psi"], dt, nsteps, nst=s["nst"])
        assert orbital_rel_err(got, ref, s["nst"]) <= 1e-12
        np.testing.assert_array_equal(got[:, s["nst"]:], s["psi"][:, s["nst"]:])
        assert pad_untouched(t, s["og"].np)
        # same system alone, same tile: bitwise equal
        alone = to_om(s["psi"], s["pad"])
        R.set_tile(s["gh"], s["nst"], tile["B"], tile["TX"], tile["TY"], tile["ZC"], tile["PD"],
                   ZM=tile["ZM"])
        R.propagate(s["gh"], alone, dt, nsteps, nst=s["nst"])
        np.testing.assert_array_equal(alone.cpu().numpy(), t.cpu().numpy())


def test_batch_graph_replays_and_autotune():
    R = rsg()
    systems = _systems(n=5, seed=44)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = [to_om(s["psi"], s["pad"]) for s in systems]
        g = [to_om(s["psi"], s["pad"]) for s in systems]
        ba = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, a)])
        bg = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, g)])
        tile, ms = bg.autotune(reps=1)
        assert ms > 0
        ba.set_tile(tile["B"], tile["TX"], tile["TY"], tile["ZC"], tile["PD"], tile["ZM"])
        for rep in range(3):
            ba.propagate(0.01, 2)
            bg.propagate(0.01, 2, graph=True)
            torch.cuda.synchronize()
            _ = sum(float((t.abs() ** 2).sum()) for t in a)  # eager work between replays
            for x, y in zip(a, g):
                np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
