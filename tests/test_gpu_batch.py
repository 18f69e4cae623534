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


def _singles(R, systems, tiles, dt, nsteps):
    """Each system propagated alone with the given tile (B, TX, TY, ZC, PD, ZM)."""
    out = []
    for s, t in zip(systems, tiles):
        alone = to_om(s["psi"], s["pad"])
        R.set_tile(s["gh"], s["nst"], t[0], t[1], t[2], t[3], t[4], ZM=t[5])
        R.propagate(s["gh"], alone, dt, nsteps, nst=s["nst"])
        out.append(alone.cpu().numpy())
    return out


def test_batch_few_workgroups_take_many_items():
    """The persistent grid capped at 1, 2 and 4 workgroups, so that every
    workgroup takes many items in turn (the work-counter loop, the plane
    buffers reused after the trailing barrier, the counter reset by the last
    workgroup out): eager steps and two graph replays per cap are bitwise
    equal to each system propagated alone."""
    R = rsg()
    systems = _systems(n=5, seed=55)
    tile = (1, 16, 8, 0, 1, 0)
    dt, nsteps = 0.005, 2
    ref = _singles(R, systems, [tile] * len(systems), dt, nsteps)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for cap in (1, 2, 4):
            tens = [to_om(s["psi"], s["pad"]) for s in systems]
            b = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, tens)])
            b.set_tile(*tile)
            b.set_grid(cap)
            info = [b.class_info(c) for c in range(int(b.classes().max()) + 1)]
            assert all(i["grid"] == cap and i["nitems"] >= 20 * cap for i in info), info
            b.propagate(dt, nsteps)
            torch.cuda.synchronize()
            for r, t in zip(ref, tens):
                np.testing.assert_array_equal(t.cpu().numpy(), r)
            g = [to_om(s["psi"], s["pad"]) for s in systems]
            bg = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, g)])
            bg.set_tile(*tile)
            bg.set_grid(cap)
            for rep in range(2):
                for s, t in zip(systems, g):
                    t.copy_(to_om(s["psi"], s["pad"]))
                bg.propagate(dt, nsteps, graph=True)
                torch.cuda.synchronize()
                _ = sum(float((t.abs() ** 2).sum()) for t in g)  # eager work between replays
                for r, t in zip(ref, g):
                    np.testing.assert_array_equal(t.cpu().numpy(), r)


def test_batch_classes_have_own_tiles():
    """Systems split into three classes, each with its own tile shape: every
    system equals the oracle and, bit for bit, itself propagated alone with
    its class's tile; the run entry point (graph replay) gives the same bits."""
    R = rsg()
    systems = _systems(n=7, seed=66)
    cls = np.array([0, 1, 2, 0, 1, 2, 1], dtype=np.int32)
    tiles = {0: (1, 8, 8, 0, 1, 0), 1: (1, 32, 8, 4, 2, 1), 2: (1, 16, 16, 0, 2, 0)}
    dt, nsteps = 0.005, 2
    ref = _singles(R, systems, [tiles[c] for c in cls], dt, nsteps)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tens = [to_om(s["psi"], s["pad"]) for s in systems]
        b = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, tens)])
        b.set_classes(cls)
        np.testing.assert_array_equal(b.classes(), cls)
        for c, t in tiles.items():
            b.set_tile(*t, cls=c)
            got = b.get_tile(cls=c)
            assert (got["TX"], got["TY"], got["ZC"], got["PD"], got["ZM"]) == (t[1], t[2], t[3], t[4], t[5])
        b.propagate(dt, nsteps)
        torch.cuda.synchronize()
        for s, r, t in zip(systems, ref, tens):
            np.testing.assert_array_equal(t.cpu().numpy(), r)
            ora = oracle.propagate(s["oh"], s["psi"], dt, nsteps, nst=s["nst"])
            assert orbital_rel_err(from_om(t, s["og"].np), ora, s["nst"]) <= 1e-12
        for s, t in zip(systems, tens):
            t.copy_(to_om(s["psi"], s["pad"]))
        b.run(nsteps, dt)
        torch.cuda.synchronize()
        for r, t in zip(ref, tens):
            np.testing.assert_array_equal(t.cpu().numpy(), r)
    with pytest.raises(R.RSGError):
        b.set_classes(np.array([0, 2, 2, 0, 2, 2, 2], dtype=np.int32))  # class 1 empty


def test_batch_uneven_spheres_at_scale():
    """48 spheres of radius U(6, 12) bohr at h = 0.25 (the large half of the
    256-system workload's range), 1..32 orbitals, 1..8 wells with
    projectors, in the default size classes and default grid: at least four
    work items per persistent workgroup in every class.  After two steps
    (eager, and replayed from a HIP graph with the same bits) one sampled
    orbital of every system equals the oracle's to 1e-12."""
    R = rsg()
    specs = synth.batch_specs(9, 48, Rmin=6.0, Rmax=12.0, h=0.25, nst_max=32, atoms_max=8)
    pick = synth.rng(9, 77)
    systems = []
    for sp in specs:
        og = oracle.Grid(sp.h, R=sp.R)
        gg = R.Grid(sp.h, R=sp.R, align=8)
        live = gg.live()
        pos = og.positions()
        V = synth.well_potential(pos, sp.wells)
        proj = synth.kb_projectors(sp.seed, pos, sp.wells.centres)
        psi = synth.white_noise(sp.seed, og.np, sp.nst, sp.h)
        Vs = np.zeros(gg.np)
        Vs[live] = V
        projs = [(torch.from_numpy(live[i].astype(np.int32)).cuda(), torch.from_numpy(p).cuda(), E)
                 for i, p, E in zip(proj.idx, proj.p, proj.E)]
        gh = R.Hamiltonian(gg, V=torch.from_numpy(Vs).cuda(), kin=-0.5, projectors=projs)
        n = int(pick.integers(0, sp.nst))
        systems.append(dict(og=og, gg=gg, gh=gh, live=live, V=V, proj=proj, psi=psi, nst=sp.nst, n=n))
    del psi

    def load():
        out = []
        for s in systems:
            t = torch.zeros((s["nst"], s["gg"].np), dtype=torch.complex128, device="cuda")
            t[:, torch.from_numpy(s["live"]).cuda()] = torch.from_numpy(s["psi"]).cuda().t()
            out.append(t)
        return out

    dt, nsteps = 0.005, 2
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tens = load()
        b = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, tens)])
        ncls = int(b.classes().max()) + 1
        assert ncls >= 2
        for c in range(ncls):
            info = b.class_info(c)
            assert info["nitems"] >= 4 * info["grid"], info
        b.propagate(dt, nsteps)
        torch.cuda.synchronize()
        eager = [t.cpu().numpy() for t in tens]
        g = load()
        bg = R.Batch([(s["gh"], t, s["nst"]) for s, t in zip(systems, g)])
        bg.propagate(dt, nsteps, graph=True)
        torch.cuda.synchronize()
        for e, t in zip(eager, g):
            np.testing.assert_array_equal(t.cpu().numpy(), e)
    for s, e in zip(systems, eager):
        oh = oracle.Ham(s["og"], V=s["V"], kin=-0.5, projectors=s["proj"])
        one = np.ascontiguousarray(s["psi"][:, [s["n"]]])
        ref = oracle.propagate(oh, one, dt, nsteps)
        got = e[s["n"], s["live"]][:, None]
        assert orbital_rel_err(got, ref, 1) <= 1e-12, (s["og"].np, s["nst"], s["n"])
        dead = np.ones(s["gg"].np, dtype=bool)
        dead[s["live"]] = False
        assert np.all(e[:, dead] == 0)


def test_batch256_workload_sampled_against_oracle():
    """The 256-system workload at full size (R ~ U(4, 12) bohr at h = 0.25,
    1..32 orbitals, 1..8 wells with projectors; 688,438,342
    point-orbitals), in its default size classes, one step as the benchmark
    runs it: every system in the batch, the step replayed from a HIP graph
    with the eager step's bits, and one orbital of each of 24 sampled
    systems equal to the oracle's step to 1e-12 (dead slots zero)."""
    R = rsg()
    cfg = dict(synth.WORKLOADS["batch256"])
    specs = synth.batch_specs(cfg["seed"], cfg["nsys"], cfg["Rmin"], cfg["Rmax"], cfg["h"], cfg["nst_max"],
                              cfg["atoms_max"])
    assert len(specs) == 256
    pick = synth.rng(cfg["seed"], 78)
    sample = set(int(k) for k in pick.choice(256, size=24, replace=False))
    systems, total = [], 0
    for k, sp in enumerate(specs):
        gg = R.Grid(sp.h, R=sp.R, align=8)
        live = gg.live()
        pos = gg.positions()[live]
        V = synth.well_potential(pos, sp.wells)
        proj = synth.kb_projectors(sp.seed, pos, sp.wells.centres)
        psi = synth.white_noise(sp.seed, gg.npoints, sp.nst, sp.h)
        Vs = np.zeros(gg.np)
        Vs[live] = V
        projs = [(torch.from_numpy(live[i].astype(np.int32)).cuda(), torch.from_numpy(p).cuda(), E)
                 for i, p, E in zip(proj.idx, proj.p, proj.E)]
        gh = R.Hamiltonian(gg, V=torch.from_numpy(Vs).cuda(), kin=-0.5, projectors=projs)
        t = torch.zeros((sp.nst, gg.np), dtype=torch.complex128, device="cuda")
        t[:, torch.from_numpy(live).cuda()] = torch.from_numpy(psi).cuda().t()
        n = int(pick.integers(0, sp.nst))
        keep = dict(sp=sp, pos=pos, V=V, proj=proj, psi=psi[:, [n]].copy(), n=n) if k in sample else None
        systems.append(dict(gg=gg, gh=gh, live=live, psi0=t.clone(), t=t, nst=sp.nst, keep=keep))
        total += gg.npoints * sp.nst
        del psi
    assert total == 688438342
    dt = cfg["dt"]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = R.Batch([(s["gh"], s["t"], s["nst"]) for s in systems])
        b.propagate(dt, 1)
        torch.cuda.synchronize()
        for s in systems:  # the graph's batch starts from the same inputs
            s["eager"] = s["t"]
            s["t"] = s["psi0"]
        bg = R.Batch([(s["gh"], s["t"], s["nst"]) for s in systems])
        bg.propagate(dt, 1, graph=True)
        torch.cuda.synchronize()
        for s in systems:
            assert torch.equal(s["t"], s["eager"])
    for s in systems:
        kp = s["keep"]
        if kp is None:
            continue
        sp = kp["sp"]
        og = oracle.Grid(sp.h, R=sp.R)
        assert og.np == s["gg"].npoints
        np.testing.assert_array_equal(og.positions(), kp["pos"])
        oh = oracle.Ham(og, V=kp["V"], kin=-0.5, projectors=kp["proj"])
        ref = oracle.propagate(oh, kp["psi"], dt, 1)
        e = s["eager"][kp["n"]].cpu().numpy()
        got = e[s["live"]][:, None]
        assert orbital_rel_err(got, ref, 1) <= 1e-12, (sp.R, sp.nst, kp["n"])
        dead = np.ones(s["gg"].np, dtype=bool)
        dead[s["live"]] = False
        assert np.all(e[dead] == 0)
