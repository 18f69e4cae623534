#!/usr/bin/env python3
"""Benchmark of the real-space Kohn-Sham H*psi / Taylor(4) propagation path.

Default workload (one GPU): the sphere of radius 18 bohr at h = 0.2 bohr
(3,053,617 points, padded box 181^3), 64 complex128 white-noise orbitals,
16 Gaussian wells with 4 separable projectors each; K Taylor(4) steps at
dt = 0.005.  One step = 4 applications of H to the whole batch.

Prints ONE JSON line: throughput in grid-point x orbital H-applications per
second, the roofline of the dominant (stencil) kernel measured with HIP
events inside the timed region, and the FP64 oracle timed on the host on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "H·ψ grid-pt·orbital updates/s"
UNIT = "pt·orb·H/s"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# the sources of the stencil kernels and their launch
STENCIL_SOURCES = ("stencil.hip", "stencil_common.h", "stencil_inst.hip", "stencil_inst_nt.hip", "stencil_kernels.h")


def stencil_source_hash() -> str:
    h = hashlib.sha256()
    for name in STENCIL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1501_05654_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def _summary_fields(path: str) -> dict:
    kv = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def read_traffic(workload: str, tile=None, align: int = 1, with_path: bool = False):
    """HBM bytes per stencil launch from a committed rocprofv3 counter
    summary (profiles/traffic_stencil_<workload>*.txt) taken on the current
    stencil source with the tile shape and grid row alignment in use; None
    if there is none.  with_path: (bytes, summary file name) or (None, None)."""
    key = None
    if tile is not None:
        key = ",".join(str(tile[k]) for k in ("B", "TX", "TY", "ZC", "PD", "PT", "BO", "ZM"))
    for p in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_stencil_{workload}*.txt"))):
        kv = _summary_fields(p)
        if kv.get("stencil_source_sha256") != stencil_source_hash():
            continue
        if key is not None and kv.get("tile") != key:
            continue
        if int(kv.get("row_align", "1")) != align:
            continue
        try:
            v = float(kv["hbm_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
        return (v, os.path.join("profiles", os.path.basename(p))) if with_path else v
    return (None, None) if with_path else None


def place_on_slots(gg, live, V, proj, psi_h, dev):
    """Per-point inputs -> the grid's slots (dead slots zero): V tensor,
    projector list with slot indices, orbital-major psi [nst, slots]."""
    import numpy as np
    import torch
    Vs = np.zeros(gg.np)
    Vs[live] = V
    projs = [(torch.from_numpy(live[i].astype(np.int32)).to(dev), torch.from_numpy(p).to(dev), E)
             for i, p, E in zip(proj.idx, proj.p, proj.E)]
    psi = torch.zeros((psi_h.shape[1], gg.np), dtype=torch.complex128, device=dev)
    psi[:, torch.from_numpy(live).to(dev)] = torch.from_numpy(psi_h).to(dev).t()
    return torch.from_numpy(Vs).to(dev), projs, psi


def build_sphere_inputs(cfg, positions):
    import synth
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], ball=cfg["well_ball"])
    V = synth.well_potential(positions, wells)
    proj = synth.kb_projectors(cfg["seed"], positions, wells.centres)
    return V, proj


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def fixed_tile(spec: str) -> list:
    """'B,TX,TY,ZC,PD,PT,BO[,ZM]' -> the eight tile fields (ZM defaults to 0)."""
    vals = [int(v) for v in spec.split(",")]
    if len(vals) not in (7, 8):
        raise SystemExit(f"a tile is B,TX,TY,ZC,PD,PT,BO[,ZM], got {spec!r}")
    return vals + [0] * (8 - len(vals))


def class_tiles_spec(spec: str) -> list:
    """batch256 --tile: one tile for every size class, or one per class
    separated by ';' (narrowest class first) -> list of eight-field tiles."""
    return [fixed_tile(t) for t in spec.split(";")]


def choose_tile(args, spec, gh, psi, reps, dtype="c128"):
    """The stencil tile of gh for psi's batch: the one spec names, else the
    autotuner's choice (the default shape with --no-autotune)."""
    import paper_1501_05654_amd as rsg

    nst = psi.shape[0]
    if spec:
        rsg.set_tile(gh, nst, *fixed_tile(spec), dtype=dtype)
    elif not args.no_autotune:
        rsg.autotune(gh, psi, dtype=dtype, reps=reps)
    return rsg.get_tile(gh, nst, dtype=dtype)


def cpu_baseline(cfg, seconds: float):
    """The FP64 oracle on the host: one Taylor(4) step over the full grid on
    a sample of the orbitals sized to take about `seconds` with every host
    thread, then the same for one orbital on a single thread."""
    import oracle
    import synth
    t0 = time.perf_counter()
    og = oracle.Grid(cfg["h"], R=cfg["R"])
    V, proj = build_sphere_inputs(cfg, og.positions())
    oh = oracle.Ham(og, V=V, kin=-0.5, projectors=proj)
    psi1 = synth.white_noise(cfg["seed"], og.np, 1, cfg["h"])
    cores = oracle.max_threads()
    t = time.perf_counter()
    oracle.hpsi(oh, psi1)
    per_orb_h = time.perf_counter() - t
    n_orb = int(max(1, min(cfg["nst"], round(seconds / (4.0 * per_orb_h)))))
    psi = synth.white_noise(cfg["seed"], og.np, n_orb, cfg["h"])
    t = time.perf_counter()
    oracle.taylor_step(oh, psi, cfg["dt"])
    el = time.perf_counter() - t
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.taylor_step(oh, psi1, cfg["dt"])
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    log(f"cpu baseline: {n_orb} orbitals, {el:.1f} s on {cores} threads; 1 orbital, {el1:.1f} s on 1 thread "
        f"(setup {t - t0:.1f} s)")
    return {
        "value": og.np * n_orb * 4 / el,
        "unit": UNIT,
        "cores": cores,
        "kind": "oracle",
        "sample": f"1 Taylor(4) step (4 H applications) over all {og.np} points for "
                  f"{n_orb} of the {cfg['nst']} orbitals, FP64 C oracle, OpenMP over points",
        "single_thread_value": og.np * 4 / el1,
        "single_thread_sample": "1 Taylor(4) step over all points for 1 orbital on 1 thread",
        "cpu_model": cpu_model(),
    }


def bench_sphere(args):
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS[args.workload])
    torch.cuda.set_device(0)
    log("grid")
    # row-aligned storage (align 8: every row starts on a 128-byte line); the
    # inputs are the same per point, placed in the live slots, zero elsewhere
    gg = rsg.Grid(cfg["h"], R=cfg["R"], align=args.align)
    live = gg.live()
    pos = gg.positions()[live]
    V, proj = build_sphere_inputs(cfg, pos)
    log(f"points={gg.npoints}, slots={gg.np}, generating {cfg['nst']} orbitals")
    psi_h = synth.white_noise(cfg["seed"], gg.npoints, cfg["nst"], cfg["h"])
    dev = torch.device("cuda:0")
    # the library's layout is orbital-major [nst, slots]
    Vt, projs, psi = place_on_slots(gg, live, V, proj, psi_h, dev)
    gh = rsg.Hamiltonian(gg, V=Vt, kin=-0.5, projectors=projs)
    del psi_h
    nst = cfg["nst"]
    ws = torch.empty(gh.workspace_bytes("step", nst, psi.shape[1]), dtype=torch.uint8, device=dev)
    dt = cfg["dt"]
    tile = None
    if args.tile:
        rsg.set_tile(gh, nst, *fixed_tile(args.tile))
        tile = rsg.get_tile(gh, nst)
    elif not args.no_autotune:
        tile, tile_ms = rsg.autotune(gh, psi, reps=4)
        log(f"autotuned tile {tile}: {tile_ms:.3f} ms of stencil work per step")
    if tile is None:
        tile = rsg.get_tile(gh, nst)
    log(f"warmup {args.warmup} steps")
    rsg.propagate(gh, psi, dt, args.warmup, ws=ws)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    with rsg.kernel_timing() as kt:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rsg.propagate(gh, psi, dt, args.steps, ws=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    el = t1 - t0
    npts = gg.npoints  # box points; dead slots are not counted
    value = npts * nst * 4 * args.steps / el
    # algorithmic HBM bytes of one stencil launch: an FP64 step runs as the
    # product of the four linear factors of the Taylor polynomial, so every
    # stage reads its input and writes its output (32 B per point-orbital)
    # and reads V (8 B per point)
    stage_bytes = npts * nst * 32 + 8 * npts
    achieved = stage_bytes / (kt.mean_ms * 1e-3) / 1e9 if kt.count else None
    traffic, traffic_src = read_traffic(args.workload, tile, gg.align, with_path=True)
    norms = rsg.norm2(gg, psi).cpu().numpy()
    # plain device copy of 1 GiB: achievable copy bandwidth, and the
    # reference kernel for scaling the HBM byte counters
    cbytes = 1 << 30
    src = torch.empty(cbytes, dtype=torch.uint8, device=dev)
    dstb = torch.empty_like(src)
    rsg.copy(src, dstb)
    with rsg.kernel_timing() as ct:
        for _ in range(3):
            rsg.copy(src, dstb)
        torch.cuda.synchronize()
    copy_gbs = 2 * cbytes / (ct.mean_ms * 1e-3) / 1e9
    del src, dstb
    log(f"{el * 1e3 / args.steps:.3f} ms/step, stencil {kt.mean_ms:.4f} ms x {kt.count}, "
        f"norm range [{norms.min():.6f}, {norms.max():.6f}]")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "np": npts, "nst": nst, "natoms": cfg["natoms"],
                   "R_bohr": cfg["R"], "h_bohr": cfg["h"], "dt": dt, "taylor_order": 4,
                   "stencil": "8th-order 25-point star", "row_align": gg.align, "slots": gg.np},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "frac_basis": "algorithmic bytes per launch / HIP-event kernel mean of this run",
                     "traffic": traffic,
                     "traffic_basis": (f"HBM bytes per launch from {traffic_src} (rocprofv3 FETCH_SIZE and "
                                       "WRITE_SIZE of this tile on this stencil source, scaled by a 1 GiB "
                                       "copy); not measured in this run") if traffic else None,
                     "traffic_over_algorithmic": (traffic / stage_bytes) if traffic else None,
                     "kernel": "k_stencil (Taylor stage, product form)",
                     "kernel_mean_ms": kt.mean_ms, "launches_timed": kt.count,
                     "algorithmic_bytes_per_launch": stage_bytes, "tile": tile,
                     "copy_gbs": copy_gbs},
    }
    del psi, ws
    torch.cuda.empty_cache()
    return out, cfg


def bench_batch(args):
    """256 independent spheres (R ~ U(4,12) bohr at h = 0.25, 1..32 orbitals,
    1..8 wells with projectors): K Taylor(4) steps of all systems (50 in the
    reference workload), every stage one persistent launch, the step sequence
    replayed from a HIP graph.  Also times the same systems propagated one by
    one (eager) for comparison."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["batch256"])
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    specs = synth.batch_specs(cfg["seed"], cfg["nsys"], cfg["Rmin"], cfg["Rmax"], cfg["h"],
                              cfg["nst_max"], cfg["atoms_max"])
    if args.nsys:
        specs = specs[: args.nsys]
    systems, keep = [], []
    tot = 0
    log(f"building {len(specs)} systems")
    for k, sp in enumerate(specs):
        gg = rsg.Grid(sp.h, R=sp.R, align=args.align)
        live = gg.live()
        pos = gg.positions()[live]
        V = synth.well_potential(pos, sp.wells)
        proj = synth.kb_projectors(sp.seed, pos, sp.wells.centres)
        Vt, projs, psi = place_on_slots(gg, live, V, proj, synth.white_noise(sp.seed, gg.npoints, sp.nst, sp.h),
                                        dev)
        gh = rsg.Hamiltonian(gg, V=Vt, kin=-0.5, projectors=projs)
        systems.append((gh, psi, sp.nst))
        keep.append(gg)
        tot += gg.npoints * sp.nst
    log(f"sum np*nst = {tot:.4e}")
    # one 1 GiB copy: the reference dispatch for scaling HBM traffic counters
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dstb = torch.empty_like(src)
    rsg.copy(src, dstb)
    torch.cuda.synchronize()
    del src, dstb
    stream = torch.cuda.Stream()
    dt = cfg["dt"]
    with torch.cuda.stream(stream):
        b = rsg.Batch(systems)
        if args.tile:
            # one tile for every size class, or one per class (';'-separated)
            tiles_t = class_tiles_spec(args.tile)
            for c, (B, TX, TY, ZC, PD, _, _, ZM) in enumerate(tiles_t):
                b.set_tile(B, TX, TY, ZC, PD, ZM, cls=None if len(tiles_t) == 1 else c)
            tile = b.get_tile()
            log(f"batch tiles {args.tile} (fixed)")
        else:
            tile, tms = b.autotune(reps=3)
            log(f"batch tile {tile}: {tms:.3f} ms per stage")
        # eager steps with per-launch HIP-event timing of the stencil kernel
        # (one persistent launch per size class and stage)
        timed_steps = max(1, args.warmup)
        with rsg.kernel_timing() as kt:
            b.propagate(dt, timed_steps)
            torch.cuda.synchronize()
        classes = b.classes()
        class_tiles = [b.get_tile(c) for c in range(int(classes.max()) + 1)]
        b.propagate(dt, args.steps, graph=True)  # capture and first replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.propagate(dt, args.steps, graph=True)  # timed replay
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # one by one (eager), a few steps
        per_steps = max(1, min(5, args.steps))
        for (gh, psi, nst), c in zip(systems, classes):
            t = class_tiles[c]
            rsg.set_tile(gh, nst, t["B"], t["TX"], t["TY"], t["ZC"], t["PD"], ZM=t["ZM"])
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        for gh, psi, nst in systems:
            rsg.propagate(gh, psi, dt, per_steps, nst=nst)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
    el = t1 - t0
    value = tot * 4 * args.steps / el
    # counter summary of this stencil source with these class tiles (one
    # tile when every class has the same, else one per class, ';'-separated)
    ctraffic, ctraffic_src = None, None
    keys = [",".join(str(t[k]) for k in ("B", "TX", "TY", "ZC", "PD", "PT", "BO", "ZM")) for t in class_tiles]
    key = keys[0] if all(k == keys[0] for k in keys) else ";".join(keys)
    for p in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_stencil_batch256_*.txt"))):
        kv = _summary_fields(p)
        if (kv.get("stencil_source_sha256") == stencil_source_hash() and kv.get("tile") == key
                and int(kv.get("row_align", "0")) == args.align):
            ctraffic, ctraffic_src = float(kv["hbm_bytes_per_stage"]), os.path.join("profiles", os.path.basename(p))
            break
    stage_bytes = tot * 32.0  # every stage of the product-form step: read its input, write its output
    stage_ms = kt.total_ms / (4 * timed_steps) if kt.count else None  # all classes' launches of a stage
    achieved = stage_bytes / (stage_ms * 1e-3) / 1e9 if kt.count else None
    return {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch256", "nsys": len(specs), "sum_np_nst": tot, "h_bohr": cfg["h"],
                   "dt": dt, "class_tiles": class_tiles,
                   "class_sizes": [int((classes == c).sum()) for c in range(len(class_tiles))],
                   "row_align": args.align},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "frac_basis": "algorithmic bytes of a stage (32 B/pt·orb) / HIP-event time of its launches",
                     "traffic": ctraffic,
                     "traffic_basis": (f"HBM bytes per stage (all class launches) from {ctraffic_src} "
                                       "(rocprofv3 FETCH_SIZE and WRITE_SIZE on this stencil source and tile, "
                                       "scaled by a 1 GiB copy); not measured in this run")
                     if ctraffic else None,
                     "kernel": "k_stencil_batch (persistent; one launch per size class and stage)",
                     "stage_ms": stage_ms, "kernel_mean_ms": kt.mean_ms, "launches_timed": kt.count},
        "per_system_eager_value": tot * 4 * per_steps / (t5 - t4),
        "cpu_baseline": None,
    }


def bench_mixed(args):
    """The 32^3 harmonic system, 4 orbitals: FP32 Hamiltonian with FP64
    accumulation against the FP64 path at steps 1, 10, 100, 1000, for
    white-noise orbitals and for smooth low harmonic-oscillator states.
    (The FP64 path itself is held to the oracle by the parity tests.)"""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["cube32_mixed"])
    n, h, nst, dt = cfg["n"], cfg["h"], cfg["nst"], cfg["dt"]
    nsteps = args.steps if args.steps else cfg["steps"]
    gg = rsg.Grid(h, n=n)
    pos = gg.positions()
    V = synth.harmonic_potential(pos)
    gh = rsg.Hamiltonian(gg, V=torch.from_numpy(V).cuda(), kin=-0.5)
    marks = [m for m in (1, 10, 100, 1000) if m <= nsteps]
    report = {}
    timing = {}
    kms = []
    for name, psi0 in (("white_noise", synth.white_noise(cfg["seed"], gg.np, nst, h)),
                       ("ho_low_states", synth.ho_low_states(pos, nst))):
        mixed = torch.from_numpy(psi0).cuda().t().contiguous()  # orbital-major
        full = torch.from_numpy(psi0).cuda().t().contiguous()
        rows, prev = [], 0
        tm = tf = 0.0
        for m in marks:
            torch.cuda.synchronize()
            t = time.perf_counter()
            with rsg.kernel_timing() as kt:
                rsg.propagate(gh, mixed, dt, m - prev, dtype="mixed")
                torch.cuda.synchronize()
            tm += time.perf_counter() - t
            if name == "white_noise" and kt.count:
                kms.append((kt.mean_ms, kt.count))
            t = time.perf_counter()
            rsg.propagate(gh, full, dt, m - prev)
            torch.cuda.synchronize()
            tf += time.perf_counter() - t
            prev = m
            gm, gf = mixed.cpu().numpy().T, full.cpu().numpy().T
            err = np.linalg.norm(gm - gf, axis=0) / np.linalg.norm(gf, axis=0)
            nm = rsg.norm2(gg, mixed).cpu().numpy()
            nf = rsg.norm2(gg, full).cpu().numpy()
            em = rsg.energy(gh, mixed).cpu().numpy().real.sum()
            ef = rsg.energy(gh, full).cpu().numpy().real.sum()
            rows.append({"step": m, "orbital_rel_err_max": float(err.max()),
                         "norm_abs_err_max": float(np.abs(nm - nf).max()),
                         "energy_rel_err": float(abs(em - ef) / abs(ef))})
            log(f"{name} step {m}: {rows[-1]}")
        report[name] = rows
        timing[name] = {"mixed_ms_per_step": tm * 1e3 / nsteps, "fp64_ms_per_step": tf * 1e3 / nsteps}
    tot = gg.np * nst
    # mixed stages per step: psi (complex128) -> y1, y1 -> y2, y2 -> y3
    # (complex64), then psi + c H y3 -> psi: 24 + 16 + 16 + 40 = 96 B/pt.orb
    # per step, 24 per launch, plus the FP32 potential (4 B/pt)
    cnt = sum(c for _, c in kms)
    mean_ms = sum(m * c for m, c in kms) / cnt if cnt else None
    mix_gbs = (24 * tot + 4 * gg.np) / (mean_ms * 1e-3) / 1e9 if mean_ms else None
    return {
        "metric": "mixed-precision orbital error vs the FP64 path", "value":
            report["white_noise"][-1]["orbital_rel_err_max"], "unit": "relative 2-norm",
        "n_gpus": 1, "steps": nsteps, "warmup": 0, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 H / f64 accumulation", "data": "synthetic",
        "config": {"workload": "cube32_mixed", "np": gg.np, "nst": nst, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": mix_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": mix_gbs / HBM_PEAK_GBS if mix_gbs else None, "traffic": None,
                     "kernel": "k_stencil mixed (FP32 arithmetic, Taylor stage)", "kernel_mean_ms": mean_ms,
                     "launches_timed": cnt,
                     "note": "2 MiB of orbitals stay in L2/MALL: a latency figure, not an HBM one"},
        "errors": report, "timing": timing,
        "mixed_value_pt_orb_H_per_s": tot * 4 * nsteps / (timing["white_noise"]["mixed_ms_per_step"] * nsteps * 1e-3),
        "cpu_baseline": None,
    }


def bench_control(args):
    """Optimal control on the 96^3 cube (h = 0.3, 8 orthonormal packets,
    4 wells, dipole along z, 64 sine coefficients): forward propagation with
    checkpoints every 50 steps, then the checkpointed discrete adjoint; the
    ratio of their times, and dJ/dc against a central difference along a
    random direction."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["cube96_control"])
    n, h, nst, dt = cfg["n"], cfg["h"], cfg["nst"], cfg["dt"]
    nsteps = args.steps if args.steps else cfg["steps"]
    ck = cfg["checkpoint"]
    gg = rsg.Grid(h, n=n)
    pos = gg.positions()
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], box=cfg["well_box"])
    V = synth.well_potential(pos, wells)
    gh = rsg.Hamiltonian(gg, V=torch.from_numpy(V).cuda(), kin=-0.5, dipole_axis=2)
    psi0 = torch.from_numpy(synth.gaussian_packets(cfg["seed"], pos, nst, h)).cuda().t().contiguous()
    coef = torch.from_numpy(synth.laser_coefficients(cfg["seed"], cfg["ncoef"])).cuda()
    psi = psi0.clone()
    rsg.control_forward(gh, psi, dt, min(nsteps, 20), coef, ck)  # warm-up (plans, tiles)
    torch.cuda.synchronize()
    psi = psi0.clone()
    t0 = time.perf_counter()
    J, store = rsg.control_forward(gh, psi, dt, nsteps, coef, ck)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad, gsteps = rsg.control_backward(gh, psi, dt, nsteps, coef, ck, store)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    # a second, untimed backward sweep with a HIP-event pair around every
    # stencil launch (the events would otherwise count in the ratio)
    with rsg.kernel_timing() as kt:
        rsg.control_backward(gh, psi, dt, nsteps, coef, ck, store)
        torch.cuda.synchronize()
    # stencil launches of the backward sweep: per step the 4 product-form
    # stages of the checkpoint recompute (keeping their outputs: 32 B/pt.orb
    # each) and the 4 adjoint factors on the costate, each of which also
    # reads the stage output its pair term needs (48 B/pt.orb each); every
    # launch reads V (8 B/pt)
    per_launch = (4 * 32 + 4 * 48) / 8 * gg.np * nst + 8 * gg.np
    st_gbs = per_launch / (kt.mean_ms * 1e-3) / 1e9 if kt.count else None
    # the whole sweep: 320 B/pt.orb + 64 B/pt per step
    sweep_gbs = (320 * gg.np * nst + 64 * gg.np) * nsteps / bwd / 1e9
    # central difference along a random unit direction d: (J(c+eps d) - J(c-eps d)) / 2 eps
    d = torch.from_numpy(synth.random_unit(cfg["seed"], cfg["ncoef"])).cuda()
    eps = 1e-4 * float(coef.abs().max())
    jp, _ = rsg.control_forward(gh, psi0.clone(), dt, nsteps, coef + eps * d, ck, keep_checkpoints=False)
    jm, _ = rsg.control_forward(gh, psi0.clone(), dt, nsteps, coef - eps * d, ck, keep_checkpoints=False)
    fd = (jp.item() - jm.item()) / (2 * eps)
    ad = float((grad * d).sum())
    log(f"forward {fwd:.3f} s, gradient {bwd:.3f} s, J = {J.item():.10f}, "
        f"d.grad = {ad:.10e}, central FD = {fd:.10e}")
    return {
        "metric": "adjoint grad time/fwd time", "value": bwd / fwd, "unit": "ratio",
        "n_gpus": 1, "steps": nsteps, "warmup": 20, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cube96_control", "np": gg.np, "nst": nst, "dt": dt, "ncoef": cfg["ncoef"],
                   "checkpoint_every": ck},
        "roofline": {"bound": "hbm", "achieved": st_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": st_gbs / HBM_PEAK_GBS if st_gbs else None, "traffic": None,
                     "kernel": "k_stencil in the backward sweep (checkpoint recompute and adjoint stages)",
                     "kernel_mean_ms": kt.mean_ms, "launches_timed": kt.count,
                     "sweep_algorithmic_GBs": sweep_gbs},
        "forward_s": fwd, "gradient_s": bwd, "J": J.item(),
        "forward_value_pt_orb_H_per_s": gg.np * nst * 4 * nsteps / fwd,
        "directional_derivative": ad, "central_fd": fd, "fd_rel_err": abs(ad - fd) / max(abs(fd), 1e-300),
        "cpu_baseline": None,
    }


def bench_cube32(args):
    """The 32^3 harmonic cube (h = 0.3, V = r^2/2, 4 white-noise orbitals):
    10 H*psi calls followed by 10 Taylor(4) steps at dt = 0.01 (50 H
    applications), captured once as a HIP graph and replayed K times.  The
    orbitals (2 MiB) stay in L2/MALL, so the rate is cache-resident, not an
    HBM figure.  (Its parity with the oracle is a test.)"""
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["cube32_ho"])
    n, h, nst, dt = cfg["n"], cfg["h"], cfg["nst"], cfg["dt"]
    torch.cuda.set_device(0)
    gg = rsg.Grid(h, n=n)
    V = synth.harmonic_potential(gg.positions())
    gh = rsg.Hamiltonian(gg, V=torch.from_numpy(V).cuda(), kin=-0.5)
    psi0 = synth.white_noise(cfg["seed"], gg.np, nst, h)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        psi = torch.from_numpy(psi0).cuda().t().contiguous()
        hp = torch.zeros_like(psi)
        ws = torch.empty(gh.workspace_bytes("step", nst, psi.shape[1]), dtype=torch.uint8, device="cuda")

        def seq():
            for _ in range(cfg["hpsi_calls"]):
                rsg.hpsi(gh, psi, out=hp)
            for _ in range(cfg["steps"]):
                rsg.propagate_step(gh, psi, dt, ws=ws)

        # launches of a few microseconds: many repetitions
        tile = choose_tile(args, args.tile, gh, psi, reps=10)
        seq()  # plans and tiles exist before capture
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            seq()
        for _ in range(max(args.warmup, 1)):
            graph.replay()
        torch.cuda.synchronize()
        reps = max(args.steps, 1)
        t0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
    napp = cfg["hpsi_calls"] + 4 * cfg["steps"]
    npo = gg.np * nst
    alg = cfg["hpsi_calls"] * (32 * npo + 8 * gg.np) + cfg["steps"] * (128 * npo + 32 * gg.np)
    return {
        "metric": METRIC, "value": npo * napp / el, "unit": UNIT, "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cube32_ho", "np": gg.np, "nst": nst, "h_bohr": h, "tile": tile,
                   "sequence": "10 hpsi + 10 Taylor(4) steps in one HIP graph (one step of this "
                               "line = one replay of the sequence)"},
        "roofline": {"bound": "hbm", "achieved": alg / el / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / el / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "note": "2 MiB of orbitals stay in L2/MALL: algorithmic bytes over wall time of the "
                             "whole graph, not an HBM measurement"},
        "cpu_baseline": None,
    }


def bench_mixed_sphere(args):
    """Mixed precision on the benchmark system (3.05 M points, 64 orbitals,
    16 wells with projectors): K Taylor(4) steps with FP32 Hamiltonian
    arithmetic on complex64 work buffers (FP64 accumulation), timed beside
    the FP64 path, and the orbital error of the mixed result against the
    FP64 one after the K steps.  The roofline is the mixed stage's: per
    step psi (complex128) is read by the first and the last stage, the
    complex64 work buffers are read three times and written three times,
    and psi is written once, 96 B/pt.orb, plus the FP32 potential (4 B/pt)
    per stage."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["sphere18_wells"])
    torch.cuda.set_device(0)
    gg = rsg.Grid(cfg["h"], R=cfg["R"], align=args.align)
    live = gg.live()
    V, proj = build_sphere_inputs(cfg, gg.positions()[live])
    dev = torch.device("cuda:0")
    nst, dt = cfg["nst"], cfg["dt"]
    Vt, projs, psi0 = place_on_slots(gg, live, V, proj, synth.white_noise(cfg["seed"], gg.npoints, nst, cfg["h"]),
                                     dev)
    gh = rsg.Hamiltonian(gg, V=Vt, kin=-0.5, projectors=projs)
    ws = torch.empty(gh.workspace_bytes("step", nst, psi0.shape[1]), dtype=torch.uint8, device=dev)
    tiles = {"c128": choose_tile(args, args.tile, gh, psi0, reps=2),
             "mixed": choose_tile(args, args.tile_mixed, gh, psi0, reps=2, dtype="mixed")}
    steps = max(args.steps, 1)

    def run(dtype):
        psi = psi0.clone()
        rsg.propagate(gh, psi, dt, max(args.warmup, 1), dtype=dtype, ws=ws)
        psi.copy_(psi0)
        torch.cuda.synchronize()
        with rsg.kernel_timing() as kt:
            t0 = time.perf_counter()
            rsg.propagate(gh, psi, dt, steps, dtype=dtype, ws=ws)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        return psi, el, kt.mean_ms

    full, el64, k64 = run("c128")
    mixed, el32, k32 = run("mixed")
    err = ((mixed - full).abs().pow(2).sum(1).sqrt() / full.abs().pow(2).sum(1).sqrt()).max().item()
    npo = gg.npoints * nst
    alg = (96 * npo + 16 * gg.npoints) / 4.0
    log(f"FP64 {el64 * 1e3 / steps:.3f} ms/step, mixed {el32 * 1e3 / steps:.3f} ms/step, error {err:.2e}")
    return {
        "metric": METRIC, "value": npo * 4 * steps / el32, "unit": UNIT, "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": el32 * 1e3 / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 H / f64 accumulation", "data": "synthetic",
        "config": {"workload": "sphere18_mixed", "np": gg.npoints, "nst": nst, "natoms": cfg["natoms"], "dt": dt,
                   "row_align": gg.align, "tile": tiles["mixed"], "tile_fp64": tiles["c128"]},
        "roofline": {"bound": "hbm", "achieved": alg / (k32 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (k32 * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stencil mixed (FP32 arithmetic, Taylor stage)", "kernel_mean_ms": k32,
                     "algorithmic_bytes_per_launch": alg},
        "fp64_value": npo * 4 * steps / el64, "fp64_stencil_ms": k64,
        "orbital_rel_err_vs_fp64": err,
        "cpu_baseline": None,
    }


def bench_cs(args):
    """Complex scaling.  (1) H_theta applications (kinetic prefactor
    -1/2 e^{-2 i theta}, continued wells potential) to 64 orbitals on the
    3.05 M-point sphere, beside plain H applications, K calls each; the
    roofline is that of the complex-scaled stencil (32 B/pt.orb + 16 B/pt
    for V and V_im).  (2) The harmonic oscillator continued to
    e^{2 i theta} r^2/2 on a 48^3 cube at h = 0.3: the eigenvalues nearest
    4 targets by inverse iteration, against the exact levels 1.5 .. 4.5."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["sphere18_cs"])
    torch.cuda.set_device(0)
    th, nst = cfg["theta"], cfg["nst"]
    gg = rsg.Grid(cfg["h"], R=cfg["R"], align=args.align)
    live = gg.live()
    pos = gg.positions()[live]
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], ball=cfg["well_ball"])
    vz = synth.well_potential_scaled(pos, wells, th)
    vre, vim = np.zeros(gg.np), np.zeros(gg.np)
    vre[live], vim[live] = vz.real, vz.imag
    psi = torch.zeros((nst, gg.np), dtype=torch.complex128, device="cuda")
    psi[:, torch.from_numpy(live).cuda()] = torch.from_numpy(
        synth.white_noise(cfg["seed"], gg.npoints, nst, cfg["h"])).cuda().t()
    gh = rsg.Hamiltonian(gg, V=torch.from_numpy(vre).cuda(), kin=-0.5)
    out = torch.empty_like(psi)
    tile = choose_tile(args, args.tile, gh, psi, reps=2)
    reps = max(args.steps, 1)

    def timed():
        for _ in range(max(args.warmup, 1)):
            rsg.hpsi(gh, psi, out=out)
        torch.cuda.synchronize()
        with rsg.kernel_timing() as kt:
            t0 = time.perf_counter()
            for _ in range(reps):
                rsg.hpsi(gh, psi, out=out)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
        return el, kt.mean_ms

    el_plain, k_plain = timed()
    gh.set_complex_scaling(th, torch.from_numpy(vim).cuda())
    el_cs, k_cs = timed()
    npo = gg.npoints * nst
    alg = 32 * npo + 16 * gg.npoints
    log(f"H {el_plain * 1e3:.3f} ms, H_theta {el_cs * 1e3:.3f} ms (stencil {k_plain:.3f} / {k_cs:.3f} ms)")
    del psi, out
    # (2) scaled oscillator
    n, h = cfg["cube_n"], cfg["cube_h"]
    gc = rsg.Grid(h, n=n)
    r2 = (gc.positions() ** 2).sum(axis=1)
    hc = rsg.Hamiltonian(gc, V=torch.from_numpy(np.cos(2 * th) * r2 / 2).cuda(), kin=-0.5)
    hc.set_complex_scaling(th, torch.from_numpy(np.sin(2 * th) * r2 / 2).cuda())
    targets = np.array(cfg["targets"])
    start = torch.from_numpy(synth.white_noise(cfg["seed"] + 1, gc.np, len(targets), h)).cuda().t().contiguous()
    t0 = time.perf_counter()
    lam, outer = rsg.cs_eigs(hc, start, targets, max_outer=60, tol=1e-10, qmr_maxiter=20000, qmr_tol=1e-11)
    el_eig = time.perf_counter() - t0
    exact = np.array([1.5, 2.5, 3.5, 4.5])
    log(f"scaled oscillator levels {lam} in {el_eig:.2f} s")
    return {
        "metric": "H_theta grid-pt·orbital applications/s", "value": npo / el_cs, "unit": "pt·orb·H/s",
        "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": el_cs * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sphere18_cs", "np": gg.npoints, "nst": nst, "theta": th, "row_align": gg.align,
                   "tile": tile, "potential": "16 wells continued to r e^{i theta}, no projectors",
                   "step": "one H_theta application to the batch"},
        "roofline": {"bound": "hbm", "achieved": alg / (k_cs * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / (k_cs * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stencil complex-scaled (H application)", "kernel_mean_ms": k_cs,
                     "algorithmic_bytes": "32 B/pt·orb + 16 B/pt"},
        "plain_H_value": npo / el_plain, "plain_H_stencil_ms": k_plain,
        "scaled_oscillator": {"grid": f"cube {n}^3, h = {h}", "targets": list(targets),
                              "eigenvalues": [[float(z.real), float(z.imag)] for z in lam],
                              "max_abs_err_vs_exact_levels": float(np.max(np.abs(lam - exact))),
                              "max_abs_imag": float(np.max(np.abs(lam.imag))),
                              "outer_iterations": int(outer.max()), "seconds": el_eig},
        "cpu_baseline": None,
    }


def bench_solve(args):
    """Shifted solves (H + sigma_n) x_n = b_n with QMR (the Sternheimer
    step) on the 5.0e5-point sphere with 16 orbitals, complex shifts
    -eps_n + omega + i eta, to a relative residual of 1e-8; K repeated
    solves from x = 0 after W warm-up solves.  value = pt x orbital x
    iterations per second; roofline over one iteration's algorithmic bytes
    (H application 32 B/pt.orb + 8 B/pt, three fused passes 32 + 64 + 208
    B/pt.orb)."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["sphere500k_qmr"])
    torch.cuda.set_device(0)
    h, R, nst = cfg["h"], cfg["R"], cfg["nst"]
    gg = rsg.Grid(h, R=R, align=args.align)
    live = gg.live()
    pos = gg.positions()[live]
    wells = synth.gaussian_wells(cfg["seed"], cfg["natoms"], ball=cfg["well_ball"])
    V = synth.well_potential(pos, wells)
    proj = synth.kb_projectors(cfg["seed"], pos, wells.centres)
    Vt, projs, b = place_on_slots(gg, live, V, proj, synth.white_noise(cfg["seed"], gg.npoints, nst, h),
                                  torch.device("cuda"))
    gh = rsg.Hamiltonian(gg, V=Vt, kin=-0.5, projectors=projs)
    rng = synth.rng(cfg["seed"], 99)
    eps = rng.uniform(cfg["eps_lo"], cfg["eps_hi"], nst)
    shifts = -eps + cfg["omega"] + 1j * cfg["eta"]
    x = torch.zeros_like(b)
    ws = torch.empty(int(rsg._lib.rsg_solve_workspace_bytes(gh._h, 1, nst, b.shape[1])), dtype=torch.uint8,
                     device="cuda")
    rsg.autotune(gh, b, reps=2)

    def solve():
        x.zero_()
        return rsg.shifted_solve(gh, b, shifts, x=x, method="qmr", tol=cfg["tol"], maxiter=cfg["maxiter"],
                                 check_every=20, ws=ws)

    for _ in range(max(args.warmup, 1)):
        solve()
    torch.cuda.synchronize()
    reps = max(args.steps, 1)
    t0 = time.perf_counter()
    iters = []
    for _ in range(reps):
        _, info = solve()
        iters.append(info["iters"])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    it = np.mean(iters, axis=0)
    hx = rsg.hpsi(gh, x)
    sig = torch.from_numpy(shifts).cuda()[:, None]
    rr = b - hx - sig * x
    rel = (rr.abs().pow(2).sum(1).sqrt() / b.abs().pow(2).sum(1).sqrt()).cpu().numpy()
    # the slowest orbital sets the number of launched iterations; every
    # orbital's passes run until it stops
    pt_orb_iter = gg.npoints * float(np.sum(it))
    alg = pt_orb_iter * 336 + float(np.max(it)) * gg.npoints * 8
    return {
        "metric": "QMR grid-pt·orbital iterations/s", "value": pt_orb_iter / el, "unit": "pt·orb·iter/s",
        "n_gpus": 1, "steps": reps, "warmup": args.warmup, "ms_per_step": el * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sphere500k_qmr", "np": gg.npoints, "nst": nst, "natoms": cfg["natoms"], "row_align": gg.align,
                   "tol": cfg["tol"], "shift": "-eps_n + 0.3 + 0.1i, eps_n ~ U(-0.6, -0.1)",
                   "step": "one full solve from x = 0"},
        "roofline": {"bound": "hbm", "achieved": alg / el / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / el / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "QMR iteration (H application + 3 fused passes)",
                     "algorithmic_bytes": "336 B/pt·orb + 8 B/pt per iteration"},
        "iterations": {"max": int(np.max(it)), "mean": float(np.mean(it)), "min": int(np.min(it))},
        "true_rel_residual_max": float(rel.max()),
        "cpu_baseline": None,
    }


def bench_gridmap(args):
    """Grid-to-memory maps (figure gpu_laplacian): the gather-form
    Laplacian on point-major batches stored in standard, brick and Hilbert
    order, on spheres of 5.0e5 and 3.05e6 points with 1..64 orbitals, timed
    with HIP events over K launches each; beside it the z-marching stencil
    (kinetic term only, orbital-major, autotuned tile) on the same grids."""
    import numpy as np
    import torch

    import paper_1501_05654_amd as rsg
    import synth

    cfg = dict(synth.WORKLOADS["sphere500k_gridmap"])
    torch.cuda.set_device(0)
    reps = max(args.steps, 1)
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg["seed"])

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # one 1 GiB copy: the reference dispatch for scaling HBM traffic counters
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rsg.copy(src, dst)
    torch.cuda.synchronize()
    del src, dst
    grids = []
    best = None
    for R, h in cfg["spheres"]:
        gg = rsg.Grid(h, R=R)
        log(f"grid R={R} h={h}: {gg.np} points")
        maps = {name: rsg.GridMap(gg, kind, param) for name, kind, param in cfg["maps"]}
        orders = {name: m.order() for name, m in maps.items()}
        gh = rsg.Hamiltonian(gg, V=None, kin=-0.5)
        rows = []
        for nst in cfg["nst_list"]:
            x_std = torch.randn(gg.np, nst, dtype=torch.complex128, device="cuda", generator=g)
            ref = None
            entry = {"nst": nst}
            alg = gg.np * nst * 32 + gg.np * 96  # psi read + out written + neighbour table
            for name, m in maps.items():
                idx = torch.from_numpy(orders[name].astype(np.int64)).cuda()
                x = x_std[idx].contiguous()
                out = torch.empty_like(x)
                ms = timed(lambda: m.laplacian(x, out, scale=1.0))
                # every map gives the same values, permuted
                back = torch.empty_like(out)
                back[idx] = out
                if ref is None:
                    ref = back
                diff = float((back - ref).abs().max())
                entry[name] = {"ms": ms, "pt_orb_per_s": gg.np * nst / (ms * 1e-3),
                               "alg_GBs": alg / (ms * 1e-3) / 1e9, "max_abs_diff_vs_standard": diff}
                log(f"  nst={nst:3d} {name:9s} {ms:8.4f} ms")
                del x, out, back
            # the z-marching stencil, kinetic term only (32 B/pt.orb)
            psi = x_std.t().contiguous()
            hp = torch.empty_like(psi)
            rsg.autotune(gh, psi, reps=2)
            ms = timed(lambda: rsg.hpsi(gh, psi, out=hp))
            entry["zmarch_hpsi"] = {"ms": ms, "pt_orb_per_s": gg.np * nst / (ms * 1e-3),
                                    "alg_GBs": gg.np * nst * 32 / (ms * 1e-3) / 1e9}
            log(f"  nst={nst:3d} zmarch    {ms:8.4f} ms")
            for name in maps:
                entry[name]["speedup_vs_standard"] = entry["standard"]["ms"] / entry[name]["ms"]
            rows.append(entry)
            del psi, hp, x_std, ref
            torch.cuda.empty_cache()
        grids.append({"R_bohr": R, "h_bohr": h, "np": gg.np, "results": rows})
        if R == cfg["spheres"][0][0]:
            last = rows[-1]
            name = max(maps, key=lambda k: last[k]["pt_orb_per_s"])
            best = (name, last[name], gg.np, last["nst"])
        del maps, gh
    name, r, npts, nst = best
    return {
        "metric": "Laplacian grid-pt·orbital applications/s", "value": r["pt_orb_per_s"],
        "unit": "pt·orb/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": r["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sphere500k_gridmap", "np": npts, "nst": nst, "best_map": name,
                   "layout": "point-major [np][nst] complex128 in map order"},
        "roofline": {"bound": "hbm", "achieved": r["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["alg_GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_map_lap", "algorithmic_bytes": "32 B/pt·orb + 96 B/pt"},
        "grids": grids,
        "cpu_baseline": None,
    }


def sub_results(args) -> dict:
    """The rest of the metric, measured in the same run: the 32^3 cube's
    50-H sequence in one graph (cache-resident), the 256-system batch, the
    mixed-precision error after 1000 steps, and the optimal-control
    gradient/forward time ratio at full size with its finite-difference
    check.  Each entry is the compact form of that workload's own line."""
    import argparse as _ap
    import gc

    import torch

    def ns(**kw):
        base = dict(vars(args))
        base.update(tile="", tile_mixed="", no_autotune=False, nsys=0)
        base.update(kw)
        return _ap.Namespace(**base)

    def run(name, fn, a):
        t0 = time.perf_counter()
        try:
            r = fn(a)
        finally:
            gc.collect()
            torch.cuda.empty_cache()
        log(f"{name}: {time.perf_counter() - t0:.1f} s")
        return r

    out = {}
    r = run("cube32_ho", bench_cube32, ns(steps=50, warmup=5))
    out["cube32_ho"] = {"value": r["value"], "unit": r["unit"], "ms_per_sequence": r["ms_per_step"],
                        "roofline_frac_cache_resident": r["roofline"]["frac"],
                        "sequence": "10 hpsi + 10 Taylor(4) steps (50 H) in one HIP graph",
                        "tile": r["config"]["tile"]}
    r = run("cube32_mixed", bench_mixed, ns(steps=1000, warmup=0))
    out["cube32_mixed"] = {"steps": r["steps"], "errors_vs_fp64_path": r["errors"],
                           "mixed_ms_per_step": r["timing"]["white_noise"]["mixed_ms_per_step"],
                           "fp64_ms_per_step": r["timing"]["white_noise"]["fp64_ms_per_step"]}
    r = run("cube96_control", bench_control, ns(steps=0, warmup=0))
    out["cube96_control"] = {"adjoint_ratio": r["value"], "unit": "gradient time / forward time",
                             "forward_s": r["forward_s"], "gradient_s": r["gradient_s"], "steps": r["steps"],
                             "checkpoint_every": r["config"]["checkpoint_every"], "ncoef": r["config"]["ncoef"],
                             "fd_rel_err": r["fd_rel_err"], "directional_derivative": r["directional_derivative"],
                             "central_fd": r["central_fd"],
                             "sweep_algorithmic_GBs": r["roofline"]["sweep_algorithmic_GBs"]}
    # one tile per size class, timed per class on this workload: 16x16 at
    # depth 2 for the narrowest and widest classes, 8x8 at depth 2 for the
    # middle one (fixed, so that the line can carry the committed counter
    # summary's traffic for exactly these tiles)
    r = run("batch256", bench_batch, ns(steps=10, warmup=2, align=8,
                                        tile="1,16,16,0,2,0,0,0;1,8,8,0,2,0,0,0;1,16,16,0,2,0,0,0"))
    out["batch256"] = {"value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
                       "stencil_stage_ms": r["roofline"]["stage_ms"], "roofline_frac": r["roofline"]["frac"],
                       "traffic_per_stage": r["roofline"]["traffic"],
                       "traffic_over_algorithmic": (r["roofline"]["traffic"] / (32.0 * r["config"]["sum_np_nst"])
                                                    if r["roofline"]["traffic"] else None),
                       "sum_np_nst": r["config"]["sum_np_nst"], "class_tiles": r["config"]["class_tiles"],
                       "class_sizes": r["config"]["class_sizes"],
                       "per_system_eager_value": r["per_system_eager_value"]}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere18_wells",
                    choices=["sphere18_wells", "batch256", "cube32_mixed", "cube96_control", "cube32_ho",
                             "sphere500k_gridmap", "sphere500k_qmr", "sphere18_cs", "sphere18_mixed"])
    ap.add_argument("--nsys", type=int, default=0, help="batch256: use only the first N systems")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sub", action="store_true",
                    help="sphere18_wells: skip the other workloads' figures (cube32_ho sequence, "
                         "cube32_mixed error, cube96_control gradient ratio, batch256)")
    ap.add_argument("--align", type=int, default=0,
                    help="sphere workloads (sphere18_wells, sphere18_mixed, sphere18_cs, sphere500k_qmr, "
                         "batch256): row alignment of the grids' storage (1 = compact rows; default 8, "
                         "16 for sphere18_mixed, whose complex64 work buffers need 16 slots per "
                         "128-byte line, and 1 for sphere500k_qmr)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default tile shape instead of timing the candidates")
    ap.add_argument("--tile", default="",
                    help="B,TX,TY,ZC,PD,PT,BO[,ZM]: use this stencil tile instead of autotuning "
                         "(sphere18_wells, batch256 (PT and BO ignored; there also one tile per size class, "
                         "';'-separated), cube32_ho, sphere18_cs, and the FP64 steps of sphere18_mixed)")
    ap.add_argument("--tile-mixed", default="",
                    help="sphere18_mixed: the same for the FP32 stencil of the mixed steps")
    args = ap.parse_args()
    if args.align <= 0:
        # measured per workload: the QMR passes are pointwise over all slots,
        # so dead slots cost them more than aligned rows gain the stencil
        args.align = {"sphere18_mixed": 16, "sphere500k_qmr": 1}.get(args.workload, 8)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the path shards over orbitals or systems "
              "with no exchange, and the benchmark measures one GPU's share only "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch256":
        out = bench_batch(args)
    elif args.workload == "cube32_mixed":
        out = bench_mixed(args)
    elif args.workload == "cube96_control":
        out = bench_control(args)
    elif args.workload == "cube32_ho":
        out = bench_cube32(args)
    elif args.workload == "sphere500k_gridmap":
        out = bench_gridmap(args)
    elif args.workload == "sphere500k_qmr":
        out = bench_solve(args)
    elif args.workload == "sphere18_cs":
        out = bench_cs(args)
    elif args.workload == "sphere18_mixed":
        out = bench_mixed_sphere(args)
    else:
        out, cfg = bench_sphere(args)
        out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(cfg, args.cpu_seconds)
        if not args.no_sub:
            out["sub"] = sub_results(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
