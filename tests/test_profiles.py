"""The committed rocprofv3 summaries match the code they describe: every
traffic summary of the benchmark's stencil was taken on the current
stencil source, names its tile and row alignment, and bench.py finds its
HBM bytes for that tile; the kernel-statistics summary lists the stencil."""
import glob
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kv(path):
    kv = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_summaries_are_used_only_when_current():
    """bench.py reports a summary's HBM bytes only for the stencil source,
    tile and row alignment it was taken on; a summary of an older source is
    never used."""
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_stencil_sphere18_wells_*.txt")))
    assert paths
    for p in paths:
        kv = _kv(p)
        B, TX, TY, ZC, PD, PT, BO, ZM = (int(v) for v in kv["tile"].split(","))
        tile = dict(B=B, TX=TX, TY=TY, ZC=ZC, PD=PD, PT=PT, BO=BO, ZM=ZM)
        got = bench.read_traffic("sphere18_wells", tile, int(kv.get("row_align", "1")))
        if kv["stencil_source_sha256"] == bench.stencil_source_hash():
            assert got == float(kv["hbm_bytes_per_launch"]), p
            assert 1.0 < got / float(kv["algorithmic_bytes_per_launch"]) < 3.0, p
        else:
            assert got is None or got != float(kv["hbm_bytes_per_launch"]), p


def test_kernel_statistics_list_the_stencil():
    text = open(os.path.join(ROOT, "profiles", "kernel_stats_sphere18_wells.txt")).read()
    assert "k_stencil<" in text and "rocprofv3 --kernel-trace --stats" in text


def test_every_workload_has_kernel_statistics():
    for w in ["sphere18_wells", "batch256", "sphere18_mixed", "sphere18_cs", "cube32_ho", "cube96_control",
              "qmr_sphere500k"]:
        text = open(os.path.join(ROOT, "profiles", f"kernel_stats_{w}.txt")).read()
        assert "rocprofv3 --kernel-trace --stats" in text and "bench.py" in text, w
        assert "k_stencil" in text, w


def test_batch_traffic_summary_is_consistent():
    """The batched stencil's counter summary adds its stage's fetch and
    write bytes, names its tile (or one per size class), and (when taken on the current source)
    reports more bytes than the algorithmic 32 B per point-orbital."""
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_stencil_batch256_*.txt")))
    assert paths
    for p in paths:
        kv = _kv(p)
        assert all(len(t.split(",")) == 8 for t in kv["tile"].split(";")), p
        hbm = float(kv["hbm_bytes_per_stage"])
        parts = float(kv["stage_fetch_bytes"]) + float(kv["stage_write_bytes"])
        assert abs(hbm - parts) <= 1e-3 * hbm, p
        assert abs(float(kv["algorithmic_bytes_per_stage"]) - 688438342 * 32.0) <= 1e-4 * 688438342 * 32.0, p
        if kv["stencil_source_sha256"] == bench.stencil_source_hash():
            assert 1.0 < hbm / float(kv["algorithmic_bytes_per_stage"]) < 4.0, p
