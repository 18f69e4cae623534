"""bench.py's command-line contract on the CPU: it measures one GPU, so a
request for more (flag or launcher environment) exits with status 2 and
says so, before touching any device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=env, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_a_multi_rank_launch_is_refused():
    r = _run([], {"WORLD_SIZE": "4", "RANK": "0", "LOCAL_RANK": "0"})
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_help_names_the_workloads():
    r = _run(["--help"])
    assert r.returncode == 0
    for w in ("sphere18_wells", "batch256", "cube96_control", "cube32_ho", "sphere18_mixed"):
        assert w in r.stdout


def test_batch_tiles_one_or_one_per_class():
    """batch256 --tile: one tile for every size class, or one per class
    separated by ';'; each tile takes its ZM default and a malformed one
    stops the run."""
    import pytest

    import bench

    assert bench.class_tiles_spec("1,16,16,0,2,0,0,0") == [[1, 16, 16, 0, 2, 0, 0, 0]]
    assert bench.class_tiles_spec("1,16,16,0,2,0,0;1,8,8,0,2,0,0,0") == [[1, 16, 16, 0, 2, 0, 0, 0],
                                                                         [1, 8, 8, 0, 2, 0, 0, 0]]
    with pytest.raises(SystemExit):
        bench.class_tiles_spec("1,16,16;1,8,8,0,2,0,0,0")
