"""The benchmark's command line on the host: it refuses more than one GPU
(by flag or by a multi-rank launch) before touching a device, and its help
lists every workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=env, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_multi_rank_launch_is_refused():
    r = _run([], {"WORLD_SIZE": "2", "RANK": "0"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_workloads():
    r = _run(["--help"])
    assert r.returncode == 0
    for w in ("c1", "c2", "c3", "c4", "c5", "loc", "cycle"):
        assert w in r.stdout


def test_form_spec_parses_panel_width():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.form_spec("mixed_f32@64") == ("mixed_f32", 64)
    assert bench.form_spec("blocked_f64") == ("blocked_f64", 0)
    assert all(bench.form_spec(f)[0] in bench.FORMS for f in bench.DEFAULT_FORMS["c3"])
