"""bench.py's command-line contract on the CPU: the library has no multi-GPU
path, so more than one GPU (by flag or by a launcher's WORLD_SIZE) ends the
run with status 2 and a message before anything is measured; the host
memory threshold below which the default run measures the AMR workload
instead of the light cone is the one the large-tree tests use."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_exits_with_status_2():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_launcher_world_size_exits_with_status_2():
    r = _run([], {"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_memory_threshold_matches_the_large_tests():
    def load(name, path):
        spec = importlib.util.spec_from_file_location(name, path)
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        return m
    b = load("bench_cli_probe", os.path.join(ROOT, "bench.py"))
    t = load("large_cli_probe", os.path.join(ROOT, "tests", "test_gpu_large.py"))
    assert b.LARGE_NEED_GIB == t.NEED_GIB
    assert b.host_available_gib() > 0
