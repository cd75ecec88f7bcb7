"""bench.py's command line on the CPU: the one-GPU contract (no GPU needed,
nothing is launched)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120, env=env)


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in ("2", "8"):
        r = _bench("--gpus", n)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""              # no JSON line for a run that did not happen


def test_a_multi_rank_launch_is_refused():
    env = dict(os.environ, WORLD_SIZE="2", RANK="1", LOCAL_RANK="1")
    r = _bench(env=env)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
