"""bench.py's command line on the host: more than one GPU is refused with a
message (the step is not sharded across GPUs), and the launch window of the
timed steps is the one the profile sets are keyed by."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_profile_sets_cover_the_default_and_the_short_command():
    import bench
    old = sys.argv
    try:
        windows = []
        for argv in (["bench.py"], ["bench.py", "--gpus", "1", "--steps", "20", "--warmup", "5"]):
            sys.argv = argv
            args = bench.parse()
            windows.append((args.warmup + 1, args.warmup + args.steps))
    finally:
        sys.argv = old
    assert windows == [(11, 110), (6, 25)]
    from paper_1304_7126_amd import profiling
    for prefix in (bench.PROFILE, bench.PROFILE_TRANSPORT):
        got = sorted(tuple(profiling.read_figures(c + "_kernel_stats.md")["window"]) for c in bench.PROFILE_SETS[prefix])
        assert got == sorted(windows)
