"""The benchmark's command-line contract on the host (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""  # no JSON line for a configuration that was not measured


class _Ctx:
    """Records the schedule settings the tuner makes."""

    def __init__(self):
        self.share, self.fork = None, None

    def set_near_share(self, s):
        self.share = s

    def set_fork(self, f):
        self.fork = f


def _tune(times, near_share=-1, fork=-2):
    import argparse
    sys.path.insert(0, ROOT)
    import bench
    ctx = _Ctx()
    a = argparse.Namespace(near_share=near_share, fork=fork)
    got = bench.tune_schedule(ctx, a, lambda s, f: times[(s, f)], 1.0, "test")
    assert (ctx.share, ctx.fork) == got  # the choice is left set on the context
    return got


def test_schedule_tuner_keeps_an_earlier_candidate_within_the_noise():
    import bench
    cands = bench.SCHEDULE_CANDIDATES
    times = {c: 1.0 for c in cands}
    times[cands[1]] = 0.9
    times[cands[2]] = 0.899  # faster, but by less than 0.5%
    assert _tune(times) == cands[1]
    times[cands[3]] = 0.85  # clearly faster
    assert _tune(times) == cands[3]


def test_schedule_tuner_respects_given_settings():
    import bench
    times = {c: 1.0 for c in bench.SCHEDULE_CANDIDATES}
    assert _tune(times, near_share=5) == (5, -1)
    assert _tune(times, near_share=5, fork=0) == (5, 0)
    shares = sorted({s for s, _ in bench.SCHEDULE_CANDIDATES})
    times = {(s, 0): 1.0 - 0.1 * i for i, s in enumerate(shares)}
    assert _tune(times, fork=0) == (shares[-1], 0)
