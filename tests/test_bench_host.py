"""Host logic of the benchmark, on the CPU: the log-log interpolation behind
the fixed-relMSE and equal-time comparisons, the relative MSE, the
comment-insensitive hash of the walk-kernel sources that keys the committed
counter summaries (and that those summaries match the sources in the tree),
and the one-GPU guard of the command line."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("p", [0.5, 1.0, 2.0])
def test_interp_loglog_is_exact_on_power_laws(p):
    """An error curve y = 3 t^-p is a straight line on log-log axes, so the
    time at which it reaches y* is (3 / y*)^(1/p) wherever y* is bracketed."""
    ts = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    ys = 3.0 * ts ** -p
    for y_star in (3.0 * 1.5 ** -p, 3.0 * 5.0 ** -p, 3.0 * 16.0 ** -p):
        t = bench._interp_loglog(ts, ys, y_star)
        assert t == pytest.approx((3.0 / y_star) ** (1.0 / p), rel=1e-12)


def test_interp_loglog_extrapolates_as_one_over_t():
    """A curve that never reaches y* is continued from its last point as
    error ~ 1/t; one that starts below y* is continued back from its first."""
    ts, ys = [1.0, 2.0], [1.0, 0.8]
    assert bench._interp_loglog(ts, ys, 0.1) == pytest.approx(2.0 * 0.8 / 0.1, rel=1e-12)
    assert bench._interp_loglog(ts, ys, 2.0) == pytest.approx(1.0 * 1.0 / 2.0, rel=1e-12)


def test_interp_loglog_takes_the_first_crossing_of_a_noisy_curve():
    """relMSE curves of heavy-tailed estimators are not monotone: the time
    reported is that of the first bracket that contains y*."""
    ts = [1.0, 2.0, 3.0, 4.0]
    ys = [4.0, 1.0, 3.0, 0.5]
    t = bench._interp_loglog(ts, ys, 2.0)
    assert 1.0 < t < 2.0
    assert t == pytest.approx(np.exp(np.log(2.0) * (np.log(2.0) - np.log(4.0)) / (np.log(1.0) - np.log(4.0))), rel=1e-12)


def test_value_at_inverts_interp_loglog():
    rng = np.random.default_rng(7)
    ts = np.cumsum(rng.uniform(0.5, 2.0, 12))
    ys = np.sort(rng.uniform(0.05, 5.0, 12))[::-1]
    for y_star in np.linspace(ys[-1] * 1.001, ys[0] * 0.999, 9):
        t = bench._interp_loglog(ts, ys, y_star)
        assert bench._value_at(ts, ys, t) == pytest.approx(y_star, rel=1e-9)
    # beyond the ends: error ~ 1/t from the nearest point
    assert bench._value_at(ts, ys, 2 * ts[-1]) == pytest.approx(ys[-1] / 2, rel=1e-12)
    assert bench._value_at(ts, ys, ts[0] / 4) == pytest.approx(ys[0] * 4, rel=1e-12)


def test_rel_mse_is_the_mean_relative_squared_error():
    est = np.array([1.0, 3.0, -2.0])
    exact = np.array([1.0, 2.0, -1.0])
    assert bench.rel_mse(est, exact, delta=0.0) == pytest.approx((0.0 + 0.25 + 1.0) / 3, rel=1e-15)
    # delta keeps points where u vanishes from dominating
    assert bench.rel_mse(np.array([0.1]), np.array([0.0]), delta=1e-2) == pytest.approx(1.0, rel=1e-12)


def _hash_of_tree(root):
    saved = bench.ROOT
    try:
        bench.ROOT = root
        return bench.walk_sources_sha256()
    finally:
        bench.ROOT = saved


def test_source_hash_ignores_comments_and_blank_space_only(tmp_path):
    """Counter summaries stay valid across comment edits of the walk-kernel
    sources and go stale on any change of the code or its build flags."""
    csrc = tmp_path / "paper_2410_18944_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = os.path.join(ROOT, "paper_2410_18944_amd", "csrc")
    for f in bench.WALK_SOURCES:
        shutil.copy(os.path.join(src, f), os.path.join(str(csrc), f))
    h0 = _hash_of_tree(str(tmp_path))
    assert h0 == bench.walk_sources_sha256()
    walk = csrc / "walk.hip"
    text = walk.read_text()
    walk.write_text("// a new leading comment\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n", 3))
    build = csrc / ".." / "build.py"
    build.write_text(build.read_text() + "\n# a trailing comment\n")
    assert _hash_of_tree(str(tmp_path)) == h0
    walk.write_text(text.replace("kDefaultPoolSlots[2] = {384, 1536}", "kDefaultPoolSlots[2] = {384, 1024}", 1))
    assert _hash_of_tree(str(tmp_path)) != h0


@pytest.mark.parametrize("workload", ["c5", "c4", "c3"])
def test_committed_counter_summaries_match_the_walk_sources(workload):
    """Each workload's committed rocprofv3 summary was taken on the walk
    kernel built from these sources, so the bench reports its measured
    traffic and VALU figures rather than falling back."""
    rec = bench.measured_traffic(workload)
    assert rec is not None, "counter summary %s is stale" % bench.COUNTER_PROFILES[workload]
    assert rec["bound"] == "alu"
    assert rec["hbm_bytes_per_launch"] > 0 and rec["valu_insts_per_launch"] > 0
    assert rec["launch_ms"] > 0 and rec["steps_per_launch"] > 0


def test_bench_measures_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
