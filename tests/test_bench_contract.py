"""Host-side checks of the benchmark script's contract (no GPU needed)."""
import json
import os
import subprocess
import time
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_fields():
    pairs = 131072.0 ** 2
    r = bench.roofline("gravity", pairs, 5.0, "k", traffic=123)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["traffic"] == 123
    # The published FP32 vector peak, 20 flop per gravity pair (the paper's count).
    assert r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(pairs * 20 / 5e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    # The issue model beside it: 17 slots per pair at 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz.
    im = r["issue_model"]
    assert im["peak_pairs_per_s"] == pytest.approx(256 * 4 * 32 * 2.4e9 / 17)
    assert im["frac"] == pytest.approx(pairs / 5e-3 / im["peak_pairs_per_s"])
    for kind, slots in (("jerk", 31), ("adjoint", 35)):
        assert bench.peak_pairs(kind) == pytest.approx(256 * 4 * 32 * 2.4e9 / slots)
    f = bench.fractions("adjoint", pairs, 5.0)
    assert f["frac"] == pytest.approx(pairs * 45 / 5e-3 / 157.3e12)


def test_default_line_lists_every_configuration():
    # The default run adds one compact entry per configuration of the workload set.
    assert set(bench.CONFIG_WORKLOADS) == {"plummer_2048", "stress_1m", "clusters_2048",
                                           "adjoint_16384"}
    body = {"config": {"workload": "w", "step": "s"}, "ms_per_step": 1.0, "value": 2.0,
            "roofline": bench.roofline("gravity", 1e6, 1.0, "k"),
            "modes": {"comp": {"value": 2.0, "errors": {"acc_rel_rms": 1e-8}}},
            "cpu_baseline": {"sample": "all"}, "error_split": {"none": {}}}
    c = bench.compact(body)
    assert c["pairs_per_s"] == 2.0 and c["roofline_frac"] == body["roofline"]["frac"]
    assert c["issue_frac"] == body["roofline"]["issue_model"]["frac"]
    assert c["modes"]["comp"] == {"errors": {"acc_rel_rms": 1e-8}} and "error_split" in c


def test_cpu_model_is_reported():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_committed_traffic_matches_the_current_sources():
    # The counter summary of the pair kernel carries the hash of the kernel sources and
    # launch shape it was measured with; the bench reports its traffic only while they match.
    text = open(bench.TRAFFIC_SUMMARY).read()
    rec = json.loads(text.split("<!-- traffic: ")[1].split(" -->")[0])
    assert rec["bytes_per_launch"] > 0
    if rec["sources_hash"] == bench.sources_hash():
        assert bench.committed_traffic() == rec["bytes_per_launch"]
    else:
        assert bench.committed_traffic() is None


def test_sources_hash_ignores_comments_only():
    src = 'x = a / b; // u m / eps\n/* block\n comment */ s = "//kept"; c = \'/\';\n'
    assert bench.code_text(src) == bench.code_text(src.replace("u m / eps", "A u (m / eps)"))
    assert bench.code_text(src) != bench.code_text(src.replace("a / b", "a * b"))
    assert '"//kept"' in bench.code_text(src)


def test_warm_up_fills_its_time_budget_or_the_given_count():
    class FakeCuda:
        @staticmethod
        def synchronize():
            pass

    class FakeTorch:
        cuda = FakeCuda

    calls = []

    def call():
        calls.append(1)
        time.sleep(0.01)

    k = bench.warm_up(FakeTorch, call, None)
    assert k == len(calls) and bench.WARMED[-1] == k
    assert k >= 2 and 0.8 * bench.WARM_SECONDS <= 0.01 * k <= 2.0 * bench.WARM_SECONDS
    calls.clear()
    assert bench.warm_up(FakeTorch, call, 3) == 3 and len(calls) == 3
    assert bench.warm_up(FakeTorch, call, 0) == 0


def test_symmetric_flag_is_parsed_and_off_by_default():
    # The default line measures the library's default engine; --symmetric asks for the
    # opt-in symmetric engine on the N = 131072 workload.
    assert bench.parse([]).symmetric is False
    assert bench.parse(["--symmetric"]).symmetric is True
