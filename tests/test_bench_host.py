"""Host-side logic of bench.py's roofline object (no GPU): the algorithmic
byte counts per kernel, the choice of the dominant gather kernel, and the
traffic summary's source check."""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


N, S, D = 1_000_000, 100_000_000, 20
E, SPK = 700_000.0, 7_000.0


def test_byte_counts(bench):
    # 8-byte pairs read from the table and written to the bucket, two 4-byte
    # run offsets per spike and delay
    assert bench.events_bytes(E, SPK, D) == 16 * E + 8 * SPK * D
    # row pointers 8 B, background count 2 B, gates 32 B per row, weights
    assert bench.rows_bytes(N, E, 4) == 42 * N + 4 * E
    assert bench.rows_bytes(N, E, 2) == 42 * N + 2 * E
    # the pull method: index + delay per synapse, weights, state, bitmaps
    assert bench.step_bytes(S, N, D, E, 4) == 5 * S + 4 * E + 44 * N + N * (D + 1) / 8
    assert bench.gather_bytes(S, N, D) == 5 * S + N * (D + 1) / 8


@pytest.mark.parametrize("t_gather,t_events", [(0.30, 0.20), (0.20, 0.30)])
def test_spike_driven_roofline_reports_the_longer_kernel(bench, t_gather, t_events):
    per = {"gather": t_gather, "events": t_events, "sums": 0.0}
    r = bench.roofline(per, 0.8, S, N, D, E, SPK, 4)
    consumer = 4 * E + bench.rows_bytes(N, E, 4)
    bucketing = bench.events_bytes(E, SPK, D)
    main, other, key = (("k_gather", "k_events", "bucketing") if t_gather > t_events
                        else ("k_events", "k_gather", "consumer"))
    assert r["kernel"] == main and r["delivery"] == "spike-driven" and r["bound"] == "hbm"
    B, t = (consumer, t_gather) if main == "k_gather" else (bucketing, t_events)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(B)
    assert r["avg_launch_ms"] == t
    assert r["achieved"] == pytest.approx(B / (t * 1e-3) / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r[key]["kernel"] == other
    assert r["step"]["pull_method_bytes"] == pytest.approx(bench.step_bytes(S, N, D, E, 4))


def test_sweep_roofline_fused_and_separate_sums(bench):
    fused = bench.roofline({"gather": 1.0, "events": 0.0, "sums": 0.0}, 2.0, S, N, D, E, SPK, 4)
    assert fused["kernel"] == "k_gather" and fused["delivery"] == "sweep"
    assert fused["algorithmic_bytes_per_launch"] == pytest.approx(
        bench.gather_bytes(S, N, D) + bench.rows_bytes(N, E, 4))
    assert "bucketing" not in fused and "sums" not in fused
    split = bench.roofline({"gather": 1.0, "events": 0.0, "sums": 0.5}, 2.0, S, N, D, E, SPK, 4)
    assert split["algorithmic_bytes_per_launch"] == pytest.approx(bench.gather_bytes(S, N, D) + S / 8)
    assert split["sums"]["algorithmic_bytes_per_launch"] == pytest.approx(bench.rows_bytes(N, E, 4) + S / 8)


def test_traffic_is_null_once_the_kernel_sources_change(bench, tmp_path, monkeypatch):
    src = [tmp_path / "k.hip", tmp_path / "k.h"]
    src[0].write_bytes(b"kernels")
    src[1].write_bytes(b"constants")
    h = hashlib.sha256(b"kernels" + b"constants").hexdigest()
    tj = tmp_path / "traffic.json"
    tj.write_text(json.dumps({"kernel_source_sha256": h,
                              "per_launch": {"k_gather": {"read_bytes": 3.0, "write_bytes": 4.0}}}))
    monkeypatch.setattr(bench, "KERNEL_SRCS", [str(p) for p in src])
    monkeypatch.setitem(bench.TRAFFIC_JSON, "spike-driven", str(tj))
    assert bench.measured_traffic("k_gather", "spike-driven") == 7.0
    assert bench.measured_traffic("k_events", "spike-driven") is None   # not in the summary
    src[1].write_bytes(b"constants, changed")
    assert bench.measured_traffic("k_gather", "spike-driven") is None
