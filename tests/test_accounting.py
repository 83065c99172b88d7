"""The byte and multiply-add accounting used to price the GPU kernels,
checked against the figures the paper prints for N = 500,000 (Section 6)."""
import json
import os

from paper_2606_27280_amd import accounting as acc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cost_model_matches_paper_figures():
    g = json.load(open(os.path.join(GOLDEN, "cost_model.json")))
    n, d = g["n"], g["d"]
    for k, b in g["major_bytes"].items():
        assert acc.major_bytes(n, int(k)) == b
    for k, b in g["minor_bytes"].items():
        assert acc.minor_bytes(n, int(k), d) == b
    assert acc.full_bytes(n, d) == g["full_bytes"]
    assert acc.score_buffer_bytes(n) == g["score_buffer_bytes"]
    for frac, cnt in g["phase2_entries"].items():
        assert round(float(frac) * n) == cnt
    assert acc.macs_full(n, d) == g["flops_full"]
    for k, f in g["flops_phase1"].items():
        assert acc.macs_phase1(n, int(k)) == f
    assert acc.macs_phase2(round(0.004 * n), 16, d) == g["flops_phase2_full_eval_k16_0.004"]
    assert acc.macs_phase2(33000, 8, d) == g["flops_phase2_k8_33000_entries"]
    pred = acc.macs_full(n, d) / (acc.macs_phase1(n, 8) + acc.macs_phase2(33000, 8, d))
    assert abs(pred - g["predicted_speedup_k8_halfdome"]) < 0.05
    assert acc.full_bytes(n) / acc.major_bytes(n, 16) == g["bandwidth_ratio_k16"]
    assert acc.full_bytes(n) / acc.major_bytes(n, 8) == g["bandwidth_ratio_k8"]


def test_gpu_counts():
    assert acc.scan_flops(10000, 1 << 20, 16) == 2 * 10000 * (1 << 20) * 16
    assert acc.bruteforce_flops(10000, 1 << 20) == 8 * acc.scan_flops(10000, 1 << 20, 16)
    assert acc.rescore_bytes(3) == 3 * 512
    assert acc.scan_stream_bytes(1 << 20, 16, 4) == 64 << 20
