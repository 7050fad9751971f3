"""bench.py's roofline bookkeeping on the CPU: the far-sum kernel with the most time per timed
solve is reported as `roofline`, each kernel against the peak of its precision with its
algorithmic flops per pair, and an HBM traffic record is used only while the kernel's sources
still hash to the value the record was taken with."""
import json
import os

import bench

PPL = 1.557114624e12


def _infos(ms_fused, ms_trac, ms32, fmm):
    return [dict(ms_fused=ms_fused, n_fused=1, ms_traction=ms_trac, n_traction=1, ms_traction32=ms32,
                 n_traction32=33, fmm_applies=33 if fmm else 0) for _ in range(2)]


def test_the_kernel_with_most_time_is_the_roofline():
    r = bench._rooflines(_infos(1720.0, 1200.0, 420.0, True), PPL, "dense4000")
    assert [x["kernel"] for x in r] == ["k_far_ts (float64 traction + Stokeslet)", "k_far<double, traction>"]
    top = r[0]
    assert top["flops_per_pair"] == 58 and top["peak"] == bench.FP64_PEAK_TFLOPS
    assert abs(top["achieved"] - 58 * PPL / 1.72 / 1e12) < 1e-9 * top["achieved"]
    assert abs(top["frac"] - top["achieved"] / 78.6) < 1e-12
    # direct float32 inner sums: their kernel enters against the float32 peak
    r = bench._rooflines(_infos(0.47, 0.33, 2.0 * 33 / 12, False), 392491008.0, "random64")
    assert r[0]["kernel"] == "k_far<float, traction>" and r[0]["peak"] == bench.FP32_PEAK_TFLOPS


def test_traffic_records_follow_the_kernel_sources(tmp_path, monkeypatch):
    for name, _, _, _, _, files in bench.FAR_KERNELS[:2]:
        t = bench._traffic(name, "dense4000", files)
        assert t is not None and t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    # a record whose source hash no longer matches is ignored
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "traffic_dense4000.json")))
    rec["source_sha256"] = "0" * 64
    (prof / "traffic_dense4000.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_1606_07428_amd").symlink_to(os.path.join(os.path.dirname(os.path.abspath(bench.__file__)),
                                                                "paper_1606_07428_amd"))
    name, _, _, _, _, files = bench.FAR_KERNELS[1]
    assert bench._traffic(name, "dense4000", files) is None
