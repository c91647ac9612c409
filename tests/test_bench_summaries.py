"""The benchmark's rocprofv3 summarizers, which write the tables and the traffic summary under
profiles/, on small synthetic inputs of rocprofv3's CSV layouts (CPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_kernel_short_names():
    assert bench.kernel_short_name(
        "void phx::(anonymous namespace)::back_kernel<false, true, 2>(phx::DevParams const*, int)"
    ) == "back_kernel<false, true, 2>"
    assert bench.kernel_short_name("phx::(anonymous namespace)::bucket_scan(unsigned int const*)") \
        == "bucket_scan"


def test_summarize_stats_sums_calls_and_durations(tmp_path):
    p = tmp_path / "kt_kernel_stats.csv"
    p.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage"\n'
                 '"void k::front_kernel<false, false>(int)","4","8000000","2000000","80"\n'
                 '"void k::back_kernel<false, false, 0>(int)","2","2000000","1000000","20"\n')
    lines = bench.summarize_stats(str(p)).splitlines()
    assert lines[1].split()[:2] == ["front_kernel<false,", "false>"]
    front = lines[1].split()
    assert front[-4:] == ["4", "2.0000", "8.00", "80.00"]
    assert lines[2].split()[-4:] == ["2", "1.0000", "2.00", "20.00"]


def _counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},"{k}",{c},{v}\n')


def test_summarize_pmc_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    k = "void phx::front_kernel<false, false>(int)"
    _counters(tmp_path / "f", [(k, "FETCH_SIZE", 100.0), (k, "FETCH_SIZE", 300.0)])
    _counters(tmp_path / "w", [(k, "WRITE_SIZE", 50.0), (k, "WRITE_SIZE", 50.0)])
    copy = "__amd_rocclr_copyBuffer"
    _counters(tmp_path / "cf", [(copy, "FETCH_SIZE", 524288.0), ("fill", "FETCH_SIZE", 1.0)])
    _counters(tmp_path / "cw", [(copy, "WRITE_SIZE", 1048576.0), ("fill", "WRITE_SIZE", 1048576.0)])
    out = tmp_path / "pmc.json"
    table = bench.summarize_pmc([str(tmp_path / "f"), str(tmp_path / "w")],
                                [str(tmp_path / "cf"), str(tmp_path / "cw")], 1e9, str(out))
    d = json.loads(out.read_text())
    assert d["calibration"]["copy_kernel"] == copy
    assert d["calibration"]["fetch_factor"] == 2.0 and d["calibration"]["write_factor"] == 1.0
    # per dispatch: FETCH 200 KiB x 2 + WRITE 50 KiB x 1
    assert d["hbm_bytes_per_launch"]["front_kernel<false, false>"] == (200 * 2 + 50) * 1024
    assert d["kernel_hash"] == bench.kernel_hash() and d["photons"] == 1000000000
    assert "front_kernel<false, false>" in table
    # the benchmark reads the summary back by kernel name when the hash matches
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(out))
    assert bench.traffic_from_profiles(1000000000, "front_kernel") == (200 * 2 + 50) * 1024
    assert bench.traffic_from_profiles(1000000000, "back_kernel") is None
    assert bench.traffic_from_profiles(5, "front_kernel") is None


def test_per_class_seconds_prices_each_class():
    rates = {"fma": 1e12, "div": 1e11, "sqrt": 5e10, "exp": 1e10, "log": 1e10, "sin": 1e10,
             "div_refined": 2e11, "sqrt_refined": 1e11}
    ops = {"add": 1e12, "mul": 1e12, "div": 2e11, "sqrt": 1e11, "trans": 1e10}
    # (add + mul) / (2 fma) + div / faster div + sqrt / faster sqrt + trans / harmonic mean
    assert abs(bench.per_class_seconds(ops, rates) - (1.0 + 1.0 + 1.0 + 1.0)) < 1e-12


def test_launch_shape_parses_widths_and_an_optional_chunk_size():
    import pytest
    assert bench.launch_shape("16,48,2") == dict(generate_blocks_per_cu=16, front_blocks_per_cu=48,
                                                 back_blocks_per_cu=2)
    assert bench.launch_shape("16,64,3,24") == dict(generate_blocks_per_cu=16,
                                                    front_blocks_per_cu=64,
                                                    back_blocks_per_cu=3, chunk_log2=24)
    for bad in ("16,48", "1,2,3,4,5"):
        with pytest.raises(SystemExit):
            bench.launch_shape(bad)
