"""Host logic of bench.py that needs no GPU: the aggregation of rocprofv3
counter rows into per-launch HBM traffic, and the rule that a traffic figure
is only reported for the kernel source and workload it was measured on."""
import csv
import json
import os

import pytest

import bench


def write_rows(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


@pytest.fixture
def traffic_file(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    return f


def test_pmc_summarize_per_launch_bytes(tmp_path, traffic_file):
    fetch = [("void kh::k_ms_pull<16>(int, int const*)", 100.0), ("void kh::k_ms_pull<16>(int, int const*)", 300.0),
             ("void kh::k_ms_pull<4>(int, int const*)", 50.0),
             ("void kh::k_union<256>(int const*)", 1000.0), ("void kh::k_union<1024>(int const*)", 500.0),
             ("void kh::k_union<256>(int const*)", 3000.0),
             ("at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<int>>", 524288.0),
             ("kh::k_reduce(long const*)", 7.0)]
    write = [(n, v / 10.0) for n, v in fetch]
    write_rows(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    write_rows(str(tmp_path / "w"), "WRITE_SIZE", write)
    bench.pmc_summarize(str(tmp_path / "f"), str(tmp_path / "w"), ["exact", "sampled"], [2])
    t = json.loads(traffic_file.read_text())
    # the pull kernel: one timed launch per dispatch of any width
    assert t["0"]["launches"] == 3
    assert t["0"]["fetch_kib_per_launch"] == pytest.approx(450.0 / 3)
    assert t["0"]["bytes_per_launch"] == int(1024 * (2.0 * 150.0 + 1.0 * 15.0))
    # the union: the hub variant runs inside the same timed launch
    assert t["1"]["launches"] == 2
    assert t["1"]["fetch_kib_per_launch"] == pytest.approx(4500.0 / 2)
    assert t["1"]["bytes_per_launch"] == int(1024 * (2.0 * 2250.0 + 1.0 * 225.0))
    assert t["0"]["source_sha256_16"] == bench.source_hash(0)
    assert any("add" in k for k in t["calibration"])


def test_traffic_only_for_same_source_and_workload(tmp_path, traffic_file):
    entry = {"source_sha256_16": bench.source_hash(1), "stage": ["exact", "sampled"], "h": [2],
             "bytes_per_launch": 1234}
    traffic_file.write_text(json.dumps({"1": entry}))
    assert bench.measured_traffic(1, ["exact", "sampled"], [2]) == 1234
    assert bench.measured_traffic(1, ["exact", "sampled"], [3]) is None
    assert bench.measured_traffic(1, ["sampled"], [2]) is None
    assert bench.measured_traffic(0, ["exact", "sampled"], [2]) is None
    traffic_file.write_text(json.dumps({"1": dict(entry, source_sha256_16="0" * 16)}))
    assert bench.measured_traffic(1, ["exact", "sampled"], [2]) is None


def test_percentile_and_gpu_count_guard(capsys, monkeypatch):
    assert bench.percentile([1, 2, 3, 4], 50) == pytest.approx(2.5)
    assert bench.percentile([], 99) is None
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().out


def test_trace_hops_numbers_hops_from_each_round(tmp_path, capsys):
    # two rounds at h = 3: hop durations 7, 14, 21 us, then a round of one hop
    p = tmp_path / "trace.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 0
        for hops in (3, 3, 1):
            w.writerow(["kh::k_select_commit(long const*)", t, t + 1000])
            t += 2000
            for hop in range(hops):
                w.writerow(["kh::k_rbfs_hop(int const*)", t, t + (hop + 1) * 7000])
                t += 50000
            w.writerow(["kh::k_decay_masked(int const*)", t, t + 500])
            t += 1000
    bench.trace_hops(str(p))
    out = json.loads(capsys.readouterr().out)
    assert out["hops"]["1"]["dispatches"] == 3 and out["hops"]["1"]["avg_us"] == 7.0
    assert out["hops"]["2"]["dispatches"] == 2 and out["hops"]["2"]["avg_us"] == 14.0
    assert out["hops"]["3"]["dispatches"] == 2 and out["hops"]["3"]["avg_us"] == 21.0
    assert sum(b["dispatches"] for b in out["buckets_us"].values()) == 7
