"""Host logic of bench.py (no GPU): the HBM traffic record written from
rocprofv3 counter CSVs, and that the bench reports it only for the kernel
source it was taken on."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    monkeypatch.setattr(m, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    return m


def _csv(d, rows):
    """A rocprofv3 counter-collection CSV with (kernel, dispatch, value) rows;
    two rows per dispatch, as a counter summed over two hardware instances."""
    os.makedirs(d / "host" / "pid", exist_ok=True)
    with open(d / "host" / "pid" / "run_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for k, disp, v in rows:
            f.write(f'{disp},"{k}",C,{v / 2}\n{disp},"{k}",C,{v / 2}\n')


def test_record_traffic_scales_by_the_copy(bench, tmp_path):
    gib_kib = (1 << 30) / 1024
    copy = "__amd_rocclr_copyBuffer"
    _csv(tmp_path / "pc_fetch", [(copy, 1, 16.0), (copy, 2, gib_kib / 2)])   # FETCH_SIZE sees half the reads
    _csv(tmp_path / "pc_write", [(copy, 1, 8.0), (copy, 2, gib_kib)])
    step32 = "void lbm::(anonymous namespace)::k_fused<0, 64, 2, 2>(lbm::FusedArgs)"
    step16 = "void lbm::(anonymous namespace)::k_fused<1, 32, 4, 2>(lbm::FusedArgs)"
    links = "void lbm::(anonymous namespace)::k_links<0>(lbm::LinkArgs)"
    _csv(tmp_path / "pb_fetch_f32", [(step32, 1, 100.0), (step32, 2, 300.0), (links, 3, 5.0)])
    _csv(tmp_path / "pb_write_f32", [(step32, 1, 50.0), (step32, 2, 50.0)])
    _csv(tmp_path / "pb_fetch_f16", [(step16, 1, 10.0)])
    _csv(tmp_path / "pb_write_f16", [(step16, 1, 4.0)])
    bench.record_traffic(str(tmp_path))
    rec = json.load(open(bench.TRAFFIC_FILE))
    assert rec["f32"]["tiles"]["64x2x2"]["kernel"] == "k_fused<0,64,2,2>"
    assert rec["f16"]["tiles"]["32x4x2"]["kernel"] == "k_fused<1,32,4,2>"
    assert rec["f32"]["fetch_scale"] == pytest.approx(2.0) and rec["f32"]["write_scale"] == pytest.approx(1.0)
    # mean over dispatches: fetch 200 KiB x 2, write 50 KiB x 1
    assert rec["f32"]["tiles"]["64x2x2"]["bytes_per_launch"] == 200 * 1024 * 2 + 50 * 1024
    assert rec["f16"]["tiles"]["32x4x2"]["bytes_per_launch"] == 10 * 1024 * 2 + 4 * 1024
    assert bench.measured_traffic("f32", "64x2x2") == 200 * 1024 * 2 + 50 * 1024
    assert bench.measured_traffic("f32", "16x8x2") is None
    assert bench.measured_traffic("bf16", "64x2x2") is None


def test_traffic_dropped_when_the_kernel_source_changes(bench, tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE, "w") as f:
        json.dump({"f32": {"kernel_sha": bench.kernel_sha(), "tiles": {"64x2x2": {"bytes_per_launch": 123}}}}, f)
    assert bench.measured_traffic("f32", "64x2x2") == 123
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic("f32", "64x2x2") is None


def test_record_traffic_per_tile_shape(bench, tmp_path):
    """The autotuner runs every tile shape: each gets its own figure; a
    shape seen by only one of the two counters gets none; a run without
    any step kernel is an error."""
    copy = "__amd_rocclr_copyBuffer"
    _csv(tmp_path / "pc_fetch", [(copy, 1, 4.0)])
    _csv(tmp_path / "pc_write", [(copy, 1, 4.0)])
    a = "void lbm::(anonymous namespace)::k_fused<0, 64, 2, 2>(lbm::FusedArgs)"
    b = "void lbm::(anonymous namespace)::k_fused<0, 32, 2, 4>(lbm::FusedArgs)"
    c = "void lbm::(anonymous namespace)::k_fused<0, 16, 8, 2>(lbm::FusedArgs)"
    _csv(tmp_path / "pb_fetch_f32", [(a, 1, 1.0), (b, 2, 2.0), (c, 3, 3.0)])
    _csv(tmp_path / "pb_write_f32", [(a, 1, 1.0), (b, 2, 1.0)])
    _csv(tmp_path / "pb_fetch_f16", [])
    _csv(tmp_path / "pb_write_f16", [])
    with pytest.raises(SystemExit):
        bench.record_traffic(str(tmp_path))
    f16 = "void lbm::(anonymous namespace)::k_fused<1, 64, 2, 2>(lbm::FusedArgs)"
    _csv(tmp_path / "pb_fetch_f16", [(f16, 1, 1.0)])
    _csv(tmp_path / "pb_write_f16", [(f16, 1, 1.0)])
    bench.record_traffic(str(tmp_path))
    rec = json.load(open(bench.TRAFFIC_FILE))
    assert sorted(rec["f32"]["tiles"]) == ["32x2x4", "64x2x2"]
    assert rec["f32"]["tiles"]["32x2x4"]["fetch_kib_per_dispatch"] == 2.0


def test_more_than_one_gpu_is_refused():
    """The bench runs on one GPU; asking for more exits with status 2 and
    says so, before any device work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
