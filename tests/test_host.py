"""Host-side logic that needs no GPU: the benchmark's refusal of several
GPUs, the numpy entry layouts handed to the C ABI, the HBM-counter scaling of
the profile summaries, and the bench's load of stored traffic figures."""
import ctypes as C
import json
import os
import subprocess
import sys
import types


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _ctypes_layout(struct):
    return [(name, getattr(struct, name).offset) for name, _ in struct._fields_], C.sizeof(struct)


def test_numpy_entry_arrays_match_the_c_structs():
    from paper_2601_08217_amd import binding as B
    for dt, st in ((B.TAPS_SRC_DTYPE, B.tt_taps_src), (B.CIR_SRC_DTYPE, B.tt_cir_src)):
        fields, size = _ctypes_layout(st)
        assert dt.itemsize == size
        assert [(n, dt.fields[n][1]) for n in dt.names] == fields


def test_counter_scaling_of_the_traffic_summary(tmp_path):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch, summed over the counter's
    instances) are scaled by what they read for a copy of known size; the
    figure per launch is the median over dispatches."""
    from paper_2601_08217_amd import profsum

    def counters(path, counter, rows):
        with open(path, "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for d, k, v in rows:
                f.write(f"{d},{k},{counter},{v}\n")

    # the kernel: three dispatches, each counter split over two instances
    counters(tmp_path / "f.csv", "FETCH_SIZE", [(1, "tt::k_fir<4>", 40), (1, "tt::k_fir<4>", 10),
                                                (2, "tt::k_fir<4>", 60), (2, "tt::k_fir<4>", 0),
                                                (3, "tt::k_fir<4>", 70), (9, "tt::k_reduce", 999)])
    counters(tmp_path / "w.csv", "WRITE_SIZE", [(1, "tt::k_fir<4>", 30), (2, "tt::k_fir<4>", 32),
                                                (3, "tt::k_fir<4>", 31)])
    # the copy: 1 MiB each way reads as 512 KiB fetched and 1024 KiB written
    counters(tmp_path / "cf.csv", "FETCH_SIZE", [(1, "tt::k_copy16", 3), (2, "tt::k_copy16", 512)])
    counters(tmp_path / "cw.csv", "WRITE_SIZE", [(1, "tt::k_copy16", 1024)])
    args = types.SimpleNamespace(
        fetch=str(tmp_path / "f.csv"), write=str(tmp_path / "w.csv"), copy_fetch=str(tmp_path / "cf.csv"),
        copy_write=str(tmp_path / "cw.csv"), kernel="k_fir", workload="w", out_json=str(tmp_path / "t.json"),
        out_md=str(tmp_path / "t.md"), cmd_fetch="f", cmd_write="w", cmd_copy="c", copy_bytes=1 << 20)
    profsum.traffic(args)
    out = json.load(open(tmp_path / "t.json"))
    assert out["fetch_scale"] == 2.0 and out["write_scale"] == 1.0
    assert out["dispatches"] == [3, 3]
    assert out["fetch_bytes_per_launch"] == 60 * 1024 * 2.0     # median of 50, 60, 70 KiB
    assert out["write_bytes_per_launch"] == 31 * 1024 * 1.0
    assert out["bytes_per_launch"] == out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    assert out["kernel_sha"] == profsum.kernel_sha()


def test_stored_traffic_is_dropped_once_the_kernel_changes(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = {"kernel": "k_fir", "workload": "c5", "kernel_sha": bench.kernel_sha(), "bytes_per_launch": 123.0}
    p = tmp_path / "fir_c5_traffic.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.load_traffic("c5") == 123.0
    assert bench.load_traffic("c4") is None            # another workload
    rec["kernel_sha"] = "0" * 16
    p.write_text(json.dumps(rec))
    assert bench.load_traffic("c5") is None            # counters of an older kernel
