"""bench.py's measurement bookkeeping on the CPU: the kernel-source hash that
ties recorded HBM counters to the code they were taken on, and the scaling of
rocprofv3 FETCH_SIZE / WRITE_SIZE readings by a copy of known size."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_text_ignores_comments_only(bench):
    src = "int a; // one\n\n   // whole-line comment\nint b;  \n"
    assert bench.code_text(src) == "int a;\nint b;"
    assert bench.code_text(src) != bench.code_text(src.replace("int b;", "int c;"))


def test_hash_follows_code_not_comments(bench):
    real = {}

    def read(path):
        if path not in real:
            with open(os.path.join(ROOT, path)) as fh:
                real[path] = fh.read()
        return real[path]

    h0 = bench.kernel_source_hash(read)
    assert h0 == bench.kernel_source_hash()
    kern = os.path.join("paper_2205_07125_amd", "csrc", "snn_kernels.hip")
    commented = lambda p: read(p) + "\n// a trailing remark\n" if p == kern else read(p)
    assert bench.kernel_source_hash(commented) == h0
    edited = lambda p: read(p) + "\nstatic int probe_only;\n" if p == kern else read(p)
    assert bench.kernel_source_hash(edited) != h0


def _pmc_dir(tmp_path, name, counter, rows):
    d = tmp_path / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for kernel, value in rows:
            w.writerow([kernel, counter, value])
    return str(d)


def test_pmc_summary_scales_by_the_copy(bench, tmp_path, capsys):
    upd = "void snn::k_update<true>(snn::KParams)"
    rl = "snn::k_recv_deliver<false>(snn::KParams)"
    # three dispatches each: the first third is dropped, then the median
    fetch = _pmc_dir(tmp_path, "f", "FETCH_SIZE",
                     [(upd, 999), (upd, 100), (upd, 102), (rl, 5), (rl, 50), (rl, 50)])
    write = _pmc_dir(tmp_path, "w", "WRITE_SIZE", [(upd, 1), (upd, 40), (upd, 40)])
    # a 1 MiB copy that FETCH_SIZE reads as 512 KiB and WRITE_SIZE as 1024 KiB
    cf = _pmc_dir(tmp_path, "cf", "FETCH_SIZE", [("copyBuffer", 512), ("fill", 4)])
    cw = _pmc_dir(tmp_path, "cw", "WRITE_SIZE", [("copyBuffer", 1024)])
    out = tmp_path / "traffic.json"
    bench.pmc_summary(fetch, write, cf, cw, 1 << 20, "demo", str(out))
    rec = json.load(open(out))["demo"]
    assert set(rec) == {"update", "recv_deliver"}
    u = rec["update"]
    assert u["fetch_scale"] == 2.0 and u["write_scale"] == 1.0
    assert u["fetch_kib"] == 101.0 and u["write_kib"] == 40.0
    assert u["bytes_per_launch"] == 101.0 * 1024 * 2 + 40.0 * 1024
    assert rec["recv_deliver"]["write_kib"] == 0.0
    assert u["kernel_hash"] == bench.kernel_source_hash()
    # a second workload is added beside the first
    bench.pmc_summary(fetch, write, cf, cw, 1 << 20, "other", str(out))
    assert set(json.load(open(out))) == {"demo", "other"}
    capsys.readouterr()


def test_cpu_baseline_runs_in_spawned_workers():
    """The oracle leg starts its workers fresh (spawn), one OpenMP thread each,
    and reports both legs; a short budget on the tiny network."""
    import sys
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench as bench_main
    import synth
    r = bench_main.cpu_baseline(synth.get_workload("tiny"), seconds_budget=0.3)
    assert r["kind"] == "oracle" and r["unit"] == "synaptic events/s"
    assert r["value"] > 0 and r["single_thread_value"] > 0
    assert 1 <= r["cores"] <= 16
    assert "processes of one thread each" in r["sample"]
