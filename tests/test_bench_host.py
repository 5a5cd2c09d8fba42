"""Host logic of bench.py, on the CPU: the one-GPU contract, the parsing of
demangled kernel names that the counter summaries select dispatches by, and the
traffic arithmetic of a counter summary (FETCH_SIZE and WRITE_SIZE in KiB per
dispatch, each scaled by what the same counter reads for a device copy of known
size) on synthetic rocprofv3 CSV files."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_template_args_of_nested_templates():
    name = ("void ebicg::(anonymous namespace)::k_bmarch<HIP_vector_type<double, 2u>, 1, -1, 0>"
            "(HIP_vector_type<double, 2u>*, HIP_vector_type<double, 2u> const*, int)")
    assert bench._template_args(name, "k_bmarch") == ["HIP_vector_type<double, 2u>", "1", "-1", "0"]
    assert bench._template_args(name, "k_bstab_v") is None
    assert bench._template_args("k_bstab_xr_f<HIP_vector_type<float, 2u>, 16>(float*)", "k_bstab_xr_f") == [
        "HIP_vector_type<float, 2u>", "16"]


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


def test_counter_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """A copy of COPY_BYTES that FETCH_SIZE reads as half its bytes and WRITE_SIZE as
    all of them gives scales 2 and 1; two dispatches of the BiCG matvec at 100 and
    102 KiB fetched, 168 KiB written, on 4^4 (V = 256: 7 units of 192 B per site
    = 344 064 algorithmic bytes) move (101 * 2 + 168) KiB = 378 880 B, 1.101x."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda cls="bicg_matvec": "0" * 16)
    (tmp_path / "profiles").mkdir()
    kib = bench.COPY_BYTES / 1024.0
    mv = "void ebicg::(anonymous namespace)::k_bicg_matvec<false>(HIP_vector_type<double, 2u>*)"
    g5 = "void ebicg::(anonymous namespace)::k_bicg_matvec<true>(HIP_vector_type<double, 2u>*)"
    cp = "__amd_rocclr_copyBuffer"
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # the gamma5 instance and an earlier, different copy are not counted
    _counter_csv(fetch, "FETCH_SIZE", [(cp, 7.0), (mv, 100.0), (g5, 999.0), (mv, 102.0)] + [(cp, kib / 2)] * 3)
    _counter_csv(write, "WRITE_SIZE", [(cp, 7.0), (mv, 168.0), (g5, 999.0), (mv, 168.0)] + [(cp, kib)] * 3)
    bench.summarize_pmc(str(fetch), str(write), "inc4")
    out = json.load(open(tmp_path / "profiles" / "pmc_bicg_matvec_inc4.json"))
    assert out["copy_calibration"]["fetch_scale"] == 2.0 and out["copy_calibration"]["write_scale"] == 1.0
    assert out["dispatches"] == {"fetch": 2, "write": 2}
    assert out["algorithmic_bytes_per_launch"] == 7 * 192 * 256
    assert out["traffic_bytes_per_launch"] == (101 * 2 + 168) * 1024
    assert out["traffic_over_algorithmic"] == round((101 * 2 + 168) * 1024 / (7 * 192 * 256), 3)
