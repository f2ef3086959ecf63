"""Host logic of bench.py (no GPU): the guarded lookup of a committed HBM
traffic figure and the averaging of a rocprofv3 per-dispatch CSV over the timed
region."""
import hashlib
import json
import os

import pytest

import bench

KERNEL = "trail_update_kernel<double,64,64>"


def _summary(path, sha, instance=KERNEL, value="1.5e+10"):
    path.write_text("# counters\n\n"
                    f"- kernel_instance: {instance}\n"
                    f"- kernel_source_sha256: {sha}\n"
                    f"- traffic_bytes_per_launch: {value}\n")


@pytest.fixture
def source(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel source\n")
    return src, hashlib.sha256(src.read_bytes()).hexdigest()


def test_traffic_read_when_source_and_instance_match(tmp_path, source):
    src, sha = source
    md = tmp_path / "summary.md"
    _summary(md, sha)
    assert bench.traffic_from_profile(str(src), str(md), KERNEL) == 1.5e10


def test_traffic_from_ratio_scales_this_runs_algorithmic_bytes(tmp_path, source):
    src, sha = source
    md = tmp_path / "summary.md"
    _summary(md, sha)
    with open(md, "a") as f:
        f.write("- traffic_alg_ratio: 1.25\n")
    assert bench.traffic_from_profile(str(src), str(md), KERNEL, 4.0e9) == 5.0e9
    # without this run's algorithmic bytes the summary's own figure is used
    assert bench.traffic_from_profile(str(src), str(md), KERNEL) == 1.5e10
    src.write_text("// kernel source, edited\n")
    assert bench.traffic_from_profile(str(src), str(md), KERNEL, 4.0e9) is None


def test_traffic_null_after_a_source_change(tmp_path, source):
    src, sha = source
    md = tmp_path / "summary.md"
    _summary(md, sha)
    src.write_text("// kernel source, edited\n")
    assert bench.traffic_from_profile(str(src), str(md), KERNEL) is None


def test_traffic_null_for_another_tile(tmp_path, source):
    src, sha = source
    md = tmp_path / "summary.md"
    _summary(md, sha)
    assert bench.traffic_from_profile(str(src), str(md), "trail_update_kernel<double,128,128>") is None


@pytest.mark.parametrize("value", ["", "n/a"])
def test_traffic_null_for_a_malformed_figure(tmp_path, source, value):
    src, sha = source
    md = tmp_path / "summary.md"
    _summary(md, sha, value=value)
    assert bench.traffic_from_profile(str(src), str(md), KERNEL) is None


def test_traffic_null_without_summary(tmp_path, source):
    src, _ = source
    assert bench.traffic_from_profile(str(src), str(tmp_path / "missing.md"), KERNEL) is None


def test_committed_summaries_carry_the_guard_fields():
    """Every committed counter summary that states a traffic figure names the
    kernel instance and the source hash it was taken on."""
    root = os.path.join(os.path.dirname(__file__), "..", "profiles")
    for name in os.listdir(root):
        with open(os.path.join(root, name)) as f:
            text = f.read()
        if "traffic_bytes_per_launch:" in text:
            assert "kernel_instance:" in text and "kernel_source_sha256:" in text, name


def _bench_json(path, kernel, launches, avg_ms):
    line = {"roofline": {"kernel": f"{kernel} (trailing update)", "launches": launches, "avg_launch_ms": avg_ms,
                         "alg_bytes_per_launch": 123.0}}
    path.write_text("log line\n" + json.dumps(line) + "\n")


def test_rocprof_window_averages_the_last_dispatches_of_the_kernel(tmp_path):
    """Kernel trace: durations of the kernel's last `launches` dispatches (in
    dispatch order, other kernels and earlier dispatches ignored)."""
    csv = tmp_path / "trace.csv"
    rows = ["Kernel_Name,Dispatch_Id,Start_Timestamp,End_Timestamp"]
    t = 0
    durations = {}
    for d in range(1, 13):
        name = f"void inla::{KERNEL}(inla::FactorDesc const*, int, int, int)" if d % 2 == 0 else "inla::other_kernel()"
        dur = 1_000_000 * d          # ns
        rows.append(f'"{name}",{d},{t},{t + dur}')
        if d % 2 == 0:
            durations[d] = dur * 1e-6
        t += dur + 10
    # dispatch ids out of order in the file
    csv.write_text("\n".join([rows[0]] + rows[:0:-1]) + "\n")
    js = tmp_path / "bench.json"
    _bench_json(js, KERNEL, 3, 10.0)
    out = bench.rocprof_window(str(csv), str(js))
    assert out["dispatches_in_csv"] == 6 and out["window"] == 3 and out["quantity"] == "duration_ms"
    assert out["window_mean"] == pytest.approx((durations[8] + durations[10] + durations[12]) / 3)
    assert out["all_mean"] == pytest.approx(sum(durations.values()) / 6)
    assert out["bench_alg_bytes_per_launch"] == 123.0


def test_rocprof_window_reads_counter_values(tmp_path):
    csv = tmp_path / "counters.csv"
    rows = ["Kernel_Name,Dispatch_Id,Counter_Name,Counter_Value"]
    for d, v in [(3, 10.0), (5, 20.0), (9, 40.0)]:
        rows.append(f'"void inla::{KERNEL}(inla::FactorDesc const*, int, int, int)",{d},FETCH_SIZE,{v}')
    rows.append('"inla::other_kernel()",11,FETCH_SIZE,999.0')
    csv.write_text("\n".join(rows) + "\n")
    js = tmp_path / "bench.json"
    _bench_json(js, KERNEL, 2, 5.0)
    out = bench.rocprof_window(str(csv), str(js))
    assert out["quantity"] == "FETCH_SIZE" and out["window"] == 2
    assert out["window_mean"] == pytest.approx(30.0)


def test_prior_pass_kernel_is_named_and_windowed_apart(tmp_path):
    """The concurrent prior pass's trailing update is a kernel of its own
    (`trail_update_aux_kernel`): the bench names it for that pass, and a window
    over one of the two symbols never counts the other's dispatches."""
    aux = bench.trail_kernel_name("fp64", 64, aux=True)
    assert aux == "trail_update_aux_kernel<double,64,64>"
    assert bench.trail_kernel_name("fp64", 64) == KERNEL
    assert bench.trail_kernel_name("fp32", 128, aux=True) == "trail_update_aux_kernel<float,128,128>"
    csv = tmp_path / "trace.csv"
    rows = ["Kernel_Name,Dispatch_Id,Start_Timestamp,End_Timestamp"]
    for d in range(1, 9):
        sym = aux if d % 2 else KERNEL
        rows.append(f'"void inla::{sym}(inla::FactorDesc const*, int, int, int)",{d},0,{1_000_000 * d}')
    csv.write_text("\n".join(rows) + "\n")
    for sym, want in ((KERNEL, (6 + 8) / 2), (aux, (5 + 7) / 2)):
        js = tmp_path / "bench.json"
        _bench_json(js, sym, 2, 1.0)
        out = bench.rocprof_window(str(csv), str(js))
        assert out["dispatches_in_csv"] == 4 and out["window_mean"] == pytest.approx(want), (sym, out)
