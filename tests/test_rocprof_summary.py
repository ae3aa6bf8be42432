"""CPU checks of the rocprofv3 summary tool used for profiles/: kernel-name
shortening, the traffic scaling by the reference copy, and the counter table."""
import csv
import io
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2506_02774_amd import rocprof_summary as rs  # noqa: E402

COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, " \
       "at::native::binary_internal::MulFunctor<float> >, std::array<char*, 2ul> >(int, float)"
BLEND = "void (anonymous namespace)::blend_jobs<true, false, false, false>(unsigned int const*, int)"


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i, k, c, v])


def test_short_names():
    assert rs.short(BLEND) == "blend_jobs<true, false, false, false>"
    assert rs.short("void (anonymous namespace)::project<true>(int const*)") == "project<true>"


def test_traffic_scaled_by_reference_copy(tmp_path):
    # the copy moves 1024 MiB each way; its counters read half of that for fetch, all of it for write
    mib = 1024
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _csv(f, [(COPY, "FETCH_SIZE", mib * 1024 / 2), (BLEND, "FETCH_SIZE", 1000.0), (BLEND, "FETCH_SIZE", 3000.0)])
    _csv(w, [(COPY, "WRITE_SIZE", mib * 1024), (BLEND, "WRITE_SIZE", 500.0), (BLEND, "WRITE_SIZE", 500.0)])
    src = tmp_path / "k.hip"
    src.write_text("kernel")
    r = subprocess.run([sys.executable, "-m", "paper_2506_02774_amd.rocprof_summary", "traffic", str(f), str(w),
                        "--copy-mib", str(mib), "--source", str(src)], capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    d = json.loads([l for l in r.stdout.splitlines() if l.startswith("{")][-1])
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0
    assert d["read_bytes_per_launch"] == 2 * 2000 * 1024 and d["write_bytes_per_launch"] == 500 * 1024
    assert d["dispatches"] == 2 and d["stage"] == "blend"


def test_counter_table(tmp_path):
    f = tmp_path / "c.csv"
    _csv(f, [(BLEND, "SQ_WAVES", 100), (BLEND, "SQ_WAVES", 300), (BLEND, "SQ_INSTS_VALU", 8)])
    out = io.StringIO()
    old = sys.stdout
    sys.stdout = out
    try:
        rs.counters([str(f)], ["blend_jobs<true, false, false, false>", "absent"])
    finally:
        sys.stdout = old
    lines = out.getvalue().splitlines()
    assert lines[0] == "| kernel | dispatches | SQ_INSTS_VALU | SQ_WAVES |"
    assert lines[2] == "| `blend_jobs<true, false, false, false>` | 2 | 8 | 200 |" and len(lines) == 3
