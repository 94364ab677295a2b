"""The rocprofv3 summaries behind profiles/ (CPU only): kernel-name matching,
copy-kernel calibration of the HBM counters, call splitting of kernel
traces and the CCD++ per-mode pass table, on small synthetic CSV files in
rocprofv3's column layout."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1910_02371_amd import rocprof_summary as S  # noqa: E402

SOLO = "void tt::k_solve_solo<tt::TrF32, 64, true, false, {rhs}, {fo}, false, {mod}>(tt::GramDev)"
HSOLO = "void tt::k_gram_solve_heavy<tt::TrF32, 32, true, false, true, false, {mod}>(tt::GramDev)"
STREAM = "void tt::k_stream<tt::TrF32, 3, 16, 2, {op}, 1024>(tt::StreamDev)"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_matches_template_arguments():
    assert S.matches("gram_solve_light", SOLO.format(rhs="true", fo="false", mod="false"))
    assert S.matches("gram_solve_light", SOLO.format(rhs="true", fo="false", mod="true"))
    assert not S.matches("gram_factor_light", SOLO.format(rhs="true", fo="false", mod="false"))
    assert S.matches("gram_factor_light", SOLO.format(rhs="false", fo="true", mod="false"))
    for mod in ("true", "false"):  # with and without the model output
        assert S.matches("gram_solve_heavy", HSOLO.format(mod=mod))
    assert S.matches("tttp", STREAM.format(op=0)) and not S.matches("tttp", STREAM.format(op=1))
    assert S.matches("gn_mttkrp", STREAM.format(op=1)) and S.matches("mttkrp", STREAM.format(op=1))
    assert S.matches("gn_matvec", STREAM.format(op=3))
    assert S.matches("gram_heavy", "void tt::k_gram_f32_heavy<tt::TrF32, 64, true, false, true, 4, false>")


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    """Counter KiB are scaled so that the calibration copy reads (writes)
    exactly copy_bytes; only the named kernel's dispatches are averaged."""
    copy_bytes = 1 << 20
    head = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    tk = STREAM.format(op=0)
    # FETCH: the copy reads 2048 "KiB" for 1 MiB (scale 0.5); two TTTP
    # dispatches of 4000 and 6000 KiB, split over two counter rows each
    fetch = [[1, "void at::native::copy_kernel", "FETCH_SIZE", 2048],
             [2, tk, "FETCH_SIZE", 1000], [2, tk, "FETCH_SIZE", 3000],
             [3, "void tt::k_fill<float>", "FETCH_SIZE", 99],
             [4, tk, "FETCH_SIZE", 6000]]
    write = [[1, "void at::native::copy_kernel", "WRITE_SIZE", 1024],
             [2, tk, "WRITE_SIZE", 10], [4, tk, "WRITE_SIZE", 30]]
    _write(str(tmp_path / "f" / "run_counter_collection.csv"), head, fetch)
    _write(str(tmp_path / "w" / "run_counter_collection.csv"), head, write)
    out = tmp_path / "prof" / "tttp_x_traffic.md"
    os.makedirs(out.parent)
    S.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "tttp", "x", "h1", copy_bytes,
              str(out), "cmd")
    db = json.load(open(out.parent / "traffic.json"))
    rec = db["tttp|x"]
    assert rec["launches"] == 2 and rec["src_hash"] == "h1"
    assert rec["fetch_scale"] == 0.5 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 0.5 * 5000 * 1024
    assert rec["write_bytes_per_launch"] == 20 * 1024
    assert rec["bytes_per_launch"] == 0.5 * 5000 * 1024 + 20 * 1024
    assert "Kernel source hash: h1" in out.read_text()


def _trace_rows(spec):
    """spec: list of (kernel name, duration us, gap us before it)."""
    rows, t = [], 1000
    for name, dur, gap in spec:
        t += int(gap * 1000)
        rows.append([name, t, t + int(dur * 1000)])
        t += int(dur * 1000)
    return rows


def test_trace_splits_calls_and_drops_warmup(tmp_path):
    spec = []
    for call in range(3):
        spec += [("tt::k_a(int)", 10 + call, 1.0), ("tt::k_b(int)", 5, 2.0),
                 ("tt::k_pcg_stats(int)", 1, 0.0)]
    p = str(tmp_path / "t.csv")
    _write(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], _trace_rows(spec))
    out = tmp_path / "t.md"
    S.trace(p, "k_pcg_stats", 1, str(out), "cmd")
    text = out.read_text()
    assert "2 calls ending with" in text
    # calls 1 and 2: 3 dispatches, summed 17 and 18 us; the spans add the
    # 2 us gap inside the call (the 1 us gap before it belongs to no call);
    # the upper median of the gaps (0, 2) is 2
    assert "| 0 | 3 | 19.0 | 17.0 | 2.00 |" in text
    assert "| 1 | 3 | 20.0 | 18.0 | 2.00 |" in text
    assert "| `tt::k_a` | 1.0 | 11.50 |" in text


def test_ccd_assigns_dispatches_to_modes(tmp_path):
    """The timed sweep is the second half of the k_ccd_tasks dispatches, and
    dispatch i of it is mode i mod 3."""
    spec = []
    for sweep in range(2):
        for col in range(2):
            spec.append(("void tt::k_ccd_column<float, float>()", 8, 0))
            for mode in range(3):
                dur = 100 * (mode + 1) + (1000 if sweep == 0 else 0) + col
                spec.append((f"void tt::k_ccd_tasks<float, float, 64, {mode % 2}>()", dur, 0))
                spec.append(("void tt::k_ccd_rows<float, float>()", 50, 0))
    p = str(tmp_path / "c.csv")
    _write(p, ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], _trace_rows(spec))
    out = tmp_path / "c.md"
    S.ccd(str(out), "cmd", p, p)
    text = out.read_text()
    assert "| mode-0 pass (k_ccd_tasks) us | 100.5 | 100.5 |" in text
    assert "| mode-2 pass (k_ccd_tasks) us | 300.5 | 300.5 |" in text
    assert "| per-row solves (k_ccd_rows) us | 50.0 | 50.0 |" in text
    assert "| columns in the sweep | 2 | 2 |" in text
