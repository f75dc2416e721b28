"""Host logic of the traffic figures: hardware byte counters scaled by the
calibration copy, restricted to the passes without guarded gates."""
import csv

import pytest

import traffic_summary as T

HEAD = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, kib) in enumerate(rows):
            w.writerow([i + 1, name, counter, kib])


def test_scaling_by_calibration_copy(tmp_path):
    mask = T.uncond_mask()
    n = len(mask)
    assert n > 0 and any(mask)
    # the copy reads and writes 4 GiB; the fetch counter reads half of it
    copy = "qsv::k_copy(HIP_vector_type<double, 2u>*, HIP_vector_type<double, 2u> const*, unsigned long)"
    fetch = [("void other_kernel()", 7.0), (copy, T.COPY_BYTES / 1024 / 2)]
    write = [("void other_kernel()", 3.0), (copy, T.COPY_BYTES / 1024)]
    # pass i reads (1000 + i) KiB by the counter (scaled x2) and writes 500 KiB
    for i in range(n):
        fetch.append((f"void qsv::k_tile_pass_d8<HIP_vector_type<double, 2u> >(int) [{i}]", 1000.0 + i))
        write.append((f"void qsv::k_tile_pass_d8<HIP_vector_type<double, 2u> >(int) [{i}]", 500.0))
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    d = T.summarize(str(fp), str(wp), "abc")
    kept = [i for i in range(n) if mask[i]]
    want = [(2 * (1000.0 + i) + 500.0) * 1024.0 for i in kept]
    assert d["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert d["calibration"]["write_factor"] == pytest.approx(1.0)
    assert d["launches"] == len(kept)
    assert d["bytes_per_launch"] == pytest.approx(sum(want) / len(want))
    assert d["per_launch_min"] == pytest.approx(min(want)) and d["per_launch_max"] == pytest.approx(max(want))


def test_mismatched_runs_are_rejected(tmp_path):
    copy = "qsv::k_copy(x)"
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, "FETCH_SIZE", [(copy, 1.0), ("qsv::k_tile_pass_r<false>(x)", 2.0)])
    _write(wp, "WRITE_SIZE", [(copy, 1.0)])
    with pytest.raises(SystemExit):
        T.summarize(str(fp), str(wp), "abc")
