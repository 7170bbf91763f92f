"""Host-side checks of bench.py: the byte model, the rocprof summarizers and
the one-GPU guard (no GPU needed)."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_entry_points_present():
    for name in ("bytes_model", "make_inputs", "run_form", "cpu_baseline", "main",
                 "summarize_stats", "summarize_pmc", "read_traffic", "stage_kernels",
                 "parse_args", "check_args", "plane_distances", "ranked_stages"):
        assert callable(getattr(bench, name)), name


def test_bytes_model_mg_level0():
    cells = 12288 * 256 * 256
    assert bench.bytes_model("mg_post_l0", 256, 12288, 12 * 2048 ** 2, 4) == cells * 14
    assert bench.bytes_model("mg_pre_l0", 256, 12288, 12 * 2048 ** 2, 4) == cells * 13
    # fused smoothing: the finest pre-smoothing runs in the first cycle only
    assert bench.bytes_model("mg_pre_l0", 256, 12288, 12 * 2048 ** 2, 4, 1.0) == cells * 10
    assert bench.bytes_model("mg_postpre_l0", 256, 12288, 12 * 2048 ** 2, 4, 3.0) == cells * 16
    assert bench.bytes_model("unknown", 256, 12288, 1, 4) is None


def test_short_name():
    k = ("void clm::(anonymous namespace)::k_mg_pre<float, 6>"
         "(clm::(anonymous namespace)::TileArgs<float>)")
    assert bench.short_name(k) == "k_mg_pre<float, 6>"


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_pmc_calibration(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    grid0 = 12288 * 16 * 512
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>(int)"
    post = "void clm::(anonymous namespace)::k_mg_post<float, 4>(int)"
    _write(tmp_path / "f.csv", hdr, [[neg, 100, "FETCH_SIZE", 524288.0],
                                     [post, grid0, "FETCH_SIZE", 1000.0],
                                     [post, grid0, "FETCH_SIZE", 3000.0]])
    _write(tmp_path / "w.csv", hdr, [[neg, 100, "WRITE_SIZE", 1048576.0],
                                     [post, grid0, "WRITE_SIZE", 500.0]])
    text = bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "F", "W")
    assert "calibration_fetch 2.000000" in text
    line = [ln for ln in text.splitlines() if ln.startswith("traffic_bytes_per_launch mg_post_l0")]
    # mean fetch 2000 KiB x 2 + write 500 KiB x 1
    assert float(line[0].split()[2]) == pytest.approx((2000 * 2 + 500) * 1024)


def test_read_traffic_needs_matching_sources(tmp_path, monkeypatch):
    p = tmp_path / "t.txt"
    p.write_text("source_sha256 deadbeef\ntraffic_bytes_per_launch mg_post_l0 123\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.read_traffic("mg_post_l0") is None
    p.write_text("source_sha256 %s\ntraffic_bytes_per_launch mg_post_l0 123\n"
                 % bench.source_digest())
    assert bench.read_traffic("mg_post_l0") == 123.0


def test_multi_gpu_request_exits():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("argv", [["--gpus", "1", "--steps", "20", "--warmup", "5"],
                                  [], ["--steps", "40", "--warmup", "30"],
                                  ["--steps", "1", "--warmup", "0"]])
def test_driver_arguments_accepted(argv):
    """The driver's command line (and other step counts) passes the checks
    that run before any GPU work."""
    args = bench.parse_args(argv)
    assert bench.check_args(args) == (0, None)


def test_defaults_match_driver_command():
    args = bench.parse_args([])
    assert (args.gpus, args.steps, args.warmup) == (1, 20, 5)


def test_bad_counts_rejected():
    assert bench.check_args(bench.parse_args(["--steps", "0"]))[0] == 2
    assert bench.check_args(bench.parse_args(["--gpus", "8"]))[0] == 2


def test_plane_distances():
    chi = bench.plane_distances(20)
    assert len(chi) == 21
    assert chi[1] - chi[0] == pytest.approx(3054.70 / 20)
    assert chi[0] == pytest.approx(0.5 * 3054.70 / 20)
    # fewer steps keep the 20-plane light cone; more steps refine the spacing
    assert len(bench.plane_distances(5)) == 21
    chi = bench.plane_distances(40)
    assert len(chi) == 41 and chi[-2] == pytest.approx(3054.70 * 39.5 / 40)
    assert (np.diff(chi) > 0).all()


def test_ranked_stages():
    st = {"mg_postpre_l0": (12.9, 3), "patch_setup": (11.3, 1), "mean": (50.0, 2),
          "ray_update": (2.6, 1)}
    # "mean" has no byte model and is never a roofline kernel; the first two
    # get the roofline and the runner-up roofline
    assert bench.ranked_stages(st, 1, 12288, 12 * 2048 ** 2) == [
        "mg_postpre_l0", "patch_setup", "ray_update"]
    st["patch_setup"] = (13.0, 1)
    assert bench.ranked_stages(st, 1, 12288, 12 * 2048 ** 2)[:2] == [
        "patch_setup", "mg_postpre_l0"]


def test_host_cpu():
    cores, visible, model = bench.host_cpu()
    assert 1 <= cores <= 16 and cores <= visible and isinstance(model, str)
