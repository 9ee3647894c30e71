"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline figure, the reader of the committed byte-counter summaries, and the
refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

V = 512 * 512 * 1024


@pytest.mark.parametrize("kernel,per_voxel", [
    ("k_zpass_r<24>", 8.0),              # read d, write T1
    ("k_yx_r<12>", 8.0),                 # read T1, write F
    ("k_yx3_r<3,6,12>", 16.0),           # read T1, write three F
    ("k_box_yz_seg<64,64>", 12.0),       # read F, write the {G1, G2} pair
    ("k_box_x_select<64>", 12.125),      # read the pair and F, write one mask bit
    ("k_threshold", 12.125),
])
def test_kernel_io_bytes(kernel, per_voxel):
    assert bench.kernel_io_bytes(kernel, V) == per_voxel * V


def test_kernel_io_bytes_unknown_kernel():
    assert bench.kernel_io_bytes("k_final_mean", V) is None


def test_roofline_uses_the_algorithmic_bytes():
    # the x walk: 6 launches per step over 10 steps, 0.774 ms each, each serving
    # one filter over the 2^28-voxel cube: 4.125 B x 2^28 / 0.774 ms
    kern = {"k_box_x_select<64>": (60, 60 * 0.774), "k_box_yz_seg<64,64>": (60, 60 * 0.61),
            "k_zpass_r<6>": (10, 10 * 0.39)}
    r = bench.roofline_for(kern, V, 6, 10, "f32", 123.0)
    assert r["kernel"] == "k_box_x_select<64>"
    assert r["voxel_filters_per_launch"] == V
    assert r["algorithmic_bytes_per_launch"] == 4.125 * V
    assert abs(r["frac"] - 4.125 * V / 0.774e-3 / 8e12) < 1e-4
    assert abs(r["frac"] - 0.179) < 0.001
    assert r["kernel_io"]["bytes_per_launch"] == 12.125 * V
    # a launch shared by three filters serves three voxel-filters per voxel
    r2 = bench.roofline_for({"k_zpass_r<6>": (20, 20.0)}, V, 6, 10, "f16", 20.0)
    assert r2["voxel_filters_per_launch"] == 3 * V
    assert r2["algorithmic_bytes_per_launch"] == 2.125 * 3 * V
    assert "kernel_io" not in r2


def test_one_read_figure():
    assert abs(bench.one_read_bytes_per_vf("f32", 6) - (4 + 6 / 8) / 6) < 1e-12
    assert abs(bench.one_read_bytes_per_vf("f16", 6) - (2 + 6 / 8) / 6) < 1e-12


def test_noise_sigma_f_matches_the_survey_table():
    # filtered-noise sigma of the measured bank for unit noise
    want = {(1.0, 2.0): 0.10612, (1.0, 8.0): 0.05312, (2.0, 2.0): 0.05314,
            (2.0, 8.0): 0.02660, (4.0, 2.0): 0.02660, (4.0, 8.0): 0.01332}
    for f, v in want.items():
        assert abs(bench.noise_sigma_f(f, 3.0) - v) < 2e-5, f


def test_traffic_file_name():
    p = bench.traffic_file("k_box_yz_seg<64,64>", "cube512x512x1024_f6_box64")
    assert os.path.basename(p) == "k_box_yz_seg_64_64_cube512x512x1024_f6_box64_traffic.txt"


def test_read_traffic_checks_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    k, wl = "k_box_x_select<64>", "w"
    assert bench.read_traffic(k, wl, "abc") is None          # no summary
    with open(bench.traffic_file(k, wl), "w") as fh:
        fh.write("# header: ignored\nkernel: k_box_x_select<64>\nsource_sha: abc\n"
                 "hbm_bytes_per_launch: 3256443692\n")
    assert bench.read_traffic(k, wl, "abc") == 3256443692.0
    assert bench.read_traffic(k, wl, "def") is None          # kernels changed since


def test_committed_summaries_parse():
    # every committed per-kernel summary names its kernel, hash and bytes
    names = [n for n in os.listdir(bench.PROFILES) if n.endswith("_traffic.txt")]
    assert names
    for n in names:
        vals = {}
        for line in open(os.path.join(bench.PROFILES, n)):
            if ":" in line and not line.startswith("#"):
                a, b = line.split(":", 1)
                vals[a.strip()] = b.strip()
        assert float(vals["hbm_bytes_per_launch"]) > 0
        assert len(vals["source_sha"]) == 16
        assert bench.traffic_file(vals["kernel"], vals["workload"]).endswith(n)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_source_hash_ignores_comments_only():
    code = "int a = 1;  // one\n/* block\n   comment */\nint b = 2;\n"
    assert bench._code_only(code) == bench._code_only("int a = 1;\n\nint b = 2;  // two\n")
    assert bench._code_only(code) != bench._code_only("int a = 1;\nint b = 3;\n")
