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
    ("k_box_yz_seg<64,64>", 12.0),       # read F, write the {G1, G2} pair
    ("k_box_x_select<64>", 12.125),      # read the pair and F, write one mask bit
    ("k_threshold", 12.125),
])
def test_algorithmic_bytes(kernel, per_voxel):
    assert bench.algorithmic_bytes(kernel, V) == per_voxel * V


def test_algorithmic_bytes_unknown_kernel():
    assert bench.algorithmic_bytes("k_final_mean", V) is None


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
