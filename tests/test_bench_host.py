"""Host-side logic of bench.py that needs no GPU: the kernel-source hash that
ties the committed HBM-traffic summary to the kernel it was measured on, the
parsing of that summary, and the refusal of runs on more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_text_ignores_comments_and_blanks_only():
    a = "int f() { return 1; } // one\n/* block\n   comment */\n  int g;\n"
    b = "int f() { return 1; }\n\n// another comment\nint g;   \n"
    c = "int f() { return 2; }\nint g;\n"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)


def test_profiled_traffic_lookup():
    # a hash no summary holds gives nothing; the committed summary's own
    # hash gives its figures
    assert bench.profiled_traffic("k_gemm_rho", "water64_pbe_100x590_fp64", "0" * 64) == (None, None)
    path = os.path.join(ROOT, "profiles", "contractions_water64_pbe_fp64_hbm_traffic.md")
    line = [l for l in open(path) if l.startswith("traffic: kernel=k_gemm_rho")][0]
    fields = dict(kv.split("=", 1) for kv in line.split()[1:])
    total, src = bench.profiled_traffic("k_gemm_rho", fields["workload"], fields["source_sha256"])
    assert total == int(fields["fetch_bytes_per_launch"]) + int(fields["write_bytes_per_launch"])
    assert src.endswith("contractions_water64_pbe_fp64_hbm_traffic.md")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
