"""Host check of the CC/SSSP push launches' vertex selection (csrc/select.h,
compiled into the library as device code) under g++ warnings and the
address and undefined-behaviour sanitizers: see tests/select_check.cpp."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_vertex_selection_under_sanitizers(tmp_path):
    exe = str(tmp_path / "select_check")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-Wuninitialized",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2010_08781_amd", "csrc"),
                    os.path.join(ROOT, "tests", "select_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
