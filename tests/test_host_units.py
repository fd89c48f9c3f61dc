"""Host-only C++ units of the runtime (LRU binding/graph cache, tuned-table
parser), compiled with g++ and run on the CPU."""
import os
import subprocess


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_22228_amd", "csrc")


def test_host_units(tmp_path):
    exe = str(tmp_path / "test_host")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra",
                    "-fsanitize=address,undefined", "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "test_host.cpp"),
                    os.path.join(CSRC, "tuning.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
