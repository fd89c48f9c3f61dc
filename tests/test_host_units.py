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


def test_autotune_table_round_trip(tmp_path):
    """A partial retune keeps the other rows: reading the shipped table and
    writing it again reproduces it byte for byte."""
    from paper_2604_22228_amd import autotune
    src = os.path.join(ROOT, "paper_2604_22228_amd", "tuned_mi355x.txt")
    rows = autotune.read_table(src)
    assert rows and all(len(r[5]) == 5 for r in rows)
    out = tmp_path / "t.txt"
    autotune.write_table(rows, str(out))
    assert out.read_text() == open(src).read()
    assert autotune.grid_for(3)[0] == autotune.TILES_8BIT
    assert autotune.grid_for(1)[0] == autotune.TILES


def test_shipped_table_covers_every_tuned_workload():
    """Every (dtype, op, ranks) the autotuner tunes has a row of its own in
    the shipped table, so no workload falls back to the catch-all row."""
    from paper_2604_22228_amd import autotune
    src = os.path.join(ROOT, "paper_2604_22228_amd", "tuned_mi355x.txt")
    have = {(r[0], r[1], r[2]) for r in autotune.read_table(src)}
    for dtype, op, ranks, _graph, _counts, _nparts in autotune.default_keys():
        key = (autotune.DTYPE_NAMES[dtype], autotune.OP_NAMES[op], ranks)
        assert key in have, key
