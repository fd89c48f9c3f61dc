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
    assert rows and all(len(r[5]) == 6 for r in rows)
    out = tmp_path / "t.txt"
    autotune.write_table(rows, str(out))
    assert out.read_text() == open(src).read()
    assert autotune.grid_for(3)[0] == autotune.TILES_8BIT
    assert autotune.grid_for(1)[0] == autotune.TILES
    assert autotune.grid_for(1, 8)[5] == autotune.UNROLL
    assert autotune.grid_for(0, 16)[5] == autotune.UNROLL
    assert autotune.grid_for(1, 2)[5] == (4,)


def test_autotune_graph_rows_precede_direct_rows(tmp_path):
    """A graph-mode row is written before the direct row of the same
    (dtype, op, ranks), whose graph column is "*": the first matching row
    wins, so graph replays take their own row and direct launches the
    other; a table of 11 columns reads with unroll 4."""
    from paper_2604_22228_amd import autotune
    rows = [("bf16", "sum", 8, "*", 29, (16384, 1, 16, 8, 64, 4), 1.0),
            ("bf16", "sum", 8, "1", 29, (32768, 2, 8, 4, 64, 2), 1.1),
            ("f32", "sum", 8, "*", 28, (8192, 2, 16, 8, 64, 4), 0.4)]
    out = tmp_path / "t.txt"
    autotune.write_table(rows, str(out))
    body = [ln.split("#")[0].split() for ln in out.read_text().splitlines()
            if not ln.startswith("#")]
    assert body[0][:4] == ["bf16", "sum", "8", "1"] and body[0][11] == "2"
    assert body[1][:4] == ["bf16", "sum", "8", "*"]
    assert sorted(autotune.read_table(str(out))) == sorted(rows)
    old = tmp_path / "old.txt"
    old.write_text("f32 sum 8 * 0 63 8192 2 16 8 64   # 0.4 at 2^28 B\n")
    assert autotune.read_table(str(old))[0][5] == (8192, 2, 16, 8, 64, 4)


def test_shipped_table_covers_every_tuned_workload():
    """Every (dtype, op, ranks) the autotuner tunes has a row of its own in
    the shipped table, so no workload falls back to the catch-all row."""
    from paper_2604_22228_amd import autotune
    src = os.path.join(ROOT, "paper_2604_22228_amd", "tuned_mi355x.txt")
    have = {(r[0], r[1], r[2]) for r in autotune.read_table(src)}
    for dtype, op, ranks, _graph, _counts, _nparts in autotune.default_keys():
        key = (autotune.DTYPE_NAMES[dtype], autotune.OP_NAMES[op], ranks)
        assert key in have, key
