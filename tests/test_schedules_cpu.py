"""Host checks of the launch-schedule table compiled into the library
(csrc/apply_schedules.inc) and of the tuner that writes it: every entry is a
schedule the apply and CG kernels accept, keyed by a real sector dimension."""

import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2012_00217_amd", "csrc", "apply_schedules.inc")
ENTRY = re.compile(r"\{\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*\{\s*(\d+),\s*(\d+),\s*(\d+),\s*(\d+)\s*\}\s*\}")


def _entries(path=TABLE):
    txt = open(path).read()
    body = txt[txt.index("kSchedTable[] = {"):]
    return [tuple(int(v) for v in m.groups()) for m in ENTRY.finditer(body)]


def _power_of_two(x):
    return x > 0 and x & (x - 1) == 0


def test_table_entries_are_valid_schedules():
    rows = _entries()
    assert len(rows) >= 2
    *entries, sentinel = rows
    assert sentinel[:4] == (0, 0, 0, 0)
    seen = set()
    for L, n, row_bytes, elem, chunk, lane, grp, slots in entries:
        assert 2 <= L <= 32
        assert n == math.comb(L, L // 2)  # keyed by the S^z = 0 (or +1/2) sector dimension
        assert elem in (4, 8)
        assert row_bytes % elem == 0 and _power_of_two(row_bytes // elem)
        assert _power_of_two(chunk) and 16 <= chunk <= 4096
        assert _power_of_two(lane) and 16 <= lane <= chunk
        assert grp >= 0 and 1 <= slots <= 256
        assert (L, row_bytes, elem) not in seen  # one schedule per shape
        seen.add((L, row_bytes, elem))


def test_tuner_writes_a_table_the_checks_accept(tmp_path):
    autotune = pytest.importorskip("paper_2012_00217_amd.autotune")
    results = [
        {"L": 20, "n": math.comb(20, 10), "b": 64, "elem": 8, "row_bytes": 512,
         "sched": (512, 64, 0, 256), "ms": 0.3, "default_ms": 0.3},
        {"L": 24, "n": math.comb(24, 12), "b": 128, "elem": 4, "row_bytes": 512,
         "sched": (512, 64, 64, 64), "ms": 4.8, "default_ms": 5.2},
    ]
    out = tmp_path / "apply_schedules.inc"
    autotune.write_table(results, str(out), device_name="test")
    rows = _entries(str(out))
    assert rows[:-1] == [(20, 184756, 512, 8, 512, 64, 0, 256),
                         (24, 2704156, 512, 4, 512, 64, 64, 64)]
    assert rows[-1][:4] == (0, 0, 0, 0)


def test_tuner_reads_back_the_committed_table_and_merges(tmp_path):
    """read_table parses every entry of the committed table; a merge keeps the
    entries of shapes that were not tuned again and replaces the others."""
    autotune = pytest.importorskip("paper_2012_00217_amd.autotune")
    rows = autotune.read_table(TABLE)
    assert [(r["L"], r["n"], r["row_bytes"], r["elem"]) + tuple(r["sched"]) for r in rows] == \
        _entries()[:-1]
    out = tmp_path / "table.inc"
    autotune.write_table(rows, str(out))
    assert _entries(str(out)) == _entries()
    new = dict(rows[0], sched=(128, 16, 0, 64), ms=0.001)
    key = lambda r: (r["L"], r["row_bytes"], r["elem"])
    merged = [r for r in rows if key(r) != key(new)] + [new]
    autotune.write_table(merged, str(out))
    back = {key(r): tuple(r["sched"]) for r in autotune.read_table(str(out))}
    assert back[key(new)] == (128, 16, 0, 64)
    assert len(back) == len(rows)
