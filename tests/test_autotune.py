"""The autotuner's committed table: its picks are the fastest of its own measurements, every pick
is a shape the tile kernel launches for that mode, and the compiled-in rows are those picks."""
import json
import os
import re

from paper_1605_01799_amd import autotune as T


def load():
    with open(T.JSON_PATH) as f:
        return json.load(f)


def test_picks_are_the_measured_minimum():
    table = load()
    assert table["picks"] == T.picks_from(table["measured"])
    for key, pick in table["picks"].items():
        mode, n_pad = (int(v) for v in key.split(":"))
        assert tuple(pick) in T.CANDIDATES[mode]
        ms = table["measured"][key]
        assert ms["%d:%d:%d" % tuple(pick)] == min(v for v in ms.values() if v is not None)


def test_compiled_rows_match_the_picks():
    table = load()
    with open(T.INC_PATH) as f:
        rows = re.findall(r"\{(-?\d+), (\d+), (\d+), (\d+), (\d+)\},", f.read())
    rows = [tuple(int(v) for v in r) for r in rows]
    assert rows[-1][0] == -1
    got = {"%d:%d" % (r[0], r[1]): list(r[2:]) for r in rows[:-1]}
    assert got == table["picks"]
    # rows of one mode in increasing size, so the first row that covers a size is its bucket
    for mode in T.CANDIDATES:
        sizes = [r[1] for r in rows if r[0] == mode]
        assert sizes == sorted(sizes)


def test_dense_source_compiles_the_table_in():
    src = os.path.join(os.path.dirname(T.INC_PATH), "dense.hip")
    with open(src) as f:
        assert '#include "tune_table.inc"' in f.read()
