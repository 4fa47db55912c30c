"""The measured tile table: tiles.json is complete and well formed, and the
header compiled into the library is the one generated from it."""
import json
import os

from paper_1105_0661_amd import gen_tile_table as gtt


def test_table_is_complete_and_the_header_is_generated_from_it(tmp_path):
    grid, bks = gtt.table()
    assert len(grid) == 2 and all(len(g) == 2 and all(len(k) == 5 for k in g) for g in grid)
    assert all(v in (1, 2, 4) for g in grid for p in g for k in p for v in k)
    assert bks[-1] >= 1 << 30 and bks == sorted(bks)
    out = tmp_path / "tile_table.h"
    gtt.generate(out=str(out))
    with open(gtt.HEADER) as f:
        assert f.read() == out.read_text()


def test_every_entry_names_a_measured_choice():
    with open(gtt.JSON) as f:
        t = json.load(f)
    for e in t["entries"]:
        if "ms" in e:
            ms = {int(k): v for k, v in e["ms"].items()}
            assert e["streams"] == min(ms, key=ms.get)


def test_incomplete_table_is_refused(tmp_path):
    with open(gtt.JSON) as f:
        t = json.load(f)
    t["entries"] = t["entries"][1:]
    p = tmp_path / "tiles.json"
    p.write_text(json.dumps(t))
    try:
        gtt.table(str(p))
    except ValueError as e:
        assert "incomplete" in str(e)
    else:
        raise AssertionError("an incomplete table was accepted")
    assert os.path.exists(gtt.HEADER)
