"""Turn tiles.json (the measured tile table) into csrc/tile_table.h.

    python -m paper_1105_0661_amd.gen_tile_table

Run by build.py before compiling, so the table in the library is always the
one in tiles.json.  tune_tiles.py writes tiles.json from timings."""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
JSON = os.path.join(HERE, "tiles.json")
HEADER = os.path.join(HERE, "csrc", "tile_table.h")

XTYPES = ["ci8", "ci16"]
PRODUCTS = ["I", "IQUV"]
KSTEPS = [4, 5, 6, 7, 8]
NBUCKETS = 5


def table(path: str = JSON):
    """grid[xtype][product][K-steps - 4][beam bucket] = streams, and the
    buckets' upper beam counts."""
    with open(path) as f:
        t = json.load(f)
    bks = t["beam_buckets"]
    if t["xtypes"] != XTYPES or t["products"] != PRODUCTS or t["ksteps"] != KSTEPS or len(bks) != NBUCKETS:
        raise ValueError("tiles.json: unexpected axes")
    if bks != sorted(bks) or bks[-1] < 1 << 30:
        raise ValueError("tiles.json: beam buckets must rise to an open last one (2^30)")
    grid = [[[[0] * NBUCKETS for _ in KSTEPS] for _ in PRODUCTS] for _ in XTYPES]
    for e in t["entries"]:
        ns = int(e["streams"])
        if ns not in (1, 2, 4):
            raise ValueError("tiles.json: streams must be 1, 2 or 4")
        grid[XTYPES.index(e["xtype"])][PRODUCTS.index(e["product"])][KSTEPS.index(int(e["ksteps"]))][
            bks.index(int(e["beams_max"]))] = ns
    if any(v == 0 for a in grid for b in a for c in b for v in c):
        raise ValueError("tiles.json: incomplete table")
    return grid, bks


def generate(path: str = JSON, out: str = HEADER) -> str:
    grid, bks = table(path)
    xt_rows = []
    for xi, xt in enumerate(XTYPES):
        pr_rows = []
        for pi, pr in enumerate(PRODUCTS):
            inner = ",\n".join("            {%s}" % ", ".join(str(v) for v in grid[xi][pi][k])
                               for k in range(len(KSTEPS)))
            pr_rows.append("        {   // %s, Stokes %s, K-steps 4..8\n%s}" % (xt, pr, inner))
        xt_rows.append("    {\n%s}" % ",\n".join(pr_rows))
    text = ("// tile_table.h -- generated from tiles.json by gen_tile_table.py; do not edit.\n"
            "// Sample streams per work item of the fast FP16/BF16 worker (1, 2 or 4: work\n"
            "// items of 256, 128 or 64 beams), by input type (complex int8, int16),\n"
            "// product (Stokes I, IQUV; voltages take the IQUV entry), K-steps of 8\n"
            "// stations (4..8) and beams per block part (at most %s).\n"
            "#pragma once\n\nnamespace lbf {\n\n"
            "constexpr int kTileBeamMax[%d] = {%s};\n"
            "constexpr unsigned char kTileStreams[2][2][5][%d] = {\n%s};\n\n}  // namespace lbf\n"
            % (", ".join(str(b) for b in bks[:-1]) + " and more", NBUCKETS, ", ".join(str(b) for b in bks),
               NBUCKETS, ",\n".join(xt_rows)))
    old = open(out).read() if os.path.exists(out) else None
    if old != text:
        with open(out, "w") as f:
            f.write(text)
    return out


def write_json(grid, bks, times=None, device: str = "", path: str = JSON):
    """tiles.json with one entry per cell; ``times`` (same shape as grid, a
    dict streams -> ms per cell) is kept beside each choice."""
    entries = []
    for xi, xt in enumerate(XTYPES):
        for pi, pr in enumerate(PRODUCTS):
            for ki, nk in enumerate(KSTEPS):
                for bi, bmax in enumerate(bks):
                    e = {"xtype": xt, "product": pr, "ksteps": nk, "beams_max": bmax,
                         "streams": grid[xi][pi][ki][bi]}
                    if times is not None:
                        e["ms"] = {str(k): round(v, 4) for k, v in sorted(times[xi][pi][ki][bi].items())}
                    entries.append(e)
    doc = {"note": "sample streams per work item of the fast FP16/BF16 worker (1, 2 or 4: items of 256, 128 "
                   "or 64 beams) by input type, Stokes product, K-steps of 8 stations and beams per block part; "
                   "written by tune_tiles.py from timings of the contraction",
           "device": device, "xtypes": XTYPES, "products": PRODUCTS, "ksteps": KSTEPS, "beam_buckets": bks,
           "entries": entries}
    with open(path, "w") as f:
        f.write("{\n")
        for k in ("note", "device", "xtypes", "products", "ksteps", "beam_buckets"):
            f.write(" %s: %s,\n" % (json.dumps(k), json.dumps(doc[k])))
        f.write(' "entries": [\n')
        f.write(",\n".join("  " + json.dumps(e) for e in entries))
        f.write("\n ]\n}\n")


if __name__ == "__main__":
    print(generate())
