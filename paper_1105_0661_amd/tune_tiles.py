"""Measure the tile table of the fast FP16/BF16 worker on this device.

    python -m paper_1105_0661_amd.tune_tiles [--out PATH] [--C 1024] [--T 768]

For every cell of the table -- input type (complex int8, int16), product
(Stokes I, IQUV, integrated 16 samples), K-steps of 8 stations (4..8: 32 to
64 stations) and beam bucket -- the contraction (lbf_beamform_channel_major,
FP16 weights) is timed with 1, 2 and 4 sample streams per work item (work
items of 256, 128 and 64 beams), forced through lbf_set_tile_streams, on two
beam counts of the bucket; the count with the least summed time goes into the
table.  Writes tiles.json (the choices with their timings); build.py turns it
into csrc/tile_table.h.  The stream count changes only speed: every choice
gives the same results.

Inputs are random samples and geometry made on the device (no oracle, no
files).  One pass takes a few seconds."""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1105_0661_amd import gen_tile_table as gtt  # noqa: E402
from paper_1105_0661_amd import lbf  # noqa: E402

BUCKETS = [32, 64, 128, 256, 1 << 30]
# two beam counts per bucket: a ragged one and its upper end (parts of more
# than 256 beams: a ragged tail of more than 128, and a multiple of 256)
BEAMS = [(8, 32), (40, 64), (96, 128), (200, 256), (400, 512)]
STREAMS = (1, 2, 4)


def log(msg):
    print(msg, flush=True)


def _geometry(torch, S, B, C, dev, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    r = 1000.0 * torch.sqrt(torch.rand(S, generator=g, dtype=torch.float64))
    ph = 2 * math.pi * torch.rand(S, generator=g, dtype=torch.float64)
    pos = torch.stack([r * torch.cos(ph), r * torch.sin(ph), torch.zeros(S, dtype=torch.float64)], 1)
    lm = 0.02 * (torch.rand(B, 2, generator=g, dtype=torch.float64) - 0.5)
    n = torch.sqrt(1 - (lm ** 2).sum(1, keepdim=True))
    dirs = torch.cat([lm, n], 1)
    freq = 150e6 + 195312.5 / 256 * torch.arange(C, dtype=torch.float64)
    return pos.to(dev), dirs.to(dev), freq.to(dev)


def _time(torch, fn, reps):
    fn()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(3):
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=gtt.JSON)
    ap.add_argument("--C", type=int, default=1024, help="channels per timed block")
    ap.add_argument("--T", type=int, default=768, help="samples per channel")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("tune_tiles needs a GPU")
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    name = "%s (%s)" % (props.name, getattr(props, "gcnArchName", "?").split(":")[0])
    log("tuning the FP16/BF16 tile table on %s (C=%d, T=%d)" % (name, a.C, a.T))
    t_start = time.time()
    nx, npr, nk, nb = len(gtt.XTYPES), len(gtt.PRODUCTS), len(gtt.KSTEPS), len(BUCKETS)
    grid = [[[[0] * nb for _ in range(nk)] for _ in range(npr)] for _ in range(nx)]
    times = [[[[None] * nb for _ in range(nk)] for _ in range(npr)] for _ in range(nx)]
    products = {"I": lbf.STOKES_I, "IQUV": lbf.STOKES_IQUV}
    t_int = 16
    try:
        for xi, xt in enumerate(gtt.XTYPES):
            dtype, amp = (torch.int8, 40) if xt == "ci8" else (torch.int16, 2000)
            for ki, NK in enumerate(gtt.KSTEPS):
                S = 8 * NK
                x = torch.randint(-amp, amp + 1, (S, a.C, a.T, 2, 2), dtype=dtype, device=dev)
                for bi in range(nb):
                    acc = {ns: {p: 0.0 for p in gtt.PRODUCTS} for ns in STREAMS}
                    for B in BEAMS[bi]:
                        pos, dirs, freq = _geometry(torch, S, B, a.C, dev, 1000 * S + B)
                        w = lbf.compute_weights(pos, dirs, freq, lbf.F16)
                        for pname, prod in products.items():
                            out = torch.empty(lbf.output_shape(prod, S, a.C, a.T, B, t_int, 1, channel_major=True),
                                              dtype=torch.float32, device=dev)
                            for ns in STREAMS:
                                lbf.set_tile_streams(ns)
                                acc[ns][pname] += _time(torch, lambda: lbf.beamform_channel_major(
                                    x, w, prod, t_int, 1, out=out), a.reps)
                            del out
                        del w
                    for pi, pname in enumerate(gtt.PRODUCTS):
                        ms = {ns: acc[ns][pname] for ns in STREAMS}
                        best = min(STREAMS, key=lambda ns: ms[ns])
                        grid[xi][pi][ki][bi] = best
                        times[xi][pi][ki][bi] = ms
                        log("%-4s %-4s S=%2d beams %s: %s -> %d streams" % (
                            xt, pname, S, "/".join(str(b) for b in BEAMS[bi]),
                            ", ".join("%d: %.3f ms" % (ns, ms[ns]) for ns in STREAMS), best))
                del x
                torch.cuda.empty_cache()
    finally:
        lbf.set_tile_streams(0)
    gtt.write_json(grid, BUCKETS, times, device=name, path=a.out)
    log("wrote %s in %.0f s" % (a.out, time.time() - t_start))


if __name__ == "__main__":
    main()
