"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/lbf.h declares, rejects malformed arguments with the documented
codes before touching the device, and its footprint arithmetic reproduces the
data rates printed in Table 1 of Mol & Romein."""
import ctypes
import os
import re

import pytest

from paper_1105_0661_amd import lbf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbf.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = lbf.lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert "gfx950" in lbf.version()


def _block(**kw):
    d = dict(d_x=1, xtype=lbf.CI16, S=4, C=8, T=64, d_w=1, ctype=lbf.F32, B=3, product=lbf.STOKES_I, t_int=16,
             f_int=1, d_out=1)
    d.update(kw)
    return lbf.Block(**d)


@pytest.mark.parametrize("kw,code", [
    (dict(S=0), lbf.E_INVAL),
    (dict(B=-1), lbf.E_INVAL),
    (dict(d_x=None), lbf.E_INVAL),
    (dict(d_out=None), lbf.E_INVAL),
    (dict(xtype=7), lbf.E_INVAL),
    (dict(ctype=9), lbf.E_INVAL),
    (dict(product=2), lbf.E_INVAL),
    (dict(T=60), lbf.E_INVAL),            # T % t_int != 0
    (dict(f_int=3), lbf.E_INVAL),         # C % f_int != 0
    (dict(t_int=0), lbf.E_INVAL),
    (dict(product=lbf.VOLTAGES, t_int=16), lbf.E_INVAL),
    (dict(t_int=3, T=63), lbf.E_UNSUPPORTED),
])
def test_beamform_rejects_malformed_blocks(kw, code):
    blk = _block(**kw)
    rc = lbf.lib().lbf_beamform(ctypes.byref(blk), None)
    assert rc == code
    assert lbf.lib().lbf_last_error().decode().startswith("lbf_beamform")


def test_other_entry_points_validate_before_device_work():
    L = lbf.lib()
    assert L.lbf_beamform(None, None) == lbf.E_INVAL
    assert L.lbf_compute_weights(None, 4, None, 2, None, None, None, 8, lbf.F32, None, None, None) == lbf.E_INVAL
    assert L.lbf_compute_weights(1, 0, 1, 2, None, None, 1, 8, lbf.F32, 1, None, None) == lbf.E_INVAL
    assert L.lbf_compute_weights(1, 4, 1, 2, None, None, 1, 8, 5, 1, None, None) == lbf.E_INVAL
    assert L.lbf_stokes(1, 2, 4, 10, lbf.STOKES_I, 3, 1, 1, None) == lbf.E_INVAL
    assert L.lbf_stokes(1, 2, 4, 12, lbf.VOLTAGES, 3, 1, 1, None) == lbf.E_INVAL
    assert L.lbf_transpose(1, 2, 3, 4, 1, 16, 2, None) == lbf.E_INVAL          # elem_bytes
    assert L.lbf_transpose(4096, 2, 3, 4, 1, 4, 4100, None) == lbf.E_INVAL     # overlap
    assert L.lbf_incoherent(1, lbf.CI8, 4, 8, 10, lbf.STOKES_I, 4, 1, 1, None) == lbf.E_INVAL
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 64, 12, None, 4096, None) == lbf.E_INVAL    # nch not a power of two
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 64, 512, None, 4096, None) == lbf.E_INVAL   # nch > 256
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 60, 16, None, 4096, None) == lbf.E_INVAL    # T_sb % nch
    assert L.lbf_channelize(16, 7, 2, 2, 64, 64, 16, None, 4096, None) == lbf.E_INVAL           # xtype
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 64, 16, None, 24, None) == lbf.E_INVAL      # alignment
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 64, 16, 2, 4096, None) == lbf.E_INVAL       # shift alignment
    assert L.lbf_channelize(4096, lbf.CI16, 2, 2, 64, 64, 16, None, 4096 + 512, None) == lbf.E_INVAL   # overlap
    assert L.lbf_channelize(16, lbf.CI16, 2, 2, 64, 64, 16, 8192, 8192, None) == lbf.E_INVAL    # shift under output
    I = ctypes.c_int
    off, mem = (I * 3)(0, 2, 3), (I * 3)(0, 1, 2)
    assert L.lbf_superstation(16, lbf.CI16, 2, 4, 8, None, 2, off, mem, 4096, None) == lbf.E_INVAL    # member 2 >= S
    assert L.lbf_superstation(16, lbf.CI16, 3, 4, 8, None, 65, off, mem, 4096, None) == lbf.E_INVAL   # G > 64
    assert L.lbf_superstation(16, lbf.CI16, 3, 4, 8, None, 2, (I * 3)(0, 2, 1), mem, 4096, None) == lbf.E_INVAL
    assert L.lbf_superstation(16, lbf.CI16, 3, 4, 8, None, 2, off, mem, 4100, None) == lbf.E_INVAL    # alignment
    assert L.lbf_superstation(4096, lbf.CI16, 3, 4, 8, None, 2, off, mem, 4096 + 64, None) == lbf.E_INVAL   # overlap
    assert L.lbf_dedisperse(16, 2, 3, 4096, 100, 16, 32, None) == lbf.E_INVAL           # n_fft
    assert L.lbf_dedisperse(16, 2, 3, 1000, 512, 16, 32, None) == lbf.E_INVAL           # T % n_fft
    assert L.lbf_dedisperse(None, 2, 3, 512, 512, 16, 32, None) == lbf.E_INVAL          # NULL
    assert L.lbf_dedisperse(16, 2, 3, 512, 512, 16, 40, None) == lbf.E_INVAL            # alignment
    assert L.lbf_dedisperse(4096, 2, 3, 512, 512, 16, 4096 + 16 * 512, None) == lbf.E_INVAL   # partial overlap
    assert L.lbf_dedisperse(1 << 40, 2, 3, 512, 512, 1 << 20, 1 << 20, None) == lbf.E_INVAL  # chirp under the output
    arr = (lbf.Block * 2)(_block(ctype=lbf.F16), _block(ctype=lbf.F16))
    assert L.lbf_beamform_batch(arr, 0, None) == lbf.E_INVAL
    assert L.lbf_beamform_batch(arr, 33, None) == lbf.E_INVAL
    arr[1] = _block(ctype=lbf.F32)
    assert L.lbf_beamform_batch(arr, 2, None) == lbf.E_UNSUPPORTED
    arr[1] = _block(ctype=lbf.F16, product=lbf.VOLTAGES, t_int=1)
    assert L.lbf_beamform_batch(arr, 2, None) == lbf.E_UNSUPPORTED
    work = ctypes.c_double()
    assert L.lbf_probe(4, 1, None, 1, 0, ctypes.byref(work), None) == lbf.E_INVAL        # unknown kind
    assert L.lbf_probe(lbf.PROBE_READ, 1, None, 1, 64, ctypes.byref(work), None) == lbf.E_INVAL   # no source
    assert L.lbf_probe(lbf.PROBE_MFMA_F16, 0, None, 1, 0, ctypes.byref(work), None) == lbf.E_INVAL
    assert L.lbf_probe(lbf.PROBE_MFMA_F32, 1, None, 1, 0, None, None) == lbf.E_INVAL
    assert L.lbf_probe(lbf.PROBE_COPY, 1, None, 1, 64, ctypes.byref(work), None) == lbf.E_INVAL
    assert L.lbf_probe(lbf.PROBE_COPY, 1, 1, 1, 8, ctypes.byref(work), None) == lbf.E_INVAL


def test_server_argument_checks_without_device():
    L = lbf.lib()
    srv = ctypes.c_void_p()
    cfg = lbf.ServerCfg(d_arena=None, arena_bytes=1 << 20, max_inflight=1, n_streams=1, queue_capacity=4,
                        max_batch=4, device=0)
    assert L.lbf_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == lbf.E_INVAL
    cfg.d_arena = 4096
    cfg.max_batch = 0
    assert L.lbf_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == lbf.E_INVAL
    st = lbf.JobStatus()
    assert L.lbf_server_poll(None, 1, ctypes.byref(st)) == lbf.E_INVAL
    assert L.lbf_server_destroy(None) == lbf.E_INVAL


def test_footprint_arithmetic():
    s = lbf.block_footprint(64, 8192, 768, 128, lbf.CI16, lbf.F32, lbf.STOKES_IQUV, 16, 1)
    assert s.input_bytes == 64 * 8192 * 768 * 2 * 4 == 3221225472
    assert s.weight_bytes == 8192 * 128 * 64 * 8
    assert s.output_bytes == 128 * 4 * 48 * 8192 * 4 == 805306368
    assert s.flops == 8 * 128 * 64 * 8192 * 768 * 2
    v = lbf.block_footprint(2, 3, 4, 5, lbf.CI8, lbf.F16, lbf.VOLTAGES)
    assert (v.input_bytes, v.weight_bytes, v.output_bytes) == (2 * 3 * 4 * 2 * 2, 3 * 5 * 2 * 4, 3 * 5 * 4 * 16)
    # Stokes staging of the fast workers: rows of B K floats padded to 32, per (channel, period)
    assert s.staging_channel_bytes == 48 * 512 * 4 and s.staging_bytes == 8192 * 48 * 512 * 4
    p = lbf.block_footprint(64, 8192, 768, 488, lbf.CI8, lbf.F16, lbf.STOKES_IQUV, 16, 1)
    assert p.staging_channel_bytes == 48 * 1952 * 4
    i = lbf.block_footprint(40, 16, 96, 150, lbf.CI16, lbf.F16, lbf.STOKES_I, 16, 1)
    assert i.staging_channel_bytes == 6 * 160 * 4
    assert v.staging_bytes == 0                                                           # voltages: none
    g = lbf.block_footprint(100, 8, 64, 40, lbf.CI8, lbf.F16, lbf.STOKES_I, 16, 1)       # > 64 stations: generic
    assert g.staging_bytes == 0
    # channel integration on the fast workers: one staging row per channel (before the channel sums)
    f = lbf.block_footprint(40, 8, 64, 40, lbf.CI8, lbf.F16, lbf.STOKES_I, 16, 2)
    assert f.staging_channel_bytes == 4 * 64 * 4 and f.staging_bytes == 8 * 4 * 64 * 4
    f3 = lbf.block_footprint(40, 9, 64, 40, lbf.CI8, lbf.F16, lbf.STOKES_I, 16, 3)        # f_int 3: generic, none
    assert f3.staging_bytes == 0


def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_rates.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                c, mode, ti, st, bm, gin, gout = line.split()
                rows.append((c, mode, int(ti), int(st), int(bm), float(gin), float(gout)))
    return rows


@pytest.mark.parametrize("row", _table1(), ids=lambda r: r[0])
def test_table1_rates_from_block_footprint(row):
    # a one-second block of the full LOFAR band: 248 subbands of 195312.5 Hz,
    # 16 channels each, complex 16-bit dual-pol input, f32 output (Section 4.6)
    case, mode, t_int, S, B, gin, gout = row
    nch, nsb = 16, 248
    T = 16 * 762                    # samples per channel in ~1 s, multiple of 16
    seconds = T * nch / 195312.5
    prod = lbf.STOKES_I if mode == "I" else lbf.STOKES_IQUV
    fp = lbf.block_footprint(S, nsb * nch, T, B, lbf.CI16, lbf.F32, prod, t_int, 1)
    rate_in = fp.input_bytes * 8 / seconds / 1e9
    rate_out = fp.output_bytes * 8 / seconds / 1e9
    # Table 1 prints whole Gb/s
    assert abs(rate_in - gin) <= 0.5, (case, rate_in)
    assert abs(rate_out - gout) <= 0.5, (case, rate_out)


def test_per_station_and_per_beam_rates():
    nch, nsb, T = 16, 248, 16 * 762
    seconds = T * nch / 195312.5
    one = lbf.block_footprint(1, nsb * nch, T, 1, lbf.CI16, lbf.F32, lbf.VOLTAGES)
    assert one.input_bytes * 8 / seconds / 1e9 == pytest.approx(3.1, abs=0.005)       # Section 2.2
    assert one.output_bytes * 8 / seconds / 1e9 == pytest.approx(6.2, abs=0.01)       # Section 4.6
    iquv = lbf.block_footprint(1, nsb * nch, T, 1, lbf.CI16, lbf.F32, lbf.STOKES_IQUV, 1)
    assert iquv.output_bytes * 8 / seconds / 1e9 == pytest.approx(6.2, abs=0.01)
    i1 = lbf.block_footprint(1, nsb * nch, T, 1, lbf.CI16, lbf.F32, lbf.STOKES_I, 1)
    assert i1.output_bytes * 8 / seconds / 1e9 == pytest.approx(1.55, abs=0.01)
    full = lbf.block_footprint(64, nsb * nch, T, 1, lbf.CI16, lbf.F32, lbf.STOKES_I, 1)
    assert full.input_bytes * 8 / seconds / 1e9 == pytest.approx(198.4, abs=0.05)     # abstract: 198 Gb/s


def test_dedisperse_stokes_argument_checks():
    L = lbf.lib()
    assert L.lbf_dedisperse_stokes(16, 1, 1, 4096, 4096, 16, lbf.STOKES_I, 3, 64, None) == lbf.E_INVAL   # t_int
    assert L.lbf_dedisperse_stokes(16, 1, 1, 4096, 4096, 16, lbf.VOLTAGES, 1, 64, None) == lbf.E_INVAL  # product
    assert L.lbf_dedisperse_stokes(16, 1, 1, 4000, 4096, 16, lbf.STOKES_I, 1, 64, None) == lbf.E_INVAL  # T
    assert L.lbf_dedisperse_stokes(16, 1, 1, 64, 64, 16, lbf.STOKES_I, 128, 64, None) == lbf.E_INVAL    # t_int > n
    assert L.lbf_dedisperse_stokes(None, 1, 1, 64, 64, 16, lbf.STOKES_I, 1, 64, None) == lbf.E_INVAL    # NULL
