"""Host-side walk of the fast workers' memory accesses (lbf_check_addressing,
no GPU): for the block shapes of the GPU tests and the uneven batch's
observations, every weight, sample and output descriptor lies inside its
buffer, no 32-bit offset wraps, and every store the epilogue means to make
lands inside its descriptor -- with the kernels' own address arithmetic, so a
base moved past the data (as once by the channel in a sample descriptor) or a
wrapping offset fails here before any kernel runs."""
import os

import pytest

from paper_1105_0661_amd import lbf, synth

pytestmark = pytest.mark.skipif(not os.path.exists(lbf.LIB_PATH), reason="liblbf.so not built")

THREADS = max(1, min(8, os.cpu_count() or 1))
X = {"ci8": lbf.CI8, "ci16": lbf.CI16, "cf32": lbf.CF32}


def _walk(S, C, T, B, xt, ct, prod, ti=1, fi=1, **kw):
    n = lbf.check_addressing(S, C, T, B, X[xt], ct, prod, ti, fi, threads=THREADS, **kw)
    assert n > 0
    return n


# (S, C, T, B, xtype, product, t_int): the fast-path shapes of the GPU parity
# tests -- ragged stations (1..64), samples (32..1100), beams (1..512, beam
# tails), every t_int, voltages and both Stokes products
TEST_SHAPES = [(13, 5, 112, 70, "ci16", lbf.VOLTAGES, 1), (1, 3, 32, 37, "ci8", lbf.STOKES_IQUV, 4),
               (7, 3, 33, 37, "ci16", lbf.STOKES_IQUV, 1), (33, 3, 100, 37, "ci8", lbf.STOKES_IQUV, 4),
               (53, 3, 80, 37, "ci16", lbf.STOKES_IQUV, 16), (64, 3, 64, 37, "ci8", lbf.STOKES_I, 4),
               (40, 2, 64, 300, "ci8", lbf.STOKES_IQUV, 16), (40, 2, 64, 385, "ci8", lbf.VOLTAGES, 1),
               (40, 2, 64, 512, "ci16", lbf.STOKES_I, 16), (11, 10, 128, 40, "ci16", lbf.STOKES_I, 2),
               (20, 3, 1100, 140, "ci8", lbf.STOKES_IQUV, 4), (20, 3, 1100, 50, "ci16", lbf.VOLTAGES, 1),
               (31, 5, 48, 1, "ci16", lbf.STOKES_I, 4), (64, 16, 768, 488, "ci8", lbf.STOKES_IQUV, 16),
               (12, 32, 64, 40, "cf32", lbf.STOKES_IQUV, 4), (13, 5, 112, 70, "cf32", lbf.VOLTAGES, 1),
               (64, 256, 48, 128, "cf32", lbf.STOKES_IQUV, 16), (40, 6, 200, 150, "cf32", lbf.STOKES_I, 8),
               (1, 1, 1, 1, "ci16", lbf.STOKES_IQUV, 1), (2, 1, 1, 1, "ci16", lbf.VOLTAGES, 1)]


@pytest.mark.parametrize("shape", TEST_SHAPES, ids=lambda s: "S%d_C%d_T%d_B%d_%s_K%d_t%d" % s)
@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16], ids=["f32", "f16"])
def test_parity_test_shapes_stay_inside_their_buffers(shape, ctype):
    S, C, T, B, xt, prod, ti = shape
    _walk(S, C, T, B, xt, ctype, prod, ti)
    if prod != lbf.VOLTAGES:
        _walk(S, C, T, B, xt, ctype, prod, ti, channel_major=True)


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16], ids=["f32", "f16"])
def test_largest_fast_path_block_stays_inside_its_buffers(ctype):
    """64 stations of complex int16, 4096 channels x 8176 samples: each
    8-station plane group just under the 2^31-byte descriptor range (the GPU
    parity test of the same shape); 16 samples more and the fast workers
    decline the block (no accesses to walk: it goes to the generic workers)."""
    assert _walk(64, 4096, 8176, 130, "ci16", ctype, lbf.STOKES_IQUV, 16) > 0
    n = lbf.check_addressing(64, 4096, 8192, 130, X["ci16"], ctype, lbf.STOKES_IQUV, 16, 1, threads=THREADS)
    assert n == 0


@pytest.mark.parametrize("j", range(12))
def test_uneven_batch_observations_stay_inside_their_buffers(j):
    js = synth.config3_jobs()[j]
    prod = lbf.PRODUCT_NAMES[js.product]
    C = js.nsb * js.nch
    n = _walk(js.S, C, js.T, js.B, js.xtype, lbf.F16, prod, js.t_int)
    # the same block through staging of a few channels at a time (the server's
    # and the no-allocation path's channel passes): every access of the whole
    # block again, and more where a pass's fewer items take shorter segments
    per = lbf.block_footprint(js.S, C, js.T, js.B, X[js.xtype], lbf.F16, prod, js.t_int).staging_channel_bytes
    assert _walk(js.S, C, js.T, js.B, js.xtype, lbf.F16, prod, js.t_int, staging_cap=7 * per) >= n


def test_staging_below_one_channel_is_refused():
    per = lbf.block_footprint(40, 8, 96, 150, lbf.CI16, lbf.F16, lbf.STOKES_IQUV, 16).staging_channel_bytes
    with pytest.raises(lbf.LbfError) as ei:
        lbf.check_addressing(40, 8, 96, 150, lbf.CI16, lbf.F16, lbf.STOKES_IQUV, 16, staging_cap=per - 4)
    assert ei.value.code == lbf.E_NOMEM


def test_blocks_outside_the_fast_path_walk_nothing():
    assert lbf.check_addressing(100, 2, 64, 30, lbf.CI8, lbf.F16, lbf.STOKES_I, 16) == 0     # > 64 stations
    assert lbf.check_addressing(20, 6, 64, 30, lbf.CI8, lbf.F16, lbf.STOKES_I, 16, 3) == 0   # f_int not a power of 2
    assert lbf.check_addressing(20, 128, 64, 30, lbf.CI8, lbf.F16, lbf.STOKES_I, 16, 128) == 0   # f_int > 64


@pytest.mark.parametrize("fi", [2, 4, 16, 64])
def test_channel_integration_walks_per_channel_staging(fi):
    # the fast workers form each channel integrated in time into staging, in
    # passes of whole f_int-channel groups, in either output order
    C = 128
    n = _walk(20, C, 96, 70, "ci16", lbf.F16, lbf.STOKES_IQUV, 16, fi)
    assert _walk(20, C, 96, 70, "ci16", lbf.F16, lbf.STOKES_IQUV, 16, fi, channel_major=True) == n
    assert n == _walk(20, C, 96, 70, "ci16", lbf.F16, lbf.STOKES_IQUV, 16, 1)      # the same accesses as f_int 1
    per = lbf.block_footprint(20, C, 96, 70, lbf.CI16, lbf.F16, lbf.STOKES_IQUV, 16, fi).staging_channel_bytes
    assert per > 0
    assert _walk(20, C, 96, 70, "ci16", lbf.F16, lbf.STOKES_IQUV, 16, fi, staging_cap=fi * per) >= n
    with pytest.raises(lbf.LbfError) as ei:
        lbf.check_addressing(20, C, 96, 70, lbf.CI16, lbf.F16, lbf.STOKES_IQUV, 16, fi, staging_cap=fi * per - 4)
    assert ei.value.code == lbf.E_NOMEM


@pytest.fixture
def streams():
    yield lbf.set_tile_streams
    lbf.set_tile_streams(0)


@pytest.mark.parametrize("ns", [1, 2, 4])
def test_every_tile_shape_stays_inside_its_buffers(ns, streams):
    # the FP16/BF16 worker's items of 256, 128 and 64 beams (1, 2, 4 sample
    # streams, forced) on the integer-sample shapes above and the uneven
    # batch's observations
    streams(ns)
    for S, C, T, B, xt, prod, ti in TEST_SHAPES:
        if xt != "cf32":
            _walk(S, C, T, B, xt, lbf.F16, prod, ti)
    for js in synth.config3_jobs()[:6]:
        _walk(js.S, js.nsb * js.nch, js.T, js.B, js.xtype, lbf.F16, lbf.PRODUCT_NAMES[js.product], js.t_int)


def test_set_tile_streams_takes_only_item_shapes(streams):
    for bad in (3, 8, -1):
        with pytest.raises(lbf.LbfError) as ei:
            streams(bad)
        assert ei.value.code == lbf.E_INVAL
    for ok in (0, 1, 2, 4):
        streams(ok)
