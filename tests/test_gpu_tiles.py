"""GPU parity of every tile shape of the FP16/BF16 fast worker: work items of
256, 128 and 64 beams (1, 2 and 4 sample streams), forced through
lbf_set_tile_streams, against the FP64 oracle (tolerances as in
test_gpu_parity), and bit for bit against each other where they must agree:
the stream count moves work between waves but every beam sample is the same
sum in the same order, so all three shapes give identical bits.  Also the
batch and incoherent-beam forms of each shape, and the measured table
(streams 0) against the forced shapes."""
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import lbf, synth
from tests._util import check_close, cplx, flush, to_dev
from tests.test_gpu_parity import CT_NAMES, TOL, _check_stokes, _check_volt, _oracle_stokes, _weights

pytestmark = pytest.mark.gpu

STREAMS = (1, 2, 4)


@pytest.fixture(autouse=True)
def _table_after():
    yield
    lbf.set_tile_streams(0)


def _torch():
    import torch
    return torch


# (S, B, nsb, nch, T, xtype): every K-step count (24..64 stations), beams
# below one 64-beam item, ragged over 64 and 128, a tail past 256 and over
# 512; ragged sample tiles and several time segments
SHAPES = [(24, 17, 1, 3, 64, "ci8"), (33, 70, 1, 3, 100, "ci16"), (41, 130, 1, 2, 96, "ci8"),
          (53, 200, 1, 2, 80, "ci16"), (64, 300, 1, 2, 64, "ci8"), (47, 520, 1, 2, 48, "ci16"),
          (29, 90, 1, 2, 1100, "ci8")]


@pytest.mark.parametrize("ctype", [lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "S%d_B%d_C%d_T%d_%s" % (s[0], s[1], s[2] * s[3], s[4], s[5]))
def test_every_stream_count_matches_oracle_and_each_other(shape, ctype):
    torch = _torch()
    S, B, nsb, nch, T, xt = shape
    blk = synth.make_block(S, B, nsb, nch, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 80))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    ti = 4 if T % 4 == 0 else 1
    got = {}
    for ns in STREAMS + (0,):
        lbf.set_tile_streams(ns)
        flush("tile streams %d %s %s" % (ns, CT_NAMES[ctype], shape))
        got[ns] = (lbf.beamform(x, w, lbf.VOLTAGES), lbf.beamform(x, w, lbf.STOKES_IQUV, ti, 1),
                   lbf.beamform(x, w, lbf.STOKES_I, ti, 1))
        torch.cuda.synchronize()
    for ns in (2, 4, 0):
        for a, b in zip(got[ns], got[1]):
            assert torch.equal(a, b), ns
    y, s4, s1 = got[1]
    _check_volt(cplx(y), orc.beamform(blk.x, orc.block_weights(blk)), TOL[ctype], "voltages")
    _check_stokes(s4.cpu().numpy(), _oracle_stokes(blk, 4, ti, 1), TOL[ctype], "IQUV", blk, ctype, ti)
    _check_stokes(s1.cpu().numpy(), _oracle_stokes(blk, 1, ti, 1), TOL[ctype], "I", blk, ctype, ti)


@pytest.mark.parametrize("ns", STREAMS)
def test_incoherent_form_of_every_stream_count(ns):
    """Blocks of at most 128 beams form the incoherent beam in the
    contraction when items have several streams (2 or 4); one stream runs
    the two kernels.  Same tied-array beams either way, incoherent beam
    against the oracle."""
    torch = _torch()
    # (the last two leave whole beam tiles idle: with two streams, and with
    # the one-accumulator form of complex int16)
    for i, (S, B, T, xt, prod, ti) in enumerate([(37, 100, 96, "ci8", lbf.STOKES_I, 4),
                                                 (64, 128, 64, "ci16", lbf.STOKES_IQUV, 16),
                                                 (26, 40, 1100, "ci8", lbf.STOKES_IQUV, 2),
                                                 (40, 20, 96, "ci16", lbf.STOKES_IQUV, 8)]):
        blk = synth.make_block(S, B, 1, 3, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 81 + i))
        x, w = to_dev(blk.x), _weights(blk, lbf.F16)
        lbf.set_tile_streams(ns)
        flush("incoherent streams %d S=%d B=%d T=%d" % (ns, S, B, T))
        out, inc = lbf.beamform_incoherent(x, w, prod, ti, 1)
        lbf.set_tile_streams(1)
        alone = lbf.beamform(x, w, prod, ti, 1)
        torch.cuda.synchronize()
        assert torch.equal(out, alone)
        K = lbf.n_stokes(prod)
        ref = orc.incoherent(blk.x, K, ti, 1)
        got = inc.cpu().numpy()
        for k in range(K):
            check_close(got[k].T[None], ref[..., k][None], 1e-5, "incoherent %s" % "IQUV"[k])


@pytest.mark.parametrize("ns", STREAMS)
def test_batch_of_every_stream_count_equals_single_launches(ns):
    torch = _torch()
    specs = [(24, 17, 2, 4, 64, "ci8", lbf.STOKES_I), (33, 200, 1, 4, 112, "ci16", lbf.STOKES_IQUV),
             (64, 70, 2, 2, 176, "ci16", lbf.STOKES_IQUV), (45, 300, 1, 3, 64, "ci8", lbf.STOKES_IQUV),
             (53, 140, 1, 3, 48, "ci16", lbf.STOKES_I)]
    lbf.set_tile_streams(ns)
    items, singles, refs = [], [], []
    for i, (S, B, nsb, nch, T, xt, prod) in enumerate(specs):
        blk = synth.make_block(S, B, nsb, nch, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 90 + i))
        x, w = to_dev(blk.x), _weights(blk, lbf.F16)
        items.append((x, w, prod, 16, 1))
        singles.append(lbf.beamform(x, w, prod, 16, 1))
        refs.append((blk, prod))
    flush("batch with %d streams" % ns)
    outs = lbf.beamform_batch(items)
    torch.cuda.synchronize()
    for o, s, (blk, prod) in zip(outs, singles, refs):
        assert torch.equal(o, s)
        _check_stokes(o.cpu().numpy(), _oracle_stokes(blk, prod, 16, 1), TOL[lbf.F16], "batch", blk, lbf.F16, 16)

