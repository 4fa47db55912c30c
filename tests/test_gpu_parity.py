"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle.

Tolerances: norm-wise relative L2 per output array and per Stokes parameter,
1e-5 for FP32 operands and 3e-3 for FP16/BF16 operands.  Element-wise, so that
a few wrong elements cannot hide inside a small norm: every Stokes element
within twice the rounding bound derived from the operand type (weights
rounded once, samples exact when representable, FP32 sums; the weights have
modulus 1, so a beam sample's error is at most eps sum_s |x_s|), and for FP32
and FP16 operands also max |got - oracle| <= 10 tol rms(oracle) per beam and
Stokes parameter.  (BF16 keeps 8 significant bits: over 10^5 elements its
largest error reaches about 12 tol rms, within its rounding bound.)  Pure data
movement (transpose) and exactly representable cases are compared bit for
bit.
"""
import types

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import lbf, synth
from tests._util import (check_close, check_stokes, check_stokes_bound, contraction_eps, cplx, flush, geometry,
                         relerr, stokes_bound, to_dev)

pytestmark = pytest.mark.gpu

TOL = {lbf.F32: 1e-5, lbf.F16: 3e-3, lbf.BF16: 3e-3}
CT_NAMES = {lbf.F32: "f32", lbf.F16: "f16", lbf.BF16: "bf16"}


def _torch():
    import torch
    return torch


def _weights(blk, ctype):
    pos, dirs, freq, ref = geometry(blk)
    return lbf.compute_weights(pos, dirs, freq, ctype, ref_dir=ref)


def _oracle_stokes(blk, K, t_int, f_int):
    return orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, K, t_int, f_int, 8)


def _samples_exact(x, ctype):
    """Integer samples the operand type holds exactly (complex f32 input
    is exact only with FP32 operands)."""
    if x.dtype == np.float32:
        return ctype == lbf.F32
    lim = {lbf.F32: 1 << 24, lbf.F16: 2048, lbf.BF16: 256}[ctype]
    return int(np.abs(x).max()) <= lim


def _check_stokes(out, ref, tol, label, blk=None, ctype=None, t_int=1, f_int=1, chans=None, scale="own"):
    """Norm-wise per parameter; element-wise against the rounding bound when
    the block is given (chans: the block's channels the output holds), and
    against 10 tol rms for FP32 / FP16 operands.  scale="I": Q, U and V
    against Stokes I (see check_stokes)."""
    check_stokes(out, ref, tol, label, scale=scale, elem_factor=10.0 if ctype != lbf.BF16 else float("inf"))
    if blk is None:
        return
    x = blk.x if chans is None else np.ascontiguousarray(blk.x[:, chans])
    freq = blk.freq_hz if chans is None else blk.freq_hz[chans]
    w = orc.weights(orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir), freq)
    y = orc.beamform(x, w)                                                       # [C][B][T][2]
    xc = x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)
    eps = contraction_eps(ctype, blk.S, _samples_exact(x, ctype))
    bound = stokes_bound(y, eps * np.abs(xc).sum(axis=0), ref.shape[1], t_int, f_int)
    check_stokes_bound(out, ref, bound, label)


def _check_volt(y, ref, tol, label):
    """y, ref: voltages [C][B][T][2] (complex); checked per beam."""
    check_close(np.asarray(y).transpose(1, 0, 2, 3), np.asarray(ref).transpose(1, 0, 2, 3), tol, label)


# --------------------------------------------------------------------------
# weights
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
def test_weights_match_oracle(ctype):
    torch = _torch()
    blk = synth.make_block(37, 45, 3, 16, 16, generate=False, tag=(1105, 661, 50))
    flush("weights %s S=37 B=45 C=48" % CT_NAMES[ctype])
    pos, dirs, freq, ref = geometry(blk)
    tau = torch.empty((45, 37), dtype=torch.float64, device="cuda:0")
    w = lbf.compute_weights(pos, dirs, freq, ctype, ref_dir=ref, tau=tau)
    torch.cuda.synchronize()
    tau_o = orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir)
    assert np.max(np.abs(tau.cpu().numpy() - tau_o)) <= 1e-15 * max(1.0, np.max(np.abs(tau_o))) + 1e-22
    w_o = orc.weights(tau_o, blk.freq_hz)
    g = cplx(w.float())
    err = np.max(np.abs(g - w_o))
    half_ulp = {lbf.F32: 2.0 ** -24, lbf.F16: 2.0 ** -11, lbf.BF16: 2.0 ** -8}[ctype]
    assert err <= half_ulp + 1e-12, err
    if ctype == lbf.F16:
        # one rounding from FP64: equal to numpy's double->half rounding
        exp = np.stack([w_o.real, w_o.imag], -1).astype(np.float16)
        same = np.mean(w.cpu().numpy() == exp)
        assert same >= 0.9999, same


def test_weights_large_phase_needs_fp64():
    # remote stations (hundreds of km) put f*tau at thousands of turns: the
    # device FP64 reduction still matches the oracle to FP32 rounding
    torch = _torch()
    blk = synth.make_block(8, 6, 2, 8, 16, generate=False, tag=(1105, 661, 51), radius_m=3.0e5)
    pos, dirs, freq, _ = geometry(blk, ref=False)
    w = lbf.compute_weights(pos, dirs, freq, lbf.F32, ref_dir=None)
    torch.cuda.synchronize()
    w_o = orc.weights(orc.delays(blk.station_xyz, blk.beam_dir, None), blk.freq_hz)
    m = np.max(np.abs(blk.freq_hz[:, None, None] * orc.delays(blk.station_xyz, blk.beam_dir, None)[None]))
    assert m > 1000
    assert np.max(np.abs(cplx(w) - w_o)) <= 2.0 ** -24 + 1e-9


# --------------------------------------------------------------------------
# the contraction: voltages
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("xtype", ["ci8", "ci16", "cf32"])
def test_voltages_match_oracle(xtype, ctype):
    torch = _torch()
    sigma = {"ci8": 20.0, "ci16": 40.0, "cf32": 30.0}[xtype]
    # ragged everywhere: 13 stations (not a multiple of 8), 70 beams (not of 32),
    # 112 samples (not of 32), several channels
    blk = synth.make_block(13, 70, 1, 5, 112, xtype, sigma, tag=(1105, 661, 52))
    flush("voltages %s %s S=13 B=70 C=5 T=112" % (xtype, CT_NAMES[ctype]))
    x = to_dev(blk.x)
    w = _weights(blk, ctype)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    torch.cuda.synchronize()
    ref = orc.beamform(blk.x, orc.block_weights(blk))          # [C][B][T][2]
    _check_volt(cplx(y), ref, TOL[ctype], "voltages")


def test_single_station_zero_delay_is_identity():
    torch = _torch()
    blk = synth.make_block(1, 1, 1, 4, 96, "ci16", 3000.0, tag=(1105, 661, 53))
    x = to_dev(blk.x)
    w = torch.zeros((4, 1, 1, 2), dtype=torch.float32, device="cuda:0")
    w[..., 0] = 1.0
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    torch.cuda.synchronize()
    assert np.array_equal(y[:, 0].cpu().numpy(), blk.x[0].astype(np.float32))


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("S,T", [(1, 32), (7, 33), (24, 96), (33, 100), (38, 64), (41, 72), (48, 64), (53, 80),
                                 (56, 40), (64, 64)])
def test_fast_path_station_and_sample_edges(ctype, S, T):
    # the fast workers pad stations to 8-station groups (zero beyond S; the
    # FP16/BF16 one to 32, 40, 48, 56 or 64 stations) and clamp the rows of a
    # ragged last sample tile
    torch = _torch()
    xt = "ci8" if ctype == lbf.BF16 else "ci16"
    blk = synth.make_block(S, 37, 1, 3, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 59))
    flush("fast edges %s S=%d T=%d" % (CT_NAMES[ctype], S, T))
    x = to_dev(blk.x)
    w = _weights(blk, ctype)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    ti = 1 if T % 2 else 4
    s = lbf.beamform(x, w, lbf.STOKES_IQUV, ti, 1)
    torch.cuda.synchronize()
    ref = orc.beamform(blk.x, orc.block_weights(blk))
    _check_volt(cplx(y), ref, TOL[ctype], "fast edges voltages")
    _check_stokes(s.cpu().numpy(), _oracle_stokes(blk, 4, ti, 1), TOL[ctype], "fast edges", blk, ctype, ti)


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("S", [1, 2, 65])
def test_one_sample_one_channel_one_beam(ctype, S):
    # the smallest block: one channel, one beam, one sample (one output sample
    # of each Stokes parameter), on the fast workers (1, 2 stations) and the
    # generic ones (65 stations)
    torch = _torch()
    blk = synth.make_block(S, 1, 1, 1, 1, "ci16", 40.0, tag=(1105, 661, 71))
    flush("one sample %s S=%d" % (CT_NAMES[ctype], S))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    s1 = lbf.beamform(x, w, lbf.STOKES_I, 1, 1)
    s4 = lbf.beamform(x, w, lbf.STOKES_IQUV, 1, 1)
    torch.cuda.synchronize()
    assert tuple(y.shape) == (1, 1, 1, 2, 2) and tuple(s4.shape) == (1, 4, 1, 1)
    _check_volt(cplx(y), orc.beamform(blk.x, orc.block_weights(blk)), TOL[ctype], "one-sample voltages")
    _check_stokes(s1.cpu().numpy(), _oracle_stokes(blk, 1, 1, 1), TOL[ctype], "one-sample I", blk, ctype, 1)
    _check_stokes(s4.cpu().numpy(), _oracle_stokes(blk, 4, 1, 1), TOL[ctype], "one-sample IQUV", blk, ctype, 1,
                  scale="I")


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("S,B,T,t_int", [(40, 150, 200, 8), (64, 300, 96, 16), (7, 20, 45, 1)])
def test_complex_float_input_on_the_fast_path(ctype, S, B, T, t_int):
    # channelised (complex f32) station samples through the fast workers: one
    # 16-byte load per sample, rounded to the operand type in the loaders.
    # BF16 rounds the (non-integer) samples as well as the weights to 8
    # significant bits: there Q, U and V (noise-like, with norms below that
    # of I) are measured against Stokes I; every element still meets its
    # rounding bound
    torch = _torch()
    blk = synth.make_block(S, B, 2, 3, T, "cf32", 30.0, tag=(1105, 661, 67))
    flush("cf32 fast %s S=%d B=%d T=%d" % (CT_NAMES[ctype], S, B, T))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    ti = t_int if T % t_int == 0 else 1
    s = lbf.beamform(x, w, lbf.STOKES_IQUV, ti, 1)
    torch.cuda.synchronize()
    _check_volt(cplx(y), orc.beamform(blk.x, orc.block_weights(blk)), TOL[ctype], "cf32 voltages")
    _check_stokes(s.cpu().numpy(), _oracle_stokes(blk, 4, ti, 1), TOL[ctype], "cf32 Stokes", blk, ctype, ti,
                  scale="I" if ctype == lbf.BF16 else "own")


@pytest.mark.parametrize("ctype", [lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("B", [300, 384, 385, 512])
def test_beam_tail_items(ctype, B):
    # beams past the last whole 256-beam group: up to 128 of them run as
    # 128-beam items (300, 384), more as one more 256-beam group (385)
    torch = _torch()
    blk = synth.make_block(40, B, 1, 2, 64, "ci8", 16.0, tag=(1105, 661, 58))
    flush("beam tail %s B=%d" % (CT_NAMES[ctype], B))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    s = lbf.beamform(x, w, lbf.STOKES_IQUV, 16, 1)
    torch.cuda.synchronize()
    _check_volt(cplx(y), orc.beamform(blk.x, orc.block_weights(blk)), TOL[ctype], "beam tail voltages")
    _check_stokes(s.cpu().numpy(), _oracle_stokes(blk, 4, 16, 1), TOL[ctype], "beam tail", blk, ctype, 16)


def test_stations_over_one_chunk_and_several_beam_groups():
    torch = _torch()
    blk = synth.make_block(100, 300, 1, 2, 64, "ci8", 12.0, tag=(1105, 661, 54))
    ref = orc.beamform(blk.x, orc.block_weights(blk))
    x = to_dev(blk.x)
    for ct in (lbf.F32, lbf.F16):
        flush("voltages S=100 B=300 %s" % CT_NAMES[ct])
        y = lbf.beamform(x, _weights(blk, ct), lbf.VOLTAGES)
        torch.cuda.synchronize()
        _check_volt(cplx(y), ref, TOL[ct], "S=100 voltages")


# --------------------------------------------------------------------------
# fused Stokes + integration + beam-major order
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("product,t_int,f_int", [
    (lbf.STOKES_I, 1, 1), (lbf.STOKES_I, 16, 1), (lbf.STOKES_IQUV, 16, 1), (lbf.STOKES_IQUV, 2, 2),
    (lbf.STOKES_IQUV, 4, 1), (lbf.STOKES_I, 8, 5), (lbf.STOKES_IQUV, 32, 1), (lbf.STOKES_I, 64, 1),
])
def test_fused_stokes_match_oracle(ctype, product, t_int, f_int):
    torch = _torch()
    xtype = "ci8" if ctype == lbf.BF16 else "ci16"
    blk = synth.make_block(11, 40, 2, 5, 128, xtype, 16.0 if xtype == "ci8" else 40.0, tag=(1105, 661, 55))
    flush("fused %s K=%d t_int=%d f_int=%d" % (CT_NAMES[ctype], product, t_int, f_int))
    x = to_dev(blk.x)
    out = lbf.beamform(x, _weights(blk, ctype), product, t_int, f_int)
    torch.cuda.synchronize()
    ref = _oracle_stokes(blk, product, t_int, f_int)
    assert out.shape == ref.shape
    _check_stokes(out.cpu().numpy(), ref, TOL[ctype], "fused", blk, ctype, t_int, f_int)


def test_unfused_chain_matches_oracle_and_fused():
    torch = _torch()
    blk = synth.make_block(9, 35, 2, 4, 96, "ci16", 50.0, tag=(1105, 661, 56))
    x = to_dev(blk.x)
    w = _weights(blk, lbf.F32)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    s = lbf.stokes(y, lbf.STOKES_IQUV, 8, 2)                   # [C'][B][T'][K]
    o = lbf.transpose(s)                                        # [B][K][T'][C']
    fused = lbf.beamform(x, w, lbf.STOKES_IQUV, 8, 2)
    torch.cuda.synchronize()
    ref = _oracle_stokes(blk, 4, 8, 2)
    _check_stokes(o.cpu().numpy(), ref, 1e-5, "unfused")
    _check_stokes(fused.cpu().numpy(), o.cpu().numpy(), 1e-5, "fused vs unfused")
    # lbf_stokes accepts any divisor, also where the fused path does not
    s3 = lbf.stokes(y, lbf.STOKES_I, 3, 1)
    torch.cuda.synchronize()
    ref3 = orc.integrate(orc.stokes(orc.beamform(blk.x, orc.block_weights(blk))), 1, 3, 1)
    check_close(s3.cpu().numpy().transpose(1, 0, 2, 3), ref3.transpose(1, 0, 2, 3), 1e-5, "lbf_stokes t_int 3")
    with pytest.raises(lbf.LbfError) as ei:
        lbf.beamform(x, w, lbf.STOKES_I, 3, 1)
    assert ei.value.code == lbf.E_UNSUPPORTED


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
@pytest.mark.parametrize("product,t_int,f_int", [(lbf.STOKES_IQUV, 16, 2), (lbf.STOKES_I, 4, 4),
                                                 (lbf.STOKES_IQUV, 8, 16), (lbf.STOKES_I, 16, 64)])
def test_channel_integration_on_the_fast_workers(ctype, product, t_int, f_int):
    """Channel integration (f_int a power of two up to 64) on the fast
    workers: each channel integrated in time into staging, then the f_int
    channel sums -- against the oracle, the same bits in both output orders
    and through lbf_beamform_noalloc."""
    torch = _torch()
    xtype = "ci8" if ctype != lbf.F32 else "ci16"
    blk = synth.make_block(37, 70, 2, 64, 128, xtype, 16.0 if xtype == "ci8" else 40.0, tag=(1105, 661, 78))
    flush("channel integration %s K=%d t_int=%d f_int=%d" % (CT_NAMES[ctype], product, t_int, f_int))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    out = lbf.beamform(x, w, product, t_int, f_int)
    cm = lbf.beamform_channel_major(x, w, product, t_int, f_int)
    na = lbf.beamform_noalloc(x, w, product, t_int, f_int)
    torch.cuda.synchronize()
    assert torch.equal(lbf.beam_major(cm), out)
    assert torch.equal(na, out)
    _check_stokes(out.cpu().numpy(), _oracle_stokes(blk, product, t_int, f_int), TOL[ctype], "channel integration",
                  blk, ctype, t_int, f_int)


def test_transpose_is_exact():
    # element-wise kernel (rows that 16-byte accesses do not fit, or
    # misaligned buffers) and the 16-byte tile kernel, with ragged tiles of
    # both: channels and (t, k) values not multiples of 64
    torch = _torch()
    g = torch.Generator(device="cuda:0").manual_seed(3)
    for shape in [(37, 5, 9, 4), (196, 5, 12, 4), (128, 7, 20, 1), (68, 2, 33, 4), (4, 1, 1, 4)]:
        a = torch.randn(shape, device="cuda:0", generator=g)
        o = lbf.transpose(a)
        torch.cuda.synchronize()
        assert torch.equal(o, a.permute(1, 3, 2, 0).contiguous()), shape
    for shape in [(33, 3, 70, 2, 2), (66, 3, 70, 2, 2), (130, 2, 65, 2, 2)]:
        v = torch.randn(shape, device="cuda:0", generator=g)
        ov = lbf.transpose(v)
        torch.cuda.synchronize()
        assert torch.equal(ov, v.permute(1, 3, 2, 0, 4).contiguous()), shape
    # a buffer 4 bytes off 16-byte alignment takes the element-wise kernel
    base = torch.randn(196 * 5 * 12 * 4 + 1, device="cuda:0", generator=g)
    a = base[1:].view(196, 5, 12, 4)
    o = lbf.transpose(a)
    torch.cuda.synchronize()
    assert torch.equal(o, a.permute(1, 3, 2, 0).contiguous())


@pytest.mark.parametrize("ctype,S,product,t_int,f_int", [
    (lbf.F32, 11, lbf.STOKES_IQUV, 16, 1),      # fast FP32 worker
    (lbf.F16, 33, lbf.STOKES_I, 4, 1),          # fast FP16 worker
    (lbf.BF16, 11, lbf.STOKES_IQUV, 8, 1),      # fast BF16 worker
    (lbf.F16, 70, lbf.STOKES_IQUV, 16, 1),      # generic worker (> 64 stations)
    (lbf.F32, 11, lbf.STOKES_IQUV, 2, 2),       # fast worker, channel sums out of the staging
    (lbf.BF16, 9, lbf.STOKES_I, 64, 1),         # generic worker (t_int >= 32)
], ids=["f32-fast", "f16-fast", "bf16-fast", "f16-S70", "f32-fint2", "bf16-tint64"])
def test_channel_major_then_beam_major_equals_fused(ctype, S, product, t_int, f_int):
    torch = _torch()
    xtype = "ci8" if ctype != lbf.F32 else "ci16"
    blk = synth.make_block(S, 75, 2, 4, 128, xtype, 16.0 if xtype == "ci8" else 40.0, tag=(1105, 661, 65))
    flush("channel-major %s S=%d K=%d t_int=%d f_int=%d" % (CT_NAMES[ctype], S, product, t_int, f_int))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    cm = lbf.beamform_channel_major(x, w, product, t_int, f_int)      # [C'][T'][B][K]
    bm = lbf.beam_major(cm)
    fused = lbf.beamform(x, w, product, t_int, f_int)
    torch.cuda.synchronize()
    assert cm.shape == (blk.C // f_int, blk.T // t_int, blk.B, product)
    assert torch.equal(bm, fused)
    assert torch.equal(bm, cm.permute(2, 3, 1, 0).contiguous())     # out[b][k][t][c] = cm[c][t][b][k]
    _check_stokes(bm.cpu().numpy(), _oracle_stokes(blk, product, t_int, f_int), TOL[ctype], "channel-major", blk,
                  ctype, t_int, f_int)


@pytest.mark.parametrize("ctype,B,xtype", [(lbf.F16, 140, "ci8"), (lbf.BF16, 50, "ci16"), (lbf.F16, 50, "ci16")],
                         ids=["f16-B140-ci8", "bf16-B50-ci16", "f16-B50-ci16"])
def test_long_block_is_cut_into_time_segments(ctype, B, xtype):
    # more than 24 tiles of 32 samples: work items cover segments of the block
    torch = _torch()
    blk = synth.make_block(20, B, 1, 3, 1100, xtype, 16.0 if xtype == "ci8" else 40.0, tag=(1105, 661, 66))
    flush("time segments %s B=%d T=1100" % (CT_NAMES[ctype], B))
    x, w = to_dev(blk.x), _weights(blk, ctype)
    out = lbf.beamform(x, w, lbf.STOKES_IQUV, 4, 1)
    y = lbf.beamform(x, w, lbf.VOLTAGES)
    torch.cuda.synchronize()
    _check_stokes(out.cpu().numpy(), _oracle_stokes(blk, 4, 4, 1), TOL[ctype], "segments", blk, ctype, 4)
    _check_volt(cplx(y), orc.beamform(blk.x, orc.block_weights(blk)), TOL[ctype], "segments voltages")


def test_beam_major_reorder_is_exact():
    torch = _torch()
    g = torch.Generator(device="cuda:0").manual_seed(4)
    for shape in [(37, 9, 70, 4), (1, 1, 1, 1), (65, 3, 129, 1), (3, 300, 5, 4)]:   # [C2][T2][B][K]
        a = torch.randn(shape, device="cuda:0", generator=g)
        o = lbf.beam_major(a)
        torch.cuda.synchronize()
        assert torch.equal(o, a.permute(2, 3, 1, 0).contiguous()), shape
    a = torch.randn((4, 4, 4, 4), device="cuda:0", generator=g)
    with pytest.raises(lbf.LbfError) as ei:
        lbf.beam_major(a, out=a)
    assert ei.value.code == lbf.E_INVAL


def test_voltages_beam_major_order_matches_oracle():
    torch = _torch()
    blk = synth.make_block(6, 33, 1, 3, 40, "ci8", 10.0, tag=(1105, 661, 57))
    x = to_dev(blk.x)
    y = lbf.beamform(x, _weights(blk, lbf.F32), lbf.VOLTAGES)
    vb = lbf.transpose(y)                                       # [B][2][T][C][2]
    torch.cuda.synchronize()
    ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, 0, 1, 1, 4)
    check_close(cplx(vb), ref, 1e-5, "beam-major voltages")


# (S, nsb, nch, T, xtype, product, t_int, f_int): power-of-two periods inside
# one lane, across lanes and across a whole wave's run, ragged row ends, 5
# stations (not a multiple of the 4-station unroll); then integrations the
# vector form does not take (t_int 12 and 3, rows of 24 bytes) and go through
# the generic kernel
INCOHERENT_CASES = [(7, 2, 4, 64, "ci16", lbf.STOKES_IQUV, 8, 2), (64, 2, 16, 768, "ci16", lbf.STOKES_IQUV, 16, 1),
                    (5, 1, 6, 520, "ci8", lbf.STOKES_I, 8, 2), (3, 1, 3, 70, "cf32", lbf.STOKES_IQUV, 2, 1),
                    (4, 1, 2, 12, "ci8", lbf.STOKES_IQUV, 1, 1), (9, 1, 3, 512, "ci8", lbf.STOKES_IQUV, 256, 3),
                    (6, 1, 2, 256, "ci16", lbf.STOKES_I, 128, 1), (2, 1, 2, 128, "cf32", lbf.STOKES_IQUV, 64, 2),
                    (8, 1, 4, 96, "ci16", lbf.STOKES_IQUV, 12, 2), (3, 1, 2, 6, "ci8", lbf.STOKES_IQUV, 3, 1)]


@pytest.mark.parametrize("case", INCOHERENT_CASES, ids=lambda c: "S%d_C%d_T%d_%s_K%d_t%d_f%d" % (
    c[0], c[1] * c[2], c[3], c[4], lbf.n_stokes(c[5]), c[6], c[7]))
def test_incoherent_beam_matches_oracle(case):
    torch = _torch()
    S, nsb, nch, T, xt, prod, ti, fi = case
    blk = synth.make_block(S, 1, nsb, nch, T, xt, 16.0 if xt == "ci8" else 30.0, tag=(1105, 661, 58))
    x = to_dev(blk.x)
    flush("incoherent %s" % (case,))
    out = lbf.incoherent(x, prod, ti, fi)
    torch.cuda.synchronize()
    K = lbf.n_stokes(prod)
    ref = orc.incoherent(blk.x, K, ti, fi)                      # [C'][T'][K]
    got = out.cpu().numpy()                                      # [K][T'][C']
    for k in range(K):
        check_close(got[k].T[None], ref[..., k][None], 1e-5, "incoherent %s" % "IQUV"[k])


# (S, B, nsb, nch, T, xtype, ctype, product, t_int): blocks of at most 128
# beams on the FP16/BF16 fast worker form the incoherent beam in the
# contraction -- every K-step count, ragged T, several time segments, every
# fused t_int, both input integer types; then blocks that run the two kernels
# (more beams, complex f32, FP32 operands, 70 stations)
INC_CASES = [(11, 40, 2, 5, 128, "ci16", lbf.F16, lbf.STOKES_IQUV, 16),
             (37, 100, 1, 4, 96, "ci8", lbf.F16, lbf.STOKES_I, 4),
             (53, 120, 1, 3, 80, "ci8", lbf.BF16, lbf.STOKES_IQUV, 8),
             (64, 128, 1, 3, 64, "ci8", lbf.F16, lbf.STOKES_IQUV, 16),
             (29, 20, 2, 3, 1100, "ci16", lbf.BF16, lbf.STOKES_I, 2),
             (40, 90, 1, 4, 208, "ci8", lbf.F16, lbf.STOKES_IQUV, 1),
             (45, 70, 1, 2, 300, "ci16", lbf.F16, lbf.STOKES_IQUV, 4),
             (64, 488, 1, 3, 64, "ci8", lbf.F16, lbf.STOKES_IQUV, 16),
             (25, 60, 1, 3, 96, "cf32", lbf.F16, lbf.STOKES_IQUV, 16),
             (12, 30, 1, 4, 64, "ci16", lbf.F32, lbf.STOKES_IQUV, 16),
             (70, 40, 1, 4, 64, "ci8", lbf.F16, lbf.STOKES_IQUV, 16)]


@pytest.mark.parametrize("case", INC_CASES, ids=lambda c: "S%d_B%d_C%d_T%d_%s_%s_K%d_t%d" % (
    c[0], c[1], c[2] * c[3], c[4], c[5], CT_NAMES[c[6]], c[7], c[8]))
def test_beamform_with_incoherent_beam(case):
    """The tied-array beams and the incoherent beam from one call: the beams
    bitwise equal to lbf_beamform, the incoherent beam against the oracle
    (1e-5; 3e-3 for complex f32 samples rounded to the operand type) and
    against lbf_incoherent."""
    torch = _torch()
    S, B, nsb, nch, T, xt, ct, prod, ti = case
    blk = synth.make_block(S, B, nsb, nch, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 68))
    flush("beamform + incoherent %s" % (case,))
    x, w = to_dev(blk.x), _weights(blk, ct)
    out, inc = lbf.beamform_incoherent(x, w, prod, ti, 1)
    alone = lbf.beamform(x, w, prod, ti, 1)
    inc2 = lbf.incoherent(x, prod, ti, 1)
    torch.cuda.synchronize()
    assert torch.equal(out, alone)
    K = lbf.n_stokes(prod)
    ref = orc.incoherent(blk.x, K, ti, 1)                       # [C'][T'][K]
    got = inc.cpu().numpy()                                      # [K][T'][C']
    tol = 3e-3 if xt == "cf32" and ct != lbf.F32 else 1e-5
    for k in range(K):
        check_close(got[k].T[None], ref[..., k][None], tol, "incoherent %s" % "IQUV"[k])
    if tol == 1e-5:
        check_close(got[None], inc2.cpu().numpy()[None], 1e-6, "fused vs lbf_incoherent")


def test_beamform_incoherent_with_channel_integration():
    """Channel integration: the tied-array beams through the staged channel
    sums, the incoherent beam by lbf_incoherent -- beams bitwise lbf_beamform,
    incoherent beam against the oracle."""
    torch = _torch()
    blk = synth.make_block(30, 50, 2, 8, 64, "ci8", 16.0, tag=(1105, 661, 77))
    x, w = to_dev(blk.x), _weights(blk, lbf.F16)
    flush("beamform + incoherent with f_int 4")
    out, inc = lbf.beamform_incoherent(x, w, lbf.STOKES_IQUV, 8, 4)
    alone = lbf.beamform(x, w, lbf.STOKES_IQUV, 8, 4)
    torch.cuda.synchronize()
    assert torch.equal(out, alone)
    ref = orc.incoherent(blk.x, 4, 8, 4)                          # [C'][T'][K]
    got = inc.cpu().numpy()                                       # [K][T'][C']
    for k in range(4):
        check_close(got[k].T[None], ref[..., k][None], 1e-5, "incoherent %s" % "IQUV"[k])


def test_beamform_incoherent_rejects_voltages_and_overlap():
    torch = _torch()
    blk = synth.make_block(8, 10, 1, 2, 64, "ci8", 16.0, tag=(1105, 661, 69))
    x, w = to_dev(blk.x), _weights(blk, lbf.F16)
    with pytest.raises(lbf.LbfError) as ei:
        lbf.beamform_incoherent(x, w, lbf.VOLTAGES)
    assert ei.value.code == lbf.E_INVAL
    out = torch.empty((10, 4, 4, 2), device="cuda:0")
    with pytest.raises(lbf.LbfError) as ei:
        lbf.beamform_incoherent(x, w, lbf.STOKES_IQUV, 16, 1, out=out, inc=out[0])
    assert ei.value.code == lbf.E_INVAL


# --------------------------------------------------------------------------
# batches: persistent launches per worker variant == separate launches, bit for bit
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctype", [lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
def test_batch_equals_single_launches_bitwise(ctype):
    torch = _torch()
    # batch-kernel blocks (t_int 16, no channel integration): one and two
    # sample streams (more / at most 128 beams), 4 to 8 K-steps, ragged
    # T, a beam tail split off a 256-beam group, two blocks of one worker
    # variant in one launch; the rest run through their own launches
    specs = [(24, 17, 2, 4, 64, "ci8", lbf.STOKES_I, 16, 1), (29, 130, 2, 3, 208, "ci8", lbf.STOKES_IQUV, 16, 1),
             (33, 200, 1, 4, 112, "ci16", lbf.STOKES_I, 16, 1), (64, 40, 2, 4, 176, "ci16", lbf.STOKES_IQUV, 16, 1),
             (40, 150, 1, 8, 96, "ci16", lbf.STOKES_IQUV, 16, 2), (45, 300, 1, 3, 64, "ci8", lbf.STOKES_IQUV, 16, 1),
             (64, 33, 3, 2, 32, "ci8", lbf.STOKES_IQUV, 32, 1), (31, 1, 1, 5, 48, "ci16", lbf.STOKES_I, 4, 1),
             (26, 20, 1, 3, 80, "ci8", lbf.STOKES_I, 16, 1), (53, 140, 1, 3, 48, "ci16", lbf.STOKES_IQUV, 16, 1),
             (38, 60, 2, 2, 64, "ci8", lbf.STOKES_I, 16, 1)]
    items, singles, refs = [], [], []
    for i, (S, B, nsb, nch, T, xt, prod, ti, fi) in enumerate(specs):
        blk = synth.make_block(S, B, nsb, nch, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 60 + i))
        x, w = to_dev(blk.x), _weights(blk, ctype)
        items.append((x, w, prod, ti, fi))
        singles.append(lbf.beamform(x, w, prod, ti, fi))
        refs.append((blk, prod, ti, fi))
    flush("batch of %d blocks %s" % (len(items), CT_NAMES[ctype]))
    outs = lbf.beamform_batch(items)
    torch.cuda.synchronize()
    for o, s, (blk, prod, ti, fi) in zip(outs, singles, refs):
        assert torch.equal(o, s)
        _check_stokes(o.cpu().numpy(), _oracle_stokes(blk, prod, ti, fi), TOL[ctype], "batch", blk, ctype, ti, fi)


def test_uneven_batch_full_size_sampled():
    """The twelve one-second observations of the uneven batch (stations
    24-64, beams 1-400, 16/64/256 channels per subband, 8-64 subbands,
    complex int8/int16, Stokes I or IQUV; 11 GB of samples) in one
    lbf_beamform_batch call: every block bitwise equal to lbf_beamform on it
    alone, and sampled channels of every block (two drawn by seed plus the
    tone's) against the oracle."""
    torch = _torch()
    jobs = synth.config3_jobs()
    items, blks = [], []
    for i, js in enumerate(jobs):
        blk = synth.block_for_job(js)
        flush("uneven batch job %d: S=%d B=%d nch=%d nsb=%d T=%d %s %s" % (i, js.S, js.B, js.nch, js.nsb, js.T,
                                                                          js.xtype, js.product))
        x = to_dev(blk.x)
        items.append((x, _weights(blk, lbf.F16), lbf.PRODUCT_NAMES[js.product], js.t_int, 1))
        blks.append(blk)
    flush("uneven batch: one lbf_beamform_batch call over %d blocks" % len(items))
    outs = lbf.beamform_batch(items)
    torch.cuda.synchronize()
    for i, (it, o, blk) in enumerate(zip(items, outs, blks)):
        single = lbf.beamform(*it)
        torch.cuda.synchronize()
        assert torch.equal(o, single), i
        del single
        chans = np.unique(np.concatenate([_sampled_channels(blk.C, 2, 100 + i), [t.channel for t in blk.tones]]))
        got = o[:, :, :, torch.from_numpy(chans).to("cuda:0")].cpu().numpy()
        xs = np.ascontiguousarray(blk.x[:, chans])
        K = it[2]
        ref = orc.pipeline(xs, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz[chans], K, 16, 1, 16)
        flush("  job %d: channels %s checked" % (i, list(chans)))
        _check_stokes(got, ref, 3e-3, "uneven batch job %d" % i, blk, lbf.F16, 16, 1, chans)


# --------------------------------------------------------------------------
# full-size blocks, sampled channels
# --------------------------------------------------------------------------

def _sampled_channels(C, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(C, size=n, replace=False))


def test_one_second_block_fp32_sampled():
    torch = _torch()
    blk = synth.config1()
    flush("full one-second block FP32: S=64 B=128 C=8192 T=768 CI16 IQUV/16")
    x = to_dev(blk.x)
    w = _weights(blk, lbf.F32)
    out = lbf.beamform(x, w, lbf.STOKES_IQUV, 16, 1)
    torch.cuda.synchronize()
    chans = _sampled_channels(blk.C, 6, 1)
    # include the channels that hold the injected tones
    chans = np.unique(np.concatenate([chans, [t.channel for t in blk.tones]]))
    got = out[:, :, :, torch.from_numpy(chans).to("cuda:0")].cpu().numpy()
    del x, w, out
    xs = np.ascontiguousarray(blk.x[:, chans])
    ref = orc.pipeline(xs, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz[chans], 4, 16, 1, 16)
    _check_stokes(got, ref, 1e-5, "one-second FP32", blk, lbf.F32, 16, 1, chans)


@pytest.mark.parametrize("ctype", [lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
def test_precision_block_sampled(ctype):
    torch = _torch()
    blk = synth.config2()
    flush("full precision block %s: S=64 B=488 C=8192 T=768 CI8 IQUV/16" % CT_NAMES[ctype])
    x = to_dev(blk.x)
    w = _weights(blk, ctype)
    out = lbf.beamform(x, w, lbf.STOKES_IQUV, 16, 1)
    torch.cuda.synchronize()
    chans = np.unique(np.concatenate([_sampled_channels(blk.C, 4, 2), [t.channel for t in blk.tones]]))
    idx = torch.from_numpy(chans).to("cuda:0")
    got = out[:, :, :, idx].cpu().numpy()
    # voltages of the sampled channels through the same kernel (channel slice)
    xs_np = np.ascontiguousarray(blk.x[:, chans])
    y = lbf.beamform(to_dev(xs_np), w[idx].contiguous(), lbf.VOLTAGES)
    torch.cuda.synchronize()
    del x, w, out
    ref = orc.pipeline(xs_np, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz[chans], 4, 16, 1, 16)
    _check_stokes(got, ref, 3e-3, "precision block", blk, ctype, 16, 1, chans)
    yo = orc.beamform(xs_np, orc.weights(orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir), blk.freq_hz[chans]))
    ev = relerr(cplx(y), yo)
    flush("  voltage rel err %s: %.3g" % (CT_NAMES[ctype], ev))
    _check_volt(cplx(y), yo, 3e-3, "precision block voltages")


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16], ids=lambda c: CT_NAMES[c])
def test_largest_fast_path_block_sampled(ctype):
    """The largest block the fast workers take: 64 stations whose 8-station
    planes of complex int16 samples (4096 channels x 8176 samples) just fit
    the 2^31-byte buffer descriptors, 130 beams, a ragged last sample tile of
    16.  The first and last 256 samples of the first, middle and last
    channels (the largest offsets) against the oracle.  Samples: seeded
    Gaussian noise (sigma 64) drawn on the device, copied back for the
    oracle."""
    torch = _torch()
    S, B, C, T = 64, 130, 4096, 8176
    assert 8 * C * T * 8 < 2 ** 31 - 4096 < 8 * C * (T + 16) * 8
    blk = synth.make_block(S, B, 16, 256, T, "ci16", generate=False)
    flush("largest fast-path block %s: S=%d B=%d C=%d T=%d CI16 IQUV/16" % (CT_NAMES[ctype], S, B, C, T))
    g = torch.Generator(device="cuda:0").manual_seed(20260)
    x = torch.empty((S, C, T, 2, 2), dtype=torch.int16, device="cuda:0")
    for s in range(S):
        v = torch.randn((C, T, 2, 2), generator=g, device="cuda:0").mul_(64.0).round_()
        x[s] = v.clamp_(-32768, 32767).to(torch.int16)
        del v
    w = _weights(blk, ctype)
    out = lbf.beamform(x, w, lbf.STOKES_IQUV, 16, 1)                     # [B][4][T'][C]
    torch.cuda.synchronize()
    chans = np.array([0, 1, C // 2, C - 1])
    idx = torch.from_numpy(chans).to("cuda:0")
    for t0 in (0, T - 256):
        xs = np.ascontiguousarray(x[:, idx, t0:t0 + 256].cpu().numpy())
        got = out[:, :, t0 // 16:t0 // 16 + 16][:, :, :, idx].cpu().numpy()
        ref = orc.pipeline(xs, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz[chans], 4, 16, 1, 16)
        part = types.SimpleNamespace(x=xs, S=S, station_xyz=blk.station_xyz, beam_dir=blk.beam_dir,
                                     ref_dir=blk.ref_dir, freq_hz=blk.freq_hz[chans])
        _check_stokes(got, ref, TOL[ctype], "largest block, samples %d.." % t0, part, ctype, 16, 1)
    del x, w, out


# --------------------------------------------------------------------------
# peak probes
# --------------------------------------------------------------------------

def test_probe_copy_is_a_copy_and_mfma_probes_report_their_work():
    torch = _torch()
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.zeros_like(src)
    work = lbf.probe(lbf.PROBE_COPY, 1, src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert work == 2 * src.numel() * 4
    sink = torch.zeros(512, dtype=torch.float32, device="cuda:0")
    for kind, flop in ((lbf.PROBE_MFMA_F16, 32768), (lbf.PROBE_MFMA_F32, 4096)):
        w = lbf.probe(kind, 3, None, sink)
        torch.cuda.synchronize()
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        assert w == 2 * cus * 4 * 3 * 8 * flop
    assert torch.count_nonzero(sink).item() == 0          # the probes never write their sink
    zeros = torch.zeros(1 << 20, dtype=torch.float32, device="cuda:0")
    w = lbf.probe(lbf.PROBE_READ, 1, zeros, sink)
    torch.cuda.synchronize()
    assert w == zeros.numel() * 4
    assert torch.count_nonzero(sink).item() == 0          # the xor of zeros never equals the key
