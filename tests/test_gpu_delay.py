"""GPU parity of delay compensation (Sec. 3): whole-sample shifts in the
channeliser, the residual sub-sample delay in the weights, then the beam
former, through the C ABI against the FP64 oracle (which applies the
residual as the paper's per-sample phase rotation).

Tolerances: weights within half an ulp of the operand type; beams and Stokes
1e-5 (FP32 operands) / 3e-3 (FP16, BF16) norm-wise relative L2, and every
element within twice the rounding bound derived from the operand type (the
channelised samples are not integers, so BF16 rounds them to 8 significant
bits, and beams near a null of a strong tone lose its power by cancellation:
their relative error is no multiple of the norm-wise one)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import lbf, synth
from tests._util import (check_stokes_bound, contraction_eps, cplx, flush, relerr, stokes_bound,
                         to_dev)

pytestmark = pytest.mark.gpu

TOL = {lbf.F32: 1e-5, lbf.F16: 3e-3, lbf.BF16: 3e-3}
CT_NAMES = {lbf.F32: "f32", lbf.F16: "f16", lbf.BF16: "bf16"}


def _torch():
    import torch
    return torch


def _scene(S, B, nsb, nch, seed):
    """Stations in a 1 km disc, beam 0 at the station-beam centre (where the
    delayed tones come from), the others on a 0.05 deg hex grid; channel
    frequencies of subbands centred on whole multiples of the subband width;
    per-station delays d_s + phi_s subband samples."""
    rng = np.random.default_rng([1105, 661, 110, seed])
    pos = synth.station_positions(rng, S)
    u0 = synth.station_beam_centre()
    dirs = synth.hex_beams(u0, B, 0.05)
    freq = synth.centred_channel_freqs(nsb, nch)
    d = rng.integers(0, 40, size=S)
    d[0] = 0
    phi = rng.uniform(-0.5, 0.5, size=S)
    return pos, dirs, u0, freq, d, phi


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
def test_weights_with_residual_delays_match_oracle(ctype):
    torch = _torch()
    pos, dirs, u0, freq, d, phi = _scene(19, 23, 2, 16, 1)
    resid = phi / synth.SUBBAND_HZ
    flush("weights with residual delays %s" % CT_NAMES[ctype])
    tau = torch.empty((23, 19), dtype=torch.float64, device="cuda:0")
    w = lbf.compute_weights(to_dev(pos), to_dev(dirs), to_dev(freq), ctype, ref_dir=u0, tau=tau,
                            station_delay=to_dev(resid))
    torch.cuda.synchronize()
    tau_o = orc.delays(pos, dirs, u0, resid=resid)
    assert np.max(np.abs(tau.cpu().numpy() - tau_o)) <= 1e-15 * np.max(np.abs(tau_o)) + 1e-22
    w_o = orc.weights(tau_o, freq)
    half_ulp = {lbf.F32: 2.0 ** -24, lbf.F16: 2.0 ** -11, lbf.BF16: 2.0 ** -8}[ctype]
    assert np.max(np.abs(cplx(w.float()) - w_o)) <= half_ulp + 1e-12


@pytest.mark.parametrize("ctype", [lbf.F32, lbf.F16, lbf.BF16], ids=lambda c: CT_NAMES[c])
def test_shift_channelise_weights_beamform_chain(ctype):
    """Stations receive three tones d_s + phi_s subband samples late.  GPU:
    lbf_channelize with the whole-sample shifts d_s, lbf_compute_weights with
    the residual delays phi_s / 195312.5 s, lbf_beamform on the complex f32
    channels.  Oracle: its channeliser with the same shifts, the per-sample
    phase correction, and the beam former with the geometric weights."""
    torch = _torch()
    S, B, nsb, nch, T, t_int = 12, 40, 2, 16, 1024, 4
    pos, dirs, u0, freq, d, phi = _scene(S, B, nsb, nch, 2)
    A = 2000.0          # channel amplitude nch A stays inside the FP16 range
    tones = [(0, 3, A, (0.4, 1.3)), (1, 11, A, (2.0, -0.7)), (1, 5, A, (0.1, 0.2))]
    x = synth.delayed_subband_tones(S, nsb, nch, T + 48, d + phi, tones)
    resid = phi / synth.SUBBAND_HZ
    flush("delay chain %s S=%d B=%d C=%d T=%d" % (CT_NAMES[ctype], S, B, nsb * nch, T // nch))

    ch = lbf.channelize(to_dev(x), nch, t_sb=T, shift=to_dev(d.astype(np.int32)))
    w = lbf.compute_weights(to_dev(pos), to_dev(dirs), to_dev(freq), ctype, ref_dir=u0,
                            station_delay=to_dev(resid))
    y = lbf.beamform(ch, w, lbf.VOLTAGES)
    st = lbf.beamform(ch, w, lbf.STOKES_IQUV, t_int, 1)
    torch.cuda.synchronize()

    ch_o = orc.phase_correct(orc.channelize(x, nch, t_sb=T, shift=d), freq, resid)
    x_o = np.ascontiguousarray(np.stack([ch_o.real, ch_o.imag], axis=-1), dtype=np.float32)
    y_o = orc.pipeline(x_o, pos, dirs, u0, freq, 0)                   # [B][2][T'][C] complex
    st_o = orc.pipeline(x_o, pos, dirs, u0, freq, 4, t_int, 1, 8)      # [B][4][T'/t_int][C]
    yv = cplx(y).transpose(1, 3, 2, 0)
    assert relerr(yv, y_o) <= TOL[ctype]
    got = st.cpu().numpy()
    for k in range(4):
        # X and Y of each tone have equal amplitude, so Q is rounding noise:
        # measure Q, U, V against Stokes I
        e = np.linalg.norm(got[:, k] - st_o[:, k]) / np.linalg.norm(st_o[:, 0])
        assert e <= TOL[ctype], ("IQUV"[k], e)
    # element-wise: the operand rounding against sum_s |x_s|, plus the GPU
    # channeliser's FP32 error, which spreads over a station's whole row (at
    # most 1e-6 of the row's largest channel sample, 4x the FFT's error of
    # about u log2(nch) max|x|)
    xs = x_o[..., 0].astype(np.float64) + 1j * x_o[..., 1]             # [S][C][T'][2]
    eps = contraction_eps(ctype, S, samples_exact=ctype == lbf.F32)
    err = eps * np.abs(xs).sum(axis=0) + 1e-6 * np.abs(xs).max(axis=(1, 2, 3)).sum()   # [C][T'][2]
    yc = y_o.transpose(3, 0, 2, 1)                                     # [C][B][T'][2]
    check_stokes_bound(got, st_o, stokes_bound(yc, err, 4, t_int, 1), "delay chain Stokes")
    ev = np.abs(yv - y_o) / (2 * (err.transpose(2, 1, 0)[None] + 2.0 ** -24 * np.abs(y_o)) + 1e-30)
    assert ev.max() <= 1.0, ev.max()
    # beam 0 looks at the tones' direction: every station adds coherently
    C = nsb * nch
    full = (S * nch * A) ** 2 * 2 * t_int                             # Stokes I of |X| = |Y| = S nch A
    for sb, q, _, _ in tones:
        c = sb * nch + q
        assert np.all(np.abs(got[0, 0, :, c] / full - 1.0) < 0.02), c
    quiet = [c for c in range(C) if c not in [sb * nch + q for sb, q, _, _ in tones]]
    assert got[0, 0][:, quiet].max() < 1e-3 * full
