"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle (``oracle/``) against something other than itself:
closed forms, an independent library routine (numpy), brute force on tiny
inputs, invariants, and values worked by hand from the paper's definitions
(``tests/golden``).  Section numbers refer to Mol & Romein, "The LOFAR Beam
Former: Implementation and Performance Analysis".
"""
import math
import os

import cmath

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C0 = 299_792_458.0


def _cx(x):
    return x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)


def _rand_block(S, B, nsb, nch, T, xtype="ci16", sigma=40.0, tag=(5, 6, 7), **kw):
    return synth.make_block(S, B, nsb, nch, T, xtype, sigma, tag=tag, **kw)


# --------------------------------------------------------------------------
# delays and weights (Sec. 3, Sec. 4.3)
# --------------------------------------------------------------------------

def test_delay_closed_forms():
    # a station displaced by d along the (unit) source direction sees the wave
    # d / c0 earlier; one displaced perpendicular to it sees no delay
    u = synth.direction(math.sin(math.radians(20)), 0.0)
    d = 1234.5
    perp = np.cross(u, [0.0, 1.0, 0.0])
    perp /= np.linalg.norm(perp)
    pos = np.stack([d * u, 77.0 * perp, np.zeros(3)])
    tau = orc.delays(pos, u[None, :])
    assert tau.shape == (1, 3)
    assert tau[0, 0] == pytest.approx(d / C0, rel=1e-15)
    assert abs(tau[0, 1]) < 1e-20
    assert tau[0, 2] == 0.0
    # with a reference direction the delay is differential: u_ref = u gives 0
    tau_ref = orc.delays(pos, u[None, :], ref=u)
    assert np.all(np.abs(tau_ref) < 1e-20)


def test_weights_unit_modulus_and_zero_delay():
    rng = np.random.default_rng(1)
    tau = rng.normal(0, 3e-6, size=(5, 7))
    f = synth.channel_freqs(2, 16)
    w = orc.weights(tau, f)
    assert w.shape == (32, 5, 7)
    assert np.max(np.abs(np.abs(w) - 1.0)) < 1e-15
    w0 = orc.weights(np.zeros((3, 4)), f)
    assert np.all(w0 == 1.0)


def test_weights_match_full_phase_exponential():
    # exp(-2 pi i f tau) evaluated by numpy on the unreduced phase: the FP64
    # reduction to the fractional turn must not change the value (phases here
    # stay below ~1e3 turns, where numpy's own error is ~1e-13)
    rng = np.random.default_rng(2)
    tau = rng.uniform(-5e-6, 5e-6, size=(4, 6))
    f = synth.channel_freqs(4, 8)
    w = orc.weights(tau, f)
    ref = np.exp(-2j * np.pi * f[:, None, None] * tau[None, :, :])
    assert np.max(np.abs(w - ref)) < 1e-11


def test_weights_periodic_in_whole_turns():
    # tau -> tau + k / f changes f*tau by exactly k turns: same weight
    f = np.array([150e6 + 12207.03125 * 3])
    tau = np.array([[1.3e-6, -2.2e-6, 0.0]])
    w1 = orc.weights(tau, f)
    for k in (1, 7, 1000):
        w2 = orc.weights(tau + k / f[0], f)
        assert np.max(np.abs(w1 - w2)) < 1e-9


def test_weights_sign_convention_worked_example():
    # station 1 km East, beam 1 deg from zenith towards East, 150 MHz, no reference:
    # tau = 1000 sin(1 deg) / c0, f tau = 0.8731... turns -> w = exp(-2 pi i frac)
    pos = np.array([[1000.0, 0.0, 0.0]])
    u = np.array([[math.sin(math.radians(1.0)), 0.0, math.cos(math.radians(1.0))]])
    tau = orc.delays(pos, u)
    m = 150e6 * 1000.0 * math.sin(math.radians(1.0)) / C0
    assert tau[0, 0] * 150e6 == pytest.approx(m, rel=1e-14)
    w = orc.weights(tau, np.array([150e6]))[0, 0, 0]
    frac = m - round(m)
    assert w.real == pytest.approx(math.cos(2 * math.pi * frac), abs=1e-14)
    assert w.imag == pytest.approx(-math.sin(2 * math.pi * frac), abs=1e-14)


# --------------------------------------------------------------------------
# the weighted complex sum (Sec. 1, Sec. 3, Sec. 4.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("xtype", ["ci8", "ci16", "cf32"])
def test_beamform_matches_numpy_einsum(xtype):
    blk = _rand_block(6, 5, 2, 4, 24, xtype, sigma=20.0)
    w = orc.block_weights(blk)
    y = orc.beamform(blk.x, w)
    ref = np.einsum("cbs,sctp->cbtp", w, _cx(blk.x))
    assert y.shape == (8, 5, 24, 2)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_beamform_channel_slice():
    blk = _rand_block(4, 3, 1, 8, 16)
    w = orc.block_weights(blk)
    full = orc.beamform(blk.x, w)
    part = orc.beamform(blk.x, w[3:6], c_lo=3, nc=3)
    assert np.array_equal(part, full[3:6])


def test_beamform_brute_force_two_stations():
    # S=2, B=1, C=1, T=1, written out in real arithmetic
    x = np.array([[[[[3, -1], [2, 5]]]], [[[[-4, 2], [0, 1]]]]], dtype=np.int16)  # [2][1][1][2][2]
    w = np.array([[[0.6 + 0.8j, -0.28 + 0.96j]]])                                  # [1][1][2]
    y = orc.beamform(x, w)
    for p in range(2):
        a, b = x[0, 0, 0, p], x[1, 0, 0, p]
        re = 0.6 * a[0] - 0.8 * a[1] + (-0.28) * b[0] - 0.96 * b[1]
        im = 0.6 * a[1] + 0.8 * a[0] + (-0.28) * b[1] + 0.96 * b[0]
        assert y[0, 0, 0, p].real == pytest.approx(re, abs=1e-13)
        assert y[0, 0, 0, p].imag == pytest.approx(im, abs=1e-13)


def test_beamform_identity_single_station_zero_delay():
    blk = _rand_block(1, 1, 1, 4, 32, "ci16", sigma=1000.0)
    w = orc.weights(np.zeros((1, 1)), blk.freq_hz)
    y = orc.beamform(blk.x, w)
    assert np.array_equal(y[:, 0], _cx(blk.x)[0])


def test_beamform_linear_in_inputs():
    b1 = _rand_block(5, 4, 1, 4, 16, "ci16", sigma=30.0, tag=(1, 1, 1))
    b2 = _rand_block(5, 4, 1, 4, 16, "ci16", sigma=30.0, tag=(2, 2, 2))
    w = orc.block_weights(b1)
    x1, x2 = b1.x.astype(np.int32), b2.x.astype(np.int32)
    comb = (3 * x1 - 2 * x2).astype(np.int16)
    y = orc.beamform(comb, w)
    ref = 3 * orc.beamform(b1.x, w) - 2 * orc.beamform(b2.x, w)
    assert np.max(np.abs(y - ref)) < 1e-9


def test_beamform_station_permutation_invariant():
    blk = _rand_block(7, 3, 1, 2, 8)
    w = orc.block_weights(blk)
    perm = np.random.default_rng(3).permutation(7)
    y = orc.beamform(blk.x, w)
    yp = orc.beamform(np.ascontiguousarray(blk.x[perm]), np.ascontiguousarray(w[:, :, perm]))
    assert np.max(np.abs(y - yp)) < 1e-9


def test_coherent_gain_of_a_plane_wave():
    # a noise-free tone of amplitude A arriving from beam 3's direction (0.5 deg
    # off the reference direction): beam 3 adds all S stations in phase,
    # |y|^2 = S^2 A^2 (up to the rounding of the tone to integers, |err| <=
    # sqrt(2)/2 per sample); other beams gain less
    S, A, hit = 24, 1.0e4, 3
    blk = synth.tone_only_block(S, 7, 4, 32, A, "ci16", beam_index=hit)
    w = orc.block_weights(blk)
    y = orc.beamform(blk.x, w)
    p0 = np.abs(y[:, hit]) ** 2
    bound = S * math.sqrt(2) * 0.5
    assert np.all(np.abs(np.abs(y[:, hit]) - S * A) <= bound)
    assert np.max(np.abs(p0 / (S * S * A * A) - 1.0)) < 2 * bound / (S * A)
    others = [b for b in range(7) if b != hit]
    assert np.all(np.abs(y[:, others]) ** 2 < 0.5 * S * S * A * A)
    # the opposite sign convention, or dropping the reference direction, would
    # not add the stations coherently
    y_conj = orc.beamform(blk.x, np.conj(w))
    assert np.max(np.abs(y_conj[:, hit])) < 0.5 * S * A
    w_noref = orc.weights(orc.delays(blk.station_xyz, blk.beam_dir), blk.freq_hz)
    assert np.max(np.abs(orc.beamform(blk.x, w_noref)[:, hit])) < 0.5 * S * A


# --------------------------------------------------------------------------
# Stokes (Sec. 4.5), integration (Sec. 3, Sec. 5.1), final order (Sec. 4.6)
# --------------------------------------------------------------------------

def _golden_stokes():
    rows = []
    with open(os.path.join(GOLDEN, "stokes_worked.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def test_stokes_worked_examples():
    g = _golden_stokes()
    y = (g[:, 0] + 1j * g[:, 1])[:, None] * np.array([1, 0]) + (g[:, 2] + 1j * g[:, 3])[:, None] * np.array([0, 1])
    st = orc.stokes(y.reshape(1, 1, -1, 2))
    assert np.array_equal(st[0, 0], g[:, 4:8])


def test_stokes_single_station_exact_on_integers():
    blk = _rand_block(1, 1, 1, 2, 64, "ci16", sigma=500.0)
    y = orc.beamform(blk.x, orc.weights(np.zeros((1, 1)), blk.freq_hz))
    st = orc.stokes(y)
    xi = blk.x[0].astype(np.int64)          # [C][T][2][2]
    inten = (xi[..., 0, 0] ** 2 + xi[..., 0, 1] ** 2 + xi[..., 1, 0] ** 2 + xi[..., 1, 1] ** 2)
    assert np.array_equal(st[:, 0, :, 0], inten.astype(np.float64))


def test_stokes_polarisation_invariants():
    blk = _rand_block(5, 3, 1, 4, 32)
    st = orc.stokes(orc.beamform(blk.x, orc.block_weights(blk)))
    I, Q, U, V = (st[..., k] for k in range(4))
    # a single sample is fully polarised
    assert np.max(np.abs(I * I - (Q * Q + U * U + V * V))) <= 1e-9 * np.max(I * I)
    assert np.all(I >= 0)
    # sums of samples are partially polarised
    s = orc.integrate(st, 4, 8, 2)
    I2, Q2, U2, V2 = (s[..., k] for k in range(4))
    assert np.all(I2 * I2 >= (Q2 * Q2 + U2 * U2 + V2 * V2) * (1 - 1e-12))


def test_integrate_is_explicit_sum_and_identity():
    rng = np.random.default_rng(4)
    st = rng.normal(size=(6, 3, 32, 4))
    s = orc.integrate(st, 4, 8, 3)
    ref = st.reshape(2, 3, 3, 4, 8, 4).sum(axis=(1, 4))
    assert np.max(np.abs(s - ref)) < 1e-12
    s1 = orc.integrate(st, 1, 4, 2)
    ref1 = st[..., :1].reshape(3, 2, 3, 8, 4, 1).sum(axis=(1, 4))
    assert np.max(np.abs(s1 - ref1)) < 1e-12
    assert np.array_equal(orc.integrate(st, 4, 1, 1), st)


def test_reorder_is_the_documented_bijection():
    rng = np.random.default_rng(5)
    s = rng.normal(size=(5, 3, 4, 4))
    out = orc.reorder(s)
    assert out.shape == (3, 4, 4, 5)
    assert np.array_equal(out, np.transpose(s, (1, 3, 2, 0)))
    sc = s + 1j * rng.normal(size=s.shape)
    assert np.array_equal(orc.reorder(sc), np.transpose(sc, (1, 3, 2, 0)))


@pytest.mark.parametrize("K,t_int,f_int", [(1, 16, 1), (4, 4, 2), (4, 1, 1), (0, 1, 1)])
def test_pipeline_equals_composition_of_steps(K, t_int, f_int):
    blk = _rand_block(5, 6, 2, 4, 32, "ci8", sigma=10.0)
    out = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, K, t_int, f_int, 3)
    y = orc.beamform(blk.x, orc.block_weights(blk))
    if K == 0:
        ref = np.transpose(y, (1, 3, 2, 0))
    else:
        ref = orc.reorder(orc.integrate(orc.stokes(y), K, t_int, f_int))
    assert np.array_equal(out, ref)


def test_incoherent_beam_is_sum_of_station_powers():
    blk = _rand_block(4, 1, 1, 4, 32, "ci16", sigma=50.0)
    inc = orc.incoherent(blk.x, 4, 8, 2)
    ref = 0.0
    for s in range(4):
        xs = np.ascontiguousarray(blk.x[s:s + 1])
        ys = orc.beamform(xs, orc.weights(np.zeros((1, 1)), blk.freq_hz))
        ref = ref + orc.integrate(orc.stokes(ys), 4, 8, 2)[:, 0]
    assert np.max(np.abs(inc - ref)) < 1e-9 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# synthetic-input constants against the paper's printed values
# --------------------------------------------------------------------------

def test_channel_constants_match_paper():
    rows = {}
    with open(os.path.join(GOLDEN, "time_freq_constants.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                name, val, unit, tol = line.split()
                rows[name] = (float(val), unit, float(tol))
    scale = {"kHz": 1e3, "Hz": 1.0, "ms": 1e-3}
    f16 = synth.channel_freqs(1, 16)
    got = {
        "subband_width": synth.SUBBAND_HZ,
        "channel_width_16": f16[1] - f16[0],
        "subchannel_4096": (f16[1] - f16[0]) / 4096,
        "channel_sample_16": 1.0 / (f16[1] - f16[0]),
    }
    for k, (val, unit, tol) in rows.items():
        assert got[k] == pytest.approx(val * scale[unit], rel=tol), k
    assert synth.samples_per_block(1.0, 256) == 768


# --------------------------------------------------------------------------
# channel-level dedispersion (Sec. 4.4)
# --------------------------------------------------------------------------

def _dd_input(C, B, T, seed):
    rng = np.random.default_rng([1105, 661, seed])
    return rng.standard_normal((C, B, T, 2)) + 1j * rng.standard_normal((C, B, T, 2))


def test_dedisperse_brute_force_dft():
    """The definition written out with explicit sums (no FFT routine): forward
    DFT with exp(-2 pi i j k / n), product with the weights, backward DFT with
    exp(+2 pi i k t / n) / n."""
    n, C, B = 8, 2, 1
    y = _dd_input(C, B, 2 * n, 1)
    rng = np.random.default_rng(7)
    chirp = np.exp(2j * np.pi * rng.random((C, n))) * (0.5 + rng.random((C, n)))
    got = orc.dedisperse(y, chirp, n)
    for c in range(C):
        for blk in range(2):
            for p in range(2):
                x = [y[c, 0, blk * n + j, p] for j in range(n)]
                X = [sum(x[j] * cmath.exp(-2j * cmath.pi * j * k / n) for j in range(n)) for k in range(n)]
                Z = [X[k] * chirp[c, k] for k in range(n)]
                for t in range(n):
                    z = sum(Z[k] * cmath.exp(2j * cmath.pi * k * t / n) for k in range(n)) / n
                    assert abs(got[c, 0, blk * n + t, p] - z) < 1e-12


def test_dedisperse_unit_weights_are_identity():
    y = _dd_input(3, 2, 3 * 64, 2)
    assert np.allclose(orc.dedisperse(y, np.ones((3, 64)), 64), y, rtol=0, atol=1e-12)


def test_dedisperse_linear_phase_is_a_circular_shift_per_channel():
    """Weights exp(-2 pi i k d_c / n) delay channel c by d_c samples, cyclically
    inside each block: out[t] = in[(t - d_c) mod n] (shift theorem)."""
    n, C, B = 64, 3, 2
    y = _dd_input(C, B, 2 * n, 3)
    d = [5, 0, 63]
    k = np.arange(n)
    chirp = np.stack([np.exp(-2j * np.pi * k * dc / n) for dc in d])
    got = orc.dedisperse(y, chirp, n)
    for c, dc in enumerate(d):
        blocks = y[c].reshape(B, 2, n, 2)
        want = np.roll(blocks, dc, axis=2).reshape(B, 2 * n, 2)
        assert np.allclose(got[c], want, rtol=0, atol=1e-12)


def test_dedisperse_unit_modulus_weights_keep_the_energy():
    n = 512
    y = _dd_input(2, 1, n, 4)
    rng = np.random.default_rng(9)
    chirp = np.exp(2j * np.pi * rng.random((2, n)))
    out = orc.dedisperse(y, chirp, n)
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(y) ** 2) - 1) < 1e-12


# --------------------------------------------------------------------------
# channeliser (Sec. 4.2)
# --------------------------------------------------------------------------

def test_channelize_brute_force_dft_and_channel_order():
    """Written out: channel q of subband sb at output time t is
    sum_j x[t nch + j] exp(-2 pi i j k / nch) with k = (q + nch/2) mod nch."""
    rng = np.random.default_rng([1105, 661, 95])
    S, NSB, nch, T = 2, 2, 8, 16
    x = rng.integers(-100, 101, size=(S, NSB, T, 2, 2)).astype(np.int16)
    got = orc.channelize(x, nch)
    assert got.shape == (S, NSB * nch, T // nch, 2)
    for s in range(S):
        for sb in range(NSB):
            for t in range(T // nch):
                for p in range(2):
                    z = [complex(int(x[s, sb, t * nch + j, p, 0]), int(x[s, sb, t * nch + j, p, 1])) for j in range(nch)]
                    for q in range(nch):
                        k = (q + nch // 2) % nch
                        want = sum(z[j] * cmath.exp(-2j * cmath.pi * j * k / nch) for j in range(nch))
                        assert abs(got[s, sb * nch + q, t, p] - want) < 1e-9


def test_channelize_tone_lands_in_its_channel():
    """A complex tone at (q0 - nch/2) channel widths from the subband centre,
    exp(2 pi i (q0 - nch/2) n / nch), puts all its power, nch per sample
    squared, into channel q0 and nothing elsewhere."""
    nch, T = 16, 64
    n = np.arange(T)
    for q0 in (0, 3, 8, 15):
        tone = np.exp(2j * np.pi * (q0 - nch / 2) * n / nch)
        x = np.zeros((1, 1, T, 2, 2), np.float32)
        x[0, 0, :, 0, 0], x[0, 0, :, 0, 1] = tone.real, tone.imag
        got = orc.channelize(x, nch)[0, :, :, 0]                 # [nch][T / nch]
        assert np.allclose(np.abs(got[q0]), nch, atol=1e-4)
        others = np.delete(got, q0, axis=0)
        assert np.abs(others).max() < 1e-4


def test_channelize_energy_and_one_channel_identity():
    rng = np.random.default_rng([1105, 661, 96])
    x = rng.integers(-128, 128, size=(2, 3, 256, 2, 2)).astype(np.int8)
    got = orc.channelize(x, 64)
    xc = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    assert abs(np.sum(np.abs(got) ** 2) / (64 * np.sum(np.abs(xc) ** 2)) - 1) < 1e-12     # Parseval
    assert np.array_equal(orc.channelize(x, 1), xc)                                      # nch = 1: no change


def test_channelize_shift_makes_delayed_stations_coherent():
    """Station 1 receives station 0's signal d samples later; shifting it by d
    (sample-level delay compensation) makes its channels equal to station 0's,
    while without the shift they differ."""
    rng = np.random.default_rng([1105, 661, 99])
    nch, T, d = 16, 256, 5
    sig = rng.integers(-500, 501, size=(1, 2, T + 32, 2, 2)).astype(np.int16)
    x = np.zeros((2, 2, T + 32, 2, 2), np.int16)
    x[0] = sig[0]
    x[1, :, d:] = sig[0, :, :T + 32 - d]                       # the same wave, d samples later
    got = orc.channelize(x, nch, t_sb=T, shift=[0, d])
    assert np.allclose(got[1], got[0], rtol=0, atol=1e-9)
    plain = orc.channelize(x, nch, t_sb=T)
    assert np.abs(plain[1] - plain[0]).max() > 1.0


def test_channelize_shift_reads_zero_outside_the_row():
    x = np.ones((1, 1, 32, 2, 2), np.float32)
    got = orc.channelize(x, 8, t_sb=32, shift=[24])            # 8 samples inside, 24 past the end
    assert np.allclose(got[0, :, 0, 0], 8 * (1 + 1j) * (np.arange(8) == 4), atol=1e-12)   # DC: channel nch/2
    assert np.abs(got[0, :, 1:]).max() == 0
    neg = orc.channelize(x, 8, t_sb=16, shift=[-8])            # the first group lies before the row
    assert np.abs(neg[0, :, 0]).max() == 0 and abs(neg[0, 4, 1, 0] - 8 * (1 + 1j)) < 1e-12


# --------------------------------------------------------------------------
# superstation beam forming (Sec. 4.2)
# --------------------------------------------------------------------------

def test_superstation_equals_the_beam_former_over_its_members():
    """With weights toward a direction, a superstation is the tied-array beam
    of its member stations in that direction: the C oracle's beam former over
    the members (an independent implementation) gives the same signal."""
    blk = synth.make_block(6, 2, 1, 4, 32, "ci16", 30.0, tag=(1105, 661, 100))
    w = orc.block_weights(blk)                                    # [C][B][S]
    groups = [[0, 2, 3], [5], [1, 4]]
    got = orc.superstation(blk.x, w[:, 1, :], groups)
    for g, members in enumerate(groups):
        want = orc.beamform(np.ascontiguousarray(blk.x[members]), np.ascontiguousarray(w[:, 1:2, members]))
        assert np.allclose(got[g], want[:, 0], rtol=0, atol=1e-9)


def test_superstation_unit_weights_brute_force_and_identity():
    rng = np.random.default_rng([1105, 661, 101])
    x = rng.integers(-50, 51, size=(4, 3, 5, 2, 2)).astype(np.int8)
    got = orc.superstation(x, None, [[1], [0, 3, 2]])
    xc = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    assert np.array_equal(got[0], xc[1])                          # one member, unit weight: the station
    for c in range(3):
        for t in range(5):
            for p in range(2):
                assert got[1, c, t, p] == xc[0, c, t, p] + xc[3, c, t, p] + xc[2, c, t, p]


# --------------------------------------------------------------------------
# delay compensation (Sec. 3): whole-sample shift, then a per-sample phase
# --------------------------------------------------------------------------

def _einsum_beams(w, xc):
    """Independent library routine: y[c][b][t][p] = sum_s w[c][b][s] x[s][c][t][p]."""
    return np.einsum("cbs,sctp->cbtp", w, xc)


def test_residual_delay_is_taken_off_every_beams_delay():
    rng = np.random.default_rng([1105, 661, 102])
    blk = synth.make_block(5, 3, 1, 4, 16, generate=False, tag=(1105, 661, 102))
    resid = rng.uniform(-3e-6, 3e-6, size=5)
    tau0 = orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir)
    tau1 = orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir, resid=resid)
    assert np.allclose(tau1, tau0 - resid[None, :], rtol=0, atol=1e-21)
    # a station exactly one period of channel c late needs no correction there
    f = synth.centred_channel_freqs(1, 4)
    late = np.zeros(5)
    late[2] = 1.0 / f[1]
    w = orc.weights(orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir, resid=late), f)
    w0 = orc.weights(tau0, f)
    assert np.max(np.abs(w[1] - w0[1])) < 1e-9
    assert np.max(np.abs(w[0, :, 2] - w0[0, :, 2])) > 1e-3


def test_residual_delay_in_the_weights_equals_the_per_sample_phase_correction():
    """Folding the residual delay into the weights gives the beams of the
    paper's per-sample complex multiplication followed by the geometric
    weights: w(tau - delta) x = w(tau) (exp(+2 pi i f delta) x).  The two
    sides run different code (the C weights and beam former against numpy's
    phase product and einsum)."""
    rng = np.random.default_rng([1105, 661, 103])
    blk = synth.make_block(6, 4, 2, 8, 24, "ci16", 40.0, tag=(1105, 661, 103))
    resid = rng.uniform(-2.5e-6, 2.5e-6, size=6)          # up to half a subband sample
    w_geo = orc.block_weights(blk)
    y_phase = _einsum_beams(w_geo, orc.phase_correct(blk.x, blk.freq_hz, resid))
    w_res = orc.weights(orc.delays(blk.station_xyz, blk.beam_dir, blk.ref_dir, resid=resid), blk.freq_hz)
    y_w = orc.beamform(blk.x, w_res)
    assert np.max(np.abs(y_w - y_phase)) <= 1e-9 * np.max(np.abs(y_phase))
    # the pipeline takes the same residual delays
    v = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, 0, resid=resid)
    assert np.max(np.abs(v - y_phase.transpose(1, 3, 2, 0))) <= 1e-9 * np.max(np.abs(y_phase))
    # a zero residual changes nothing
    assert np.array_equal(orc.phase_correct(blk.x, blk.freq_hz, np.zeros(6)), _cx(blk.x))


def test_shift_and_residual_phase_make_fractionally_delayed_stations_coherent():
    """Stations receive the same tones d_s + phi_s subband samples late (d_s
    whole, |phi_s| <= 1/2).  Shifting each series by d_s (channeliser) and
    removing the residual phi_s / 195312.5 s with the per-sample phase adds
    every station coherently in every tone channel: |sum_s| = S nch A, up to
    the rounding of the samples to integers (at most sqrt(2)/2 per sample, so
    S nch sqrt(2)/2 after the FFT and the station sum).  Without the shift,
    without the residual phase, with the opposite sign, or with the
    baseband instead of the sky frequency, the stations do not add up."""
    S, nsb, nch, T = 6, 2, 16, 256
    rng = np.random.default_rng([1105, 661, 104])
    d = rng.integers(0, 40, size=S)
    d[0] = 0
    phi = rng.uniform(-0.5, 0.5, size=S)
    A = 6000.0
    tones = [(0, 3, A, (0.4, 1.3)), (1, 11, A, (2.0, -0.7)), (1, 5, A, (0.1, 0.2))]
    x = synth.delayed_subband_tones(S, nsb, nch, T + 48, d + phi, tones)
    freq = synth.centred_channel_freqs(nsb, nch)
    resid = phi / synth.SUBBAND_HZ
    full = S * nch * A
    bound = S * nch * math.sqrt(2) / 2
    tone_ch = [sb * nch + q for sb, q, _, _ in tones]

    ch = orc.channelize(x, nch, t_sb=T, shift=d)                      # [S][C][T/nch][2]
    good = orc.phase_correct(ch, freq, resid).sum(axis=0)             # unit weights, zero geometric delay
    for c in tone_ch:
        assert np.all(np.abs(np.abs(good[c]) - full) <= bound), c
    quiet = np.delete(good, tone_ch, axis=0)
    assert np.abs(quiet).max() <= bound

    def worst(summed):
        return min(np.abs(summed[c]).min() for c in tone_ch) / full

    assert worst(ch.sum(axis=0)) < 0.9                                              # no residual phase
    assert worst(orc.phase_correct(ch, freq, -resid).sum(axis=0)) < 0.9            # opposite sign
    f_mix = np.repeat((768 + np.arange(nsb)) * synth.SUBBAND_HZ, nch)
    assert worst(orc.phase_correct(ch, freq - f_mix, resid).sum(axis=0)) < 0.9     # baseband frequency
    plain = orc.channelize(x, nch, t_sb=T)
    assert worst(orc.phase_correct(plain, freq, resid).sum(axis=0)) < 0.9          # no whole-sample shift
