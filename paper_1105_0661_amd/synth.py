"""Seeded synthetic station data for the tied-array beam former.

This module only *synthesises inputs*: station positions, tied-array beam
directions, channel frequencies and channelised complex station samples
(Gaussian noise plus optional plane-wave tones).  It contains none of the
beam former's arithmetic (no delays-to-weights step, no weighted sum, no
Stokes); both the FP64 oracle and the GPU path read the arrays it returns.

The shapes follow the paper's data model:

* stations produce subbands of 195,312.5 Hz, each split into ``nch``
  channels, with dual-polarisation (X, Y) complex integer samples
  (Section 3; Section 4.2 for the channel split);
* the array is ``x[s][c][t][p][ri]`` -- station, channel, time, polarisation,
  real/imaginary -- as ``int8`` (complex int8), ``int16`` (complex int16) or
  ``float32`` (complex float32).

Geometry is a local East-North-Up frame: station positions in metres,
directions as unit vectors ``(l, m, n)`` with ``n = sqrt(1 - l^2 - m^2)``.
A tone from direction ``u`` reaches station ``s`` with the phase of a plane
wave, ``exp(+2 pi i f p_s.(u - u_ref) / c0)``: the geometric delay of Section 3,
seen as a phase at the channel's frequency.

Randomness: geometry and tones come from ``default_rng([1105, 661, tag])``;
the noise of station ``s`` in subband ``sb`` from
``default_rng([1105, 661, tag, 1 + s, sb])``, so any (station, subband) slice can
be regenerated on its own and blocks are generated in parallel.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

C0 = 299_792_458.0            # speed of light, m/s
SUBBAND_HZ = 195_312.5        # LOFAR subband width (Section 3 "195 kHz")
BASE_HZ = 150e6               # frequency of the first subband used here
SUBBANDS_PER_STATION = 248    # Section 3
XTYPES = ("ci8", "ci16", "cf32")
_NP_X = {"ci8": np.int8, "ci16": np.int16, "cf32": np.float32}
_QMAX = {"ci8": 127, "ci16": 32767}
_QMIN = {"ci8": -128, "ci16": -32768}


@dataclass
class Tone:
    """A monochromatic plane wave injected in one channel."""
    channel: int
    direction: np.ndarray          # [3] unit vector
    amplitude: float
    cycles_per_sample: float = 0.1
    phase_xy: Tuple[float, float] = (0.0, 0.0)


@dataclass
class Block:
    """One beam-forming block: geometry, frequencies and station samples."""
    S: int
    B: int
    nsb: int
    nch: int
    T: int
    xtype: str
    station_xyz: np.ndarray        # [S][3] float64, metres
    beam_dir: np.ndarray           # [B][3] float64, unit vectors
    ref_dir: np.ndarray            # [3] float64, station-beam centre
    freq_hz: np.ndarray            # [C] float64
    x: Optional[np.ndarray] = None  # [S][C][T][2][2]
    sigma: float = 0.0
    tones: List[Tone] = field(default_factory=list)
    tag: Tuple[int, ...] = ()

    @property
    def C(self) -> int:
        return self.nsb * self.nch

    @property
    def bytes_per_complex(self) -> int:
        return {"ci8": 2, "ci16": 4, "cf32": 8}[self.xtype]


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def direction(l: float, m: float) -> np.ndarray:
    return np.array([l, m, math.sqrt(max(0.0, 1.0 - l * l - m * m))])


def station_beam_centre(zenith_deg: float = 30.0, azimuth_deg: float = 0.0) -> np.ndarray:
    za = math.radians(zenith_deg)
    az = math.radians(azimuth_deg)
    return direction(math.sin(za) * math.sin(az), math.sin(za) * math.cos(az))


def station_positions(rng: np.random.Generator, S: int, radius_m: float = 1000.0) -> np.ndarray:
    """Uniform in a disc of the given radius (r = R sqrt(U), theta = 2 pi U), z = 0."""
    u = rng.random((S, 2))
    r = radius_m * np.sqrt(u[:, 0])
    th = 2.0 * np.pi * u[:, 1]
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(S)], axis=1)


def hex_offsets(n: int, spacing_deg: float) -> np.ndarray:
    """The ``n`` hexagonal-lattice points nearest the origin, ordered by
    distance and then by angle in [0, 2 pi); returns [n][2] (dl, dm) radians."""
    a = math.radians(spacing_deg)
    R = int(math.ceil(math.sqrt(n))) + 2
    pts = []
    for j in range(-R, R + 1):
        for i in range(-R - abs(j), R + abs(j) + 1):
            x = i + j / 2.0
            y = j * math.sqrt(3.0) / 2.0
            d2 = x * x + y * y
            ang = math.atan2(y, x) % (2.0 * math.pi)
            pts.append((round(d2, 9), round(ang, 12), x * a, y * a))
    pts.sort()
    if len(pts) < n:
        raise ValueError("hex lattice too small")
    return np.array([[p[2], p[3]] for p in pts[:n]])


def hex_beams(u0: np.ndarray, n: int, spacing_deg: float) -> np.ndarray:
    off = hex_offsets(n, spacing_deg)
    return np.stack([direction(u0[0] + dl, u0[1] + dm) for dl, dm in off])


def channel_freqs(nsb: int, nch: int, base_hz: float = BASE_HZ) -> np.ndarray:
    """f[sb*nch + k] = base + sb*195312.5 + k*195312.5/nch (Hz)."""
    sb = np.arange(nsb, dtype=np.float64)[:, None]
    k = np.arange(nch, dtype=np.float64)[None, :]
    return (base_hz + sb * SUBBAND_HZ + k * (SUBBAND_HZ / nch)).reshape(-1)


def centred_channel_freqs(nsb: int, nch: int, first_subband: int = 768) -> np.ndarray:
    """Channel frequencies of subbands centred on whole multiples of the
    subband width, as a station's polyphase filter bank forms them (subband k
    centred at k * 195312.5 Hz): f[sb*nch + q] = (first_subband + sb) *
    195312.5 + (q - nch/2) * 195312.5 / nch, so channel nch/2 sits at the
    subband's centre (FFT bin 0 of the channeliser)."""
    sb = np.arange(nsb, dtype=np.float64)[:, None]
    q = np.arange(nch, dtype=np.float64)[None, :]
    return ((first_subband + sb) * SUBBAND_HZ + (q - nch / 2) * (SUBBAND_HZ / nch)).reshape(-1)


def delayed_subband_tones(S: int, nsb: int, nch: int, T_in: int, delay_samples, tones, xtype: str = "ci16",
                          first_subband: int = 768) -> np.ndarray:
    """Subband samples [S][nsb][T_in][2][2] of stations that all receive the
    same tones, station s ``delay_samples[s]`` subband samples late (any real
    number).  ``tones``: (subband, channel q, amplitude, (phase X, phase Y))
    tuples; the tone sits at the centre of channel q, nu = (q - nch/2) / nch
    cycles per subband sample from the subband's centre f_mix, i.e. at sky
    frequency f = f_mix + nu * 195312.5 Hz (``centred_channel_freqs``).  The
    station mixes its delayed signal down by f_mix and samples it every
    1/195312.5 s, which gives
        x_s[sb][n][p] = sum_tones A exp(i (2 pi (nu n - f D_s) + phase_p)),
    D_s = delay_samples[s] / 195312.5 s; quantised with clip(rint(.))."""
    d = np.asarray(delay_samples, dtype=np.float64)
    if d.shape != (S,):
        raise ValueError("one delay per station")
    n = np.arange(T_in, dtype=np.float64)
    v = np.zeros((S, nsb, T_in, 2), np.complex128)
    for sb, q, amp, ph in tones:
        nu = (q - nch / 2) / nch
        f = (first_subband + sb) * SUBBAND_HZ + nu * SUBBAND_HZ
        D = d / SUBBAND_HZ                                              # seconds
        arg = 2.0 * np.pi * (nu * n[None, :] - (f * D)[:, None])       # [S][T_in]
        for p in range(2):
            v[:, sb, :, p] += amp * np.exp(1j * (arg + ph[p]))
    out = np.stack([v.real, v.imag], axis=-1)
    return _quantise(out, xtype)


def samples_per_block(seconds: float, nch: int) -> int:
    """Channel samples in a block of ``seconds``, rounded up to a multiple of 16."""
    return 16 * int(math.ceil(seconds * SUBBAND_HZ / (nch * 16)))


# --------------------------------------------------------------------------
# samples
# --------------------------------------------------------------------------

def _tone_field(tone: Tone, pos: np.ndarray, ref: np.ndarray, f: float, T: int) -> np.ndarray:
    """Complex tone for every station/time/pol: [S][T][2] complex128."""
    geo = 2.0 * np.pi * f * (pos @ (tone.direction - ref)) / C0          # [S]
    t = np.arange(T, dtype=np.float64)
    rot = 2.0 * np.pi * tone.cycles_per_sample * t                       # [T]
    ph = np.array(tone.phase_xy, dtype=np.float64)                        # [2]
    return tone.amplitude * np.exp(1j * (geo[:, None, None] + rot[None, :, None] + ph[None, None, :]))


def _quantise(v: np.ndarray, xtype: str) -> np.ndarray:
    if xtype == "cf32":
        return v.astype(np.float32, copy=False)
    np.rint(v, out=v)
    np.clip(v, _QMIN[xtype], _QMAX[xtype], out=v)
    return v.astype(_NP_X[xtype])


def fill_samples(blk: Block, threads: int = 8, stations: Optional[Sequence[int]] = None,
                 subbands: Optional[Sequence[int]] = None, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Generate ``x[s][c][t][p][ri]`` for the given stations/subbands (default all).

    Noise: re and im each N(0, sigma^2), drawn per (station, subband) from its own
    seeded stream; tones are added before quantisation (clip(rint(.)))."""
    st = list(range(blk.S)) if stations is None else list(stations)
    sbs = list(range(blk.nsb)) if subbands is None else list(subbands)
    if out is None:
        out = np.empty((len(st), len(sbs) * blk.nch, blk.T, 2, 2), dtype=_NP_X[blk.xtype])
    tones_by_ch = {}
    for tn in blk.tones:
        tones_by_ch.setdefault(tn.channel, []).append(tn)

    def work(args):
        i, s, j, sb = args
        rng = np.random.default_rng(list(blk.tag) + [1 + s, sb])
        v = rng.standard_normal((blk.nch, blk.T, 2, 2), dtype=np.float32)
        v *= np.float32(blk.sigma)
        for k in range(blk.nch):
            c = sb * blk.nch + k
            for tn in tones_by_ch.get(c, ()):
                fld = _tone_field(tn, blk.station_xyz[s:s + 1], blk.ref_dir, blk.freq_hz[c], blk.T)[0]
                v[k, :, :, 0] += fld.real.astype(np.float32)
                v[k, :, :, 1] += fld.imag.astype(np.float32)
        out[i, j * blk.nch:(j + 1) * blk.nch] = _quantise(v, blk.xtype)

    jobs = [(i, s, j, sb) for i, s in enumerate(st) for j, sb in enumerate(sbs)]
    if threads > 1 and len(jobs) > 1:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, jobs))
    else:
        for a in jobs:
            work(a)
    return out


def make_block(S: int, B: int, nsb: int, nch: int, T: int, xtype: str = "ci16", sigma: float = 32.0,
               tag: Sequence[int] = (1105, 661, 99), n_tones: int = 1, tone_amp: float = 64.0,
               beam_spacing_deg: float = 0.05, generate: bool = True, threads: int = 8,
               radius_m: float = 1000.0) -> Block:
    """A generic block: S stations in a disc, B beams on a hex grid around the
    station-beam centre, ``n_tones`` tones aimed at beams drawn from the seed."""
    if xtype not in XTYPES:
        raise ValueError(xtype)
    rng = np.random.default_rng(list(tag))
    pos = station_positions(rng, S, radius_m)
    u0 = station_beam_centre()
    beams = hex_beams(u0, B, beam_spacing_deg)
    C = nsb * nch
    freqs = channel_freqs(nsb, nch)
    tones = []
    for _ in range(n_tones):
        b = int(rng.integers(0, B))
        c = int(rng.integers(0, C))
        ph = tuple(float(v) for v in rng.random(2) * 2 * np.pi)
        tones.append(Tone(channel=c, direction=beams[b].copy(), amplitude=tone_amp, phase_xy=ph))
    blk = Block(S=S, B=B, nsb=nsb, nch=nch, T=T, xtype=xtype, station_xyz=pos, beam_dir=beams,
                ref_dir=u0, freq_hz=freqs, sigma=sigma, tones=tones, tag=tuple(tag))
    if generate:
        blk.x = fill_samples(blk, threads=threads)
    return blk


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def config0(generate: bool = True) -> Block:
    """Tiny: 8 stations, 1 subband x 16 channels, 1024 samples, CI16 sigma=32 plus a
    unit-amplitude tone from beam 0's direction in channel 5; 4 beams (beam 0 at
    the tone, three uniform within +-1 deg of the station-beam centre)."""
    tag = (1105, 661, 0)
    rng = np.random.default_rng(list(tag))
    S, nsb, nch, T = 8, 1, 16, 1024
    pos = station_positions(rng, S)
    u0 = station_beam_centre()
    d = np.radians(1.0)
    off = rng.uniform(-d, d, size=(4, 2))
    beams = np.stack([direction(u0[0] + a, u0[1] + b) for a, b in off])
    ph = tuple(float(v) for v in rng.random(2) * 2 * np.pi)
    tones = [Tone(channel=5, direction=beams[0].copy(), amplitude=1.0, phase_xy=ph)]
    blk = Block(S=S, B=4, nsb=nsb, nch=nch, T=T, xtype="ci16", station_xyz=pos, beam_dir=beams,
                ref_dir=u0, freq_hz=channel_freqs(nsb, nch), sigma=32.0, tones=tones, tag=tag)
    if generate:
        blk.x = fill_samples(blk)
    return blk


def config1(generate: bool = True, threads: int = 16) -> Block:
    """One-second block: 64 stations, 32 subbands x 256 channels, 768 samples,
    CI16 sigma=64 with 3 tones (amplitude 64), 128 beams on a 0.05 deg hex grid."""
    return make_block(64, 128, 32, 256, 768, "ci16", 64.0, tag=(1105, 661, 1), n_tones=3,
                      tone_amp=64.0, generate=generate, threads=threads)


def config2(generate: bool = True, threads: int = 16) -> Block:
    """As the one-second block but complex int8 (sigma=16) and 488 beams."""
    return make_block(64, 488, 32, 256, 768, "ci8", 16.0, tag=(1105, 661, 2), n_tones=3,
                      tone_amp=16.0, generate=generate, threads=threads)


@dataclass
class JobSpec:
    S: int
    B: int
    nch: int
    nsb: int
    xtype: str
    product: str          # "I" or "IQUV"
    t_int: int
    T: int
    seconds: float = 1.0
    tag: Tuple[int, ...] = ()


def config3_jobs(n_jobs: int = 12, seed_tag=(1105, 661, 3), seconds: float = 1.0) -> List[JobSpec]:
    """Uneven batch: stations U{24..64}, beams U{1..400}, 16/64/256 channels per
    subband, U{8..64} subbands, CI8/CI16 and Stokes I/IQUV 50/50, 1 s blocks."""
    rng = np.random.default_rng(list(seed_tag))
    jobs = []
    for j in range(n_jobs):
        S = int(rng.integers(24, 65))
        B = int(rng.integers(1, 401))
        nch = int(rng.choice([16, 64, 256]))
        nsb = int(rng.integers(8, 65))
        xt = "ci8" if rng.random() < 0.5 else "ci16"
        prod = "I" if rng.random() < 0.5 else "IQUV"
        T = samples_per_block(seconds, nch)
        jobs.append(JobSpec(S=S, B=B, nch=nch, nsb=nsb, xtype=xt, product=prod, t_int=16, T=T,
                            seconds=seconds, tag=tuple(seed_tag) + (100 + j,)))
    return jobs


def block_for_job(js: JobSpec, generate: bool = True, threads: int = 16) -> Block:
    sigma = 16.0 if js.xtype == "ci8" else 64.0
    return make_block(js.S, js.B, js.nsb, js.nch, js.T, js.xtype, sigma, tag=js.tag, n_tones=1,
                      tone_amp=sigma, generate=generate, threads=threads)


def poisson_arrivals(rate_hz: float, duration_s: float, seed_tag=(1105, 661, 4)) -> np.ndarray:
    rng = np.random.default_rng(list(seed_tag))
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.array(out)
        out.append(t)


def tone_only_block(S: int, B: int, nch: int, T: int, amplitude: float, xtype: str = "ci16",
                    beam_index: int = 3, tag=(1105, 661, 7), beam_spacing_deg: float = 0.5) -> Block:
    """A noise-free block holding one loud tone aimed exactly at beam ``beam_index``
    in every channel (used for the coherent-gain check)."""
    blk = make_block(S, B, 1, nch, T, xtype, 0.0, tag=tag, n_tones=0, generate=False,
                     beam_spacing_deg=beam_spacing_deg)
    ph = (0.3, 1.1)
    blk.tones = [Tone(channel=c, direction=blk.beam_dir[beam_index].copy(), amplitude=amplitude,
                      phase_xy=ph) for c in range(blk.C)]
    blk.x = fill_samples(blk)
    return blk
