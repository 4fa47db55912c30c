"""FP64 CPU oracle of the tied-array beam former -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The GPU library never calls it and shares
no code with it.  The arithmetic lives in ``lbf_oracle.c`` (plain C, FP64);
this file compiles it with gcc and marshals numpy arrays.  The superstation
sum, the channeliser and dedispersion are written here in numpy (complex128),
with numpy's FFT as the FFT step.

Definitions followed (Mol & Romein, "The LOFAR Beam Former"):

* ``delays``     -- tau[b][s] = p_s . (u_b - u_ref) / c0 - delta_s (Sec. 3; Sec. 4.3:
  weights depend on station location, channel frequency and beam coordinates;
  delta_s is an optional per-station residual delay, see ``phase_correct``)
* ``phase_correct`` -- sub-sample delay compensation (Sec. 3): after the
  station series are shifted by whole samples, each sample is multiplied by a
  complex phase that removes the station's remaining delay at the channel's
  frequency
* ``weights``    -- w[c][b][s] = exp(-2 pi i frac(f_c tau)) (Sec. 3, phase shift
  by a complex multiplication per sample)
* ``beamform``   -- y[c][b][t][p] = sum_s w[c][b][s] x[s][c][t][p] (Sec. 1,
  Sec. 3, Sec. 4.3: weighted addition of the station signals)
* ``stokes``     -- I, Q, U, V as defined in Sec. 4.5
* ``integrate``  -- sums over t_int samples and f_int channels (Sec. 3, Sec. 5.1)
* ``reorder``    -- final per-beam, per-Stokes order [b][k][t'][c'] (Sec. 4.6)
* ``incoherent`` -- sum over stations of per-station Stokes (Sec. 3)
* ``superstation`` -- superstation beam forming (Sec. 4.2): member stations
  combined, with their weights, into one station signal
* ``channelize`` -- the FFT that splits each subband into channels (Sec. 4.2):
  nch consecutive subband samples -> nch channels, lowest frequency first
* ``dedisperse`` -- channel-level dedispersion (Sec. 4.4): per block of
  n_fft samples a forward FFT, a product with the channel's precomputed
  complex chirp weights, and a backward FFT; numpy's FFT is the FFT step

Parity pins for every function are in ``tests/test_oracle_pins.py``; the
absolute values of the beam former have no worked example in the paper, so
they are pinned by closed forms, invariants, brute force and an independent
library routine (numpy einsum), not by printed numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbf_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "liboracle.so")
_XT = {"ci8": 0, "ci16": 1, "cf32": 2}
_lock = threading.Lock()
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile lbf_oracle.c into _build/liboracle.so with gcc (plain -O2)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_SO)
            vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
            lib.lbfo_delays.argtypes = [_dp, i, _dp, i, vp, vp, _dp]
            lib.lbfo_weights.argtypes = [_dp, i, i, _dp, i, _dp]
            lib.lbfo_beamform.argtypes = [vp, i, i, i, i, i, i, _dp, i, _dp]
            lib.lbfo_stokes.argtypes = [_dp, i, i, i, _dp]
            lib.lbfo_integrate.argtypes = [_dp, i, i, i, i, i, i, _dp]
            lib.lbfo_reorder.argtypes = [_dp, i, i, i, i, i, _dp]
            lib.lbfo_incoherent.argtypes = [vp, i, i, i, i, i, i, i, _dp]
            lib.lbfo_pipeline.argtypes = [vp, i, i, i, i, _dp, _dp, i, vp, vp, _dp, i, i, i, i, _dp]
            lib.lbfo_pipeline.restype = i
            for f in ("lbfo_delays", "lbfo_weights", "lbfo_beamform", "lbfo_stokes", "lbfo_integrate",
                      "lbfo_reorder", "lbfo_incoherent"):
                getattr(lib, f).restype = None
            _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _xtype_of(x: np.ndarray) -> int:
    if x.dtype == np.int8:
        return _XT["ci8"]
    if x.dtype == np.int16:
        return _XT["ci16"]
    if x.dtype == np.float32:
        return _XT["cf32"]
    raise TypeError("station samples must be int8, int16 or float32, got %s" % x.dtype)


def delays(pos, dirs, ref=None, resid=None) -> np.ndarray:
    """tau[b][s] in seconds; ``resid`` [S]: residual delays (seconds, positive
    for a station whose signal arrives late), subtracted from every beam's
    delay of that station."""
    pos, dirs = _f64(pos), _f64(dirs)
    S, B = pos.shape[0], dirs.shape[0]
    tau = np.empty((B, S))
    refp = None if ref is None else _f64(ref)
    rp = None if resid is None else _f64(resid)
    if rp is not None and rp.shape != (S,):
        raise ValueError("resid must hold one delay per station")
    _load().lbfo_delays(pos, S, dirs, B, None if refp is None else refp.ctypes.data,
                        None if rp is None else rp.ctypes.data, tau)
    return tau


def weights(tau, freq) -> np.ndarray:
    """w[c][b][s] complex128."""
    tau, freq = _f64(tau), _f64(freq)
    B, S = tau.shape
    C = freq.shape[0]
    w = np.empty((C, B, S, 2))
    _load().lbfo_weights(tau, B, S, freq, C, w)
    return w[..., 0] + 1j * w[..., 1]


def beamform(x: np.ndarray, w: np.ndarray, c_lo: int = 0, nc: int | None = None) -> np.ndarray:
    """y[nc][B][T][2] complex128 for channels [c_lo, c_lo+nc) of x[S][C][T][2][2];
    w holds the weights of those channels only: w[nc][B][S]."""
    x = np.ascontiguousarray(x)
    S, C, T = x.shape[:3]
    if nc is None:
        nc = C - c_lo
    B = w.shape[1]
    wr = np.ascontiguousarray(np.stack([w.real, w.imag], axis=-1), dtype=np.float64)
    assert wr.shape == (nc, B, S, 2)
    y = np.empty((nc, B, T, 2, 2))
    _load().lbfo_beamform(x.ctypes.data, _xtype_of(x), S, C, T, c_lo, nc, wr, B, y)
    return y[..., 0] + 1j * y[..., 1]


def stokes(y: np.ndarray) -> np.ndarray:
    """st[c][b][t][4] = (I, Q, U, V) float64 from y[c][b][t][2] complex."""
    C, B, T = y.shape[:3]
    yr = np.ascontiguousarray(np.stack([y.real, y.imag], axis=-1), dtype=np.float64)
    st = np.empty((C, B, T, 4))
    _load().lbfo_stokes(yr, C, B, T, st)
    return st


def integrate(st: np.ndarray, K: int, t_int: int, f_int: int) -> np.ndarray:
    """s[c'][b][t'][K] (sums)."""
    C, B, T = st.shape[:3]
    assert C % f_int == 0 and T % t_int == 0
    s = np.empty((C // f_int, B, T // t_int, K))
    _load().lbfo_integrate(_f64(st), C, B, T, K, t_int, f_int, s)
    return s


def reorder(s: np.ndarray) -> np.ndarray:
    """[c'][b][t'][k] -> [b][k][t'][c'] (real or complex)."""
    C2, B, T2, K = s.shape
    if np.iscomplexobj(s):
        sr = np.ascontiguousarray(np.stack([s.real, s.imag], axis=-1), dtype=np.float64)
        out = np.empty((B, K, T2, C2, 2))
        _load().lbfo_reorder(sr, C2, B, T2, K, 2, out)
        return out[..., 0] + 1j * out[..., 1]
    out = np.empty((B, K, T2, C2))
    _load().lbfo_reorder(_f64(s), C2, B, T2, K, 1, out)
    return out


def incoherent(x: np.ndarray, K: int, t_int: int, f_int: int) -> np.ndarray:
    """Incoherent beam inc[c'][t'][K]: sum over stations of per-station Stokes."""
    x = np.ascontiguousarray(x)
    S, C, T = x.shape[:3]
    inc = np.empty((C // f_int, T // t_int, K))
    _load().lbfo_incoherent(x.ctypes.data, _xtype_of(x), S, C, T, K, t_int, f_int, inc)
    return inc


def pipeline(x: np.ndarray, pos, dirs, ref, freq, K: int, t_int: int = 1, f_int: int = 1,
             nthreads: int = 1, resid=None) -> np.ndarray:
    """Whole chain: out[B][K][T/t_int][C/f_int] (K in {1, 4}) or, for K == 0,
    voltages [B][2][T][C] complex128.  ``resid``: per-station residual delays
    folded into the weights (see ``delays``)."""
    x = np.ascontiguousarray(x)
    S, C, T = x.shape[:3]
    pos, dirs, freq = _f64(pos), _f64(dirs), _f64(freq)
    B = dirs.shape[0]
    refp = None if ref is None else _f64(ref)
    rp = None if resid is None else _f64(resid)
    if rp is not None and rp.shape != (S,):
        raise ValueError("resid must hold one delay per station")
    if K == 0:
        out = np.empty((B, 2, T, C, 2))
    else:
        out = np.empty((B, K, T // t_int, C // f_int))
    rc = _load().lbfo_pipeline(x.ctypes.data, _xtype_of(x), S, C, T, pos, dirs, B,
                               None if refp is None else refp.ctypes.data,
                               None if rp is None else rp.ctypes.data, freq, K, t_int, f_int,
                               nthreads, out)
    if rc != 0:
        raise ValueError("oracle pipeline rejected its arguments")
    if K == 0:
        return out[..., 0] + 1j * out[..., 1]
    return out


def phase_correct(x: np.ndarray, freq, resid) -> np.ndarray:
    """Sub-sample delay compensation (Sec. 3): once station series have been
    shifted against each other by whole samples, the delay that remains,
    resid[s] seconds (positive: station s's signal arrives late), is removed
    by one complex multiplication per sample that advances its phase at the
    sample's frequency:
        out[s][c][t][p] = x[s][c][t][p] * exp(+2 pi i frac(f_c resid[s])).
    The fractional turn is taken in FP64 as for the weights.  x: channelised
    samples [S][C][T][2] (complex) or [S][C][T][2][2] (re, im last); freq [C]
    Hz; resid [S] s.  Returns complex128 [S][C][T][2]."""
    x = np.asarray(x)
    if not np.iscomplexobj(x):
        x = x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)
    freq, resid = _f64(freq), _f64(resid)
    S, C = x.shape[:2]
    if freq.shape != (C,) or resid.shape != (S,):
        raise ValueError("freq must be [C] and resid [S]")
    m = resid[:, None] * freq[None, :]                        # turns, [S][C]
    r = m - np.rint(m)
    rot = np.cos(2.0 * np.pi * r) + 1j * np.sin(2.0 * np.pi * r)
    return x.astype(np.complex128) * rot[:, :, None, None]


def block_weights(blk, use_ref: bool = True) -> np.ndarray:
    """Weights of a synthetic block (complex128 [C][B][S])."""
    return weights(delays(blk.station_xyz, blk.beam_dir, blk.ref_dir if use_ref else None), blk.freq_hz)


def dedisperse(y: np.ndarray, chirp: np.ndarray, n_fft: int) -> np.ndarray:
    """Channel-level dedispersion (Sec. 4.4) of beam voltages y[C][B][T][2]
    (complex): every polarisation's time series is cut into blocks of n_fft
    consecutive samples; each block is Fourier transformed (forward sign
    exp(-2 pi i j k / n_fft)), multiplied bin by bin with the channel's chirp
    weights chirp[C][n_fft] (bin k at index k), and transformed back.  The
    backward transform carries the 1/n_fft factor, so all-one weights give
    the input back.  Returns complex128 [C][B][T][2]."""
    y = np.asarray(y, dtype=np.complex128)
    chirp = np.asarray(chirp, dtype=np.complex128)
    C, B, T, P = y.shape
    if T % n_fft or chirp.shape != (C, n_fft):
        raise ValueError("T must be a multiple of n_fft and chirp must be [C][n_fft]")
    blocks = y.reshape(C, B, T // n_fft, n_fft, P)
    spec = np.fft.fft(blocks, axis=3)                       # forward, per block and polarisation
    spec = spec * chirp[:, None, None, :, None]              # the channel's chirp, same for every beam
    out = np.fft.ifft(spec, axis=3)                          # backward, with the 1/n_fft factor
    return out.reshape(C, B, T, P)


def channelize(x: np.ndarray, nch: int, t_sb: int | None = None, shift=None) -> np.ndarray:
    """Channeliser (Sec. 4.2) with sample-granularity delay compensation
    (Sec. 3: station series are shifted against each other by whole samples).
    Station s contributes its subband samples [shift[s], shift[s] + t_sb) of
    x (samples outside the row count as zero); each subband's complex time
    series (per station and polarisation) is then cut into consecutive groups
    of nch samples, and the FFT of a group (forward sign, no window, no
    scaling) gives its nch channels.  Channel q of subband sb is FFT bin
    (q + nch/2) mod nch, so channels run from the lowest frequency (q = 0,
    nch/2 channel widths below the subband's centre) upwards.
    x: [S][NSB][T_in][2][2] (re, im last; int8, int16 or float32); t_sb
    defaults to T_in and shift to zeros.  Returns complex128
    [S][NSB nch][t_sb / nch][2]."""
    x = np.asarray(x)
    S, NSB, Tin = x.shape[:3]
    Tsb = Tin if t_sb is None else t_sb
    if Tsb % nch:
        raise ValueError("T_sb must be a multiple of nch")
    xin = x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)     # [S][NSB][T_in][2]
    xc = np.zeros((S, NSB, Tsb, 2), np.complex128)
    for st in range(S):                                                         # the shifted window
        d = 0 if shift is None else int(shift[st])
        lo, hi = max(d, 0), min(d + Tsb, Tin)
        if hi > lo:
            xc[st, :, lo - d:hi - d] = xin[st, :, lo:hi]
    groups = xc.reshape(S, NSB, Tsb // nch, nch, 2)
    spec = np.fft.fft(groups, axis=3)                                           # bin k
    spec = np.fft.fftshift(spec, axes=3)                                        # channel q = bin (q + nch/2) mod nch
    return spec.transpose(0, 1, 3, 2, 4).reshape(S, NSB * nch, Tsb // nch, 2)


def superstation(x: np.ndarray, w, groups) -> np.ndarray:
    """Superstation beam forming (Sec. 4.2: a simplified beam former that
    combines several stations as if they were one): for each group g of
    member stations, out[g][c][t][p] = sum over members s of
    w[c][s] x[s][c][t][p].  x: [S][C][T][2][2] (re, im last); w: complex
    [C][S], or None for unit weights; groups: a list of member-index lists.
    Returns complex128 [G][C][T][2]."""
    x = np.asarray(x)
    S, C, T = x.shape[:3]
    xc = x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)      # [S][C][T][2]
    wt = np.ones((C, S), np.complex128) if w is None else np.asarray(w, np.complex128)
    out = np.zeros((len(groups), C, T, 2), np.complex128)
    for g, members in enumerate(groups):
        for s in members:                                                       # the member sum, in member order
            out[g] += wt[:, s, None, None] * xc[s]
    return out
