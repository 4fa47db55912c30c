"""Benchmark of the beam-forming hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the one-second block -- 64 stations, 32 subbands x 256 channels
(8192 channels), 768 samples per channel, dual-pol complex int16 (sigma 64,
3 injected tones), 128 tied-array beams on a 0.05 deg hexagonal grid, Stokes
IQUV integrated 16x in time, beam-major f32 output.  Synthetic data (seeded),
resident in HBM before timing starts.

One step = one block through the whole hot path: FP64 weights
(lbf_compute_weights) + the fused beam former (contraction, Stokes,
integration, beam-major store; lbf_beamform).  ``value`` is the FP32-operand
path in beam-samples/s (one dual-pol sample of one beam in one channel);
the FP16-MFMA and BF16-MFMA paths on the same block are reported beside it,
with every path's error against the FP64 oracle on sampled channels.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "f32_TFLOPs": 157.3, "f16_TFLOPs": 2500.0, "bf16_TFLOPs": 2500.0}
SUBBAND_HZ = 195312.5


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-extra", action="store_true", help="skip the 488-beam precision block")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    p.add_argument("--only", default="", help="comma list of paths to time: f32,f16,bf16 (profiling runs)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--profile-precision", action="store_true",
                   help="profiling run: time only the 488-beam block paths (no JSON line)")
    p.add_argument("--serve-seconds", type=float, default=60.0, help="measured seconds of the streaming run")
    p.add_argument("--serve-warmup", type=float, default=5.0, help="warm-up seconds of the streaming run")
    p.add_argument("--profile-batch", action="store_true",
                   help="profiling run: time only the uneven batch (no JSON line)")
    p.add_argument("--profile-aux", action="store_true",
                   help="profiling run: only the kernels beside the beam former -- incoherent beam, "
                        "dedispersion, the case-E chain, channeliser, superstations (no JSON line)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="counter calibration run: three plain 1 GiB device-to-device copies (no JSON line)")
    return p.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def relerr(g, o):
    g = np.asarray(g, dtype=np.float64)
    return float(np.linalg.norm((g - o).ravel()) / max(np.linalg.norm(o.ravel()), 1e-300))


def max_over_rms(g, o):
    """max |g - o| / rms(o): the largest single error against the typical size."""
    g = np.asarray(g, dtype=np.float64)
    return float(np.max(np.abs(g - o)) / max(np.sqrt(np.mean(o * o)), 1e-300))


def host_threads():
    """Cores this process may run on (its affinity), and the machine's count."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return aff, os.cpu_count() or aff


def time_path(lbf, torch, x, geo, ctype, product, t_int, f_int, steps, warmup):
    """Time `steps` blocks through the whole path on torch's current stream:
    FP64 weights (lbf_compute_weights), the contraction kernel with fused Stokes
    and integration (lbf_beamform_channel_major, one kernel launch) and the
    reorder into the beam-major final order (lbf_beam_major).  HIP events on
    that stream bracket each call.  Returns per-step and per-call ms and the
    beam-major output of the last step."""
    pos, dirs, freq, ref = geo
    S, C, T = x.shape[:3]
    B = dirs.shape[0]
    w = torch.empty((C, B, S, 2), dtype=lbf.weight_dtype(ctype), device=x.device)
    cm = torch.empty(lbf.output_shape(product, S, C, T, B, t_int, f_int, channel_major=True), dtype=torch.float32,
                     device=x.device)
    out = torch.empty(lbf.output_shape(product, S, C, T, B, t_int, f_int), dtype=torch.float32, device=x.device)
    n = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n)]
    torch.cuda.synchronize()
    t0 = None
    for i in range(n):
        if i == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        ev[i][0].record()
        lbf.compute_weights(pos, dirs, freq, ctype, ref_dir=ref, out=w)
        ev[i][1].record()
        lbf.beamform_channel_major(x, w, product, t_int, f_int, out=cm)
        ev[i][2].record()
        lbf.beam_major(cm, out=out)
        ev[i][3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def span(a, b):
        return np.array([ev[i][a].elapsed_time(ev[i][b]) for i in range(warmup, n)])

    return dict(wall_s=wall, step_ms=span(0, 3), weights_ms=span(0, 1), beamform_ms=span(1, 2),
                reorder_ms=span(2, 3), out=out, w=w)


def unfused(lbf, torch, x, geo, nch, steps, warmup):
    """The unfused chain on the first `nch` channels of a block: FP32 voltages
    (lbf_beamform VOLTAGES), Stokes IQUV integrated x16 (lbf_stokes) and the
    final order (lbf_transpose), each timed with HIP events on the current
    stream, against the fused product of the same channels."""
    pos, dirs, freq, ref = geo
    xs = x[:, :nch].contiguous()
    S, C, T = xs.shape[:3]
    B = dirs.shape[0]
    w = lbf.compute_weights(pos, dirs, freq[:nch].contiguous(), lbf.F32, ref_dir=ref)
    n = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n)]
    y = s = o = None
    for i in range(n):
        ev[i][0].record()
        y = lbf.beamform(xs, w, lbf.VOLTAGES, out=y)
        ev[i][1].record()
        s = lbf.stokes(y, lbf.STOKES_IQUV, 16, 1, out=s)
        ev[i][2].record()
        o = lbf.transpose(s, out=o)
        ev[i][3].record()
    fused = lbf.beamform(xs, w, lbf.STOKES_IQUV, 16, 1)
    torch.cuda.synchronize()

    def span(a, b):
        return float(np.mean([ev[i][a].elapsed_time(ev[i][b]) for i in range(warmup, n)]))

    v_ms, s_ms, t_ms = span(0, 1), span(1, 2), span(2, 3)
    y_bytes = C * B * T * 16
    s_bytes = C * B * (T // 16) * 4 * 4
    v_bytes = S * C * T * 8 + C * B * S * 8 + y_bytes
    err = relerr(o.cpu().numpy(), fused.cpu().numpy())
    del xs, y, s, o, fused
    return {"workload": "first %d channels of the one-second block, FP32 voltages -> Stokes IQUV x16 -> final order"
                        % nch,
            "voltages_kernel_ms": v_ms, "voltages_hbm_GBps": v_bytes / (v_ms / 1e3) / 1e9,
            "stokes_kernel_ms": s_ms, "stokes_hbm_GBps": (y_bytes + s_bytes) / (s_ms / 1e3) / 1e9,
            "transpose_kernel_ms": t_ms, "transpose_hbm_GBps": 2 * s_bytes / (t_ms / 1e3) / 1e9,
            "rel_err_vs_fused": err}


def incoherent(lbf, torch, x, steps, warmup, mp, geo=None):
    """The incoherent beam (sum over stations of the station powers) of the
    whole one-second block, Stokes IQUV integrated x16: an HBM-bound read of
    every sample once.  HIP events on the current stream around each launch.
    With the block's geometry, also both products from one read of the
    samples (lbf_beamform_incoherent, FP16 MFMA) against lbf_beamform then
    lbf_incoherent."""
    S, C, T = x.shape[:3]
    n = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n)]
    out = None
    for i in range(n):
        ev[i][0].record()
        out = lbf.incoherent(x, lbf.STOKES_IQUV, 16, 1, out=out)
        ev[i][1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(warmup, n)]))
    nbytes = S * C * T * x.element_size() * 4 + 4 * (T // 16) * C * 4
    gbps = nbytes / (ms / 1e3) / 1e9
    r = {"workload": "incoherent beam of the one-second block (64 stations, 8192 channels, 768 samples, "
                     "complex int16), Stokes IQUV x16",
         "kernel_ms": ms, "algorithmic_bytes": nbytes, "hbm_GBps": gbps, "bound": "hbm",
         "frac": gbps / PEAK["hbm_GBps"]}
    if mp:
        r["frac_of_measured_hbm"] = gbps / max(mp["hbm_GBps"], mp["hbm_read_GBps"])
    if geo is not None:
        pos, dirs, freq, ref = geo
        B = dirs.shape[0]
        w = lbf.compute_weights(pos, dirs, freq, lbf.F16, ref_dir=ref)
        bf = torch.empty((B, 4, T // 16, C), dtype=torch.float32, device=x.device)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n)]
        for i in range(n):
            ev[i][0].record()
            lbf.beamform_incoherent(x, w, lbf.STOKES_IQUV, 16, 1, out=bf, inc=out)
            ev[i][1].record()
            lbf.beamform(x, w, lbf.STOKES_IQUV, 16, 1, out=bf)
            ev[i][2].record()
            lbf.incoherent(x, lbf.STOKES_IQUV, 16, 1, out=out)
            ev[i][3].record()
        torch.cuda.synchronize()

        def span(a, b):
            return float(np.mean([ev[i][a].elapsed_time(ev[i][b]) for i in range(warmup, n)]))

        r["with_beams"] = {"workload": "128 tied-array beams (FP16 MFMA, Stokes IQUV x16, final order) and the "
                                       "incoherent beam of the one-second block",
                           "one_read_ms": span(0, 1), "two_reads_ms": span(1, 3),
                           "beamform_ms": span(1, 2), "incoherent_ms": span(2, 3)}
        del w, bf
    return r


def superstations(lbf, torch, dev, steps, warmup, mp):
    """Superstation beam forming on the one-second block's shape: 64 stations
    (complex int16, 8192 channels, 768 samples) into 8 superstations of 8
    stations each, unit-modulus weights per (channel, station).  HBM-bound:
    every station sample read once, every superstation sample written once."""
    S, C, T, G = 64, 8192, 768, 8
    gen = torch.Generator(device=dev).manual_seed(1105662)
    x = torch.randint(-300, 301, (S, C, T, 2, 2), generator=gen, device=dev, dtype=torch.int16)
    ph = torch.rand((C, S), generator=gen, device=dev, dtype=torch.float64) * 2 * np.pi
    w = torch.stack([torch.cos(ph), torch.sin(ph)], dim=-1).float().contiguous()
    groups = [list(range(8 * g, 8 * g + 8)) for g in range(G)]
    out = torch.empty((G, C, T, 2, 2), dtype=torch.float32, device=dev)
    nrep = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nrep)]
    for i in range(nrep):
        ev[i][0].record()
        lbf.superstation(x, groups, w, out=out)
        ev[i][1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(warmup, nrep)]))
    nbytes = S * C * T * 8 + G * C * T * 16 + C * S * 8
    gbps = nbytes / (ms / 1e3) / 1e9
    r = {"workload": "superstation beam forming: 64 stations (complex int16, 8192 channels, 768 samples, 2 pols) "
                     "-> 8 superstations of 8 stations, weighted",
         "kernel_ms": ms, "algorithmic_bytes": nbytes, "hbm_GBps": gbps, "bound": "hbm",
         "frac": gbps / PEAK["hbm_GBps"]}
    if mp:
        r["frac_of_measured_hbm"] = gbps / max(mp["hbm_GBps"], mp["hbm_read_GBps"])
    del x, w, out
    return r


def channelizer(lbf, torch, dev, steps, warmup, mp, geo=None):
    """The channeliser ahead of the one-second block: 64 stations x 32
    subbands of 196608 complex int16 samples (1.0066 s at 195 kHz), 256
    channels per subband -> the block's [64][8192][768][2] channels in
    complex f32.  Seeded uniform int16 samples generated on the device.
    HBM-bound: every sample read once, every channel sample written once.
    With the block's geometry, also the chain channelise -> beam form (128
    beams, Stokes IQUV x16) on those complex f32 channels, FP16 MFMA and FP32."""
    S, NSB, nch = 64, 32, 256
    T_sb = 768 * nch
    gen = torch.Generator(device=dev).manual_seed(1105661)
    # rows 64 samples longer than the window, so that shifted windows stay inside them
    x = torch.randint(-300, 301, (S, NSB, T_sb + 64, 2, 2), generator=gen, device=dev, dtype=torch.int16)
    shift = torch.randint(0, 64, (S,), generator=gen, device=dev, dtype=torch.int32)
    out = torch.empty((S, NSB * nch, T_sb // nch, 2, 2), dtype=torch.float32, device=dev)
    nrep = warmup + steps

    def timed(sh):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nrep)]
        for i in range(nrep):
            ev[i][0].record()
            lbf.channelize(x, nch, t_sb=T_sb, shift=sh, out=out)
            ev[i][1].record()
        torch.cuda.synchronize()
        return float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(warmup, nrep)]))

    ms = timed(None)
    ms_shift = timed(shift)
    nbytes = S * NSB * T_sb * 8 + S * NSB * T_sb * 16
    gbps = nbytes / (ms / 1e3) / 1e9
    r = {"workload": "channeliser of the one-second block: 64 stations, 32 subbands x 196608 complex int16 "
                     "samples, 2 pols -> 256 channels per subband, complex f32",
         "kernel_ms": ms, "algorithmic_bytes": nbytes, "hbm_GBps": gbps, "bound": "hbm",
         "frac": gbps / PEAK["hbm_GBps"],
         "input_Gbps": S * NSB * T_sb * 64 / (ms / 1e3) / 1e9,
         "kernel_ms_with_station_shifts": ms_shift,
         "station_shifts": "seeded per-station whole-sample shifts U{0..63} (delay compensation)"}
    if mp:
        r["frac_of_measured_hbm"] = gbps / max(mp["hbm_GBps"], mp["hbm_read_GBps"])
    if geo is not None:
        pos, dirs, freq, ref = geo
        B = dirs.shape[0]
        chain = {}
        for name, ct in (("f16", lbf.F16), ("f32", lbf.F32)):
            w = lbf.compute_weights(pos, dirs, freq, ct, ref_dir=ref)
            bf = torch.empty((B, 4, 48, NSB * nch), dtype=torch.float32, device=dev)
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(nrep)]
            for i in range(nrep):
                ev[i][0].record()
                lbf.channelize(x, nch, t_sb=T_sb, shift=shift, out=out)
                ev[i][1].record()
                lbf.beamform(out, w, lbf.STOKES_IQUV, 16, 1, out=bf)
                ev[i][2].record()
            torch.cuda.synchronize()
            bms = float(np.mean([ev[i][1].elapsed_time(ev[i][2]) for i in range(warmup, nrep)]))
            tms = float(np.mean([ev[i][0].elapsed_time(ev[i][2]) for i in range(warmup, nrep)]))
            fpc = lbf.block_footprint(S, NSB * nch, 768, B, lbf.CF32, ct, lbf.STOKES_IQUV, 16, 1)
            chain[name] = {"beamform_ms": bms, "chain_ms": tms,
                           "beamform_hbm_GBps": (fpc.input_bytes + fpc.weight_bytes + fpc.output_bytes)
                           / (bms / 1e3) / 1e9,
                           "beam_samples_per_s": B * NSB * nch * 768 / (tms / 1e3)}
            del w, bf
        r["channelise_then_beamform"] = dict(chain, workload="channelise with the station shifts (above) -> "
                                                             "lbf_beamform on the complex f32 channels: 128 beams, "
                                                             "Stokes IQUV x16, final order")
    del x, out
    return r


def dedispersion(lbf, torch, dev, steps, warmup, mp):
    """Channel-level dedispersion at Table 1 case E's shape on one GPU's share
    of the subbands: 32 subbands x 16 channels (12.2 kHz), 10 beams, three
    4096-sample blocks (1.007 s), seeded Gaussian voltages and unit-modulus
    chirp weights.  FFT, chirp product and inverse FFT in one kernel that
    reads and writes every voltage once: HBM-bound."""
    C, B, T, n = 512, 10, 3 * 4096, 4096
    gen = torch.Generator().manual_seed(1105661)
    y = (torch.randn((C, B, T, 2, 2), generator=gen) * 100.0).to(dev)
    ph = torch.rand((C, n), generator=gen, dtype=torch.float64) * 2 * np.pi
    h = torch.stack([torch.cos(ph), torch.sin(ph)], dim=-1).float().to(dev)
    out = torch.empty_like(y)
    nrep = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(nrep)]
    for i in range(nrep):
        ev[i][0].record()
        lbf.dedisperse(y, h, n, out=out)
        ev[i][1].record()
    torch.cuda.synchronize()
    ms = float(np.mean([ev[i][0].elapsed_time(ev[i][1]) for i in range(warmup, nrep)]))
    nbytes = 2 * C * B * T * 16 + C * n * 8
    gbps = nbytes / (ms / 1e3) / 1e9
    r = {"workload": "channel-level dedispersion, Table 1 case E share: 512 channels of 12.2 kHz, 10 beams, "
                     "3 blocks of 4096 samples, 2 pols, FP32 FFT -> chirp -> inverse FFT",
         "kernel_ms": ms, "algorithmic_bytes": nbytes, "hbm_GBps": gbps, "bound": "hbm",
         "frac": gbps / PEAK["hbm_GBps"],
         "beam_samples_per_s": C * B * T / (ms / 1e3)}
    if mp:
        r["frac_of_measured_hbm"] = gbps / max(mp["hbm_GBps"], mp["hbm_read_GBps"])
    del y, h, out
    return r


def pulsar_chain(lbf, torch, synth, dev, steps, warmup, mp):
    """Table 1 case E end to end on one GPU's share of the subbands: 64
    stations of complex int16 (32 subbands x 16 channels of 12.2 kHz, 3 x
    4096 samples = 1.007 s), 10 tied-array beams formed as voltages (FP16
    MFMA), channel-level dedispersion (4096-point FFT, chirp, inverse FFT),
    Stokes IQUV at full time resolution (case E's 6.2 Gb/s per beam) and the
    final per-beam order.  Fused: lbf_dedisperse_stokes keeps the dedispersed
    voltages on chip; unfused: lbf_dedisperse, lbf_stokes.  Both end with
    lbf_transpose, and their outputs agree."""
    S, B, nsb, nch, n = 64, 10, 32, 16, 4096
    T = 3 * n
    blk = synth.make_block(S, B, nsb, nch, T, "ci16", 64.0, tag=(1105, 661, 5), n_tones=2, tone_amp=64.0,
                           threads=16)
    x = torch.from_numpy(blk.x).to(dev)
    del blk.x
    C = blk.C
    w = lbf.compute_weights(torch.from_numpy(blk.station_xyz).to(dev), torch.from_numpy(blk.beam_dir).to(dev),
                            torch.from_numpy(blk.freq_hz).to(dev), lbf.F16, ref_dir=blk.ref_dir)
    gen = torch.Generator().manual_seed(1105662)
    ph = torch.rand((C, n), generator=gen, dtype=torch.float64) * 2 * np.pi
    h = torch.stack([torch.cos(ph), torch.sin(ph)], dim=-1).float().to(dev)
    y = torch.empty((C, B, T, 2, 2), device=dev)
    yd = torch.empty_like(y)
    s = torch.empty((C, B, T, 4), device=dev)
    s2 = torch.empty_like(s)
    o = torch.empty((B, 4, T, C), device=dev)
    o2 = torch.empty_like(o)
    nrep = warmup + steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(8)] for _ in range(nrep)]
    for i in range(nrep):
        e = ev[i]
        e[0].record()
        lbf.beamform(x, w, lbf.VOLTAGES, out=y)
        e[1].record()
        lbf.dedisperse_stokes(y, h, n, lbf.STOKES_IQUV, 1, out=s)
        e[2].record()
        lbf.transpose(s, out=o)
        e[3].record()
        lbf.beamform(x, w, lbf.VOLTAGES, out=y)
        e[4].record()
        lbf.dedisperse(y, h, n, out=yd)
        e[5].record()
        lbf.stokes(yd, lbf.STOKES_IQUV, 1, 1, out=s2)
        e[6].record()
        lbf.transpose(s2, out=o2)
        e[7].record()
    torch.cuda.synchronize()

    def span(a, b):
        return float(np.mean([ev[i][a].elapsed_time(ev[i][b]) for i in range(warmup, nrep)]))

    fused = {"beamform_ms": span(0, 1), "dedisperse_stokes_ms": span(1, 2), "transpose_ms": span(2, 3),
             "total_ms": span(0, 3)}
    unf = {"beamform_ms": span(3, 4), "dedisperse_ms": span(4, 5), "stokes_ms": span(5, 6),
           "transpose_ms": span(6, 7), "total_ms": span(3, 7)}
    vb = C * B * T * 16                                     # voltages, or Stokes IQUV at full resolution
    dd_bytes = vb + C * n * 8 + vb                          # fused: voltages in, Stokes out
    diff = float((o - o2).norm() / o2.norm())
    r = {"workload": "Table 1 case E share: 64 stations ci16, 512 channels (32 x 16 of 12.2 kHz), 12288 samples, "
                     "10 beams: voltages (FP16 MFMA) -> dedispersion (4096-point) -> Stokes IQUV x1 -> final order",
         "fused": fused, "unfused": unf, "rel_diff_fused_vs_unfused": diff,
         "beam_samples_per_s": C * B * T / (fused["total_ms"] / 1e3),
         "input_Gbps": S * C * T * 8 * 8 / (fused["total_ms"] / 1e3) / 1e9,
         "dedisperse_stokes_hbm_GBps": dd_bytes / (fused["dedisperse_stokes_ms"] / 1e3) / 1e9,
         "realtime_factor": (T * nch / SUBBAND_HZ) / (fused["total_ms"] / 1e3)}
    if mp:
        r["dedisperse_stokes_frac_of_measured_hbm"] = r["dedisperse_stokes_hbm_GBps"] / max(mp["hbm_GBps"],
                                                                                            mp["hbm_read_GBps"])
    del x, w, h, y, yd, s, s2, o, o2
    return r


def measured_peaks(lbf, torch, dev):
    """What this device sustains: register-only MFMA loops in the contraction's
    instruction forms (FP16 32x32x16, FP32 32x32x2), a 4 GiB device copy
    (read + write) and a 4 GiB read stream, each timed with HIP events
    (lbf_probe)."""
    sink = torch.empty(512, dtype=torch.float32, device=dev)
    src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    out = {}
    for name, kind, iters, scale in (("f16_TFLOPs", lbf.PROBE_MFMA_F16, 16000, 1e12),
                                     ("f32_TFLOPs", lbf.PROBE_MFMA_F32, 8000, 1e12),
                                     ("hbm_GBps", lbf.PROBE_COPY, 1, 1e9),
                                     ("hbm_read_GBps", lbf.PROBE_READ, 1, 1e9)):
        s_, d_ = (src, dst) if kind == lbf.PROBE_COPY else (src, sink) if kind == lbf.PROBE_READ else (None, sink)
        lbf.probe(kind, max(1, iters // 4), s_, d_)                # warm-up (clocks)
        reps = 10 if kind in (lbf.PROBE_COPY, lbf.PROBE_READ) else 2
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        work = sum(lbf.probe(kind, iters, s_, d_) for _ in range(reps))
        e1.record()
        torch.cuda.synchronize()
        out[name] = work / (e0.elapsed_time(e1) / 1e3) / scale
    del src, dst
    return out


def t_roof_s(fp):
    """Roofline time of one FP16-MFMA block: max(MFMA, HBM) at the datasheet peaks."""
    return max(fp.flops / (PEAK["f16_TFLOPs"] * 1e12),
               (fp.input_bytes + fp.weight_bytes + fp.output_bytes) / (PEAK["hbm_GBps"] * 1e9))


def make_jobs(lbf, torch, synth, dev, log_every=4):
    """The uneven batch: 12 one-second blocks of random shape, resident in HBM,
    with their FP16 weights."""
    jobs = []
    for i, js in enumerate(synth.config3_jobs()):
        blk = synth.block_for_job(js, threads=16)
        x = torch.from_numpy(blk.x).to(dev)
        del blk.x
        geo = (torch.from_numpy(blk.station_xyz).to(dev), torch.from_numpy(blk.beam_dir).to(dev),
               torch.from_numpy(blk.freq_hz).to(dev), blk.ref_dir)
        prod = lbf.STOKES_I if js.product == "I" else lbf.STOKES_IQUV
        w = lbf.compute_weights(*geo[:3], lbf.F16, ref_dir=geo[3])
        jobs.append(dict(spec=js, blk=blk, x=x, w=w, prod=prod, geo=geo))
        if (i + 1) % log_every == 0:
            log("generated %d uneven-batch jobs" % (i + 1))
    return jobs


def precision_errors(lbf, torch, b2, x2, geo2):
    """Voltage and Stokes errors of the precision block's FP16 and BF16 paths
    against the FP64 oracle, on the subband that holds the first tone (256
    channels x 488 beams x 768 samples; the whole block's voltages would be
    49 GB, and the work is linear in the channels)."""
    from oracle import oracle as orc
    nthreads, _ = host_threads()
    sb = b2.tones[0].channel // b2.nch
    chans = np.arange(sb * b2.nch, (sb + 1) * b2.nch)
    xs = np.ascontiguousarray(b2.x[:, chans])
    t0 = time.perf_counter()
    vref = orc.pipeline(xs, b2.station_xyz, b2.beam_dir, b2.ref_dir, b2.freq_hz[chans], 0, 1, 1, nthreads)
    sref = orc.pipeline(xs, b2.station_xyz, b2.beam_dir, b2.ref_dir, b2.freq_hz[chans], 4, 16, 1, nthreads)
    cpu_s = time.perf_counter() - t0
    xd = x2[:, torch.from_numpy(chans).to(x2.device)].contiguous()
    pos, dirs, freq, ref = geo2
    out = {"sample": "subband %d (channels %d..%d, holding a tone), all 488 beams and 768 samples; oracle %.1f s "
                     "on %d threads" % (sb, chans[0], chans[-1], cpu_s, nthreads)}
    vr = vref                                                 # [B][2][T][C] complex128
    for name, ct in (("f16", lbf.F16), ("bf16", lbf.BF16)):
        w = lbf.compute_weights(pos, dirs, freq[torch.from_numpy(chans).to(x2.device)].contiguous(), ct, ref_dir=ref)
        y = lbf.beamform(xd, w, lbf.VOLTAGES)                 # [C][B][T][2][2]
        st = lbf.beamform(xd, w, lbf.STOKES_IQUV, 16, 1)      # [B][4][T'][C]
        torch.cuda.synchronize()
        yc = y.cpu().numpy().astype(np.float64)
        yc = (yc[..., 0] + 1j * yc[..., 1]).transpose(1, 3, 2, 0)   # [B][2][T][C]
        got = st.cpu().numpy()
        out[name] = {"voltages_rel_l2": float(np.linalg.norm(yc - vr) / np.linalg.norm(vr)),
                     "voltages_max_over_rms": float(np.max(np.abs(yc - vr)) / np.sqrt(np.mean(np.abs(vr) ** 2))),
                     "stokes_rel_l2": {k: relerr(got[:, i], sref[:, i]) for i, k in enumerate("IQUV")},
                     "stokes_max_over_rms": {k: max_over_rms(got[:, i], sref[:, i]) for i, k in enumerate("IQUV")}}
        del w, y, st
    del xd
    return out


def batched(lbf, torch, jobs, steps, warmup):
    """One persistent launch over all jobs (lbf_beamform_batch) against one
    lbf_beamform per job, FP16 MFMA, weights resident."""
    items, bs, froof, fl = [], 0.0, 0.0, 0.0
    for j in jobs:
        js = j["spec"]
        out = torch.empty(lbf.output_shape(j["prod"], js.S, j["x"].shape[1], js.T, js.B, 16, 1), dtype=torch.float32,
                          device=j["x"].device)
        items.append((j["x"], j["w"], j["prod"], 16, 1, out))
        fp = lbf.block_footprint(js.S, j["x"].shape[1], js.T, js.B, lbf.CI8 if js.xtype == "ci8" else lbf.CI16,
                                 lbf.F16, j["prod"], 16, 1)
        bs += float(js.B) * j["x"].shape[1] * js.T
        froof += t_roof_s(fp)
        fl += fp.flops

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_batch = run(lambda: lbf.beamform_batch(items))
    ms_seq = run(lambda: [lbf.beamform(*it[:5], out=it[5]) for it in items])
    per_job = [run(lambda it=it: lbf.beamform(*it[:5], out=it[5])) for it in items]
    return {"workload": "12 concurrent one-second observations: stations U{24..64}, beams U{1..400}, "
                        "16/64/256 channels x U{8..64} subbands, ci8/ci16, Stokes I or IQUV x16, FP16 MFMA, "
                        "one persistent launch per worker variant",
            "jobs": [{"S": j["spec"].S, "B": j["spec"].B, "C": int(j["x"].shape[1]), "T": j["spec"].T,
                      "xtype": j["spec"].xtype, "product": j["spec"].product, "ms_alone": pj}
                     for j, pj in zip(jobs, per_job)],
            "ms_per_batch": ms_batch, "ms_sequential": ms_seq,
            "beam_samples_per_s": bs / (ms_batch / 1e3), "TFLOPs": fl / (ms_batch / 1e3) / 1e12,
            "roofline_ms": froof * 1e3, "roofline_frac": froof * 1e3 / ms_batch,
            "batch_vs_sequential": ms_seq / ms_batch}


def serving(lbf, torch, synth, jobs, blk1, x1, blk2, x2, seconds, warm_s):
    """Streaming request loop: Poisson arrivals of 0.25/0.5/1 s blocks of 16
    fixed observations (shapes of the one-second block, the precision block and
    the uneven batch), offered at the full array's 198.4 Gb/s, through the
    lbf_server (footprint admission, device weight cache, persistent batches
    on a stream pool), FP16 MFMA.  Then a closed loop for the sustainable rate."""
    dev = x1.device
    rng = np.random.default_rng([1105, 661, 4])
    base = [(blk1, x1, lbf.STOKES_IQUV), (blk2, x2, lbf.STOKES_IQUV)]
    base += [(j["blk"], j["x"], j["prod"]) for j in jobs]
    obs = []
    for i in range(16):
        blk, x, prod = base[i % len(base)]
        d = float(rng.choice([0.25, 0.5, 1.0]))
        T = synth.samples_per_block(d, blk.nch)
        T = min(T, x.shape[2]) // 16 * 16
        xs = x[:, :, :T].contiguous() if T < x.shape[2] else x
        outs = [torch.empty(lbf.output_shape(prod, blk.S, blk.C, T, blk.B, 16, 1), dtype=torch.float32, device=dev)
                for _ in range(3)]
        obs.append(dict(blk=blk, x=xs, prod=prod, T=T, outs=outs, seconds=d, nbytes=xs.numel() * xs.element_size(),
                        next=0))
    mean_bytes = float(np.mean([o["nbytes"] for o in obs]))
    rate_bps = 198.4e9 / 8
    lam = rate_bps / mean_bytes
    arena = torch.empty(24 << 30, dtype=torch.uint8, device=dev)

    def submit(srv, o):
        out = o["outs"][o["next"] % 3]
        o["next"] += 1
        b = o["blk"]
        return srv.submit(id(o) & 0xffffffff, b.station_xyz, b.beam_dir, b.freq_hz, o["x"], lbf.F16, o["prod"], 16, 1,
                          out=out, ref_dir=b.ref_dir)

    res = {}
    with lbf.Server(arena, max_inflight=8, n_streams=2, queue_capacity=256, max_batch=8) as srv:
        # open loop at the real-time rate
        arrivals = synth.poisson_arrivals(lam, warm_s + seconds, seed_tag=(1105, 661, 4))
        pick = rng.integers(0, len(obs), size=len(arrivals))
        t0 = time.monotonic_ns()
        pending = []
        for a, k in zip(arrivals, pick):
            due = t0 + int(a * 1e9)
            while time.monotonic_ns() < due:
                pass
            pending.append((due, a, obs[k], submit(srv, obs[k])))
        lat, bits, first_due, last_due, done_last = [], 0.0, None, 0, 0
        for due, a, o, t in pending:
            st = srv.wait(t, 60000)
            if st.state != lbf.JOB_DONE:
                raise RuntimeError("serving job failed: state %d error %d" % (st.state, st.error))
            if a >= warm_s:
                lat.append((st.t_done_ns - due) / 1e6)
                bits += o["nbytes"] * 8
                first_due = due if first_due is None else first_due
                last_due = due
                done_last = max(done_last, st.t_done_ns)
            srv.release(t)
        offered_s = (last_due - first_due) / 1e9          # arrival span of the measured blocks
        served_s = (done_last - first_due) / 1e9          # first arrival to last completion
        res["open_loop"] = {"offered_Gbps_nominal": 198.4, "arrival_rate_hz": lam, "blocks": len(lat),
                            "warmup_s": warm_s, "measured_s": seconds,
                            "offered_Gbps": bits / offered_s / 1e9, "completed_Gbps": bits / served_s / 1e9,
                            "sustain_ratio": bits / served_s / 198.4e9,
                            "p50_block_latency_ms": float(np.percentile(lat, 50)),
                            "p99_block_latency_ms": float(np.percentile(lat, 99)),
                            "latency": "completion minus arrival, per block"}
        # closed loop: keep the queue full
        n = 96
        order = rng.integers(0, len(obs), size=n)
        t1 = time.monotonic_ns()
        tickets = [(obs[k], submit(srv, obs[k])) for k in order]
        lat2, bits2, last = [], 0.0, t1
        for o, t in tickets:
            st = srv.wait(t, 60000)
            if st.state != lbf.JOB_DONE:
                raise RuntimeError("serving job failed: state %d error %d" % (st.state, st.error))
            lat2.append((st.t_done_ns - st.t_submit_ns) / 1e6)
            bits2 += o["nbytes"] * 8
            last = max(last, st.t_done_ns)
            srv.release(t)
        res["closed_loop"] = {"blocks": n, "sustainable_Gbps": bits2 / ((last - t1) / 1e9) / 1e9,
                              "realtime_factor": bits2 / ((last - t1) / 1e9) / 198.4e9}
    res["workload"] = ("Poisson arrivals of 0.25/0.5/1 s blocks of 16 observations (one-second-block, precision-block "
                       "and uneven-batch shapes), offered at 198.4 Gb/s of station input, device-resident input, "
                       "lbf_server with weight cache, FP16 MFMA; sustain ratio = completed bits/s / 198.4 Gb/s")
    res["mean_block_GB"] = mean_bytes / 1e9
    return res


KERNEL_SOURCES = ["lbf_device.h", "bf_addr.h", "bf_common.h", "bf_workers.h", "bf_fast_impl.h", "bf_fast_f32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_one_second_fp32.txt")


def kernel_source_hash():
    """sha256 over the code of the FP32 contraction kernel's sources: comments
    and blank lines are dropped, so that only a change of code invalidates the
    counter measurements."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1105_0661_amd", "csrc", f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the FP32 contraction kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    device copy), or None if the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if line.startswith("TRAFFIC "):
                    kv = dict(t.split("=", 1) for t in line.split()[1:])
                    if kv.get("sources") == kernel_source_hash():
                        return float(kv["read_bytes"]) + float(kv["write_bytes"])
    except OSError:
        pass
    return None


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs the beam former on a single MI355X "
              "(channels shard across GPUs with no exchange in the hot path; multi-GPU runs are not part "
              "of it). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1105_0661_amd import lbf, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    only = set(v for v in a.only.split(",") if v)

    if a.copy_calibration:
        n = 1 << 28                                  # 1 GiB of float32
        src = torch.ones(n, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes three times" % (4 * n))
        return

    if a.profile_precision:
        b2 = synth.config2(threads=16)
        x2 = torch.from_numpy(b2.x).to(dev)
        geo2 = (torch.from_numpy(b2.station_xyz).to(dev), torch.from_numpy(b2.beam_dir).to(dev),
                torch.from_numpy(b2.freq_hz).to(dev), b2.ref_dir)
        for name, ct in (("f16", lbf.F16), ("bf16", lbf.BF16)):
            if only and name not in only:
                continue
            r = time_path(lbf, torch, x2, geo2, ct, lbf.STOKES_IQUV, 16, 1, a.steps, a.warmup)
            log("precision %s: beam former %.3f ms" % (name, np.mean(r["beamform_ms"])))
        return

    if a.profile_aux:
        blk = synth.config1(threads=16)
        x = torch.from_numpy(blk.x).to(dev)
        del blk.x
        log("incoherent beam: %s" % incoherent(lbf, torch, x, a.steps, a.warmup, None))
        del x
        log("dedispersion: %s" % dedispersion(lbf, torch, dev, a.steps, a.warmup, None))
        log("pulsar chain (case E): %s" % pulsar_chain(lbf, torch, synth, dev, a.steps, a.warmup, None))
        log("channeliser: %s" % channelizer(lbf, torch, dev, a.steps, a.warmup, None))
        log("superstations: %s" % superstations(lbf, torch, dev, a.steps, a.warmup, None))
        return

    if a.profile_batch:
        jobs = make_jobs(lbf, torch, synth, dev)
        r = batched(lbf, torch, jobs, a.steps, a.warmup)
        log("batched: %.3f ms per batch, sequential %.3f ms" % (r["ms_per_batch"], r["ms_sequential"]))
        return

    # ---------------- the one-second block ----------------
    t = time.time()
    blk = synth.config1(threads=16)
    log("generated one-second block in %.1f s (%.2f GB)" % (time.time() - t, blk.x.nbytes / 1e9))
    S, C, T, B = blk.S, blk.C, blk.T, blk.B
    prod, t_int, f_int = lbf.STOKES_IQUV, 16, 1
    x = torch.from_numpy(blk.x).to(dev)
    geo = (torch.from_numpy(blk.station_xyz).to(dev), torch.from_numpy(blk.beam_dir).to(dev),
           torch.from_numpy(blk.freq_hz).to(dev), blk.ref_dir)
    fp = lbf.block_footprint(S, C, T, B, lbf.CI16, lbf.F32, prod, t_int, f_int)
    bsamp = float(B) * C * T
    block_seconds = T * blk.nch / SUBBAND_HZ

    # sampled channels for the oracle: whole subbands, timed until ~cpu-seconds
    res = {}
    for name, ct in (("f32", lbf.F32), ("f16", lbf.F16), ("bf16", lbf.BF16)):
        if only and name not in only:
            continue
        r = time_path(lbf, torch, x, geo, ct, prod, t_int, f_int, a.steps, a.warmup)
        log("%s: step %.3f ms (weights %.3f, contraction %.3f, reorder %.3f)" % (
            name, np.median(r["step_ms"]), np.median(r["weights_ms"]), np.median(r["beamform_ms"]),
            np.median(r["reorder_ms"])))
        res[name] = r
    mp = None if only else measured_peaks(lbf, torch, dev)
    if mp:
        log("measured peaks: %s" % mp)

    # ---------------- oracle on sampled subbands (CPU baseline + errors) ----------------
    cpu = None
    errs = {}
    if not a.no_cpu:
        from oracle import oracle as orc
        ncpu, nproc = host_threads()
        ncpu = min(ncpu, 256)
        done_ch, cpu_s, sb = [], 0.0, 0
        refs = []
        while cpu_s < a.cpu_seconds and sb < blk.nsb:
            chans = np.arange(sb * blk.nch, (sb + 1) * blk.nch)
            xs = np.ascontiguousarray(blk.x[:, chans])
            t1 = time.perf_counter()
            ref = orc.pipeline(xs, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz[chans], 4, t_int, f_int,
                               ncpu)
            cpu_s += time.perf_counter() - t1
            refs.append(ref)
            done_ch.append(chans)
            sb += 1
        chans = np.concatenate(done_ch)
        ref = np.concatenate(refs, axis=3)
        cpu = {"value": float(B * len(chans) * T / cpu_s), "unit": "beam-samples/s", "cores": ncpu,
               "nproc": nproc, "kind": "oracle",
               "sample": "%d of %d subbands (%d channels x %d beams x %d samples, all 64 stations), FP64 C oracle "
                         "with %d threads, %.1f s" % (sb, blk.nsb, len(chans), B, T, ncpu, cpu_s)}
        idx = torch.from_numpy(chans).to(dev)
        for name, r in res.items():
            got = r["out"][:, :, :, idx].cpu().numpy()
            errs[name] = {"rel_l2": {k: relerr(got[:, i], ref[:, i]) for i, k in enumerate("IQUV")},
                          "max_over_rms": {k: max_over_rms(got[:, i], ref[:, i]) for i, k in enumerate("IQUV")}}
        log("cpu baseline: %s" % cpu)

    # ---------------- the 488-beam precision block (MFMA-bound) ----------------
    extra = None
    batch_res = serve_res = unfused_res = inc_res = dd_res = ch_res = ss_res = pc_res = None
    if not a.no_extra and not only:
        unfused_res = unfused(lbf, torch, x, geo, 1024, max(3, a.steps // 4), 1)
        log("unfused chain: %s" % unfused_res)
        inc_res = incoherent(lbf, torch, x, max(5, a.steps // 2), a.warmup, mp, geo)
        log("incoherent beam: %s" % inc_res)
        dd_res = dedispersion(lbf, torch, dev, max(5, a.steps // 2), a.warmup, mp)
        log("dedispersion: %s" % dd_res)
        pc_res = pulsar_chain(lbf, torch, synth, dev, max(5, a.steps // 2), a.warmup, mp)
        log("pulsar chain (case E): %s" % pc_res)
        ch_res = channelizer(lbf, torch, dev, max(5, a.steps // 2), a.warmup, mp, geo)
        log("channeliser: %s" % ch_res)
        ss_res = superstations(lbf, torch, dev, max(5, a.steps // 2), a.warmup, mp)
        log("superstations: %s" % ss_res)
        b2 = synth.config2(threads=16)
        x2 = torch.from_numpy(b2.x).to(dev)
        geo2 = (torch.from_numpy(b2.station_xyz).to(dev), torch.from_numpy(b2.beam_dir).to(dev),
                torch.from_numpy(b2.freq_hz).to(dev), b2.ref_dir)
        extra = {"workload": "precision block: 64 stations, 8192 channels, 768 samples, complex int8, 488 beams, "
                             "Stokes IQUV x16"}
        fp2 = lbf.block_footprint(b2.S, b2.C, b2.T, b2.B, lbf.CI8, lbf.F16, prod, t_int, f_int)
        for name, ct in (("f16", lbf.F16), ("bf16", lbf.BF16)):
            r = time_path(lbf, torch, x2, geo2, ct, prod, t_int, f_int, max(5, a.steps // 2), a.warmup)
            kms = float(np.mean(r["beamform_ms"]))
            extra[name] = {"beam_samples_per_s": b2.B * b2.C * b2.T / (np.median(r["step_ms"]) / 1e3),
                           "ms_per_step": float(np.median(r["step_ms"])), "contraction_kernel_ms": kms,
                           "reorder_kernel_ms": float(np.mean(r["reorder_ms"])),
                           "weights_kernel_ms": float(np.mean(r["weights_ms"])),
                           "mfma_TFLOPs": fp2.flops / (kms / 1e3) / 1e12,
                           "mfma_frac": fp2.flops / (kms / 1e3) / 1e12 / PEAK["f16_TFLOPs"]}
            if mp:
                extra[name]["mfma_frac_of_measured_peak"] = extra[name]["mfma_TFLOPs"] / mp["f16_TFLOPs"]
            log("precision %s: %s" % (name, extra[name]))
        if not a.no_cpu:
            extra["errors_vs_oracle"] = precision_errors(lbf, torch, b2, x2, geo2)
            log("precision errors: %s" % extra["errors_vs_oracle"])
        del b2.x

        # ---------------- uneven batch and streaming service ----------------
        jobs = make_jobs(lbf, torch, synth, dev)
        batch_res = batched(lbf, torch, jobs, max(3, a.steps // 4), 1)
        log("batched: %.3f ms per batch, %.3g beam-samples/s, %.2f of roofline, %.2fx sequential"
            % (batch_res["ms_per_batch"], batch_res["beam_samples_per_s"], batch_res["roofline_frac"],
               batch_res["batch_vs_sequential"]))
        log("batched, per job alone (ms): %s" % ["%.3f" % jb["ms_alone"] for jb in batch_res["jobs"]])
        serve_res = serving(lbf, torch, synth, jobs, blk, x, b2, x2, a.serve_seconds, a.serve_warmup)
        log("serving: %s" % serve_res["open_loop"])
        log("serving closed loop: %s" % serve_res["closed_loop"])
        del jobs, x2

    # ---------------- the JSON line ----------------
    main_name = "f32" if "f32" in res else sorted(res)[0]
    r = res[main_name]
    ms = float(np.median(r["step_ms"]))
    kms = float(np.mean(r["beamform_ms"]))
    flops = fp.flops
    achieved = flops / (kms / 1e3) / 1e12
    alg_bytes = fp.input_bytes + fp.weight_bytes + fp.output_bytes
    line = {
        "metric": "tied-array beam-samples/s, FP16-MFMA vs FP32 at <=3e-3 rel err; p99 block latency",
        "value": bsamp / (ms / 1e3),
        "unit": "beam-samples/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_name == "f32" else main_name,
        "data": "synthetic (seeded Gaussian noise + plane-wave tones), resident in HBM",
        "config": {"workload": "one-second block: 64 stations, 32 subbands x 256 channels, 768 samples, complex "
                               "int16, 128 beams, Stokes IQUV integrated x16, beam-major f32 out",
                   "S": S, "C": C, "T": T, "B": B, "xtype": "ci16", "product": "IQUV", "t_int": t_int,
                   "f_int": f_int,
                   "step": "lbf_compute_weights + lbf_beamform_channel_major (fused contraction, Stokes, "
                           "integration) + lbf_beam_major (final order)"},
        "p50_step_ms": float(np.percentile(r["step_ms"], 50)),
        "p99_step_ms": float(np.percentile(r["step_ms"], 99)),
        "input_Gbps_equiv": fp.input_bytes * 8 / (ms / 1e3) / 1e9,
        "realtime_factor": block_seconds / (ms / 1e3),
        "TFLOPs": flops / (ms / 1e3) / 1e12,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32_TFLOPs"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["f32_TFLOPs"],
                     "traffic": measured_traffic() if main_name == "f32" else None,
                     "kernel": "bf_f32_fast_kernel<ci16, IQUV, t_int 16>", "kernel_ms": kms,
                     "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_sources": kernel_source_hash()},
        "measured_peaks": mp,
        "cpu_baseline": cpu,
    }
    paths = {}
    for name, rr in res.items():
        m = float(np.median(rr["step_ms"]))
        k = float(np.mean(rr["beamform_ms"]))
        ro = float(np.mean(rr["reorder_ms"]))
        ent = {"beam_samples_per_s": bsamp / (m / 1e3), "ms_per_step": m, "contraction_kernel_ms": k,
               "weights_kernel_ms": float(np.mean(rr["weights_ms"])), "reorder_kernel_ms": ro,
               "reorder_hbm_GBps": 2 * fp.output_bytes / (ro / 1e3) / 1e9,
               "p99_step_ms": float(np.percentile(rr["step_ms"], 99)),
               "err_vs_oracle": errs.get(name)}
        if name != "f32":
            fpn = lbf.block_footprint(S, C, T, B, lbf.CI16, lbf.F16, prod, t_int, f_int)
            byts = fpn.input_bytes + fpn.weight_bytes + fpn.output_bytes
            ent["hbm_GBps"] = byts / (k / 1e3) / 1e9
            ent["hbm_frac"] = ent["hbm_GBps"] / PEAK["hbm_GBps"]
            if mp:
                ent["hbm_frac_of_measured_hbm"] = ent["hbm_GBps"] / max(mp["hbm_GBps"], mp["hbm_read_GBps"])
            ent["bound"] = "hbm"
        paths[name] = ent
    line["paths"] = paths
    if mp:
        line["roofline"]["frac_of_measured_peak"] = achieved / mp["f32_TFLOPs"]
    if "f16" in paths and "f32" in paths:
        line["fp16_mfma_vs_fp32_speedup"] = paths["f16"]["beam_samples_per_s"] / paths["f32"]["beam_samples_per_s"]
    if extra:
        line["precision_block"] = extra
    if unfused_res:
        line["unfused_chain"] = unfused_res
    if inc_res:
        line["incoherent_beam"] = inc_res
    if dd_res:
        line["dedispersion"] = dd_res
    if pc_res:
        line["pulsar_chain_case_E"] = pc_res
    if ch_res:
        line["channeliser"] = ch_res
    if ss_res:
        line["superstation"] = ss_res
    if batch_res:
        line["batched"] = batch_res
    if serve_res:
        line["serving"] = serve_res
        line["p50_block_latency_ms"] = serve_res["open_loop"]["p50_block_latency_ms"]
        line["p99_block_latency_ms"] = serve_res["open_loop"]["p99_block_latency_ms"]
    line["context"] = "paper: 198 Gb/s station input sustained on one Blue Gene/P rack (Sections 1, 5)"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
