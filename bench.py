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
    p.add_argument("--copy-calibration", action="store_true",
                   help="counter calibration run: three plain 1 GiB device-to-device copies (no JSON line)")
    return p.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def relerr(g, o):
    g = np.asarray(g, dtype=np.float64)
    return float(np.linalg.norm((g - o).ravel()) / max(np.linalg.norm(o.ravel()), 1e-300))


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


KERNEL_SOURCES = ["lbf_device.h", "bf_common.h", "bf_workers.h", "bf_fast_impl.h", "bf_fast_f32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_one_second_fp32.txt")


def kernel_source_hash():
    """sha256 over the sources of the FP32 contraction kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1105_0661_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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

    # ---------------- oracle on sampled subbands (CPU baseline + errors) ----------------
    cpu = None
    errs = {}
    if not a.no_cpu:
        from oracle import oracle as orc
        ncpu = min(os.cpu_count() or 1, 16)
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
               "kind": "oracle",
               "sample": "%d of %d subbands (%d channels x %d beams x %d samples, all 64 stations), FP64 C oracle "
                         "with %d threads, %.1f s" % (sb, blk.nsb, len(chans), B, T, ncpu, cpu_s)}
        idx = torch.from_numpy(chans).to(dev)
        for name, r in res.items():
            got = r["out"][:, :, :, idx].cpu().numpy()
            errs[name] = {k: relerr(got[:, i], ref[:, i]) for i, k in enumerate("IQUV")}
        log("cpu baseline: %s" % cpu)

    # ---------------- the 488-beam precision block (MFMA-bound) ----------------
    extra = None
    if not a.no_extra and not only:
        del x
        torch.cuda.empty_cache()
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
            log("precision %s: %s" % (name, extra[name]))
        del x2

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
        "p50_block_latency_ms": float(np.percentile(r["step_ms"], 50)),
        "p99_block_latency_ms": float(np.percentile(r["step_ms"], 99)),
        "input_Gbps_equiv": fp.input_bytes * 8 / (ms / 1e3) / 1e9,
        "realtime_factor": block_seconds / (ms / 1e3),
        "TFLOPs": flops / (ms / 1e3) / 1e12,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["f32_TFLOPs"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["f32_TFLOPs"],
                     "traffic": measured_traffic() if main_name == "f32" else None,
                     "kernel": "bf_f32_fast_kernel<ci16, IQUV, t_int 16>", "kernel_ms": kms,
                     "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_sources": kernel_source_hash()},
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
               "p99_block_latency_ms": float(np.percentile(rr["step_ms"], 99)),
               "rel_err_vs_oracle": errs.get(name)}
        if name != "f32":
            fpn = lbf.block_footprint(S, C, T, B, lbf.CI16, lbf.F16, prod, t_int, f_int)
            byts = fpn.input_bytes + fpn.weight_bytes + fpn.output_bytes
            ent["hbm_GBps"] = byts / (k / 1e3) / 1e9
            ent["hbm_frac"] = ent["hbm_GBps"] / PEAK["hbm_GBps"]
            ent["bound"] = "hbm"
        paths[name] = ent
    line["paths"] = paths
    if "f16" in paths and "f32" in paths:
        line["fp16_mfma_vs_fp32_speedup"] = paths["f16"]["beam_samples_per_s"] / paths["f32"]["beam_samples_per_s"]
    if extra:
        line["precision_block"] = extra
    line["context"] = "paper: 198 Gb/s station input sustained on one Blue Gene/P rack (Sections 1, 5)"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
