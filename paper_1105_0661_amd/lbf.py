"""Python binding of liblbf (ctypes).  Argument marshalling only: every step of
the beam former runs in the HIP kernels of liblbf.so; torch provides device
memory and streams.  If the library has not been built, importing works but
every call raises ``LbfUnavailable`` -- there is no fallback.

Names mirror include/lbf.h (``lbf_beamform`` -> ``beamform`` ...).
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbf.so")

# enums (include/lbf.h)
OK, E_INVAL, E_UNSUPPORTED, E_NOMEM, E_HIP, E_BUSY, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
CI8, CI16, CF32 = 0, 1, 2
F32, F16, BF16 = 0, 1, 2
VOLTAGES, STOKES_I, STOKES_IQUV = 0, 1, 4
MAX_BATCH = 32
JOB_QUEUED, JOB_ADMITTED, JOB_RUNNING, JOB_DONE, JOB_FAILED = range(5)
XTYPE_NAMES = {"ci8": CI8, "ci16": CI16, "cf32": CF32}
CTYPE_NAMES = {"f32": F32, "f16": F16, "bf16": BF16}
PRODUCT_NAMES = {"voltages": VOLTAGES, "I": STOKES_I, "IQUV": STOKES_IQUV}


class LbfUnavailable(RuntimeError):
    pass


class LbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("lbf error %d: %s" % (code, msg))
        self.code = code


class Block(ctypes.Structure):
    _fields_ = [("d_x", ctypes.c_void_p), ("xtype", ctypes.c_int), ("S", ctypes.c_int), ("C", ctypes.c_int),
                ("T", ctypes.c_int), ("d_w", ctypes.c_void_p), ("ctype", ctypes.c_int), ("B", ctypes.c_int),
                ("product", ctypes.c_int), ("t_int", ctypes.c_int), ("f_int", ctypes.c_int),
                ("d_out", ctypes.c_void_p)]


class BlockSizes(ctypes.Structure):
    _fields_ = [("input_bytes", ctypes.c_uint64), ("weight_bytes", ctypes.c_uint64),
                ("output_bytes", ctypes.c_uint64), ("flops", ctypes.c_double),
                ("staging_bytes", ctypes.c_uint64), ("staging_channel_bytes", ctypes.c_uint64)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("d_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int),
                ("n_streams", ctypes.c_int), ("queue_capacity", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("device", ctypes.c_int), ("staging_cap", ctypes.c_uint64)]


class Job(ctypes.Structure):
    _fields_ = [("obs_id", ctypes.c_uint64),
                ("station_xyz", ctypes.c_void_p), ("S", ctypes.c_int),
                ("beam_dir", ctypes.c_void_p), ("B", ctypes.c_int),
                ("ref_dir", ctypes.c_void_p), ("station_delay", ctypes.c_void_p),
                ("freq_hz", ctypes.c_void_p), ("C", ctypes.c_int),
                ("x", ctypes.c_void_p), ("xtype", ctypes.c_int), ("T", ctypes.c_int),
                ("x_on_host", ctypes.c_int),
                ("ctype", ctypes.c_int), ("product", ctypes.c_int), ("t_int", ctypes.c_int), ("f_int", ctypes.c_int),
                ("d_out", ctypes.c_void_p), ("stream_id", ctypes.c_uint64)]


class JobStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("error", ctypes.c_int), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("batch_size", ctypes.c_int), ("periods", ctypes.c_int)]


_lock = threading.Lock()
_lib = None

_PROTOS = {
    "lbf_last_error": (ctypes.c_char_p, []),
    "lbf_version": (ctypes.c_char_p, []),
    "lbf_compute_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_beamform": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_void_p]),
    "lbf_beamform_channel_major": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_void_p]),
    "lbf_beamform_noalloc": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_void_p]),
    "lbf_beamform_incoherent": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_beam_major": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_beamform_batch": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_int, ctypes.c_void_p]),
    "lbf_stokes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_transpose": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_incoherent": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_superstation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_channelize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_dedisperse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbf_dedisperse_stokes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "lbf_block_footprint": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.POINTER(BlockSizes)]),
    "lbf_set_tile_streams": (ctypes.c_int, [ctypes.c_int]),
    "lbf_check_addressing": (ctypes.c_int, [ctypes.POINTER(Block), ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "lbf_probe": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "lbf_server_create": (ctypes.c_int, [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]),
    "lbf_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]),
    "lbf_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(JobStatus)]),
    "lbf_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(JobStatus)]),
    "lbf_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "lbf_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}


def lib():
    """The loaded liblbf.so; raises LbfUnavailable if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise LbfUnavailable("liblbf.so is not built (%s); run `python -m paper_1105_0661_amd.build`"
                                     % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _PROTOS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LbfError(rc, lib().lbf_last_error().decode())


def version() -> str:
    return lib().lbf_version().decode()


# --------------------------------------------------------------------------
# torch marshalling helpers
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def xtype_of(x) -> int:
    torch = _torch()
    m = {torch.int8: CI8, torch.int16: CI16, torch.float32: CF32}
    if x.dtype not in m:
        raise TypeError("station samples must be int8, int16 or float32 (got %s)" % x.dtype)
    return m[x.dtype]


def ctype_of(w) -> int:
    torch = _torch()
    m = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
    if w.dtype not in m:
        raise TypeError("weights must be float32, float16 or bfloat16 pairs (got %s)" % w.dtype)
    return m[w.dtype]


def weight_dtype(ctype: int):
    torch = _torch()
    return {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[ctype]


def n_stokes(product: int) -> int:
    return {STOKES_I: 1, STOKES_IQUV: 4}[product]


def output_shape(product: int, S: int, C: int, T: int, B: int, t_int: int = 1, f_int: int = 1,
                 channel_major: bool = False):
    if product == VOLTAGES:
        return (C, B, T, 2, 2)
    if channel_major:
        return (C // f_int, T // t_int, B, n_stokes(product))
    return (B, n_stokes(product), T // t_int, C // f_int)


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------

def compute_weights(station_xyz, beam_dir, freq_hz, wtype: int = F32, ref_dir=None, out=None, tau=None,
                    station_delay=None, stream=None):
    """w[C][B][S] (complex as a trailing pair axis) from device f64 geometry;
    ``station_delay``: device f64 [S] residual delays in seconds, or None."""
    torch = _torch()
    S, B, C = station_xyz.shape[0], beam_dir.shape[0], freq_hz.shape[0]
    if out is None:
        out = torch.empty((C, B, S, 2), dtype=weight_dtype(wtype), device=station_xyz.device)
    ref = None
    if ref_dir is not None:
        ref = (ctypes.c_double * 3)(*[float(v) for v in ref_dir])
    if station_delay is not None and (station_delay.dtype != torch.float64 or tuple(station_delay.shape) != (S,)):
        raise ValueError("station_delay must be a float64 tensor of shape (S,)")
    _check(lib().lbf_compute_weights(_dev_ptr(station_xyz, "station_xyz"), S, _dev_ptr(beam_dir, "beam_dir"), B,
                                     ref, _dev_ptr(station_delay, "station_delay"), _dev_ptr(freq_hz, "freq_hz"), C,
                                     wtype, _dev_ptr(out, "out"), _dev_ptr(tau, "tau"), _stream(stream)))
    return out


def make_block(x, w, product: int, t_int: int = 1, f_int: int = 1, out=None) -> Block:
    S, C, T = x.shape[0], x.shape[1], x.shape[2]
    B = w.shape[1]
    return Block(d_x=_dev_ptr(x, "x"), xtype=xtype_of(x), S=S, C=C, T=T, d_w=_dev_ptr(w, "w"),
                 ctype=ctype_of(w), B=B, product=product, t_int=t_int, f_int=f_int,
                 d_out=_dev_ptr(out, "out") if out is not None else None)


def beamform(x, w, product: int, t_int: int = 1, f_int: int = 1, out=None, stream=None):
    """x [S][C][T][2][2] (int8/int16/float32), w [C][B][S][2] -> voltages
    [C][B][T][2][2] f32, or Stokes [B][K][T'][C'] f32."""
    torch = _torch()
    S, C, T = x.shape[0], x.shape[1], x.shape[2]
    B = w.shape[1]
    if out is None:
        out = torch.empty(output_shape(product, S, C, T, B, t_int, f_int), dtype=torch.float32, device=x.device)
    blk = make_block(x, w, product, t_int, f_int, out)
    _check(lib().lbf_beamform(ctypes.byref(blk), _stream(stream)))
    return out


def beamform_incoherent(x, w, product: int, t_int: int = 1, f_int: int = 1, out=None, inc=None, stream=None):
    """``beamform`` and the incoherent beam [K][T'][C'] of the same block
    (one read of the samples on the FP16/BF16 fast path): (out, inc)."""
    torch = _torch()
    S, C, T = x.shape[0], x.shape[1], x.shape[2]
    B = w.shape[1]
    if out is None:
        out = torch.empty(output_shape(product, S, C, T, B, t_int, f_int), dtype=torch.float32, device=x.device)
    if inc is None:
        K = n_stokes(product) if product in (STOKES_I, STOKES_IQUV) else 1   # voltages: refused by the library
        inc = torch.empty((K, T // t_int, C // f_int), dtype=torch.float32, device=x.device)
    blk = make_block(x, w, product, t_int, f_int, out)
    _check(lib().lbf_beamform_incoherent(ctypes.byref(blk), _dev_ptr(inc, "inc"), _stream(stream)))
    return out, inc


def beamform_noalloc(x, w, product: int, t_int: int = 1, f_int: int = 1, out=None, stream=None):
    """``beamform`` through lbf_beamform_noalloc: the library allocates
    nothing (pass ``out`` to allocate nothing here either)."""
    torch = _torch()
    S, C, T = x.shape[0], x.shape[1], x.shape[2]
    B = w.shape[1]
    if out is None:
        out = torch.empty(output_shape(product, S, C, T, B, t_int, f_int), dtype=torch.float32, device=x.device)
    blk = make_block(x, w, product, t_int, f_int, out)
    _check(lib().lbf_beamform_noalloc(ctypes.byref(blk), _stream(stream)))
    return out


def beamform_channel_major(x, w, product: int, t_int: int = 1, f_int: int = 1, out=None, stream=None):
    """As ``beamform`` but Stokes stay channel-major: [C'][T'][B][K] f32."""
    torch = _torch()
    S, C, T = x.shape[0], x.shape[1], x.shape[2]
    B = w.shape[1]
    if out is None:
        out = torch.empty(output_shape(product, S, C, T, B, t_int, f_int, channel_major=True), dtype=torch.float32,
                          device=x.device)
    blk = make_block(x, w, product, t_int, f_int, out)
    _check(lib().lbf_beamform_channel_major(ctypes.byref(blk), _stream(stream)))
    return out


def beam_major(inp, out=None, stream=None):
    """[C2][T2][B][K] f32 -> [B][K][T2][C2] (final order)."""
    torch = _torch()
    C2, T2, B, K = inp.shape
    if out is None:
        out = torch.empty((B, K, T2, C2), dtype=torch.float32, device=inp.device)
    _check(lib().lbf_beam_major(_dev_ptr(inp, "inp"), C2, K, T2, B, _dev_ptr(out, "out"), _stream(stream)))
    return out


def beamform_batch(items: Sequence[tuple], stream=None) -> List:
    """items: (x, w, product, t_int, f_int[, out]) tuples -> list of outputs."""
    torch = _torch()
    n = len(items)
    arr = (Block * max(n, 1))()
    outs = []
    for i, it in enumerate(items):
        x, w, product, t_int, f_int = it[:5]
        out = it[5] if len(it) > 5 else None
        if out is None:
            S, C, T = x.shape[:3]
            out = torch.empty(output_shape(product, S, C, T, w.shape[1], t_int, f_int), dtype=torch.float32,
                              device=x.device)
        outs.append(out)
        arr[i] = make_block(x, w, product, t_int, f_int, out)
    _check(lib().lbf_beamform_batch(arr, n, _stream(stream)))
    return outs


def stokes(y, product: int, t_int: int = 1, f_int: int = 1, out=None, stream=None):
    """y [C][B][T][2][2] f32 -> s [C'][B][T'][K] f32 (unfused path)."""
    torch = _torch()
    C, B, T = y.shape[:3]
    if out is None:
        out = torch.empty((C // f_int, B, T // t_int, n_stokes(product)), dtype=torch.float32, device=y.device)
    _check(lib().lbf_stokes(_dev_ptr(y, "y"), B, C, T, product, t_int, f_int, _dev_ptr(out, "out"),
                            _stream(stream)))
    return out


def transpose(inp, out=None, stream=None):
    """[C2][B][T2][K] f32 -> [B][K][T2][C2]; a trailing pair axis of 2 means complex elements."""
    torch = _torch()
    if inp.dim() == 5:
        C2, B, T2, K, _ = inp.shape
        elem, shape = 8, (B, K, T2, C2, 2)
    else:
        C2, B, T2, K = inp.shape
        elem, shape = 4, (B, K, T2, C2)
    if out is None:
        out = torch.empty(shape, dtype=inp.dtype, device=inp.device)
    _check(lib().lbf_transpose(_dev_ptr(inp, "inp"), C2, B, T2, K, elem, _dev_ptr(out, "out"), _stream(stream)))
    return out


def incoherent(x, product: int, t_int: int = 1, f_int: int = 1, out=None, stream=None):
    """Incoherent beam [K][T'][C'] f32 of x [S][C][T][2][2]."""
    torch = _torch()
    S, C, T = x.shape[:3]
    if out is None:
        out = torch.empty((n_stokes(product), T // t_int, C // f_int), dtype=torch.float32, device=x.device)
    _check(lib().lbf_incoherent(_dev_ptr(x, "x"), xtype_of(x), S, C, T, product, t_int, f_int,
                                _dev_ptr(out, "out"), _stream(stream)))
    return out


def superstation(x, groups, w=None, out=None, stream=None):
    """Superstations [G][C][T][2][2] f32 from stations x [S][C][T][2][2]:
    group g sums its member stations ``groups[g]`` (a list of station
    indices), each weighted by w [C][S][2] f32 (None: unit weights)."""
    torch = _torch()
    S, C, T = x.shape[:3]
    G = len(groups)
    offs = [0]
    for members in groups:
        offs.append(offs[-1] + len(members))
    off_arr = (ctypes.c_int * (G + 1))(*offs)
    flat = [int(s) for members in groups for s in members]
    mem_arr = (ctypes.c_int * max(1, len(flat)))(*flat)
    if w is not None and tuple(w.shape) != (C, S, 2):
        raise ValueError("w must be [C][S][2]")
    if out is None:
        out = torch.empty((G, C, T, 2, 2), dtype=torch.float32, device=x.device)
    _check(lib().lbf_superstation(_dev_ptr(x, "x"), xtype_of(x), S, C, T, _dev_ptr(w, "w"), G, off_arr, mem_arr,
                                  _dev_ptr(out, "out"), _stream(stream)))
    return out


def channelize(x, nch: int, t_sb: int = None, shift=None, out=None, stream=None):
    """Subband samples x [S][NSB][T_in][2][2] (int8/int16/float32) -> channels
    [S][NSB nch][t_sb / nch][2][2] f32, lowest frequency first.  ``shift``: a
    device int32 tensor [S] of per-station sample shifts (station s uses row
    samples shift[s] .. shift[s] + t_sb - 1, zeros outside the row)."""
    torch = _torch()
    S, NSB, Tin = x.shape[:3]
    Tsb = Tin if t_sb is None else t_sb
    if shift is not None and (shift.dtype != torch.int32 or tuple(shift.shape) != (S,)):
        raise ValueError("shift must be an int32 tensor of shape (S,)")
    if out is None:
        out = torch.empty((S, NSB * nch, Tsb // nch, 2, 2), dtype=torch.float32, device=x.device)
    _check(lib().lbf_channelize(_dev_ptr(x, "x"), xtype_of(x), S, NSB, Tin, Tsb, nch, _dev_ptr(shift, "shift"),
                                _dev_ptr(out, "out"), _stream(stream)))
    return out


def dedisperse(y, chirp, n_fft: int = 4096, out=None, stream=None):
    """Channel-level dedispersion of voltages y [C][B][T][2][2] f32 with chirp
    weights [C][n_fft][2] f32; returns [C][B][T][2][2] f32 (``out`` may be y)."""
    torch = _torch()
    C, B, T = y.shape[:3]
    if out is None:
        out = torch.empty_like(y)
    _check(lib().lbf_dedisperse(_dev_ptr(y, "y"), C, B, T, n_fft, _dev_ptr(chirp, "chirp"), _dev_ptr(out, "out"),
                                _stream(stream)))
    return out


def dedisperse_stokes(y, chirp, n_fft: int, product: int, t_int: int, out=None, stream=None):
    """Dedispersion then Stokes and integration of voltages y [C][B][T][2][2]
    f32 with chirp weights [C][n_fft][2] f32: [C][B][T/t_int][K] f32."""
    torch = _torch()
    C, B, T = y.shape[:3]
    if out is None:
        out = torch.empty((C, B, T // t_int, n_stokes(product)), dtype=torch.float32, device=y.device)
    _check(lib().lbf_dedisperse_stokes(_dev_ptr(y, "y"), C, B, T, n_fft, _dev_ptr(chirp, "chirp"), product, t_int,
                                       _dev_ptr(out, "out"), _stream(stream)))
    return out


def set_tile_streams(streams: int):
    """lbf_set_tile_streams: force 1, 2 or 4 sample streams per FP16/BF16
    work item (0: the measured table).  A tuning hook; results do not change."""
    _check(lib().lbf_set_tile_streams(streams))


def block_footprint(S: int, C: int, T: int, B: int, xtype: int, ctype: int, product: int, t_int: int = 1,
                    f_int: int = 1) -> BlockSizes:
    blk = Block(d_x=None, xtype=xtype, S=S, C=C, T=T, d_w=None, ctype=ctype, B=B, product=product, t_int=t_int,
                f_int=f_int, d_out=None)
    out = BlockSizes()
    _check(lib().lbf_block_footprint(ctypes.byref(blk), ctypes.byref(out)))
    return out


def check_addressing(S: int, C: int, T: int, B: int, xtype: int, ctype: int, product: int, t_int: int = 1,
                     f_int: int = 1, channel_major: bool = False, staging_cap: int = 0, threads: int = 8) -> int:
    """lbf_check_addressing on a block of these sizes (host only): raises
    LbfError on a bad access, returns the number of accesses walked."""
    blk = Block(d_x=1, xtype=xtype, S=S, C=C, T=T, d_w=1, ctype=ctype, B=B, product=product, t_int=t_int,
                f_int=f_int, d_out=1)
    n = ctypes.c_uint64()
    _check(lib().lbf_check_addressing(ctypes.byref(blk), int(channel_major), staging_cap, threads, ctypes.byref(n)))
    return n.value


# --------------------------------------------------------------------------
# streaming server
# --------------------------------------------------------------------------

PROBE_MFMA_F16, PROBE_MFMA_F32, PROBE_COPY, PROBE_READ = 0, 1, 2, 3


def probe(kind: int, iters: int = 1, src=None, dst=None, stream=None) -> float:
    """lbf_probe: launch one peak probe on the stream; returns its work (flop,
    or bytes moved for the copy).  The caller times it."""
    work = ctypes.c_double()
    nbytes = 0 if src is None else src.numel() * src.element_size()
    _check(lib().lbf_probe(kind, iters, _dev_ptr(src, "src"), _dev_ptr(dst, "dst"), nbytes, ctypes.byref(work),
                           _stream(stream)))
    return work.value


class Server:
    """lbf_server_* over a caller-owned device arena (a torch uint8 tensor).

    ``submit`` copies the geometry; station samples (device tensor, or host
    array / CPU tensor staged through the arena) and the output tensor are kept
    referenced here until the ticket is released."""

    def __init__(self, arena, max_inflight: int = 8, n_streams: int = 2, queue_capacity: int = 64,
                 max_batch: int = 8, device: int = 0, staging_cap: int = 0):
        self.arena = arena
        cfg = ServerCfg(d_arena=_dev_ptr(arena, "arena"), arena_bytes=arena.numel() * arena.element_size(),
                        max_inflight=max_inflight, n_streams=n_streams, queue_capacity=queue_capacity,
                        max_batch=max_batch, device=device, staging_cap=staging_cap)
        h = ctypes.c_void_p()
        _check(lib().lbf_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}      # ticket -> (samples, output tensor, stream block?) kept alive until release

    def submit(self, obs_id: int, station_xyz, beam_dir, freq_hz, x, ctype: int, product: int, t_int: int = 1,
               f_int: int = 1, out=None, ref_dir=None, stream_id: int = 0, station_delay=None) -> int:
        """Queue one block.  With a non-zero ``stream_id`` the block continues
        that stream in time and its output holds (carried + T) // t_int
        periods, carried being the samples the server kept from the stream's
        earlier blocks; the output buffer made here has room for the most a
        block can complete, (t_int - 1 + T) // t_int, and ``output`` views the
        periods the server reports for the ticket."""
        import numpy as np
        torch = _torch()
        pos = np.ascontiguousarray(station_xyz, dtype=np.float64)
        dirs = np.ascontiguousarray(beam_dir, dtype=np.float64)
        freq = np.ascontiguousarray(freq_hz, dtype=np.float64)
        ref = None if ref_dir is None else (ctypes.c_double * 3)(*[float(v) for v in ref_dir])
        delay = None if station_delay is None else np.ascontiguousarray(station_delay, dtype=np.float64)
        if isinstance(x, np.ndarray):
            x = torch.from_numpy(np.ascontiguousarray(x))
        on_host = not x.is_cuda
        if not x.is_contiguous():
            raise ValueError("x must be contiguous")
        S, C, T = x.shape[:3]
        B = dirs.shape[0]
        if pos.shape != (S, 3) or dirs.shape != (B, 3) or freq.shape != (C,):
            raise ValueError("geometry shapes %s %s %s do not match samples [S=%d][C=%d]"
                             % (pos.shape, dirs.shape, freq.shape, S, C))
        if delay is not None and delay.shape != (S,):
            raise ValueError("station_delay must hold one delay per station")
        Tq = (t_int - 1 + T) // t_int * t_int if stream_id else T
        if out is None:
            # a block that completes no period still gets a one-period buffer (never written)
            out = torch.empty(output_shape(product, S, C, max(Tq, t_int), B, t_int, f_int), dtype=torch.float32,
                              device=self.arena.device)
        job = Job(obs_id=obs_id, station_xyz=pos.ctypes.data, S=S, beam_dir=dirs.ctypes.data, B=B,
                  ref_dir=ctypes.addressof(ref) if ref is not None else None,
                  station_delay=delay.ctypes.data if delay is not None else None,
                  freq_hz=freq.ctypes.data, C=C, x=x.data_ptr(), xtype=xtype_of(x), T=T, x_on_host=int(on_host),
                  ctype=ctype, product=product, t_int=t_int, f_int=f_int, d_out=_dev_ptr(out, "out"),
                  stream_id=stream_id)
        t = ctypes.c_uint64()
        _check(lib().lbf_server_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        self._keep[t.value] = (x, out, bool(stream_id))
        return t.value

    def output(self, ticket: int):
        """The ticket's output (call after ``wait``).  For a stream block, the
        [B][K][P][C'] view of the P periods the server wrote, P from the
        ticket's status (empty when the block completed none)."""
        x, out, is_stream = self._keep[ticket]
        if not is_stream:
            return out
        B, K, _, C2 = out.shape
        P = self.poll(ticket).periods
        return out.reshape(-1)[:B * K * P * C2].view(B, K, P, C2)

    def poll(self, ticket: int) -> JobStatus:
        st = JobStatus()
        _check(lib().lbf_server_poll(self._h, ticket, ctypes.byref(st)))
        return st

    def wait(self, ticket: int, timeout_ms: int = 60000) -> JobStatus:
        st = JobStatus()
        _check(lib().lbf_server_wait(self._h, ticket, timeout_ms, ctypes.byref(st)))
        return st

    def release(self, ticket: int):
        _check(lib().lbf_server_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def close(self):
        if self._h:
            _check(lib().lbf_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
