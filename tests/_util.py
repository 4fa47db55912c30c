"""Shared helpers of the GPU tests (marshalling and error metrics only)."""
import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def geometry(blk, ref=True):
    """Device f64 geometry of a synthetic block, plus the host reference direction."""
    return (to_dev(blk.station_xyz), to_dev(blk.beam_dir), to_dev(blk.freq_hz),
            blk.ref_dir if ref else None)


def relerr(got, ref):
    """Norm-wise relative L2 error ||got - ref|| / ||ref||."""
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((got - ref).ravel())
    if den == 0:
        return num
    return num / den


def cplx(t):
    """[..., 2] float tensor/array -> complex128 numpy."""
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    a = a.astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def flush(msg):
    print(msg, flush=True)
