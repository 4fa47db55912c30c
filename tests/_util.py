"""Shared helpers of the GPU tests (marshalling and error metrics only)."""
import math

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


def max_err_over_rms(got, ref):
    """max |got - ref| / rms(ref) over an array (rms 0: the plain max)."""
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    ref = np.asarray(ref)
    rms = math.sqrt(float(np.mean(np.abs(ref) ** 2))) if ref.size else 0.0
    m = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    return m / rms if rms > 0 else m


def check_close(got, ref, tol, label, elem_factor=10.0):
    """Norm-wise relative L2 error <= tol over the whole array, and for every
    index of the first axis (a beam) the element-wise bound
    max |got - ref| <= elem_factor * tol * rms(ref), so that a few wrong
    elements cannot hide inside a small norm-wise error."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, "%s: shape %s != %s" % (label, got.shape, ref.shape)
    e = relerr(got, ref)
    assert e <= tol, "%s: rel err %.3g > %.1g" % (label, e, tol)
    if ref.ndim == 0:
        return
    for b in range(ref.shape[0]):
        m = max_err_over_rms(got[b], ref[b])
        assert m <= elem_factor * tol, "%s: index %d: max|g-o|/rms(o) %.3g > %.3g" % (label, b, m,
                                                                                       elem_factor * tol)


def check_stokes(got, ref, tol, label, scale="own", elem_factor=10.0):
    """Stokes arrays [B][K][T'][C']: per parameter, the norm-wise relative L2
    error <= tol, and per (beam, parameter) max |g - o| <= elem_factor * tol *
    rms(o).  scale="I" measures Q, U and V against Stokes I of the same beam
    (for data whose Q, U or V vanish, where their own norm is rounding noise)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, "%s: shape %s != %s" % (label, got.shape, ref.shape)
    K = ref.shape[1]
    for k in range(K):
        den = ref[:, 0] if scale == "I" else ref[:, k]
        nd = np.linalg.norm(den.ravel())
        e = np.linalg.norm((got[:, k] - ref[:, k]).ravel()) / nd if nd > 0 else np.abs(got[:, k] - ref[:, k]).max()
        assert e <= tol, "%s: Stokes %s rel err %.3g > %.1g" % (label, "IQUV"[k], e, tol)
        for b in range(ref.shape[0]):
            rms = math.sqrt(float(np.mean(den[b] ** 2)))
            m = float(np.max(np.abs(got[b, k] - ref[b, k])))
            bound = elem_factor * tol * rms
            assert m <= bound or (rms == 0 and m == 0), \
                "%s: beam %d Stokes %s max|g-o| %.3g > %.3g (rms %.3g)" % (label, b, "IQUV"[k], m, bound, rms)


# unit roundoff of the contraction's operand types (lbf.F32, F16, BF16)
UNIT_ROUNDOFF = {0: 2.0 ** -24, 1: 2.0 ** -11, 2: 2.0 ** -8}


def contraction_eps(ctype, S, samples_exact=True, extra=0.0):
    """Relative bound of one beam sample's error against sum_s |w_s x_s|:
    weights rounded once to the operand type (unit roundoff u), samples exact
    (integers in range) or rounded once too, S products accumulated in FP32
    in any order, plus ``extra`` (an error already in the samples)."""
    u = UNIT_ROUNDOFF[ctype]
    ux = 0.0 if samples_exact else u
    return u + ux + u * ux + S * 2.0 ** -23 + extra


def stokes_bound(y, err, K, t_int, f_int):
    """Element-wise error bound [B][K][T'][C'] of fused Stokes products from
    the oracle's voltages y [C][B][T][2] (complex) and a bound err [C][T][2]
    on every beam sample's error (the weights have modulus 1, so with
    operand rounding alone it is eps * sum_s |x_s|): the first-order
    propagation of those errors into |X|^2 +- |Y|^2 and 2 X conj(Y), their
    FP32 rounding, and the FP32 sums over the t_int x f_int group."""
    e = err[:, None]                                              # [C][1][T][2]
    ax, ay = np.abs(y[..., 0]), np.abs(y[..., 1])
    ex, ey = e[..., 0], e[..., 1]
    n = t_int * f_int + 8
    bI = 2 * ax * ex + ex * ex + 2 * ay * ey + ey * ey + n * 2.0 ** -24 * (ax * ax + ay * ay)
    bU = 2 * (ax * ey + ay * ex + ex * ey) + n * 2.0 ** -23 * ax * ay
    C, B, T = y.shape[:3]
    parts = [bI] if K == 1 else [bI, bI, bU, bU]
    out = []
    for b in parts:
        g = b.reshape(C // f_int, f_int, B, T // t_int, t_int).sum(axis=(1, 4))    # [C'][B][T']
        out.append(g.transpose(1, 2, 0))                                              # [B][T'][C']
    return np.stack(out, axis=1)                                                      # [B][K][T'][C']


def check_stokes_bound(got, ref, bound, label, slack=2.0):
    """Every element within slack x its derived rounding bound."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    worst = float(np.max(err / (slack * bound + 1e-30)))
    assert worst <= 1.0, "%s: an element exceeds %g x its rounding bound by %.3g" % (label, slack, worst)


def stokes_errors(got, ref):
    """(norm-wise relative L2, max |g - o| / rms(o)) per Stokes parameter,
    for reports: lists of K floats each."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return ([relerr(got[:, k], ref[:, k]) for k in range(ref.shape[1])],
            [max_err_over_rms(got[:, k], ref[:, k]) for k in range(ref.shape[1])])


def cplx(t):
    """[..., 2] float tensor/array -> complex128 numpy."""
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    a = a.astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def flush(msg):
    print(msg, flush=True)
