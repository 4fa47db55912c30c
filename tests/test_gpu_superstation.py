"""GPU parity of superstation beam forming (Sec. 4.2) through the C ABI
against the FP64 oracle: 1e-5 norm-wise relative L2 per (group, channel)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import lbf, synth
from tests._util import cplx, flush, geometry, relerr, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    return torch


def _stations(S, C, T, xtype, seed):
    rng = np.random.default_rng([1105, 661, 102, seed])
    if xtype == "cf32":
        return (rng.standard_normal((S, C, T, 2, 2)) * 40.0).astype(np.float32)
    lim = 127 if xtype == "ci8" else 3000
    return rng.integers(-lim, lim + 1, size=(S, C, T, 2, 2)).astype(np.int8 if xtype == "ci8" else np.int16)


def _weights(C, S, seed):
    rng = np.random.default_rng([1105, 661, 103, seed])
    ph = 2 * np.pi * rng.random((C, S))
    return np.stack([np.cos(ph), np.sin(ph)], axis=-1).astype(np.float32)       # [C][S][2]


# (S, C, T, xtype, groups): single members, a station in two groups, ragged
# T (not a multiple of the work group's samples); T a multiple of the
# samples per 16-byte vector (vector kernel) and not (one sample per thread)
CASES = [(6, 3, 300, "ci16", [[0, 1, 2], [3], [4, 5, 0]]), (9, 2, 64, "ci8", [[8, 7, 6, 5, 4, 3, 2, 1, 0]]),
         (4, 5, 513, "cf32", [[1, 3], [2], [0, 2]]), (5, 2, 301, "ci16", [[4, 0], [1, 2, 3]]),
         (3, 2, 66, "ci8", [[2, 1], [0]])]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "S%d_C%d_T%d_%s_G%d" % (c[0], c[1], c[2], c[3], len(c[4])))
def test_superstation_matches_oracle(case):
    torch = _torch()
    S, C, T, xt, groups = case
    x, w = _stations(S, C, T, xt, S), _weights(C, S, S)
    flush("superstation %s" % (case[:4],))
    out = lbf.superstation(to_dev(x), groups, to_dev(w))
    torch.cuda.synchronize()
    want = orc.superstation(x, cplx(w), groups)
    got = cplx(out)
    for g in range(len(groups)):
        for c in range(C):
            assert relerr(got[g, c], want[g, c]) <= TOL, (g, c)


def test_superstation_unit_weights_single_member_is_the_station():
    torch = _torch()
    x = _stations(3, 2, 100, "ci16", 5)
    out = lbf.superstation(to_dev(x), [[2], [0]])
    torch.cuda.synchronize()
    assert np.array_equal(out[0].cpu().numpy(), x[2].astype(np.float32))
    assert np.array_equal(out[1].cpu().numpy(), x[0].astype(np.float32))


def test_superstation_equals_the_beam_former_over_its_members():
    """Weights toward a direction (lbf_compute_weights with one beam): the
    superstation is the FP32 tied-array beam of its members."""
    torch = _torch()
    blk = synth.make_block(8, 2, 1, 16, 96, "ci16", 30.0, tag=(1105, 661, 104))
    pos, dirs, freq, ref = geometry(blk)
    w = lbf.compute_weights(pos, dirs, freq, lbf.F32, ref_dir=ref)        # [C][B][S][2]
    members = [1, 4, 6, 7]
    xd = to_dev(blk.x)
    flush("superstation vs beam former, 4 of 8 stations")
    ss = lbf.superstation(xd, [members], w[:, 0].contiguous())
    sub = xd[members].contiguous()
    bw = w[:, :1, members].contiguous()
    beam = lbf.beamform(sub, bw, lbf.VOLTAGES)                            # [C][1][T][2][2]
    torch.cuda.synchronize()
    got, want = cplx(ss[0]), cplx(beam[:, 0])
    for c in range(blk.C):
        assert relerr(got[c], want[c]) <= TOL, c


def test_superstation_one_second_block_sampled():
    """64 stations of the one-second block shape into 8 superstations of 8
    stations; sampled channels against the oracle."""
    torch = _torch()
    S, C, T = 64, 8192, 768
    gen = torch.Generator(device="cuda").manual_seed(1105662)
    x = torch.randint(-300, 301, (S, C, T, 2, 2), generator=gen, device="cuda", dtype=torch.int16)
    w = to_dev(_weights(C, S, 9))
    groups = [list(range(8 * g, 8 * g + 8)) for g in range(8)]
    flush("superstation one-second block: 64 -> 8 stations")
    out = lbf.superstation(x, groups, w)
    torch.cuda.synchronize()
    chans = np.random.default_rng(14).choice(C, 5, replace=False)
    idx = torch.from_numpy(chans).to("cuda")
    xs = x[:, idx].cpu().numpy()
    want = orc.superstation(xs, cplx(w[idx].cpu().numpy()), groups)
    got = cplx(out[:, idx])
    for g in range(8):
        for k in range(len(chans)):
            assert relerr(got[g, k], want[g, k]) <= TOL, (g, chans[k])
