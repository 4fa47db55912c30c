"""GPU parity of channel-level dedispersion (Sec. 4.4) through the C ABI
against the FP64 oracle: 1e-5 norm-wise relative L2 per (channel, beam)
array (FP32 arithmetic), bit for bit where only the buffer differs."""
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


def _voltages(C, B, T, seed):
    """Seeded complex Gaussian voltages [C][B][T][2][2] f32 (re, im last)."""
    rng = np.random.default_rng([1105, 661, 90, seed])
    return (rng.standard_normal((C, B, T, 2, 2)) * 100.0).astype(np.float32)


def _chirp(C, n, seed):
    """Seeded unit-modulus weights with a quadratic phase in the bin index
    (a chirp) plus a random part, [C][n][2] f32."""
    rng = np.random.default_rng([1105, 661, 91, seed])
    k = np.arange(n)
    ph = np.pi * rng.random((C, 1)) * (k[None, :] - n / 2) ** 2 / n + 2 * np.pi * rng.random((C, n))
    return np.stack([np.cos(ph), np.sin(ph)], axis=-1).astype(np.float32)


def _oracle(y, h, n):
    return orc.dedisperse(cplx(y), cplx(h), n)


# (C, B, T, n_fft): every supported length, one and several blocks per series
CASES = [(3, 2, 24, 8), (2, 3, 192, 64), (2, 2, 1024, 512), (2, 2, 8192, 4096), (1, 1, 4096, 4096)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "C%d_B%d_T%d_n%d" % c)
def test_dedisperse_matches_oracle(case):
    torch = _torch()
    C, B, T, n = case
    y, h = _voltages(C, B, T, n), _chirp(C, n, n)
    flush("dedisperse %s" % (case,))
    out = lbf.dedisperse(to_dev(y), to_dev(h), n)
    torch.cuda.synchronize()
    got, ref = cplx(out), _oracle(y, h, n)
    for c in range(C):
        for b in range(B):
            assert relerr(got[c, b], ref[c, b]) <= TOL, (c, b)


def test_dedisperse_in_place_equals_out_of_place_bitwise():
    torch = _torch()
    C, B, T, n = 2, 3, 8192, 4096
    y, h = to_dev(_voltages(C, B, T, 5)), to_dev(_chirp(C, n, 5))
    flush("dedisperse in place")
    a = lbf.dedisperse(y, h, n)
    yy = y.clone()
    b = lbf.dedisperse(yy, h, n, out=yy)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_dedisperse_unit_weights_return_the_input():
    torch = _torch()
    C, B, T, n = 2, 2, 1024, 512
    y = _voltages(C, B, T, 6)
    ones = np.zeros((C, n, 2), np.float32)
    ones[..., 0] = 1.0
    out = lbf.dedisperse(to_dev(y), to_dev(ones), n)
    torch.cuda.synchronize()
    assert relerr(cplx(out), cplx(y)) <= TOL


def test_dedisperse_of_beam_former_voltages():
    """Beam former (FP32 voltages) then dedispersion, against the oracle's
    beam former then the oracle's dedispersion."""
    torch = _torch()
    blk = synth.make_block(8, 3, 1, 16, 4096, "ci16", 32.0, tag=(1105, 661, 92))
    pos, dirs, freq, ref = geometry(blk)
    w = lbf.compute_weights(pos, dirs, freq, lbf.F32, ref_dir=ref)
    h = _chirp(blk.C, 4096, 7)
    flush("beam former + dedispersion, 16 channels x 4096 samples")
    v = lbf.beamform(to_dev(blk.x), w, lbf.VOLTAGES)
    out = lbf.dedisperse(v, to_dev(h), 4096)
    torch.cuda.synchronize()
    yo = orc.beamform(blk.x, orc.block_weights(blk))                 # [C][B][T][2] complex128
    want = orc.dedisperse(yo, cplx(h), 4096)
    got = cplx(out)
    for c in range(blk.C):
        assert relerr(got[c], want[c]) <= TOL, c


def test_dedisperse_case_e_share_sampled():
    """Table 1 case E at one GPU's share: 512 channels of 12.2 kHz, 10 beams,
    three 4096-sample blocks; sampled (channel, beam) series against the
    oracle."""
    torch = _torch()
    C, B, T, n = 512, 10, 3 * 4096, 4096
    gen = torch.Generator().manual_seed(1105661)
    y = (torch.randn((C, B, T, 2, 2), generator=gen) * 100.0).to("cuda")
    h = to_dev(_chirp(C, n, 8))
    flush("dedisperse case E share: C=512 B=10 T=12288")
    out = lbf.dedisperse(y, h, n)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    for c, b in zip(rng.choice(C, 6, replace=False), rng.choice(B, 6)):
        yc = y[c:c + 1, b:b + 1].cpu().numpy()
        want = orc.dedisperse(cplx(yc), cplx(h[c:c + 1].cpu().numpy()), n)
        assert relerr(cplx(out[c:c + 1, b:b + 1]), want) <= TOL, (c, b)
