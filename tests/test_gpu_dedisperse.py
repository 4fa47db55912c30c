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


# (C, B, T, n_fft, product, t_int): periods inside a thread (t_int <= n_fft / 256),
# across lanes (up to 64 lanes: t_int 1024 at 4096), the small transforms
# with fewer threads than the block's work group, both products
STOKES_CASES = [(2, 3, 8192, 4096, lbf.STOKES_IQUV, 16), (1, 2, 4096, 4096, lbf.STOKES_I, 1),
                (2, 2, 8192, 4096, lbf.STOKES_IQUV, 1024), (2, 2, 4096, 4096, lbf.STOKES_IQUV, 64),
                (3, 2, 1024, 512, lbf.STOKES_IQUV, 2), (2, 2, 1024, 512, lbf.STOKES_I, 128),
                (3, 2, 192, 64, lbf.STOKES_IQUV, 4), (2, 1, 128, 64, lbf.STOKES_I, 64),
                (3, 2, 24, 8, lbf.STOKES_IQUV, 8), (2, 2, 16, 8, lbf.STOKES_I, 1)]


@pytest.mark.parametrize("case", STOKES_CASES, ids=lambda c: "C%d_B%d_T%d_n%d_K%d_t%d" % c)
def test_dedisperse_stokes_matches_oracle_and_the_two_step_chain(case):
    """Dedispersion then Stokes and integration in one kernel, against the
    oracle's dedispersion followed by its Stokes and integration steps, and
    against lbf_dedisperse + lbf_stokes on the GPU."""
    torch = _torch()
    C, B, T, n, prod, ti = case
    K = lbf.n_stokes(prod)
    y, h = _voltages(C, B, T, 7 * n + ti), _chirp(C, n, n + 1)
    flush("dedisperse+Stokes %s" % (case,))
    yd, hd = to_dev(y), to_dev(h)
    s = lbf.dedisperse_stokes(yd, hd, n, prod, ti)                         # [C][B][T'][K]
    two = lbf.stokes(lbf.dedisperse(yd, hd, n), prod, ti, 1)
    torch.cuda.synchronize()
    ref = orc.integrate(orc.stokes(_oracle(y, h, n)), K, ti, 1)            # [C][B][T'][K]
    got = s.cpu().numpy()
    assert got.shape == ref.shape
    for k in range(K):
        # Q, U and V of independent Gaussian polarisations average out: measure
        # every parameter against Stokes I of the same (channel, beam)
        for c in range(C):
            for b in range(B):
                den = np.linalg.norm(ref[c, b, :, 0])
                assert np.linalg.norm(got[c, b, :, k] - ref[c, b, :, k]) <= TOL * den, (k, c, b)
    assert np.linalg.norm(got - two.cpu().numpy()) <= 1e-6 * np.linalg.norm(got[..., 0])


def test_dedisperse_stokes_rejects_unsupported_integrations():
    torch = _torch()
    y = torch.zeros((1, 1, 4096, 2, 2), device="cuda:0")
    h = torch.zeros((1, 4096, 2), device="cuda:0")
    for ti in (3, 2048, 8192):
        with pytest.raises(lbf.LbfError) as ei:
            lbf.dedisperse_stokes(y, h, 4096, lbf.STOKES_IQUV, ti)
        assert ei.value.code == lbf.E_INVAL
    with pytest.raises(lbf.LbfError):
        lbf.dedisperse_stokes(y[:, :, :512].contiguous(), h[:, :512].contiguous(), 512, lbf.STOKES_I, 256)
