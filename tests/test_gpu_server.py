"""GPU tests of the streaming server (lbf_server_*): continuous batching of
blocks of different shapes, each result the same alone and in the mix, host
staging, admission by arena footprint with weight-cache eviction, and the
status codes of the queue."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1105_0661_amd import lbf, synth
from tests._util import check_stokes, flush, to_dev

pytestmark = pytest.mark.gpu

TOL = {lbf.F32: 1e-5, lbf.F16: 3e-3, lbf.BF16: 3e-3}
CT_NAMES = {lbf.F32: "f32", lbf.F16: "f16", lbf.BF16: "bf16"}

# (S, B, nsb, nch, T, xtype, product, t_int, f_int, obs_id)
MIX = [
    (24, 17, 2, 16, 64, "ci8", lbf.STOKES_I, 16, 1, 1),
    (40, 150, 1, 16, 96, "ci16", lbf.STOKES_IQUV, 16, 1, 2),
    (64, 33, 3, 8, 32, "ci8", lbf.STOKES_IQUV, 32, 1, 3),
    (31, 1, 1, 5, 48, "ci16", lbf.STOKES_I, 4, 1, 4),
    (70, 90, 1, 4, 64, "ci8", lbf.STOKES_IQUV, 16, 2, 5),     # > 64 stations, channel integration
    (24, 17, 2, 16, 64, "ci8", lbf.STOKES_I, 16, 1, 1),       # same observation as the first: cached weights
    (48, 70, 2, 16, 64, "ci16", lbf.STOKES_IQUV, 16, 4, 6),   # channel integration on the fast workers
]


def _torch():
    import torch
    return torch


def _blocks():
    out = []
    for i, (S, B, nsb, nch, T, xt, prod, ti, fi, obs) in enumerate(MIX):
        blk = synth.make_block(S, B, nsb, nch, T, xt, 16.0 if xt == "ci8" else 40.0, tag=(1105, 661, 70 + obs))
        out.append((blk, prod, ti, fi, obs))
    return out


def _arena(nbytes):
    torch = _torch()
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")


def _submit(srv, blk, prod, ti, fi, obs, ctype, x):
    return srv.submit(obs, blk.station_xyz, blk.beam_dir, blk.freq_hz, x, ctype, prod, ti, fi, ref_dir=blk.ref_dir)


@pytest.mark.parametrize("ctype", [lbf.F16, lbf.BF16, lbf.F32], ids=["f16", "bf16", "f32"])
def test_results_alone_equal_results_in_the_mix(ctype):
    torch = _torch()
    blocks = _blocks()
    xs = [to_dev(b[0].x) for b in blocks]
    # alone: one job on the device at a time
    alone = []
    with lbf.Server(_arena(256 << 20), max_inflight=1, n_streams=1, max_batch=1) as srv:
        for (blk, prod, ti, fi, obs), x in zip(blocks, xs):
            flush("server alone %s S=%d B=%d" % (CT_NAMES[ctype], blk.S, blk.B))
            t = _submit(srv, blk, prod, ti, fi, obs, ctype, x)
            st = srv.wait(t)
            assert st.state == lbf.JOB_DONE and st.batch_size == 1, (st.state, st.error)
            alone.append(srv.output(t).clone())
            srv.release(t)
    # mix: all submitted at once, fused into shared launches on two streams
    flush("server mix %s" % CT_NAMES[ctype])
    with lbf.Server(_arena(256 << 20), max_inflight=16, n_streams=2, max_batch=8) as srv:
        tickets = [_submit(srv, blk, prod, ti, fi, obs, ctype, x) for (blk, prod, ti, fi, obs), x in zip(blocks, xs)]
        sts = [srv.wait(t) for t in tickets]
        assert all(s.state == lbf.JOB_DONE for s in sts), [(s.state, s.error) for s in sts]
        mixed = [srv.output(t).clone() for t in tickets]
        if ctype != lbf.F32:
            assert max(s.batch_size for s in sts) > 1      # admitted together, batched
        for s in sts:
            assert s.t_submit_ns <= s.t_admit_ns <= s.t_start_ns <= s.t_done_ns
    torch.cuda.synchronize()
    for i, ((blk, prod, ti, fi, obs), a, m) in enumerate(zip(blocks, alone, mixed)):
        assert torch.equal(a, m), "job %d differs alone vs mix" % i
        direct = lbf.beamform(xs[i], lbf.compute_weights(to_dev(blk.station_xyz), to_dev(blk.beam_dir),
                                                         to_dev(blk.freq_hz), ctype, ref_dir=blk.ref_dir),
                              prod, ti, fi)
        torch.cuda.synchronize()
        assert torch.equal(a, direct), "job %d differs from lbf_beamform" % i
        ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, prod, ti, fi, 8)
        check_stokes(a.cpu().numpy(), ref, TOL[ctype], "server job %d" % i)


def test_host_staged_input_equals_device_input():
    torch = _torch()
    blk, prod, ti, fi, obs = _blocks()[1]
    with lbf.Server(_arena(64 << 20), max_inflight=2, n_streams=2, max_batch=2) as srv:
        t_dev = _submit(srv, blk, prod, ti, fi, obs, lbf.F16, to_dev(blk.x))
        t_host = _submit(srv, blk, prod, ti, fi, obs, lbf.F16, blk.x)          # host array, staged in the arena
        a, b = srv.wait(t_dev), srv.wait(t_host)
        assert a.state == lbf.JOB_DONE and b.state == lbf.JOB_DONE
        assert torch.equal(srv.output(t_dev), srv.output(t_host))


def _align(v):
    return (v + 255) // 256 * 256


def _footprint(blk, prod, ti, fi, ctype=lbf.F16):
    """Arena bytes of one job: its weights (with the geometry) and its Stokes staging."""
    fp = lbf.block_footprint(blk.S, blk.C, blk.T, blk.B, lbf.XTYPE_NAMES[blk.xtype], ctype, prod, ti, fi)
    return (_align(fp.weight_bytes) + _align(8 * (4 * blk.S + 3 * blk.B + blk.C)), _align(fp.staging_bytes))


def test_admission_by_footprint_evicts_idle_weights():
    # an arena that holds one observation's weights (and one job's Stokes
    # staging) at a time: jobs of alternating observations still all
    # complete, with the right results
    torch = _torch()
    blocks = _blocks()[:2]
    xs = [to_dev(b[0].x) for b in blocks]
    need = max(sum(_footprint(*b[:4])) for b in blocks)
    with lbf.Server(_arena(need + 256), max_inflight=4, n_streams=2, max_batch=4) as srv:
        order = [0, 1, 0, 1, 1, 0]
        tickets = [_submit(srv, *blocks[i], lbf.F16, xs[i]) for i in order]
        outs = []
        for t in tickets:
            st = srv.wait(t)
            assert st.state == lbf.JOB_DONE, (st.state, st.error)
            outs.append(srv.output(t).clone())
    torch.cuda.synchronize()
    for i in range(2):
        blk, prod, ti, fi, obs = blocks[i]
        ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, prod, ti, fi, 8)
        first = outs[order.index(i)]
        check_stokes(first.cpu().numpy(), ref, TOL[lbf.F16], "eviction %d" % i)
        for j, o in zip(order, outs):
            if j == i:
                assert torch.equal(o, first)


def test_admission_waits_for_stokes_staging():
    # two blocks of one observation (weights cached once) in an arena that
    # holds the Stokes staging of only one of them: the second is admitted
    # once the first has finished and given its staging back, and both
    # results are right
    torch = _torch()
    blk, prod, ti, fi, obs = _blocks()[1]
    x = to_dev(blk.x)
    w_bytes, st_bytes = _footprint(blk, prod, ti, fi)
    assert st_bytes > 0
    with lbf.Server(_arena(w_bytes + st_bytes + st_bytes // 2), max_inflight=2, n_streams=2, max_batch=2) as srv:
        flush("server staging wait")
        tickets = [_submit(srv, blk, prod, ti, fi, obs, lbf.F16, x) for _ in range(2)]
        sts = [srv.wait(t) for t in tickets]
        assert all(s.state == lbf.JOB_DONE for s in sts), [(s.state, s.error) for s in sts]
        assert sts[1].t_admit_ns >= sts[0].t_done_ns
        outs = [srv.output(t).clone() for t in tickets]
    # a staging cap below one channel's staging can never run that block
    with lbf.Server(_arena(64 << 20), max_inflight=1, n_streams=1, staging_cap=256) as srv:
        with pytest.raises(lbf.LbfError) as ei:
            _submit(srv, blk, prod, ti, fi, obs, lbf.F16, x)
        assert ei.value.code == lbf.E_NOMEM
    # a cap of a few channels: the block runs in channel passes, same result
    fp = lbf.block_footprint(blk.S, blk.C, blk.T, blk.B, lbf.XTYPE_NAMES[blk.xtype], lbf.F16, prod, ti, fi)
    with lbf.Server(_arena(64 << 20), max_inflight=1, n_streams=1,
                    staging_cap=5 * fp.staging_channel_bytes) as srv:
        t = _submit(srv, blk, prod, ti, fi, obs, lbf.F16, x)
        assert srv.wait(t).state == lbf.JOB_DONE
        passes = srv.output(t).clone()
    torch.cuda.synchronize()
    ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, prod, ti, fi, 8)
    check_stokes(outs[0].cpu().numpy(), ref, TOL[lbf.F16], "staging wait")
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(passes, outs[0])


@pytest.mark.parametrize("ctype", [lbf.F16, lbf.F32], ids=["f16", "f32"])
def test_channel_integration_through_staging_passes(ctype):
    # channel integration on the fast workers: per-channel staging in passes
    # of whole f_int-channel groups (4 channels of a 6-channel cap), the same
    # bits as lbf_beamform; a cap below one group is refused at submit
    torch = _torch()
    blk = synth.make_block(40, 100, 2, 16, 64, "ci8", 16.0, tag=(1105, 661, 79))
    prod, ti, fi = lbf.STOKES_IQUV, 16, 4
    x = to_dev(blk.x)
    w = lbf.compute_weights(to_dev(blk.station_xyz), to_dev(blk.beam_dir), to_dev(blk.freq_hz), ctype,
                            ref_dir=blk.ref_dir)
    direct = lbf.beamform(x, w, prod, ti, fi)
    per = lbf.block_footprint(blk.S, blk.C, blk.T, blk.B, lbf.CI8, ctype, prod, ti, fi).staging_channel_bytes
    assert per > 0
    flush("server channel integration passes %s" % CT_NAMES[ctype])
    with lbf.Server(_arena(64 << 20), max_inflight=1, n_streams=1, staging_cap=6 * per) as srv:
        t = _submit(srv, blk, prod, ti, fi, 79, ctype, x)
        assert srv.wait(t).state == lbf.JOB_DONE
        got = srv.output(t).clone()
    with lbf.Server(_arena(64 << 20), max_inflight=1, n_streams=1, staging_cap=3 * per) as srv:
        with pytest.raises(lbf.LbfError) as ei:
            _submit(srv, blk, prod, ti, fi, 79, ctype, x)
        assert ei.value.code == lbf.E_NOMEM
    torch.cuda.synchronize()
    assert torch.equal(got, direct)
    ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, prod, ti, fi, 8)
    check_stokes(got.cpu().numpy(), ref, TOL[ctype], "channel integration passes")


def test_queue_status_codes():
    blk, prod, ti, fi, obs = _blocks()[1]
    x = to_dev(blk.x)
    # footprint beyond the arena: refused at submit
    with lbf.Server(_arena(4096), max_inflight=1, n_streams=1) as srv:
        with pytest.raises(lbf.LbfError) as ei:
            _submit(srv, blk, prod, ti, fi, obs, lbf.F16, x)
        assert ei.value.code == lbf.E_NOMEM
    # a bounded queue refuses work rather than growing: one job on the device,
    # one queued, blocks that take a fraction of a millisecond each (their
    # Stokes staging capped at 16 MiB, so they run in channel passes)
    big = synth.make_block(64, 300, 8, 64, 768, "ci8", 16.0, tag=(1105, 661, 79))
    xb = to_dev(big.x)
    with lbf.Server(_arena(64 << 20), max_inflight=1, n_streams=1, queue_capacity=1, max_batch=1,
                    staging_cap=16 << 20) as srv:
        codes, tickets = [], []
        flush("server queue bound")
        for _ in range(32):
            try:
                tickets.append(_submit(srv, big, lbf.STOKES_IQUV, 16, 1, 7, lbf.F16, xb))
            except lbf.LbfError as e:
                codes.append(e.code)
        assert lbf.E_BUSY in codes
        assert set(codes) == {lbf.E_BUSY}
        for t in tickets:
            assert srv.wait(t).state == lbf.JOB_DONE
        with pytest.raises(lbf.LbfError) as ei:
            srv.poll(10 ** 9)
        assert ei.value.code == lbf.E_NOTFOUND
        srv.release(tickets[0])
        with pytest.raises(lbf.LbfError) as ei:
            srv.poll(tickets[0])
        assert ei.value.code == lbf.E_NOTFOUND


# blocks of one stream whose integration periods span block boundaries: 256
# samples cut at 100, 110, 184 (the 10-sample block completes no period)
STREAM_CUTS = [0, 100, 110, 184, 256]


@pytest.mark.parametrize("ctype,prod,t_int,f_int,periods", [
    (lbf.F16, lbf.STOKES_IQUV, 16, 1, [6, 0, 5, 5]),
    (lbf.F32, lbf.STOKES_IQUV, 16, 1, [6, 0, 5, 5]),
    (lbf.BF16, lbf.STOKES_I, 8, 2, [12, 1, 10, 9]),       # channel integration: the generic workers
], ids=["f16", "f32", "bf16-I-t8-f2"])
def test_stream_carry_equals_the_concatenated_block(ctype, prod, t_int, f_int, periods):
    torch = _torch()
    streams = [synth.make_block(24, 17, 2, 16, 256, "ci8", 16.0, tag=(1105, 661, 90)),
               synth.make_block(40, 9, 1, 8, 256, "ci16", 40.0, tag=(1105, 661, 91))]
    xs = [to_dev(b.x) for b in streams]
    plain = synth.make_block(24, 17, 2, 16, 64, "ci8", 16.0, tag=(1105, 661, 92))
    with lbf.Server(_arena(64 << 20), max_inflight=8, n_streams=2, max_batch=4) as srv:
        tickets = {0: [], 1: []}
        # the two streams interleaved, with an independent block between them,
        # so that consecutive blocks of a stream run on different HIP streams
        for a, b in zip(STREAM_CUTS[:-1], STREAM_CUTS[1:]):
            for i, (blk, x) in enumerate(zip(streams, xs)):
                flush("server stream %d samples [%d, %d) %s" % (i, a, b, CT_NAMES[ctype]))
                tickets[i].append(srv.submit(300 + i, blk.station_xyz, blk.beam_dir, blk.freq_hz,
                                             x[:, :, a:b].contiguous(), ctype, prod, t_int, f_int,
                                             ref_dir=blk.ref_dir, stream_id=7 + i))
            t_plain = _submit(srv, plain, prod, 16, 1, 310, ctype, to_dev(plain.x))
            assert srv.wait(t_plain).state == lbf.JOB_DONE
        for i, blk in enumerate(streams):
            outs = []
            for t, a, b in zip(tickets[i], STREAM_CUTS[:-1], STREAM_CUTS[1:]):
                st = srv.wait(t)
                assert st.state == lbf.JOB_DONE, (st.state, st.error)
                assert st.periods == srv.output(t).shape[2]
                outs.append(srv.output(t).clone())
            assert [o.shape[2] for o in outs] == periods
            got = torch.cat(outs, dim=2)
            torch.cuda.synchronize()
            ref = orc.pipeline(blk.x, blk.station_xyz, blk.beam_dir, blk.ref_dir, blk.freq_hz, prod, t_int, f_int, 8)
            check_stokes(got.cpu().numpy(), ref, TOL[ctype], "stream %d" % i)


def test_stream_block_rules():
    blk = synth.make_block(24, 17, 2, 16, 40, "ci8", 16.0, tag=(1105, 661, 93))
    x = to_dev(blk.x)
    with lbf.Server(_arena(16 << 20), max_inflight=2, n_streams=1) as srv:
        for bad in (dict(product=lbf.VOLTAGES, t_int=1), dict(x=blk.x)):
            args = dict(x=x, product=lbf.STOKES_I, t_int=16)
            args.update(bad)
            with pytest.raises(lbf.LbfError) as ei:
                srv.submit(1, blk.station_xyz, blk.beam_dir, blk.freq_hz, args["x"], lbf.F16, args["product"],
                           args["t_int"], 1, ref_dir=blk.ref_dir, stream_id=5)
            assert ei.value.code == lbf.E_INVAL
        # 40 samples at t_int 16: two periods, 8 carried
        t = srv.submit(1, blk.station_xyz, blk.beam_dir, blk.freq_hz, x, lbf.F16, lbf.STOKES_I, 16, 1,
                       ref_dir=blk.ref_dir, stream_id=5)
        st = srv.wait(t)
        assert st.state == lbf.JOB_DONE and st.periods == 2
        # a live stream keeps its t_int
        with pytest.raises(lbf.LbfError) as ei:
            srv.submit(1, blk.station_xyz, blk.beam_dir, blk.freq_hz, x, lbf.F16, lbf.STOKES_I, 8, 1,
                       ref_dir=blk.ref_dir, stream_id=5)
        assert ei.value.code == lbf.E_INVAL
        # the same t_int continues it: 8 + 40 = 48 samples, three periods
        t = srv.submit(1, blk.station_xyz, blk.beam_dir, blk.freq_hz, x, lbf.F16, lbf.STOKES_I, 16, 1,
                       ref_dir=blk.ref_dir, stream_id=5)
        st = srv.wait(t)
        assert st.state == lbf.JOB_DONE and st.periods == 3
