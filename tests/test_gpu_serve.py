"""GPU: segmented decoding and the continuous-batching server.

A request's frames must decode exactly as a standalone decode with the
request's seed and frame index would decode them (and as the oracle does),
whichever requests share its launch and whichever slots it occupies.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1402_2773_amd as ng
from synth import channel, codes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    ng.lib()
    oracle.build(force=False)
    return torch


P_C1 = oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=100)
P_SM = oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)

_CODES = {}


def dev_code(name):
    if name not in _CODES:
        c = codes.named_code(name)
        _CODES[name] = (c, ng.Code.from_ldpc(c))
    return _CODES[name]


def test_segments_equal_oracle(torch_dev):
    """Three segments scattered over a pool, keyed by their own seeds and frame
    indices; slots outside every segment stay untouched."""
    torch = torch_dev
    c, dc = dev_code("C96")
    pool = 256
    sig = channel.frame_sigmas(pool, 2.5, 4.5, c.rate, seed=11).astype(np.float32)
    y = channel.bpsk_awgn(pool, c.n, sig, seed=12)
    # (first_slot, length, seed, frame_base)
    segs = [(200, 40, 5, 1000), (0, 17, 7, 0), (90, 33, 5, 2000)]
    host_segs = (ng.ngdbf_segment * len(segs))()
    off = 0
    for i, (fs, ln, sd, fb) in enumerate(segs):
        host_segs[i] = ng.ngdbf_segment(fs, off, sd, fb)
        off += ln
    seg_dev = torch.frombuffer(bytearray(bytes(host_segs)), dtype=torch.uint8).cuda()
    y_dev = torch.from_numpy(y).cuda()
    s_dev = torch.from_numpy(sig).cuda()
    bits = torch.full((pool, (c.n + 7) // 8), 0xAB, dtype=torch.uint8, device="cuda")
    iters = torch.full((pool,), -7, dtype=torch.int32, device="cuda")
    conv = torch.full((pool,), 0xCD, dtype=torch.uint8, device="cuda")
    say("segments C96", segs)
    ng.ngdbf_decode_segments(dc.handle, y_dev, s_dev, 0.0, pool, ng.Params(**P_SM.__dict__).c(
        ng.NGDBF_Y_F32), seg_dev, len(segs), off, bits, iters, conv, None)
    torch.cuda.synchronize()
    b, it, cv = bits.cpu().numpy(), iters.cpu().numpy(), conv.cpu().numpy()
    covered = np.zeros(pool, dtype=bool)
    for fs, ln, sd, fb in segs:
        r = oracle.decode(c, y[fs:fs + ln], sig[fs:fs + ln], P_SM, sd, frame_base=fb, threads=8)
        assert (it[fs:fs + ln] == r.iters).all()
        assert (b[fs:fs + ln] == r.bits).all()
        assert (cv[fs:fs + ln] == r.converged).all()
        covered[fs:fs + ln] = True
    assert (b[~covered] == 0xAB).all() and (it[~covered] == -7).all() and (cv[~covered] == 0xCD).all()


def test_segments_skip_slots_outside_pool(torch_dev):
    """A segment running past the pool decodes its in-pool frames only."""
    torch = torch_dev
    c, dc = dev_code("C96")
    pool = 64
    y = channel.bpsk_awgn(pool, c.n, 0.7, seed=3)
    segs = (ng.ngdbf_segment * 1)(ng.ngdbf_segment(50, 0, 9, 0))
    seg_dev = torch.frombuffer(bytearray(bytes(segs)), dtype=torch.uint8).cuda()
    y_dev = torch.from_numpy(y).cuda()
    bits = torch.zeros((pool, 12), dtype=torch.uint8, device="cuda")
    iters = torch.full((pool,), -1, dtype=torch.int32, device="cuda")
    ng.ngdbf_decode_segments(dc.handle, y_dev, None, 0.7, pool, ng.Params(**P_C1.__dict__).c(
        ng.NGDBF_Y_F32), seg_dev, 1, 30, bits, iters, None, None)
    torch.cuda.synchronize()
    r = oracle.decode(c, y[50:], 0.7, P_C1, 9, threads=4)
    assert (iters.cpu().numpy()[50:] == r.iters).all()
    assert (bits.cpu().numpy()[50:] == r.bits).all()
    assert (iters.cpu().numpy()[:50] == -1).all()


def _requests(rng, n_req, code_names, max_frames):
    reqs = []
    for i in range(n_req):
        ci = int(rng.integers(len(code_names)))
        nf = int(np.exp(rng.uniform(0, np.log(max_frames))))
        ebn0 = float(rng.uniform(2.0, 5.0))
        reqs.append(dict(code=ci, frames=max(nf, 1), ebn0=ebn0, seed=int(rng.integers(1 << 62)),
                         base=int(rng.integers(1 << 40)), data_seed=1000 + i))
    return reqs


def _serve(torch, srv, code_list, reqs, order, pump_every=1):
    """Admit / fill / commit / pump / poll / release until every request of
    ``order`` is done; returns per-request (bits, iters, conv) on the host."""
    results = {}
    pending = list(order)
    live = {}
    steps = 0
    while pending or live:
        steps += 1
        assert steps < 100000, "server made no progress"
        if pending:
            batch = pending[:8]
            t, first = srv.admit([reqs[i]["code"] for i in batch], [reqs[i]["frames"] for i in batch],
                                 [reqs[i]["seed"] for i in batch], [reqs[i]["base"] for i in batch])
            for k in range(len(t)):
                i = batch[k]
                q = reqs[i]
                c, _ = code_list[q["code"]]
                p = srv.pools[q["code"]]
                s = channel.sigma_from_ebn0(q["ebn0"], c.rate)
                y = channel.bpsk_awgn(q["frames"], c.n, s, seed=q["data_seed"])
                fs = int(first[k])
                p.y[fs:fs + q["frames"]].copy_(torch.from_numpy(y), non_blocking=False)
                p.sigma[fs:fs + q["frames"]].fill_(s)
                live[int(t[k])] = (i, fs)
            if len(t):
                srv.commit(t)
            pending = pending[len(t):]
        if steps % pump_every == 0 or not pending:
            srv.pump()
        done = srv.poll()
        for t in done:
            i, fs = live.pop(int(t))
            q = reqs[i]
            p = srv.pools[q["code"]]
            sl = slice(fs, fs + q["frames"])
            results[i] = (p.bits[sl].cpu().numpy(), p.iters[sl].cpu().numpy(),
                          p.converged[sl].cpu().numpy())
        if len(done):
            srv.release(done)
    return results


def test_server_alone_equals_mix_equals_decode(torch_dev):
    """Every request gives the same result served alone, served in a mix of
    two codes under slot pressure, and decoded standalone with ngdbf_decode;
    small requests also match the oracle."""
    torch = torch_dev
    names = ["C96", "C1008"]
    code_list = [dev_code(n) for n in names]
    params = [P_C1, P_SM]
    rng = np.random.default_rng(5)
    reqs = _requests(rng, 40, names, 300)
    say("server mix: sizes", [r["frames"] for r in reqs])
    srv = ng.Server([dc for _, dc in code_list], [ng.Params(**p.__dict__) for p in params],
                    [700, 700], n_streams=3)
    try:
        mixed = _serve(torch, srv, code_list, reqs, list(range(len(reqs))), pump_every=3)
        alone = {}
        for i in range(0, len(reqs), 5):
            alone.update(_serve(torch, srv, code_list, reqs, [i]))
    finally:
        srv.close()
    # the unbatched baseline: one launch per request
    srv1 = ng.Server([dc for _, dc in code_list], [ng.Params(**p.__dict__) for p in params],
                     [700, 700], n_streams=2, max_requests_per_launch=1, launches_per_stream=8)
    try:
        single = _serve(torch, srv1, code_list, reqs, list(range(len(reqs))), pump_every=2)
    finally:
        srv1.close()
    for i, q in enumerate(reqs):
        c, dc = code_list[q["code"]]
        s = channel.sigma_from_ebn0(q["ebn0"], c.rate)
        y = channel.bpsk_awgn(q["frames"], c.n, s, seed=q["data_seed"])
        out = ng.decode(dc, torch.from_numpy(y).cuda(), s, ng.Params(**params[q["code"]].__dict__),
                        q["seed"], frame_base=q["base"])
        torch.cuda.synchronize()
        ref = (out.bits.cpu().numpy(), out.iters.cpu().numpy(), out.converged.cpu().numpy())
        for a, b in zip(mixed[i], ref):
            assert (a == b).all(), f"request {i} differs in the mix"
        for a, b in zip(single[i], ref):
            assert (a == b).all(), f"request {i} differs launched alone"
        if i in alone:
            for a, b in zip(alone[i], ref):
                assert (a == b).all(), f"request {i} differs alone"
        if q["code"] == 0 and q["frames"] <= 64:
            r = oracle.decode(c, y, s, params[0], q["seed"], frame_base=q["base"], threads=4)
            assert (mixed[i][1] == r.iters).all() and (mixed[i][0] == r.bits).all()


def test_server_admission_is_bounded_by_the_pool(torch_dev):
    torch = torch_dev
    c, dc = dev_code("C96")
    srv = ng.Server([dc], [ng.Params(**P_C1.__dict__)], [100], n_streams=1)
    try:
        t, first = srv.admit([0, 0, 0], [60, 30, 20], [1, 2, 3], [0, 0, 0])
        assert len(t) == 2 and list(first) == [0, 60]
        with pytest.raises(ng.NgdbfError, match="frames for a pool of 100"):
            srv.admit([0], [101], [1], [0])
        with pytest.raises(ng.NgdbfError, match="not a finished request"):
            srv.release(t[:1])
        srv.pools[0].y[:90].fill_(1.0)
        srv.pools[0].sigma[:90].fill_(0.5)
        srv.commit(t)
        done = []
        for _ in range(100000):
            srv.pump()
            done += list(srv.poll())
            if len(done) == 2:
                break
        assert sorted(done) == sorted(int(x) for x in t)
        assert (srv.pools[0].iters[:90].cpu().numpy() == 0).all()  # noiseless-like input: x(0) valid
        srv.release(done)
        t2, first2 = srv.admit([0], [100], [1], [0])
        assert len(t2) == 1 and first2[0] == 0  # slots coalesced after release
    finally:
        srv.close()
