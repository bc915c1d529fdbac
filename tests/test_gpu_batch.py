"""GPU: launch shapes, the autotuner, batched multi-code decoding and its
hipGraph capture all give the oracle's results bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import paper_1402_2773_amd as ng
from synth import channel, codes

pytestmark = pytest.mark.gpu

# (waves per frame, quads per lane) pairs built into the library
SHAPES = [(1, 1), (1, 2), (1, 4), (2, 2), (2, 4), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2), (16, 1)]


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


def heur(ebn0):
    lam = 0.99 if ebn0 < 3.5 else 0.97 if ebn0 < 4.0 else 0.94 if ebn0 < 4.25 else 0.90
    return oracle.Params(w=0.75, theta=-0.9, lam=lam, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)


P_HIGH = oracle.Params(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0, t_max=300)


def fitting_shapes(n):
    nq = (n + 3) // 4
    out = []
    for w, q in SHAPES:
        if nq <= 64 * w * q:
            for fpb in ([2, 4, 8, 16] if w == 1 else [1]):
                out.append((w, q, fpb))
    return out


def host(out):
    return out.bits.cpu().numpy(), out.iters.cpu().numpy(), out.converged.cpu().numpy()


def same(g, r):
    assert (g[1] == r.iters).all(), np.nonzero(g[1] != r.iters)[0][:10]
    assert (g[0] == r.bits).all()
    assert (g[2] == r.converged).all()


@pytest.mark.parametrize("name,frames,ebn0", [("C96", 600, 3.0), ("C1008", 300, 3.0),
                                              ("C2048", 120, 4.0), ("C4000", 60, 3.0)])
def test_every_shape_gives_the_same_result(torch_dev, name, frames, ebn0):
    torch = torch_dev
    c = codes.named_code(name)
    sig = np.float32(channel.sigma_from_ebn0(ebn0, c.rate))
    y = channel.bpsk_awgn(frames, c.n, sig, seed=81)
    p = P_HIGH if name == "C2048" else heur(ebn0)
    r = oracle.decode(c, y, sig, p, 82, threads=8)
    dc = ng.Code.from_ldpc(c)
    yd = torch.from_numpy(y).cuda()
    tried = 0
    for w, q, fpb in fitting_shapes(c.n):
        try:
            ng.ngdbf_code_set_shape(dc.handle, w, q, fpb)
        except ng.NgdbfError as e:
            assert e.status == -4  # not buildable in LDS: refused on the host
            continue
        say(name, "shape", w, q, fpb)
        out = ng.decode(dc, yd, float(sig), ng.Params(**p.__dict__), 82)
        torch.cuda.synchronize()
        same(host(out), r)
        tried += 1
    assert tried >= 2
    dc.close()


def test_shape_validation(torch_dev):
    c = codes.named_code("C1008")
    dc = ng.Code.from_ldpc(c)
    with pytest.raises(ng.NgdbfError, match="hold"):
        ng.ngdbf_code_set_shape(dc.handle, 1, 2, 8)  # 128 quads < 252
    with pytest.raises(ng.NgdbfError, match="workgroup of its own"):
        ng.ngdbf_code_set_shape(dc.handle, 2, 2, 2)
    with pytest.raises(ng.NgdbfError, match="no kernel"):
        ng.ngdbf_code_set_shape(dc.handle, 3, 4, 1)
    ng.ngdbf_code_set_shape(dc.handle, 4, 1, 1)
    assert ng.ngdbf_code_get_shape(dc.handle) == (4, 1, 1)
    ng.ngdbf_code_set_shape(dc.handle, 0, 0, 0)
    assert ng.ngdbf_code_get_shape(dc.handle) == (1, 4, 16)
    # the extended decoders default to at most two quads per lane, except the
    # packed quantized one and the single-bit one with per-bit draws
    ps = ng.Params(variant=ng.NGDBF_SINGLE).c(ng.NGDBF_Y_F32)
    assert ng.ngdbf_code_get_shape(dc.handle, ps) == (1, 4, 16)
    pr = ng.Params(variant=ng.NGDBF_SINGLE, noise_reuse=1).c(ng.NGDBF_Y_F32)
    assert ng.ngdbf_code_get_shape(dc.handle, pr) == (2, 2, 1)
    pq = ng.Params(quant_bits=4, noise_reuse=1, ymax=1.75, t_max=300).c(ng.NGDBF_Y_F32)
    assert ng.ngdbf_code_get_shape(dc.handle, pq) == (1, 4, 16)
    # a long schedule's stream leaves LDS for fewer frames per workgroup
    pl = ng.Params(quant_bits=4, noise_reuse=1, ymax=1.75, t_max=4000).c(ng.NGDBF_Y_F32)
    assert ng.ngdbf_code_get_shape(dc.handle, pl)[:2] == (1, 4)
    dc.close()
    # longer codes: the fewest waves that hold them (the base decoder's frames
    # of several waves read their tables from global memory)
    for name, shape in (("C2048", (2, 4, 1)), ("C4000", (4, 4, 1))):
        dl = ng.Code.from_ldpc(codes.named_code(name))
        assert ng.ngdbf_code_get_shape(dl.handle) == shape, name
        dl.close()


def test_autotune_keeps_results(torch_dev):
    torch = torch_dev
    c = codes.named_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(3.5, c.rate))
    y = channel.bpsk_awgn(2048, c.n, sig, seed=91)
    p = heur(3.5)
    dc = ng.Code.from_ldpc(c)
    yd = torch.from_numpy(y).cuda()
    best, ms = ng.autotune(dc, yd, float(sig), ng.Params(**p.__dict__), 92)
    say("autotune", best, ms)
    assert best in [tuple(s) for s in fitting_shapes(c.n)] and ms > 0
    assert ng.ngdbf_code_get_shape(dc.handle) == best
    out = ng.decode(dc, yd, float(sig), ng.Params(**p.__dict__), 92)
    torch.cuda.synchronize()
    same(host(out), oracle.decode(c, y, sig, p, 92, threads=8))
    dc.close()


def _mixed_jobs(torch):
    """Four codes, per-frame Eb/N0 uniform in [2, 5] dB, int8 y for C2048."""
    spec = [("C96", 800, heur(3.5), "f32"), ("C1008", 400, heur(3.5), "f32"),
            ("C2048", 150, P_HIGH, "i8"), ("C4000", 100, heur(3.5), "f32")]
    items = []
    for idx, (name, frames, p, fmt) in enumerate(spec):
        c = codes.named_code(name)
        sig = channel.frame_sigmas(frames, 2.0, 5.0, c.rate, seed=100 + idx)
        y = channel.bpsk_awgn(frames, c.n, sig, seed=110 + idx)
        if fmt == "i8":
            y = channel.quantize_int8(y)
        dc = ng.Code.from_ldpc(c)
        yd = torch.from_numpy(y).cuda()
        sd = torch.from_numpy(sig).cuda()
        out = ng.alloc_outputs(dc, frames, "cuda")
        items.append(dict(c=c, dc=dc, y=y, yd=yd, sig=sig, sd=sd, p=p, out=out,
                          seed=120 + idx, base=1000 * idx))
    return items


def test_batch_equals_oracle(torch_dev):
    torch = torch_dev
    items = _mixed_jobs(torch)
    jobs = [ng.job(it["dc"], it["yd"], it["sd"], ng.Params(**it["p"].__dict__), it["seed"],
                   it["out"], frame_base=it["base"]) for it in items]
    say("batch of", len(jobs))
    ng.ngdbf_decode_batch(jobs, None)
    torch.cuda.synchronize()
    for it in items:
        r = oracle.decode(it["c"], it["y"], it["sig"], it["p"], it["seed"], frame_base=it["base"],
                          threads=8)
        same(host(it["out"]), r)
    for it in items:
        it["dc"].close()


def test_batch_of_many_parameter_sets(torch_dev):
    """A parameter-search step: 27 parameter sets on one code and the same
    received frames, all concurrent on the library's streams (jobs below the
    full-device size), equal to one-at-a-time decodes and, on sampled jobs
    and frames, to the oracle."""
    torch = torch_dev
    c = codes.named_code("C1008")
    dc = ng.Code.from_ldpc(c)
    F = 384
    sig = float(np.float32(channel.sigma_from_ebn0(3.0, c.rate)))
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=411)
    base = heur(3.0)
    sets = [oracle.Params(**dict(base.__dict__, w=w, theta=th, eta=eta))
            for w in (0.6, 0.75, 0.9) for th in (-0.7, -0.9, -1.1) for eta in (0.85, 0.95, 1.05)]
    outs = [ng.alloc_outputs(dc, F, "cuda") for _ in sets]
    jobs = [ng.job(dc, y, sig, ng.Params(**p.__dict__), 500 + i, o) for i, (p, o) in enumerate(zip(sets, outs))]
    say("batch of", len(jobs), "parameter sets")
    ng.ngdbf_decode_batch(jobs, None)
    torch.cuda.synchronize()
    for i, (p, o) in enumerate(zip(sets, outs)):
        r = ng.decode(dc, y, sig, ng.Params(**p.__dict__), 500 + i)
        assert torch.equal(o.bits, r.bits) and torch.equal(o.iters, r.iters) and torch.equal(o.converged, r.converged)
    yh = y[:24].cpu().numpy()
    for i in (0, 13, 26):
        r = oracle.decode(c, yh, sig, sets[i], 500 + i, threads=8)
        same(host(ng.Outputs(outs[i].bits[:24], outs[i].iters[:24], outs[i].converged[:24])), r)
    dc.close()


def test_batch_graph_replays(torch_dev):
    """The batch captured into a graph: every replay (with eager work and
    synchronisation between replays) reproduces the eager results."""
    torch = torch_dev
    items = _mixed_jobs(torch)
    jobs = [ng.job(it["dc"], it["yd"], it["sd"], ng.Params(**it["p"].__dict__), it["seed"],
                   it["out"], frame_base=it["base"]) for it in items]
    ng.ngdbf_decode_batch(jobs, None)  # eager run (also creates the library streams)
    torch.cuda.synchronize()
    ref = [host(it["out"]) for it in items]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ng.ngdbf_decode_batch(jobs, s)
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:
            it["out"].bits.fill_(0xAA)
            it["out"].iters.fill_(-1)
        torch.cuda.synchronize()
        say("replay", rep)
        g.replay()
        torch.cuda.synchronize()
        for it, rf in zip(items, ref):
            h = host(it["out"])
            assert (h[0] == rf[0]).all() and (h[1] == rf[1]).all() and (h[2] == rf[2]).all()
    del g
    for it in items:
        it["dc"].close()


def test_batch_with_full_device_jobs_and_graph(torch_dev):
    """Jobs of 65536 frames or more run in order on the caller's stream beside
    the forked small ones; eager and graph-replayed results equal
    one-at-a-time decodes (and the oracle on samples)."""
    torch = torch_dev
    c = codes.named_code("C96")
    dc = ng.Code.from_ldpc(c)
    p = oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=60)
    sizes = [70000, 300, 65536, 90]
    ys, outs, refs = [], [], []
    for i, F in enumerate(sizes):
        sig = float(np.float32(channel.sigma_from_ebn0(3.0 + 0.25 * i, c.rate)))
        y = channel.bpsk_awgn_device(F, c.n, sig, seed=200 + i)
        ys.append((y, sig))
        outs.append(ng.alloc_outputs(dc, F, "cuda"))
        refs.append(ng.decode(dc, y, sig, ng.Params(**p.__dict__), 300 + i, frame_base=7 * i))
    torch.cuda.synchronize()
    jobs = [ng.job(dc, y, sig, ng.Params(**p.__dict__), 300 + i, outs[i], frame_base=7 * i)
            for i, (y, sig) in enumerate(ys)]
    say("batch with full-device jobs")
    ng.ngdbf_decode_batch(jobs, None)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert (o.bits == r.bits).all().item() and (o.iters == r.iters).all().item()
    y0, sig0 = ys[0]
    rs = oracle.decode(c, y0[:64].cpu().numpy(), sig0, p, 300, frame_base=0, threads=4)
    same(host(ng.Outputs(outs[0].bits[:64], outs[0].iters[:64], outs[0].converged[:64])), rs)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ng.ngdbf_decode_batch(jobs, s)
    torch.cuda.synchronize()
    for rep in range(2):
        for o in outs:
            o.iters.fill_(-1)
        torch.cuda.synchronize()
        say("replay", rep)
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert (o.bits == r.bits).all().item() and (o.iters == r.iters).all().item()
    del g
    dc.close()
