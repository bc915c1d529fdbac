"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle.

Decoded words, iteration counts, convergence flags and per-round flip masks
must be identical (integer results: bit-exact).  Inputs come from the seeded
generators in ``synth``; the oracle sees the same host copy of y.
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
    ng.lib()  # fail loudly if the library is missing
    oracle.build(force=False)
    return torch


_CODES = {}


def dev_code(name_or_code):
    c = codes.named_code(name_or_code) if isinstance(name_or_code, str) else name_or_code
    if c.name not in _CODES:
        _CODES[c.name] = (c, ng.Code.from_ldpc(c))
    return _CODES[c.name]


def run_both(torch, code, y_host, sigma, params, seed, frame_base=0, trace=False):
    """Decode y on the GPU and with the oracle; return both results."""
    c, dc = dev_code(code)
    y_dev = torch.from_numpy(y_host).cuda()
    sig_dev = torch.from_numpy(np.asarray(sigma, dtype=np.float32)).cuda() if np.ndim(sigma) else float(sigma)
    gp = ng.Params(**params.__dict__)
    out = ng.decode(dc, y_dev, sig_dev, gp, seed, frame_base=frame_base, trace=trace)
    torch.cuda.synchronize()
    g = (out.bits.cpu().numpy(), out.iters.cpu().numpy(), out.converged.cpu().numpy(),
         out.trace.cpu().numpy() if trace else None)
    r = oracle.decode(c, y_host, sigma, params, seed, frame_base=frame_base, trace=trace, threads=8)
    return g, r


def assert_same(g, r, trace=False):
    bits, iters, conv, tr = g
    assert (iters == r.iters).all(), f"iters differ at frames {np.nonzero(iters != r.iters)[0][:10]}"
    assert (conv == r.converged).all()
    assert (bits == r.bits).all(), f"bits differ at frames {np.nonzero((bits != r.bits).any(1))[0][:10]}"
    if trace:
        assert (tr == r.trace).all()


P_C1 = oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=100, smooth_window=0)


def p_heur(ebn0):
    lam = 0.99 if ebn0 < 3.5 else 0.97 if ebn0 < 4.0 else 0.94 if ebn0 < 4.25 else 0.90
    return oracle.Params(w=0.75, theta=-0.9, lam=lam, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)


# ------------------------------------------------------------- noise source

def test_noise_radius_exhaustive(torch_dev):
    """rho(m) on the device equals the oracle's for all m in [1, 2^24]."""
    torch = torch_dev
    say("probe radius 2^24")
    out = torch.empty(1 << 24, dtype=torch.float32, device="cuda")
    ng.ngdbf_noise_probe(0, 1, 1 << 24, 0, 0, 0, out, None, None)
    got = out.cpu().numpy()
    ref = oracle.rho_range(1, 1 << 24)
    bad = np.nonzero(got.view(np.uint32) != ref.view(np.uint32))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first m = {bad[:5] + 1}"


def test_noise_angle_exhaustive(torch_dev):
    """cos/sin of 2 pi i 2^-24 on the device equal the oracle's for every i."""
    torch = torch_dev
    say("probe angle 2^24")
    c = torch.empty(1 << 24, dtype=torch.float32, device="cuda")
    s = torch.empty(1 << 24, dtype=torch.float32, device="cuda")
    ng.ngdbf_noise_probe(1, 0, 1 << 24, 0, 0, 0, c, s, None)
    rc, rs = oracle.sincos_range(0, 1 << 24)
    assert (c.cpu().numpy().view(np.uint32) == rc.view(np.uint32)).all()
    assert (s.cpu().numpy().view(np.uint32) == rs.view(np.uint32)).all()


@pytest.mark.parametrize("seed,frame,it", [(1, 0, 0), (2**40 + 3, 2**32 + 5, 299), (7, 123456, 17)])
def test_noise_quads(torch_dev, seed, frame, it):
    torch = torch_dev
    say("probe quads", seed, frame, it)
    nq = 1 << 16
    out = torch.empty(4 * nq, dtype=torch.float32, device="cuda")
    ng.ngdbf_noise_probe(2, 0, nq, seed, frame, it, out, None, None)
    ref = oracle.noise_block(seed, frame, it, 0, nq)
    assert (out.cpu().numpy().view(np.uint32) == ref.view(np.uint32)).all()


# ------------------------------------------------------------- decode parity

def test_config1_plain_c96_10000_frames(torch_dev):
    """Plain M-NGDBF, (3,6) N=96, 4 dB, eta 0.9, w 0.75, theta -0.6, T 100,
    10,000 frames, seed 1: bit-exact."""
    c = codes.named_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(4.0, c.rate))
    y = channel.bpsk_awgn(10000, c.n, sig, seed=1)
    say("config1 C96 10000")
    g, r = run_both(torch_dev, "C96", y, sig, P_C1, seed=1)
    assert_same(g, r)
    assert (r.iters == 100).sum() > 100 and (r.iters == 0).sum() > 10  # both ends exercised


@pytest.mark.parametrize("name,frames,ebn0", [("C96", 600, 2.0), ("C1008", 200, 2.5)])
def test_trace_parity(torch_dev, name, frames, ebn0):
    """Every flip decision of every round matches (Sec. III-B Step 3b)."""
    c = codes.named_code(name)
    sig = np.float32(channel.sigma_from_ebn0(ebn0, c.rate))
    y = channel.bpsk_awgn(frames, c.n, sig, seed=31)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=120, smooth_window=64)
    say("trace", name, frames)
    g, r = run_both(torch_dev, name, y, sig, p, seed=32, trace=True)
    assert_same(g, r, trace=True)


@pytest.mark.parametrize("ebn0", [2.0, 3.5, 5.0])
def test_heuristic_sm_ngdbf_c1008(torch_dev, ebn0):
    """Adaptive threshold + smoothing, T = 300, the lambda schedule by SNR."""
    c = codes.named_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(ebn0, c.rate))
    y = channel.bpsk_awgn(1500, c.n, sig, seed=int(ebn0 * 10))
    say("SM C1008", ebn0)
    g, r = run_both(torch_dev, "C1008", y, sig, p_heur(ebn0), seed=2000 + int(ebn0 * 10))
    assert_same(g, r)


@pytest.mark.parametrize("variant", ["plain", "heur"])
def test_c4000(torch_dev, variant):
    c = codes.named_code("C4000")
    sig = np.float32(channel.sigma_from_ebn0(2.5, c.rate))
    y = channel.bpsk_awgn(300, c.n, sig, seed=41)
    p = p_heur(2.5) if variant == "heur" else oracle.Params(**{**P_C1.__dict__, "t_max": 300})
    say("C4000", variant)
    g, r = run_both(torch_dev, "C4000", y, sig, p, seed=42)
    assert_same(g, r)


@pytest.mark.parametrize("fmt", ["f32", "i8"])
def test_c2048_high_rate(torch_dev, fmt):
    """(6,32) N=2048 high-rate code, theta -0.7, eta 0.65, Y_max 2.0, w 0.125,
    T 300; float32 and int8 storage."""
    c = codes.named_code("C2048")
    sig = np.float32(channel.sigma_from_ebn0(4.0, c.rate))
    y = channel.bpsk_awgn(500, c.n, sig, seed=51)
    if fmt == "i8":
        y = channel.quantize_int8(y)
    p = oracle.Params(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0, t_max=300)
    say("C2048", fmt)
    g, r = run_both(torch_dev, "C2048", y, sig, p, seed=52)
    assert_same(g, r)


# ------------------------------------------------------------- edge cases

def test_empty_batch_is_a_no_op(torch_dev):
    torch = torch_dev
    c, dc = dev_code("C96")
    y = torch.empty((0, c.n), dtype=torch.float32, device="cuda")
    out = ng.decode(dc, y, 0.7, ng.Params(), 1)
    torch.cuda.synchronize()
    assert out.bits.shape == (0, 12)


@pytest.mark.parametrize("case", ["T0", "eta0", "noclamp", "window_gt_T", "per_frame_sigma",
                                  "frame_base", "noiseless", "lambda_small"])
def test_edge_cases(torch_dev, case):
    c = codes.named_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(2.5, c.rate))
    y = channel.bpsk_awgn(700, c.n, sig, seed=61)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.98, eta=0.95, ymax=2.5, t_max=60, smooth_window=64)
    s = sig
    fb = 0
    if case == "T0":
        p.t_max = 0
    elif case == "eta0":
        p.eta = 0.0
    elif case == "noclamp":
        p.ymax = 0.0
        y = (y * 2.0).astype(np.float32)
    elif case == "window_gt_T":
        p.smooth_window = 200
    elif case == "per_frame_sigma":
        s = channel.frame_sigmas(700, 2.0, 5.0, c.rate, seed=62)
    elif case == "frame_base":
        fb = 2**33 + 17
    elif case == "noiseless":
        y = np.ones_like(y)
    elif case == "lambda_small":
        p.lam = 0.5
    say("edge", case)
    g, r = run_both(torch_dev, "C96", y, s, p, seed=63, frame_base=fb, trace=True)
    assert_same(g, r, trace=True)


@pytest.mark.parametrize("shape", [(1, 4, 8), (2, 2, 1), (4, 1, 1), (8, 1, 1), (16, 1, 1)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("t_max", [200, 300])
def test_base_kernel_every_shape(torch_dev, shape, t_max):
    """The base kernel on every launch shape that holds C1008: code tables in
    LDS (one and two waves per frame) or read from global memory (four or more
    waves), 8-bit (T <= 255) or 16-bit flip counts."""
    c, dc = dev_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(2.5, c.rate))
    y = channel.bpsk_awgn(150, c.n, sig, seed=66)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=t_max, smooth_window=64)
    say("base shape", shape, t_max)
    ng.ngdbf_code_set_shape(dc.handle, *shape)
    try:
        g, r = run_both(torch_dev, "C1008", y, sig, p, seed=67, trace=True)
    finally:
        ng.ngdbf_code_set_shape(dc.handle, 0, 0, 0)
    assert_same(g, r, trace=True)


def test_frame_queue_reuse(torch_dev):
    """Frames come from a per-launch queue taken from a ring of 1024 and reset
    by the launch's last taker: 4200 launches in a row (every queue used more
    than once, the first ones again) give the same decode each time."""
    torch = torch_dev
    c, dc = dev_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(3.0, c.rate))
    y = channel.bpsk_awgn(40, c.n, sig, seed=70)
    p = ng.Params(**P_C1.__dict__)
    y_dev = torch.from_numpy(y).cuda()
    ref = ng.decode(dc, y_dev, float(sig), p, 71)
    out = ng.decode(dc, y_dev, float(sig), p, 71)
    say("queue reuse: 4200 launches")
    for i in range(4200):
        ng.decode(dc, y_dev, float(sig), p, 71, out=out)
        if i % 700 == 699:
            torch.cuda.synchronize()
            assert torch.equal(out.iters, ref.iters) and torch.equal(out.bits, ref.bits), f"launch {i}"
    torch.cuda.synchronize()
    assert torch.equal(out.iters, ref.iters) and torch.equal(out.bits, ref.bits)
    r = oracle.decode(c, y, sig, P_C1, 71)
    assert (ref.iters.cpu().numpy() == r.iters).all()


def test_graph_replays_beside_direct_launches(torch_dev):
    """Launches recorded into a graph take their queues from a ring of their
    own: replays of a captured decode (and a captured traced decode, whose
    trace rows are cleared by a kernel on every replay) interleaved with 1100
    direct launches on another stream, more than the direct ring holds,
    reproduce the eager results every time."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(3.5, c.rate))
    y = channel.bpsk_awgn(4096, c.n, sig, seed=75)
    gp = ng.Params(**p_heur(3.5).__dict__)
    y_dev = torch.from_numpy(y).cuda()
    ref = ng.decode(dc, y_dev, float(sig), gp, 76)
    ref_tr = ng.decode(dc, y_dev[:16], float(sig), gp, 78, trace=True)
    out_g = ng.decode(dc, y_dev, float(sig), gp, 76)
    out_tr = ng.decode(dc, y_dev[:16], float(sig), gp, 78, trace=True)
    y2 = y_dev[:64].contiguous()
    ref2 = ng.decode(dc, y2, float(sig), gp, 77)
    out2 = ng.decode(dc, y2, float(sig), gp, 77)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            ng.decode(dc, y_dev, float(sig), gp, 76, out=out_g, stream=cs)
            ng.decode(dc, y_dev[:16], float(sig), gp, 78, trace=True, out=out_tr, stream=cs)
    torch.cuda.synchronize()
    other = torch.cuda.Stream()
    say("graph replays beside 1100 direct launches")
    for i in range(1100):
        ng.decode(dc, y2, float(sig), gp, 77, out=out2, stream=other)
        if i % 100 == 50:
            out_g.iters.fill_(-1)
            out_tr.trace.fill_(0xFF)
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                g.replay()
        if i % 100 == 99:
            torch.cuda.synchronize()
            assert torch.equal(out_g.iters, ref.iters) and torch.equal(out_g.bits, ref.bits), f"replay {i}"
            assert torch.equal(out_tr.trace, ref_tr.trace) and torch.equal(out_tr.iters, ref_tr.iters)
            assert torch.equal(out2.iters, ref2.iters) and torch.equal(out2.bits, ref2.bits), f"direct {i}"
    torch.cuda.synchronize()
    del g


def test_long_launch_beside_many_short_ones(torch_dev):
    """A direct launch passes over ring queues still held: eight long decodes
    queued on one stream (a C4000 frame that never converges, 65535 rounds
    each) hold their queues while 1100 one-frame decodes on another stream
    take and free the rest of the ring, more than it holds; every short decode
    equals the oracle and every long one the same decode run alone.  The short
    decodes go to a stream that runs beside the long ones (streams can share a
    hardware queue, whose launches then run one after another)."""
    import time

    torch = torch_dev
    c4, dc4 = dev_code("C4000")
    sig4 = np.float32(channel.sigma_from_ebn0(0.0, c4.rate))
    y4 = channel.bpsk_awgn(1, c4.n, sig4, seed=83)
    p_long = ng.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=65535, smooth_window=0)
    y4_dev = torch.from_numpy(y4).cuda()
    c, dc = dev_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(3.0, c.rate))
    y = channel.bpsk_awgn(1100, c.n, sig, seed=84)
    y_dev = torch.from_numpy(y).cuda()
    gp = ng.Params(**P_C1.__dict__)
    outs = [ng.alloc_outputs(dc, 1, "cuda") for _ in range(1100)]
    probe = ng.alloc_outputs(dc, 1, "cuda")
    torch.cuda.synchronize()
    long_s = torch.cuda.Stream()
    candidates = [torch.cuda.Stream() for _ in range(4)]
    say("eight 65535-round C4000 decodes beside 1100 one-frame C96 decodes")
    t0 = time.perf_counter()
    longs = [ng.decode(dc4, y4_dev, float(sig4), p_long, 85, stream=long_s) for _ in range(8)]
    long_done = torch.cuda.Event()
    long_done.record(long_s)
    short_s = None
    for cand in candidates:
        ng.decode(dc, y_dev[:1], float(sig), gp, 86, out=probe, stream=cand)
        cand.synchronize()
        if not long_done.query():
            short_s = cand
            break
    if short_s is None:
        torch.cuda.synchronize()
        pytest.skip("no stream ran beside the long decodes")
    for i in range(1100):
        # frame i has its own noise key (seed, i), as in one decode of all 1100
        ng.decode(dc, y_dev[i:i + 1], float(sig), gp, 86, frame_base=i, out=outs[i], stream=short_s)
        if i % 100 == 99:
            short_s.synchronize()
    short_s.synchronize()
    t_short = time.perf_counter() - t0
    exercised = not long_done.query()
    torch.cuda.synchronize()
    t_long = time.perf_counter() - t0
    say(f"short decodes done after {t_short * 1e3:.1f} ms, long decodes after {t_long * 1e3:.1f} ms")
    assert exercised, "the long decodes ended before the short ones wrapped the ring"
    r = oracle.decode(c, y, sig, P_C1, 86)
    assert (torch.cat([o.iters for o in outs]).cpu().numpy() == r.iters).all()
    assert (torch.cat([o.bits for o in outs]).cpu().numpy() == r.bits).all()
    alone = ng.decode(dc4, y4_dev, float(sig4), p_long, 85)
    torch.cuda.synchronize()
    assert int(alone.iters[0]) == 65535 and not bool(alone.converged[0])
    for o in longs:
        assert torch.equal(o.bits, alone.bits) and torch.equal(o.iters, alone.iters)


def test_settle_statistics(torch_dev):
    """The settle-test counters: every round of every frame evaluates ceil(n/2)
    pairs, a minority of them is transformed, and the decode is unchanged."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(3.5, c.rate))
    y = channel.bpsk_awgn(400, c.n, sig, seed=68)
    p = p_heur(3.5)
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    ng.ngdbf_code_set_stats(dc.handle, counters)
    try:
        g, r = run_both(torch, "C1008", y, sig, p, seed=69)
    finally:
        ng.ngdbf_code_set_stats(dc.handle, None)
    assert_same(g, r)
    evaluated, transformed = counters.cpu().tolist()
    say("pairs evaluated", evaluated, "transformed", transformed)
    assert evaluated == int(r.iters.astype(np.int64).sum()) * ((c.n + 1) // 2)
    assert 0 < transformed < evaluated // 4
    # detached: the counters stay as they are
    run_both(torch, "C1008", y[:8], sig, p, seed=69)
    assert counters.cpu().tolist() == [evaluated, transformed]


def test_every_frame_once_mixed_lengths(torch_dev):
    """2^18 frames of very different lengths (Eb/N0 drawn per frame from 1.5
    to 6 dB): the queue's takers drain their own counter and then the
    others'.  Every frame is decoded exactly once (outputs start at a
    sentinel; the settle counters equal the rounds summed over frames), and
    sampled frames equal the oracle's."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    F = 1 << 18
    s = channel.frame_sigmas(F, 1.5, 6.0, c.rate, seed=72)
    s_dev = torch.from_numpy(s).cuda()
    y = channel.bpsk_awgn_device(F, c.n, s_dev, seed=73)
    p = p_heur(3.5)
    gp = ng.Params(**p.__dict__)
    say("every frame once: 2^18 frames, 1.5 .. 6 dB")
    out = ng.decode(dc, y, s_dev, gp, 74)
    torch.cuda.synchronize()
    first = out.iters.clone()
    out.iters.fill_(-1)
    out.converged.fill_(2)
    out.bits.fill_(0xA5)
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    ng.ngdbf_code_set_stats(dc.handle, counters)
    try:
        ng.decode(dc, y, s_dev, gp, 74, out=out)
        torch.cuda.synchronize()
    finally:
        ng.ngdbf_code_set_stats(dc.handle, None)
    iters = out.iters.cpu().numpy()
    assert (iters >= 0).all() and (iters <= p.t_max).all(), "a frame was not decoded"
    assert (out.converged.cpu().numpy() <= 1).all()
    assert torch.equal(out.iters, first)
    evaluated = int(counters[0].item())
    assert evaluated == int(iters.astype(np.int64).sum()) * ((c.n + 1) // 2), "a frame was decoded twice"
    assert iters.min() < 20 and iters.max() == p.t_max
    for start in (0, F // 2 + 3, F - 32):
        yh = y[start:start + 32].cpu().numpy()
        r = oracle.decode(c, yh, s[start:start + 32], p, 74, frame_base=start, threads=8)
        g = (out.bits[start:start + 32].cpu().numpy(), iters[start:start + 32],
             out.converged[start:start + 32].cpu().numpy(), None)
        assert_same(g, r)


@pytest.mark.parametrize("t_max", [5000, 9000])
def test_long_adaptive_schedule(torch_dev, t_max):
    """Adaptive thresholds over thousands of rounds: the base kernel's table of
    theta lambda^u (T = 5000, fewer frames per workgroup to fit it) and the
    multi-bit kernel that keeps thresholds in registers (T = 9000)."""
    c = codes.named_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(1.0, c.rate))
    y = channel.bpsk_awgn(60, c.n, sig, seed=64)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.999, eta=0.95, ymax=2.5, t_max=t_max,
                      smooth_window=64)
    say("long schedule", t_max)
    g, r = run_both(torch_dev, "C96", y, sig, p, seed=65)
    assert (r.iters == t_max).any(), "some frame should use the whole schedule"
    assert_same(g, r)


def test_ragged_irregular_code(torch_dev):
    """n not a multiple of 4 or 8, irregular row and column degrees."""
    rng = np.random.Generator(np.random.PCG64(71))
    n, m = 103, 47
    rows = []
    for i in range(m):
        deg = int(rng.integers(3, 9))
        rows.append(sorted(rng.choice(n, size=deg, replace=False).tolist()))
    covered = set(b for r in rows for b in r)
    for b in range(n):
        if b not in covered:
            rows[b % m].append(b)
    code = codes.from_rows("irr103", n, rows)
    sig = np.float32(0.75)
    y = channel.bpsk_awgn(900, n, sig, seed=72)
    p = oracle.Params(w=0.6, theta=-0.8, lam=0.99, eta=0.9, ymax=2.5, t_max=80, smooth_window=16)
    say("ragged irregular")
    g, r = run_both(torch_dev, code, y, sig, p, seed=73, trace=True)
    assert_same(g, r, trace=True)


# ------------------------------------------------------------- full size, sampled

def test_full_size_c1008_sampled(torch_dev):
    """2^20 frames of C1008 at 3.5 dB (the benchmark's launch): decode all on
    the GPU, then check sampled blocks (first, middle, last frames) against
    the oracle run on the same samples with the same frame indices."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    F = 1 << 20
    sig = float(np.float32(channel.sigma_from_ebn0(3.5, c.rate)))
    say("full size C1008 2^20")
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=99)
    p = p_heur(3.5)
    out = ng.decode(dc, y, sig, ng.Params(**p.__dict__), 2035)
    torch.cuda.synchronize()
    for start in (0, F // 2 + 13, F - 64):
        yh = y[start:start + 64].cpu().numpy()
        r = oracle.decode(c, yh, np.float32(sig), p, 2035, frame_base=start, threads=8)
        g = (out.bits[start:start + 64].cpu().numpy(), out.iters[start:start + 64].cpu().numpy(),
             out.converged[start:start + 64].cpu().numpy(), None)
        assert_same(g, r)
    it = out.iters.double().mean().item()
    say("mean iterations", it)
    assert 5 < it < 100
