"""GPU parity for the parameter corners and full-size configurations the
measurements use: thresholds theta >= 0 with adaptation, per-frame sigma
arrays holding zeros and negative values, the (6,32) code's searched
parameter set, the N=4000 SM-NGDBF point and the default benchmark's 2^22-frame
four-code batch sampled from full-size launches, and the binary32 decoder
against the binary64 oracle at the headline point.

Integer results (decoded words, iteration counts, flags, flip masks) must be
identical to the oracle's; the binary64 comparison is statistical (FER and
BER within binomial intervals, Sec. IV-A simulates in double precision).
"""
import math
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


_CODES = {}


def dev_code(name):
    if name not in _CODES:
        c = codes.named_code(name)
        _CODES[name] = (c, ng.Code.from_ldpc(c))
    return _CODES[name]


def run_both(torch, name, y_host, sigma, params, seed, trace=False):
    c, dc = dev_code(name)
    y_dev = torch.from_numpy(y_host).cuda()
    sig_dev = torch.from_numpy(np.asarray(sigma, dtype=np.float32)).cuda() if np.ndim(sigma) else float(sigma)
    out = ng.decode(dc, y_dev, sig_dev, ng.Params(**params.__dict__), seed, trace=trace)
    torch.cuda.synchronize()
    r = oracle.decode(c, y_host, sigma, params, seed, trace=trace, threads=8)
    assert (out.iters.cpu().numpy() == r.iters).all(), \
        f"iters differ at frames {np.nonzero(out.iters.cpu().numpy() != r.iters)[0][:10]}"
    assert (out.converged.cpu().numpy() == r.converged).all()
    assert (out.bits.cpu().numpy() == r.bits).all()
    if trace:
        assert (out.trace.cpu().numpy() == r.trace).all(), "flip decisions differ"
    return r


# ------------------------------------------------------------- threshold signs

# (theta, lambda, eta): Sec. III-B takes theta < 0; the decoder accepts any
# finite theta, and with theta > 0 and lambda < 1 a bit that flips keeps a
# larger threshold than one that does not (theta lambda^u falls with u)
THETA_CASES = {
    "theta_pos_0.4": (0.4, 0.9, 0.3),
    "theta_pos_1.0": (1.0, 0.8, 0.1),
    "theta_zero": (0.0, 0.95, 0.9),
    "theta_pos_plain": (0.2, 1.0, 0.6),
}


@pytest.mark.parametrize("name,frames,ebn0", [("C96", 500, 2.5), ("C1008", 150, 3.0)])
@pytest.mark.parametrize("case", sorted(THETA_CASES))
def test_threshold_signs_trace(torch_dev, case, name, frames, ebn0):
    theta, lam, eta = THETA_CASES[case]
    c, _ = dev_code(name)
    sig = np.float32(channel.sigma_from_ebn0(ebn0, c.rate))
    y = channel.bpsk_awgn(frames, c.n, sig, seed=81)
    p = oracle.Params(w=0.75, theta=theta, lam=lam, eta=eta, ymax=2.5, t_max=80, smooth_window=32)
    say("threshold sign", case, name)
    r = run_both(torch_dev, name, y, sig, p, seed=82, trace=True)
    # the flips the settle test must not miss happen: some frames run long
    assert r.trace.any()


# ------------------------------------------------------------- sigma arrays

def odd_sigmas(frames, rate, seed):
    """Channel sigma per frame from 2 to 5 dB, and the sigma handed to the
    decoder: the same with every third frame negated (the draw enters as
    fl(eta sigma) z, whose magnitude the noise skip bounds), every fifth
    frame 0 (no perturbation: the deterministic GDBF rule on a noisy frame)
    and every tenth -0."""
    s = channel.frame_sigmas(frames, 2.0, 5.0, rate, seed=seed)
    idx = np.arange(frames)
    d = np.where(idx % 3 == 1, -s, s)
    d = np.where(idx % 5 == 2, np.float32(0.0), d)
    d[idx % 10 == 7] = np.float32(-0.0)
    return s, d.astype(np.float32)


SIGMA_DECODERS = {
    # base decoder: adaptive thresholds, smoothing, exact noise skip
    "multi_adaptive": dict(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=100, smooth_window=64),
    "multi_plain": dict(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=100, smooth_window=0),
    # single-bit argmin by bounds on the draws
    "single": dict(w=0.75, theta=-0.6, lam=1.0, eta=1.0, ymax=2.5, t_max=60, smooth_window=0, variant=1),
    # quantized multi-bit with per-bit draws (settle test in half steps)
    "quantized": dict(w=0.75, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75, t_max=100, smooth_window=64,
                      quant_bits=4),
}


@pytest.mark.parametrize("name,frames", [("C96", 600), ("C1008", 120)])
@pytest.mark.parametrize("dec", sorted(SIGMA_DECODERS))
def test_sigma_array_with_zero_and_negative_values(torch_dev, dec, name, frames):
    c, _ = dev_code(name)
    s_channel, s = odd_sigmas(frames, c.rate, seed=83)
    y = channel.bpsk_awgn(frames, c.n, s_channel, seed=84)
    p = oracle.Params(**SIGMA_DECODERS[dec])
    say("sigma array", dec, name)
    r = run_both(torch_dev, name, y, s, p, seed=85, trace=p.variant == 0)
    assert (r.iters[s == 0] > 0).any(), "the zero-sigma frames should need rounds"


# ------------------------------------------------------------- full-size configurations

def sampled_blocks(torch, name, y_dev, sigma, params, seed, out, frames, block=48):
    """Oracle parity on the first, a middle and the last frames of a launch."""
    c, _ = dev_code(name)
    for start in (0, frames // 2 + 11, frames - block):
        yh = y_dev[start:start + block].cpu().numpy()
        r = oracle.decode(c, yh, np.float32(sigma), params, seed, frame_base=start, threads=8)
        assert (out.iters[start:start + block].cpu().numpy() == r.iters).all(), f"iters, block {start}"
        assert (out.converged[start:start + block].cpu().numpy() == r.converged).all()
        assert (out.bits[start:start + block].cpu().numpy() == r.bits).all(), f"bits, block {start}"


SEARCHED_C2048 = oracle.Params(w=0.162, theta=-0.287, lam=1.0, eta=0.613, ymax=2.0, t_max=300)


@pytest.mark.parametrize("fmt", ["f32", "i8"])
def test_c2048_searched_set_full_size(torch_dev, fmt):
    """The (6,32) N=2048 code with the successive-approximation parameters
    (w 0.162, theta -0.287, eta 0.613, Y_max 2.0, T 300) at 4.5 dB: a whole
    2^21-frame launch (float32 or int8 samples), sampled blocks against the
    oracle; plus 400 host frames decoded whole."""
    torch = torch_dev
    c, dc = dev_code("C2048")
    sig = float(np.float32(channel.sigma_from_ebn0(4.5, c.rate)))
    yh = channel.bpsk_awgn(400, c.n, sig, seed=86)
    if fmt == "i8":
        yh = channel.quantize_int8(yh)
    say("C2048 searched, 400 frames", fmt)
    run_both(torch, "C2048", yh, sig, SEARCHED_C2048, seed=87)
    F = 1 << 21
    say("C2048 searched, 2^21 frames", fmt)
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=88)
    if fmt == "i8":
        y = channel.quantize_int8(y)
    out = ng.decode(dc, y, sig, ng.Params(**SEARCHED_C2048.__dict__), 2045)
    torch.cuda.synchronize()
    sampled_blocks(torch, "C2048", y, sig, SEARCHED_C2048, 2045, out, F)
    it = out.iters.double().mean().item()
    say("mean iterations", it)
    assert 5 < it < 40
    del y, out
    torch.cuda.empty_cache()


def test_c4000_sm_ngdbf_full_size(torch_dev):
    """SM-NGDBF on the (3,6) N=4000 code at 3.5 dB (theta -0.9, eta 0.95,
    lambda 0.97, W 64, T 300): a whole 2^20-frame launch, sampled blocks
    against the oracle."""
    torch = torch_dev
    c, dc = dev_code("C4000")
    F = 1 << 20
    sig = float(np.float32(channel.sigma_from_ebn0(3.5, c.rate)))
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)
    say("C4000 SM 3.5 dB, 2^20 frames")
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=89)
    out = ng.decode(dc, y, sig, ng.Params(**p.__dict__), 2035)
    torch.cuda.synchronize()
    sampled_blocks(torch, "C4000", y, sig, p, 2035, out, F, block=32)
    del y, out
    torch.cuda.empty_cache()


def test_mix4_full_size_batch_sampled(torch_dev):
    """The default benchmark's batch as bench.py times it: C96 : C1008 : C2048
    : C4000 = 2^21 : 2^20 : 2^19 : 2^19 frames, per-frame Eb/N0 uniform in
    2..5 dB, per-code parameters, frames from the device channel, each code at
    the shape the autotuner picks on a tuning sample of its own, one
    ngdbf_decode_batch; the first, a middle and the last frames of every code
    against the oracle."""
    import bench
    from paper_1402_2773_amd import sweep

    torch = torch_dev
    items = []
    for idx, (name, frames, params) in enumerate(bench.MIX4):
        c = codes.named_code(name)
        dc = ng.Code.from_ldpc(c)  # a handle of its own: the tuned shape stays on it
        p = ng.Params(**params)
        n_s = min(frames, 1 << 17)
        sig_s = torch.from_numpy(channel.frame_sigmas(n_s, 2.0, 5.0, c.rate, seed=900 + idx)).cuda()
        y_s = ng.channel(c.n, n_s, sig_s, seed=sweep.channel_seed(920 + idx))
        best, _ = ng.autotune(dc, y_s, sig_s, p, 940 + idx)
        del y_s, sig_s
        sig_h = channel.frame_sigmas(frames, 2.0, 5.0, c.rate, seed=300 + idx)
        sig = torch.from_numpy(sig_h).cuda()
        y = ng.channel(c.n, frames, sig, seed=sweep.channel_seed(320 + idx))
        say(name, frames, "frames at the tuned shape", list(best))
        items.append(dict(c=c, dc=dc, y=y, sig=sig, sig_h=sig_h, params=params, p=p, seed=320 + idx,
                          frames=frames, out=ng.alloc_outputs(dc, frames, "cuda")))
    jobs = [ng.job(it["dc"], it["y"], it["sig"], it["p"], it["seed"], it["out"]) for it in items]
    say("one batch of 2^22 frames")
    ng.ngdbf_decode_batch(jobs, None)
    torch.cuda.synchronize()
    block = 16
    for it in items:
        F, c = it["frames"], it["c"]
        for start in (0, F // 2 + 5, F - block):
            yh = it["y"][start:start + block].cpu().numpy()
            r = oracle.decode(c, yh, it["sig_h"][start:start + block], oracle.Params(**it["params"]),
                              it["seed"], frame_base=start, threads=8)
            o = it["out"]
            assert (o.iters[start:start + block].cpu().numpy() == r.iters).all(), f"{c.name} iters {start}"
            assert (o.converged[start:start + block].cpu().numpy() == r.converged).all()
            assert (o.bits[start:start + block].cpu().numpy() == r.bits).all(), f"{c.name} bits {start}"
    for it in items:
        it["dc"].close()
    del items, jobs
    torch.cuda.empty_cache()


# ------------------------------------------------------------- binary32 against binary64

def wilson(k, n, z):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


def test_binary32_against_binary64_headline(torch_dev):
    """C1008 SM-NGDBF at 3.5 dB (lambda 0.97, W 64, T 300): the GPU's binary32
    decode of 2^20 frames and the oracle's binary64 decoder (adaptive
    thresholds and smoothing in double, draws from the same Philox words) on
    the first 16384 of them agree in FER and BER within 99.9% intervals
    (frame errors binomial; bit errors clustered by frame)."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    F, F64 = 1 << 20, 1 << 14
    sig = float(np.float32(channel.sigma_from_ebn0(3.5, c.rate)))
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)
    say("binary32 2^20 frames on the GPU")
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=90)
    out = ng.decode(dc, y, sig, ng.Params(**p.__dict__), 2035)
    torch.cuda.synchronize()
    e32 = oracle.unpack_bits(out.bits.cpu().numpy(), c.n).sum(1).astype(np.int64)
    say("binary64 oracle, 2^14 frames")
    r64 = oracle.decode(c, y[:F64].cpu().numpy(), np.float32(sig), p, 2035, threads=16, f64=True)
    e64 = oracle.unpack_bits(r64.bits, c.n).sum(1).astype(np.int64)
    z = 3.29
    fer32, fer64 = (e32 > 0).mean(), (e64 > 0).mean()
    lo, hi = wilson(int((e64 > 0).sum()), F64, z)
    say("FER binary32", fer32, "binary64", fer64, "interval", lo, hi)
    assert lo <= fer32 <= hi
    # the difference of the two proportions, pooled
    pp = ((e32 > 0).sum() + (e64 > 0).sum()) / (F + F64)
    assert abs(fer32 - fer64) <= z * math.sqrt(pp * (1 - pp) * (1 / F + 1 / F64))
    # BER: per-frame error counts, normal interval on their mean
    ber32, ber64 = e32.mean() / c.n, e64.mean() / c.n
    sd = math.sqrt(e64.var(ddof=1) / F64 + e32.var(ddof=1) / F) / c.n
    say("BER binary32", ber32, "binary64", ber64, "sd", sd)
    assert abs(ber32 - ber64) <= z * sd
    # on the common frames most trajectories are identical
    same = (out.iters[:F64].cpu().numpy() == r64.iters).mean()
    say("frames with identical iteration counts", same)
    assert same > 0.99
    del y, out
    torch.cuda.empty_cache()


# ------------------------------------------------------------- busy rounds

def _round_stats(c, y, trace, iters):
    """Per round: unsatisfied checks at its start and checks it toggles."""
    ht = c.dense().astype(np.float32).T
    x0 = (y < 0).astype(np.float32)
    fl = oracle.unpack_bits(trace, c.n).astype(np.float32)
    unsat, events = [], []
    for f in range(len(y)):
        m = fl[f, : int(iters[f])]
        if not len(m):
            continue
        xe = (x0[f] + np.vstack([np.zeros((1, c.n), np.float32), np.cumsum(m, 0)[:-1]])) % 2
        unsat.append(((xe @ ht).astype(np.int64) & 1).sum(1))
        events.append(((m @ ht).astype(np.int64) & 1).sum(1))
    return np.concatenate(unsat), np.concatenate(events)


@pytest.mark.parametrize("name,frames,event_list", [("C1008", 200, 256), ("C4000", 40, 1024)])
def test_busy_rounds_unlisted_and_full_event_list(torch_dev, name, frames, event_list):
    """A threshold above most a_k with strong perturbation flips about half
    the bits of a round (Sec. III-B Step 3b), so about half the checks
    toggle: rounds that start with more than 64 unsatisfied checks have their
    events applied by the owners of s without a list, and rounds that start
    with fewer can toggle more checks than the frame's event list holds (256
    per wave), so the owners apply the excess themselves.  Whole flip traces
    must still match the oracle's."""
    c, _ = dev_code(name)
    y = channel.bpsk_awgn(frames, c.n, 0.3, seed=41)
    p = oracle.Params(w=0.75, theta=3.0, lam=1.0, eta=1.0, ymax=2.5, t_max=12, smooth_window=0)
    say(f"busy rounds {name} frames={frames}")
    r = run_both(torch_dev, name, y, 1.0, p, seed=43, trace=True)
    unsat, events = _round_stats(c, y, r.trace, r.iters)
    assert (unsat > 64).sum() > 50, "the case must hold rounds applied without a list"
    assert ((unsat <= 64) & (events > event_list)).sum() >= 1, "the case must overflow the event list"


# ------------------------------------------------------------- int8 samples, one wave per frame

@pytest.mark.parametrize("name,frames,ebn0,params", [
    ("C96", 800, 3.0, oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=100)),
    ("C1008", 200, 3.0, oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=300,
                                      smooth_window=64)),
])
def test_int8_samples_one_wave_per_frame(torch_dev, name, frames, ebn0, params):
    """int8 storage (y_q = clamp(rint(16 y)), decoded as y_q / 16) through the
    one-wave instances of the base kernel, with a share of exact zeros
    (sign(0) = +1) and saturated samples: whole flip traces must match."""
    c, _ = dev_code(name)
    sig = float(np.float32(channel.sigma_from_ebn0(ebn0, c.rate)))
    y = channel.quantize_int8(channel.bpsk_awgn(frames, c.n, sig, seed=95))
    rng = np.random.Generator(np.random.PCG64(96))
    y[rng.random(y.shape) < 0.02] = 0
    y[rng.random(y.shape) < 0.01] = 127
    assert (y == 0).mean() > 0.01
    say(f"int8 {name} frames={frames}")
    run_both(torch_dev, name, y, sig, params, seed=97, trace=True)
