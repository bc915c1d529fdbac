"""GPU parity of the extended decoders against the oracle: single-bit flips
(S-NGDBF, S-GDBF), mode switching, the quantized decoder and shift-register
noise reuse, on single- and multi-wave frames, plus the objective kernel.
Decoded words, iteration counts, flags and per-round flip masks must match
bit for bit."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1402_2773_amd as ng
from synth import channel, codes

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def dev_code(code):
    c = codes.named_code(code) if isinstance(code, str) else code
    if c.name not in _CODES:
        _CODES[c.name] = (c, ng.Code.from_ldpc(c))
    return _CODES[c.name]


def run_both(torch, code, y_host, sigma, p, seed, frame_base=0, trace=True, shape=None):
    c, dc = dev_code(code)
    if shape:
        ng.ngdbf_code_set_shape(dc.handle, *shape)
    try:
        y_dev = torch.from_numpy(y_host).cuda()
        sig = torch.from_numpy(np.asarray(sigma, dtype=np.float32)).cuda() if np.ndim(sigma) else float(sigma)
        out = ng.decode(dc, y_dev, sig, ng.Params(**p.__dict__), seed, frame_base=frame_base, trace=trace)
        torch.cuda.synchronize()
    finally:
        if shape:
            ng.ngdbf_code_set_shape(dc.handle, 0, 0, 0)
    g = (out.bits.cpu().numpy(), out.iters.cpu().numpy(), out.converged.cpu().numpy(),
         out.trace.cpu().numpy() if trace else None)
    r = oracle.decode(c, y_host, sigma, p, seed, frame_base=frame_base, trace=trace, threads=8)
    return g, r


def assert_same(g, r, trace=True):
    bits, iters, conv, tr = g
    assert (iters == r.iters).all(), f"iters differ at frames {np.nonzero(iters != r.iters)[0][:10]}"
    assert (conv == r.converged).all()
    assert (bits == r.bits).all(), f"bits differ at frames {np.nonzero((bits != r.bits).any(1))[0][:10]}"
    if trace:
        assert (tr == r.trace).all()


def P(**kw):
    base = dict(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=60, smooth_window=0)
    base.update(kw)
    return oracle.Params(**base)


CASES = {
    "s_ngdbf": P(variant=1, eta=1.0),
    "s_gdbf": P(variant=1, w=1.0, eta=0.0),
    "s_ngdbf_smoothed": P(variant=1, eta=0.8, smooth_window=16),
    "mode_switch_gdbf": P(variant=2, w=1.0, eta=0.0),
    "mode_switch_noisy": P(variant=2, eta=0.9, lam=0.97),
    "quant3": P(quant_bits=3, theta=-0.7, lam=0.98, eta=0.9, ymax=1.75, smooth_window=16),
    "quant4_reuse": P(quant_bits=4, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75, smooth_window=16,
                      noise_reuse=1),
    "quant5_reuse_plain": P(quant_bits=5, theta=-0.7, eta=0.9, ymax=1.75, noise_reuse=1),
    "reuse_fp32": P(noise_reuse=1, theta=-0.9, lam=0.98, eta=0.95, smooth_window=16),
    "quant4_single_reuse": P(variant=1, quant_bits=4, eta=0.9, ymax=1.75, noise_reuse=1),
    "quant1": P(quant_bits=1, theta=-0.5, eta=0.9, ymax=1.0),
    "quant3_single": P(variant=1, quant_bits=3, eta=0.9, ymax=1.75),
    "s_ngdbf_low_noise": P(variant=1, eta=0.05),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_variant_parity_c96(torch_dev, name):
    c = codes.named_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(3.0, c.rate))
    y = channel.bpsk_awgn(600, c.n, sig, seed=101)
    say("variant", name)
    g, r = run_both(torch_dev, "C96", y, sig, CASES[name], seed=102, frame_base=5)
    assert_same(g, r)


@pytest.mark.parametrize("name", ["s_ngdbf", "mode_switch_noisy", "quant4_reuse", "reuse_fp32"])
def test_variant_parity_c1008_per_frame_sigma(torch_dev, name):
    c = codes.named_code("C1008")
    s = channel.frame_sigmas(300, 2.5, 4.5, c.rate, seed=103)
    y = channel.bpsk_awgn(300, c.n, s, seed=104)
    p = oracle.Params(**{**CASES[name].__dict__, "t_max": 120})
    say("variant C1008", name)
    g, r = run_both(torch_dev, "C1008", y, s, p, seed=105)
    assert_same(g, r)


# (waves per frame, quads per lane, frames per block) covering single- and
# multi-wave frames for C1008 (252 quads)
SHAPES_1008 = [(1, 4, 2), (1, 4, 8), (1, 4, 12), (2, 2, 1), (4, 1, 1), (8, 1, 1), (16, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES_1008, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("name", ["s_ngdbf", "quant3_single", "mode_switch_noisy", "quant4_reuse"])
def test_variant_every_shape(torch_dev, name, shape):
    """The frame-wide reductions (argmin, objective) across 1..16 waves."""
    c = codes.named_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(3.0, c.rate))
    y = channel.bpsk_awgn(96, c.n, sig, seed=106)
    p = oracle.Params(**{**CASES[name].__dict__, "t_max": 80})
    say("variant shape", name, shape)
    g, r = run_both(torch_dev, "C1008", y, sig, p, seed=107, shape=shape)
    assert_same(g, r)


def test_variant_irregular_ragged_int8(torch_dev):
    """n = 103 (ragged), irregular degrees, int8 samples, quantized + reuse and
    single-bit, against the oracle."""
    rng = np.random.Generator(np.random.PCG64(108))
    n, m = 103, 47
    rows = []
    for i in range(m):
        rows.append(sorted(rng.choice(n, size=int(rng.integers(3, 9)), replace=False).tolist()))
    covered = set(b for r in rows for b in r)
    for b in range(n):
        if b not in covered:
            rows[b % m].append(b)
    code = codes.from_rows("irr103v", n, rows)
    sig = np.float32(0.75)
    y = channel.quantize_int8(channel.bpsk_awgn(500, n, sig, seed=109))
    for name in ("quant4_reuse", "s_ngdbf", "mode_switch_noisy"):
        say("irregular int8", name)
        g, r = run_both(torch_dev, code, y, sig, CASES[name], seed=110)
        assert_same(g, r)


def test_variant_golden_examples(torch_dev):
    """The hand-derived examples (tests/golden) on the device."""
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        exs = json.load(f)["examples"]
    for ex in exs:
        code = codes.from_rows("g_" + ex["name"], ex["n"], ex["rows"])
        d = ex["params"]
        p = oracle.Params(w=d["w"], theta=d["theta"], lam=d["lam"], eta=d["eta"], ymax=d["ymax"],
                          t_max=d["t_max"], smooth_window=d["smooth_window"],
                          variant=d.get("variant", 0), quant_bits=d.get("quant_bits", 0),
                          noise_reuse=d.get("noise_reuse", 0))
        y = np.array([ex["y"]], dtype=np.float32)
        say("golden", ex["name"])
        g, r = run_both(torch_dev, code, y, ex["sigma"], p, seed=123)
        assert_same(g, r)
        assert oracle.unpack_bits(g[0], code.n)[0].tolist() == ex["bits"]
        assert int(g[1][0]) == ex["iters"]


def test_reuse_long_T_and_T0(torch_dev):
    """Noise reuse with T = 0 (no stream), with a long T (large stream) and
    with T beyond the packed decoder's threshold table (general path)."""
    c = codes.named_code("C96")
    sig = np.float32(channel.sigma_from_ebn0(2.0, c.rate))
    y = channel.bpsk_awgn(200, c.n, sig, seed=111)
    for T in (0, 1, 1500, 5000):
        p = oracle.Params(**{**CASES["quant4_reuse"].__dict__, "t_max": T, "smooth_window": 0})
        say("reuse T", T)
        g, r = run_both(torch_dev, "C96", y, sig, p, seed=112, trace=T <= 100)
        assert_same(g, r, trace=T <= 100)


def test_objective_kernel_and_convergence_error(torch_dev):
    """f(x) of Sec. III-B on the device equals the oracle's, for decoded words
    and for the sent codeword (int8 and float32 samples); the convergence
    error of Sec. VI follows."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    sig = np.float32(channel.sigma_from_ebn0(5.0, c.rate))
    y = channel.bpsk_awgn(100, c.n, sig, seed=113)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=100, smooth_window=0)
    r = oracle.decode(c, y, sig, p, 114, threads=8)
    for yy in (y, channel.quantize_int8(y)):
        y_dev = torch.from_numpy(yy).cuda()
        bits_dev = torch.from_numpy(r.bits).cuda()
        zero_dev = torch.zeros_like(bits_dev)
        f_out = ng.objective(dc, y_dev, 2.5, bits_dev)
        f_max = ng.objective(dc, y_dev, 2.5, zero_dev)
        torch.cuda.synchronize()
        assert (f_out.cpu().numpy() == oracle.objective(c, yy, 2.5, r.bits)).all()
        assert (f_max.cpu().numpy() == oracle.objective(c, yy, 2.5, np.zeros_like(r.bits))).all()
        eps = (f_out - f_max).double().mean().item() / 2.0 ** 20
        say("convergence error", eps)


def test_full_size_quantized_reuse_sampled(torch_dev):
    """The benchmark's quantized workload at full size (2^20 frames of C1008
    at 3.5 dB, default launch shape): sampled frames against the oracle."""
    torch = torch_dev
    c, dc = dev_code("C1008")
    F = 1 << 20
    sig = float(np.float32(channel.sigma_from_ebn0(3.5, c.rate)))
    p = oracle.Params(w=0.75, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75, t_max=300,
                      smooth_window=64, quant_bits=4, noise_reuse=1)
    say("full size quantized C1008 2^20")
    y = channel.bpsk_awgn_device(F, c.n, sig, seed=2035)
    out = ng.decode(dc, y, sig, ng.Params(**p.__dict__), 2035)
    torch.cuda.synchronize()
    for start in (0, F // 2 + 5, F - 64):
        yh = y[start:start + 64].cpu().numpy()
        r = oracle.decode(c, yh, np.float32(sig), p, 2035, frame_base=start, threads=8)
        g = (out.bits[start:start + 64].cpu().numpy(), out.iters[start:start + 64].cpu().numpy(),
             out.converged[start:start + 64].cpu().numpy(), None)
        assert_same(g, r, trace=False)
