"""Pins of the CPU oracle against facts fixed outside it.

Each test ties the oracle to something it does not compute itself: values
worked out by hand from the paper (tests/golden), a library implementation of
the same generator, closed forms, libm, GF(2) algebra, or brute force.
"""
import json
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
from synth import channel, codes
from tests import gf2

HERE = os.path.dirname(os.path.abspath(__file__))


def _params(d):
    return oracle.Params(w=d["w"], theta=d["theta"], lam=d["lam"], eta=d["eta"],
                         ymax=d["ymax"], t_max=d["t_max"], smooth_window=d["smooth_window"],
                         variant=d.get("variant", 0), quant_bits=d.get("quant_bits", 0),
                         noise_reuse=d.get("noise_reuse", 0))


# ---------------------------------------------------------------- worked examples

def _golden():
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_worked_example(oracle_lib, ex):
    """Hand-derived decodes (Sec. III-B..E, IV-A) of tiny codes with eta = 0."""
    code = codes.from_rows(ex["name"], ex["n"], ex["rows"])
    y = np.array([ex["y"]], dtype=np.float32)
    p = _params(ex["params"])
    r = oracle.decode(code, y, ex["sigma"], p, seed=123, trace=True)
    assert oracle.unpack_bits(r.bits, code.n)[0].tolist() == ex["bits"]
    assert int(r.iters[0]) == ex["iters"]
    assert int(r.converged[0]) == ex["converged"]
    tr = oracle.unpack_bits(r.trace[0], code.n)
    for t in range(p.t_max):
        expect = ex["trace"][t] if t < len(ex["trace"]) else []
        assert np.nonzero(tr[t])[0].tolist() == expect, f"round {t}"


# ---------------------------------------------------------------- noise generator

_TORCH_PHILOX = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def test_philox_matches_torch_engine(oracle_lib):
    """Philox4x32-10 equals PyTorch's philox_engine (a library implementation
    of the same SC'11 generator): key = seed, counter = (offset, subsequence)."""
    import torch.utils.cpp_extension as ce

    inc = ce.include_paths()
    rng = np.random.Generator(np.random.PCG64(5))
    cases = [(0, 0, 0), (1, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1)]
    for _ in range(200):
        cases.append(tuple(int(v) for v in rng.integers(0, 2**63, size=3, dtype=np.int64)))
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "p.cpp")
        exe = os.path.join(td, "p")
        with open(src, "w") as f:
            f.write(_TORCH_PHILOX)
        subprocess.check_call(["g++", "-std=c++17", "-O1", *[f"-I{i}" for i in inc], src, "-o", exe])
        inp = "".join(f"{s} {u} {o}\n" for s, u, o in cases)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.strip().split("\n")
    assert len(lines) == len(cases)
    for (seed, sub, off), line in zip(cases, lines):
        ref = [int(v) for v in line.split()]
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert oracle.philox4x32_10(ctr, key).tolist() == ref


def test_rho_exhaustive_against_libm(oracle_lib):
    """rho(m) = sqrt(-2 ln(m 2^-24)) for every m in [1, 2^24], against float64
    libm: relative error below 4e-7 (a few binary32 ulps) everywhere."""
    m = np.arange(1, (1 << 24) + 1, dtype=np.float64)
    exact = np.sqrt(-2.0 * np.log(m * 2.0**-24))
    got = oracle.rho_range(1, 1 << 24).astype(np.float64)
    assert got[-1] == 0.0 and exact[-1] == 0.0
    rel = np.abs(got[:-1] - exact[:-1]) / exact[:-1]
    assert rel.max() < 4e-7, rel.max()
    # the radius never exceeds the closed-form bound sqrt(48 ln 2)
    assert got.max() <= math.sqrt(48 * math.log(2)) * (1 + 2e-7)


def test_sincos_exhaustive_against_libm(oracle_lib):
    """cos/sin of 2 pi i 2^-24 for every i in [0, 2^24), against float64 libm:
    absolute error below 2^-23, and never above 1 in magnitude."""
    i = np.arange(1 << 24, dtype=np.float64)
    phi = 2.0 * np.pi * i * 2.0**-24
    c, s = oracle.sincos_range(0, 1 << 24)
    assert np.abs(c.astype(np.float64) - np.cos(phi)).max() < 2.0**-23
    assert np.abs(s.astype(np.float64) - np.sin(phi)).max() < 2.0**-23
    assert np.abs(c).max() <= 1.0 and np.abs(s).max() <= 1.0
    # the quarter turn (the angle word's top two bits) fixes the signs, zeros
    # aside: cos >= 0 in quarters 0 and 3, <= 0 in 1 and 2; sin >= 0 in 0 and
    # 1, <= 0 in 2 and 3
    q = np.arange(1 << 24, dtype=np.uint32) >> 22
    assert not (c[(q == 0) | (q == 3)] < 0).any() and not (c[(q == 1) | (q == 2)] > 0).any()
    assert not (s[q <= 1] < 0).any() and not (s[q >= 2] > 0).any()


def test_noise_is_standard_normal(oracle_lib):
    """The draws q_k / (eta sigma) are N(0,1) (Sec. III-C): moments, KS test,
    no correlation between neighbours, iterations or frames."""
    z = np.concatenate([oracle.noise_block(11, f, t, 0, 1 << 16) for f in range(2) for t in range(4)])
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(z[: 1 << 20], "norm").pvalue > 1e-4
    kurt = stats.kurtosis(z)
    assert abs(kurt) < 5 * math.sqrt(24.0 / n)
    a = oracle.noise_block(11, 0, 0, 0, 1 << 16)
    b = oracle.noise_block(11, 0, 1, 0, 1 << 16)
    c = oracle.noise_block(11, 1, 0, 0, 1 << 16)
    lim = 5 / math.sqrt(a.size)
    assert abs(np.corrcoef(a, b)[0, 1]) < lim
    assert abs(np.corrcoef(a, c)[0, 1]) < lim
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < lim
    assert np.abs(z).max() <= 5.7682


# ---------------------------------------------------------------- channel model

def test_sigma_convention_matches_paper_example():
    """Sec. VII: sigma = 0.668 is E_b/N_0 = 3.50 dB for a (3,6) code and the
    initial error probability is p_e(0) = 0.0672."""
    assert abs(channel.ebn0_from_sigma(0.668, 0.5) - 3.50) < 0.01
    assert abs(channel.sigma_from_ebn0(3.5, 0.5) - 0.668) < 0.001
    assert abs(stats.norm.cdf(-1.0 / 0.668) - 0.0672) < 5e-5


def test_channel_initial_error_rate():
    """Fraction of sign errors in y equals Phi(-1/sigma) (Sec. III-A, VII)."""
    sig = channel.sigma_from_ebn0(3.5, 0.5)
    y = channel.bpsk_awgn(2000, 1008, sig, seed=3)
    p = stats.norm.cdf(-1.0 / sig)
    frac = (y < 0).mean()
    assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / y.size)


# ---------------------------------------------------------------- decoder properties

@pytest.fixture(scope="module")
def c96():
    return codes.named_code("C96")


P_PLAIN = oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=100)
P_SM = oracle.Params(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)


def test_noiseless_codewords_decode_in_zero_rounds(oracle_lib, c96):
    """Sec. III-A/B Step 1: if y is a bipolar codeword, x(0) satisfies every
    check, so decoding stops before any round and returns it."""
    cw = gf2.random_codewords(c96.dense(), 50, seed=4)
    y = (1.0 - 2.0 * cw).astype(np.float32)
    for p in (P_PLAIN, P_SM):
        r = oracle.decode(c96, y, 0.7, p, seed=9)
        assert (r.iters == 0).all() and (r.converged == 1).all()
        assert (oracle.unpack_bits(r.bits, c96.n) == cw).all()


def test_converged_output_is_codeword(oracle_lib, c96):
    """Stop rule (Sec. III-B Step 1): converged frames satisfy H c = 0; frames
    that hit T without smoothing do not."""
    h = c96.dense()
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(3000, c96.n, sig, seed=5)
    r = oracle.decode(c96, y, sig, P_PLAIN, seed=6, threads=4)
    c = oracle.unpack_bits(r.bits, c96.n)
    syn = gf2.syndrome(h, c).any(axis=1)
    assert (~syn[r.converged == 1]).all()
    assert syn[r.converged == 0].all()
    assert (r.converged == 0).sum() > 10  # the case is exercised
    assert (r.iters[r.converged == 0] == P_PLAIN.t_max).all()


def _replay(code, y_row, ymax, trace_f):
    """x(t) for t = 0..len(trace) from x(0) = sign(sat(y)) and the flip masks."""
    v = np.clip(y_row, -ymax, ymax) if ymax > 0 else y_row
    x = np.where(v < 0, -1, 1)
    xs = [x.copy()]
    for t in range(trace_f.shape[0]):
        x = np.where(trace_f[t].astype(bool), -x, x)
        xs.append(x.copy())
    return np.array(xs)


def test_trace_replay_matches_stop_rule_and_smoothing(oracle_lib):
    """Replaying the flip trace from x(0) gives a trajectory whose syndrome
    is nonzero before the stop and zero at it (Sec. III-B), and whose
    smoothed output is the majority of x(t), t = T-W..T (Sec. III-E)."""
    code = codes.named_code("C96")
    h = code.dense()
    sig = channel.sigma_from_ebn0(2.0, code.rate)
    y = channel.bpsk_awgn(300, code.n, sig, seed=7)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=80, smooth_window=20)
    r = oracle.decode(code, y, sig, p, seed=8, trace=True)
    out = oracle.unpack_bits(r.bits, code.n)
    smoothed = 0
    for f in range(y.shape[0]):
        tr = oracle.unpack_bits(r.trace[f], code.n)
        xs = _replay(code, y[f], p.ymax, tr)
        it = int(r.iters[f])
        assert not tr[it:].any()  # no flips after the stop
        syn = gf2.syndrome(h, ((1 - xs[: it + 1]) // 2).astype(np.uint8)).any(axis=1)
        assert syn[:it].all()
        if r.converged[f]:
            assert not syn[it]
            assert (out[f] == (1 - xs[it]) // 2).all()
        else:
            assert it == p.t_max and syn[it]
            X = xs[p.t_max - p.smooth_window: p.t_max + 1].sum(axis=0)
            assert (out[f] == (X < 0).astype(np.uint8)).all()
            smoothed += 1
    assert smoothed > 5


def test_codeword_symmetry(oracle_lib, c96):
    """For a codeword c, decoding (1-2c) * y gives the decode of y shifted by
    c, round by round: x y, s and E are unchanged (Sec. III-A, III-C)."""
    h = c96.dense()
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(400, c96.n, sig, seed=10)
    cw = gf2.random_codewords(h, 400, seed=11)
    sign = (1.0 - 2.0 * cw).astype(np.float32)
    for p in (P_PLAIN, P_SM):
        a = oracle.decode(c96, y, sig, p, seed=12, trace=True)
        b = oracle.decode(c96, (y * sign).astype(np.float32), sig, p, seed=12, trace=True)
        assert (a.iters == b.iters).all() and (a.converged == b.converged).all()
        assert (oracle.unpack_bits(a.bits, c96.n) ^ cw == oracle.unpack_bits(b.bits, c96.n)).all()
        assert (a.trace == b.trace).all()


def test_eta_zero_is_seed_independent(oracle_lib, c96):
    """eta = 0 removes the perturbation (Sec. III-C): the GDBF decoder of
    Sec. III-B/D is deterministic."""
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(300, c96.n, sig, seed=13)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.95, eta=0.0, ymax=2.5, t_max=50)
    a = oracle.decode(c96, y, sig, p, seed=1)
    b = oracle.decode(c96, y, sig, p, seed=2)
    assert (a.bits == b.bits).all() and (a.iters == b.iters).all()
    q = oracle.decode(c96, y, sig, oracle.Params(**{**p.__dict__, "eta": 0.9}), seed=1)
    assert not (q.iters == a.iters).all()


def test_first_round_flip_probability_closed_form(oracle_lib):
    """Sec. III-E: a bit flips with p_f = Pr(x y + w S + q < theta),
    q ~ N(0, (eta sigma)^2).  With a single wrong bit j, bits sharing a
    check with j have S = d_v - 2, the others S = d_v, and j has S = -d_v;
    observed first-round flips match the Gaussian tail per class."""
    code = codes.named_code("C96")
    h = code.dense()
    dv = 3
    F = 2500
    rng = np.random.Generator(np.random.PCG64(14))
    y = rng.uniform(0.05, 2.4, size=(F, code.n)).astype(np.float32)
    j = 17
    y[:, j] = -1.0
    sig, eta, w, theta = 0.7, 1.5, 0.75, -0.6
    p = oracle.Params(w=w, theta=theta, lam=1.0, eta=eta, ymax=2.5, t_max=1)
    r = oracle.decode(code, y, sig, p, seed=15, trace=True)
    flips = oracle.unpack_bits(r.trace[:, 0, :], code.n).astype(np.float64)
    qs = float(np.float32(np.float32(eta) * np.float32(sig)))
    neighbours = np.nonzero(h[h[:, j] == 1].sum(axis=0))[0]
    S = np.full(code.n, dv)
    S[neighbours] = dv - 2
    S[j] = -dv
    xy = np.abs(y.astype(np.float64))
    prob = stats.norm.cdf((theta - (w * S[None, :] + xy)) / qs)
    for cls in (dv, dv - 2, -dv):
        sel = S == cls
        obs = flips[:, sel].sum()
        exp = prob[:, sel].sum()
        var = (prob[:, sel] * (1 - prob[:, sel])).sum()
        assert abs(obs - exp) < 5 * math.sqrt(var) + 1, (cls, obs, exp)


def test_fp32_and_fp64_decoders_agree_statistically(oracle_lib, c96):
    """The binary32 decoder (with its own log/sin/cos) and a binary64 decoder
    drawing from libm agree in FER and average iterations within sampling
    error at 3 dB (the FP32 rounding changes trajectories only rarely)."""
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(4000, c96.n, sig, seed=16)
    a = oracle.decode(c96, y, sig, P_PLAIN, seed=17, threads=8)
    b = oracle.decode(c96, y, sig, P_PLAIN, seed=17, threads=8, f64=True)
    fa = oracle.unpack_bits(a.bits, c96.n).any(axis=1)
    fb = oracle.unpack_bits(b.bits, c96.n).any(axis=1)
    n = len(fa)
    # paired comparison: discordant frames are few and balanced
    d01, d10 = int((fa & ~fb).sum()), int((~fa & fb).sum())
    assert (d01 + d10) < 0.05 * n
    assert abs(d01 - d10) <= 5 * math.sqrt(d01 + d10 + 1)
    assert abs(a.iters.mean() - b.iters.mean()) < 5 * a.iters.std() / math.sqrt(n)


def test_ml_bound_on_tiny_code(oracle_lib):
    """Brute force over all 2^K codewords of a K = 12 code: NGDBF never finds a
    codeword more likely than ML (objective of Sec. III-B / VI) and its FER is
    not below the ML FER."""
    code = codes.regular_code(24, 3, 6, seed=24, name="C24", girth6=False)
    h = code.dense()
    basis = gf2.nullspace_basis(h)
    k = basis.shape[0]
    assert k >= 12
    allc = np.array([[(i >> b) & 1 for b in range(k)] for i in range(1 << k)], dtype=np.int64)
    cws = (allc @ basis.astype(np.int64)) % 2
    bip = 1.0 - 2.0 * cws
    sig = channel.sigma_from_ebn0(2.0, code.rate)
    y = channel.bpsk_awgn(3000, code.n, sig, seed=18)
    p = oracle.Params(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=100, smooth_window=0)
    r = oracle.decode(code, y, sig, p, seed=19)
    corr = y.astype(np.float64) @ bip.T
    ml = corr.argmax(axis=1)
    ml_err = cws[ml].any(axis=1)
    out = oracle.unpack_bits(r.bits, code.n).astype(np.int64)
    got = (1.0 - 2.0 * out) * y
    conv = r.converged == 1
    assert (got.sum(axis=1)[conv] <= corr.max(axis=1)[conv] + 1e-4).all()
    ngdbf_err = out.any(axis=1)
    assert ngdbf_err.sum() >= ml_err.sum() - 3 * math.sqrt(ml_err.sum() + 1)


def test_int8_storage_equals_its_float_value(oracle_lib, c96):
    """int8 samples y_q decode exactly as float32 y_q/16 (exact conversion)."""
    sig = channel.sigma_from_ebn0(3.5, c96.rate)
    y = channel.bpsk_awgn(300, c96.n, sig, seed=20)
    q = channel.quantize_int8(y)
    a = oracle.decode(c96, q, sig, P_SM, seed=21)
    b = oracle.decode(c96, (q.astype(np.float32) / 16.0).astype(np.float32), sig, P_SM, seed=21)
    assert (a.bits == b.bits).all() and (a.iters == b.iters).all()


def test_threads_and_frame_base_do_not_change_results(oracle_lib, c96):
    """Frames are independent and the noise is keyed by the global frame
    index: threading and chunking leave every result unchanged."""
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(200, c96.n, sig, seed=22)
    a = oracle.decode(c96, y, sig, P_SM, seed=23, threads=1)
    b = oracle.decode(c96, y, sig, P_SM, seed=23, threads=7)
    c = oracle.decode(c96, y[50:120], sig, P_SM, seed=23, frame_base=50)
    assert (a.bits == b.bits).all() and (a.iters == b.iters).all()
    assert (a.bits[50:120] == c.bits).all() and (a.iters[50:120] == c.iters).all()


@pytest.mark.parametrize("ebn0,lam,frames", [(3.0, 0.99, 2048), (3.5, 0.97, 3072)])
def test_binary64_decoder_with_adaptation_and_smoothing(oracle_lib, ebn0, lam, frames):
    """SM-NGDBF on C1008 (theta -0.9, eta 0.95, W 64, T 300; the headline point
    is 3.5 dB): the binary32 decoder and the binary64 one (thresholds adapted
    and smoothing sums kept in double, draws from the same Philox words) agree
    in FER and BER within 99.9% intervals, their trajectories coincide on
    almost every frame, and the frames that end unconverged (where smoothing
    decides the output) give the same smoothed words.  Sec. IV-A simulates in
    double precision; this pins the binary64 decoder's adaptive and smoothing
    paths beside its plain one."""
    c = codes.named_code("C1008")
    sig = channel.sigma_from_ebn0(ebn0, c.rate)
    y = channel.bpsk_awgn(frames, c.n, sig, seed=18)
    p = oracle.Params(w=0.75, theta=-0.9, lam=lam, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)
    a = oracle.decode(c, y, sig, p, seed=19, threads=8)
    b = oracle.decode(c, y, sig, p, seed=19, threads=8, f64=True)
    ea = oracle.unpack_bits(a.bits, c.n).sum(1).astype(np.int64)
    eb = oracle.unpack_bits(b.bits, c.n).sum(1).astype(np.int64)
    z = 3.29
    k = int((eb > 0).sum())
    ph = k / frames
    half = z * math.sqrt(ph * (1 - ph) / frames + z * z / (4 * frames * frames)) / (1 + z * z / frames)
    mid = (ph + z * z / (2 * frames)) / (1 + z * z / frames)
    assert mid - half <= (ea > 0).mean() <= mid + half
    sd = math.sqrt((ea.var(ddof=1) + eb.var(ddof=1)) / frames)
    assert abs(ea.mean() - eb.mean()) <= z * sd + 1e-12
    same = a.iters == b.iters
    assert same.mean() > 0.98
    unconv = same & (a.converged == 0)
    assert unconv.sum() >= 3, "some frames must reach T (smoothing in use)"
    assert (a.bits[unconv] == b.bits[unconv]).all(axis=1).mean() > 0.9


# ------------------------------------------------------------- the synthetic channel

def test_channel_hard_decision_error_rate_closed_form(oracle_lib):
    """Sec. III-A with sigma = 0.668 (3.50 dB for a rate-1/2 code, the paper's
    Sec. VII example): the fraction of samples below zero is Phi(-1/sigma) =
    0.0672 within a 99.9% binomial interval on 2.0e6 independent samples."""
    sig = np.float32(0.668)
    y = oracle.channel(1000, 2000, sig, seed=31)
    k, n = int((y < 0).sum()), y.size
    p = stats.norm.cdf(-1.0 / float(sig))
    assert abs(p - 0.0672) < 5e-5
    assert abs(k / n - p) < 3.29 * math.sqrt(p * (1 - p) / n)


def test_channel_noise_moments_and_normality(oracle_lib):
    sig = np.float32(0.8)
    y = oracle.channel(512, 400, sig, seed=32).astype(np.float64)
    z = (y - 1.0) / float(sig)
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z.ravel()[:20000], "norm").pvalue > 1e-3


def test_channel_special_cases(oracle_lib):
    """sigma = 0 gives the BPSK symbols exactly (c_hat = 1 - 2c); the frame
    index keys the noise (a shifted frame_base reproduces the same frames);
    int8 storage is clamp(rint(16 y), -127, 127) of the float32 samples."""
    rng = np.random.Generator(np.random.PCG64(33))
    cw = rng.integers(0, 256, size=(6, 13), dtype=np.uint8)
    y0 = oracle.channel(100, 6, 0.0, seed=34, codewords=cw)
    bits = oracle.unpack_bits(cw, 100)
    assert (y0 == (1.0 - 2.0 * bits).astype(np.float32)).all()
    sig = channel.frame_sigmas(9, 2.0, 5.0, 0.5, seed=35)
    a = oracle.channel(100, 9, sig, seed=36, frame_base=1000)
    b = oracle.channel(100, 9 + 4, np.concatenate([np.ones(4, np.float32), sig]), seed=36, frame_base=996)
    assert (a == b[4:]).all()
    q = oracle.channel(100, 9, sig, seed=36, frame_base=1000, int8=True)
    ref = np.clip(np.rint(a.astype(np.float64) * 16.0), -127, 127).astype(np.int8)
    assert (q == ref).all()
    # the channel's draws are not the decoder's round-0 draws of the same frame
    z0 = oracle.noise_block(36, 1000, 0, 0, 25)
    zc = (a[0].astype(np.float64) - 1.0) / float(sig[0])
    assert abs(np.corrcoef(z0, zc)[0, 1]) < 0.5
