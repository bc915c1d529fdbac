"""Pins of the oracle's single-bit, mode-switching, quantized and noise-reuse
decoders (Sec. III-B, IV-E, V-A, V-B) and of its objective function.

As in test_oracle_pins, each test ties the oracle to something outside it:
the paper's Table II, hand-computed quantizer values, GF(2) codeword
symmetry, brute-force evaluation of the objective with dense H, or the shift
property that defines the noise chain.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from synth import channel, codes
from tests import gf2

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def c96(oracle_lib):
    return codes.named_code("C96")


# ---------------------------------------------------------------- quantizer

def test_table2_threshold_events(oracle_lib):
    """Sec. V-A, Table II: the quantized threshold values and the non-flip
    counts at which they become active, for Q = 3, 4, 5."""
    with open(os.path.join(HERE, "golden", "table2_threshold_events.json")) as f:
        g = json.load(f)
    for q, expect in g["events"].items():
        got = oracle.threshold_events(g["theta"], g["lambda"], g["ymax"], int(q), g["t_max"])
        assert [t for _, t in got] == [t for _, t in expect], q
        for (v, _), (e, _) in zip(got, expect):
            assert abs(v - e) <= 5e-5, (q, v, e)


# (Q, Y_max, v, g(v)) worked out by hand from Sec. IV-E eq. (quantization):
# g(v) = sign(v) (floor(|v| N_Q / 2Y_max) + 1/2) (2 Y_max / N_Q)
HAND_G = [
    (3, 2.5, 0.9, 0.9375),      # 1.44 -> 1 -> 1.5 * 0.625
    (3, 2.5, 0.3, 0.3125),      # 0.48 -> 0 -> 0.5 * 0.625
    (3, 2.5, -1.3, -1.5625),    # 2.08 -> 2 -> 2.5 * 0.625
    (3, 2.5, 2.49, 2.1875),     # 3.984 -> 3 -> 3.5 * 0.625 (top level)
    (3, 2.5, 7.0, 2.1875),      # beyond Y_max: top level
    (3, 2.5, 0.0, 0.0),         # signum(0) = 0
    (4, 1.75, 0.5, 0.546875),   # 2.2857 -> 2 -> 2.5 * 0.21875
    (4, 1.75, -1.0, -0.984375),  # 4.571 -> 4 -> 4.5 * 0.21875
    (4, 1.75, 1.7, 1.640625),   # 7.771 -> 7 -> 7.5 * 0.21875
    (5, 2.5, -0.05, -0.078125),  # 0.64 -> 0 -> 0.5 * 0.15625
]


@pytest.mark.parametrize("q,ymax,v,g", HAND_G)
def test_quantizer_hand_values(oracle_lib, q, ymax, v, g):
    half = oracle.quant_half(v, q, ymax)
    assert half * ymax / (1 << q) == pytest.approx(g, abs=1e-12)
    assert half == 0.0 or int(half) % 2 != 0  # odd multiples of half a step


def test_quantizer_is_odd_and_monotone(oracle_lib):
    """g(-v) = -g(v) and g is non-decreasing (a uniform quantizer)."""
    v = np.linspace(-3.0, 3.0, 6001, dtype=np.float32)
    for q in (2, 3, 4, 5, 8):
        a = np.array([oracle.quant_half(float(x), q, 2.5) for x in v])
        b = np.array([oracle.quant_half(float(-x), q, 2.5) for x in v])
        assert (a == -b).all()
        assert (np.diff(a) >= 0).all()
        assert np.abs(a).max() == (1 << q) - 1


# ---------------------------------------------------------------- noise reuse

def test_noise_reuse_is_a_shift_register(oracle_lib):
    """Sec. V-B: each round one new sample enters the chain at bit 0 and every
    other bit takes the sample its predecessor held the round before."""
    n, seed, frame = 96, 77, 5
    rng = np.random.default_rng(0)
    for _ in range(300):
        k = int(rng.integers(1, n))
        t = int(rng.integers(1, 400))
        assert oracle.reuse_sample(seed, frame, n, t, k) == oracle.reuse_sample(seed, frame, n, t - 1, k - 1)
    # bit 0 gets a different sample every round; the samples are N(0, 1)
    z0 = np.array([oracle.reuse_sample(seed, frame, n, t, 0) for t in range(4000)])
    assert len(np.unique(z0)) == len(z0)
    assert stats.kstest(z0, "norm").pvalue > 1e-3


def test_noise_reuse_one_round_brute_force(oracle_lib):
    """One round on a 3-bit check with reuse: each bit's flip is the Step 3b
    decision with the chain's sample at that bit, element n - 1 - k of the
    stream (Sec. V-B with the preload read as the stream's first n samples)."""
    code = codes.from_rows("spc3", 3, [[0, 1, 2]])
    rng = np.random.default_rng(3)
    F = 3000
    y = rng.uniform(-1.0, 1.0, size=(F, 3)).astype(np.float32)
    sig, eta, w, theta = 0.8, 1.0, 0.75, -0.6
    p = oracle.Params(w=w, theta=theta, lam=1.0, eta=eta, ymax=2.5, t_max=1, noise_reuse=1)
    r = oracle.decode(code, y, sig, p, seed=21, trace=True)
    flips = oracle.unpack_bits(r.trace[:, 0, :], 3)
    x = np.where(y < 0, -1.0, 1.0)
    s = x.prod(axis=1)
    qs = np.float32(np.float32(eta) * np.float32(sig))
    n_checked = 0
    for f in range(F):
        if s[f] > 0:
            continue  # stopped before round 0
        stream = np.concatenate([oracle.noise_quad(21, f, 0xFFFFFFFF, 0)])
        for k in range(3):
            z = stream[3 - 1 - k]
            a = np.float32(np.float32(w) * np.float32(s[f]) + np.float32(x[f, k] * y[f, k]))
            e = float(np.float64(qs) * np.float64(z) + np.float64(a))
            if abs(e - theta) < 1e-5:
                continue  # too close to call outside binary32
            assert flips[f, k] == (e < theta), (f, k)
            n_checked += 1
    assert n_checked > 3000


# ---------------------------------------------------------------- objective

def _dense_objective(h, y, x):
    s = np.where((h @ (x < 0).astype(np.int64).T).T % 2 == 1, -1.0, 1.0)
    return (x * y).sum(axis=1) + s.sum(axis=1)


def test_objective_matches_dense_evaluation(oracle_lib, c96):
    """f(x) = sum x y + sum s (Sec. III-B) against a dense GF(2) evaluation,
    and the transmitted word's value sum y + m (Sec. VI, f_max)."""
    h = c96.dense().astype(np.int64)
    y = channel.bpsk_awgn(200, c96.n, 0.7, seed=31)
    ysat = np.clip(y, -2.5, 2.5).astype(np.float64)
    rng = np.random.default_rng(32)
    bits = rng.integers(0, 2, size=(200, c96.n)).astype(np.uint8)
    bits[:20] = 0  # the all-zero codeword
    packed = np.packbits(bits, axis=1, bitorder="little")
    F = oracle.objective(c96, y, 2.5, packed).astype(np.float64) / 2.0 ** 20
    x = 1.0 - 2.0 * bits
    ref = _dense_objective(h, ysat, x)
    assert np.abs(F - ref).max() <= c96.n * 2.0 ** -21 + 1e-9
    assert np.abs(F[:20] - (ysat[:20].sum(axis=1) + c96.m)).max() <= c96.n * 2.0 ** -21


def test_objective_single_flip_identity(oracle_lib, c96):
    """Flipping bit k changes F by -2 (x_k Y_k + 2^20 S_k) exactly: the
    gradient identity that defines E_k (Sec. III-B, w = 1, eta = 0)."""
    h = c96.dense().astype(np.int64)
    y = channel.bpsk_awgn(1, c96.n, 0.8, seed=33)
    rng = np.random.default_rng(34)
    bits = rng.integers(0, 2, size=c96.n).astype(np.uint8)
    x = 1 - 2 * bits.astype(np.int64)
    s = np.where((h @ bits.astype(np.int64)) % 2 == 1, -1, 1)
    Yf = np.rint(np.clip(y[0], -2.5, 2.5).astype(np.float64) * 2.0 ** 20).astype(np.int64)
    base = oracle.objective(c96, y, 2.5, np.packbits(bits, bitorder="little")[None])[0]
    for k in range(0, c96.n, 7):
        b2 = bits.copy()
        b2[k] ^= 1
        fk = oracle.objective(c96, y, 2.5, np.packbits(b2, bitorder="little")[None])[0]
        S = int(s[h[:, k] == 1].sum())
        assert fk - base == -2 * (x[k] * Yf[k] + (1 << 20) * S)


# ---------------------------------------------------------------- single-bit

def _replay(code, y, r, f):
    """x(t) for t = 0 .. iters from x(0) = sign(y) and the flip trace."""
    x = np.where(y[f] < 0, -1.0, 1.0)
    xs = [x.copy()]
    tr = oracle.unpack_bits(r.trace[f], code.n)
    for t in range(int(r.iters[f])):
        x = np.where(tr[t] == 1, -x, x)
        xs.append(x.copy())
    return np.array(xs), tr


def test_single_bit_gdbf_takes_the_best_single_flip(oracle_lib, c96):
    """S-GDBF (Step 3a, w = 1, eta = 0): every round flips exactly one bit,
    and no other single flip would raise the objective more (brute force
    over all n flips with dense H)."""
    h = c96.dense().astype(np.int64)
    sig = channel.sigma_from_ebn0(2.5, c96.rate)
    y = channel.bpsk_awgn(60, c96.n, sig, seed=35)
    ysat = np.clip(y, -2.5, 2.5).astype(np.float64)
    p = oracle.Params(w=1.0, theta=-0.6, lam=1.0, eta=0.0, ymax=2.5, t_max=30, variant=1)
    r = oracle.decode(c96, y, sig, p, seed=36, trace=True)
    rounds = 0
    for f in range(60):
        xs, tr = _replay(c96, y, r, f)
        for t in range(int(r.iters[f])):
            assert tr[t].sum() == 1
            x = xs[t]
            base = _dense_objective(h, ysat[f:f + 1], x[None])[0]
            flipped = np.repeat(x[None], c96.n, axis=0) * (1 - 2 * np.eye(c96.n))
            gains = _dense_objective(h, np.repeat(ysat[f:f + 1], c96.n, axis=0), flipped) - base
            k = int(np.nonzero(tr[t])[0][0])
            assert gains[k] >= gains.max() - 1e-5, (f, t)
            rounds += 1
    assert rounds > 100


def test_single_bit_ngdbf_flips_one_bit_and_is_codeword_symmetric(oracle_lib, c96):
    """S-NGDBF (Sec. III-C with Step 3a): one flip per executed round, and
    decoding (1-2c) y for a codeword c shifts every decision by c."""
    h = c96.dense()
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(150, c96.n, sig, seed=37)
    cw = gf2.random_codewords(h, 150, seed=38)
    sign = (1.0 - 2.0 * cw).astype(np.float32)
    p = oracle.Params(w=0.75, theta=-0.6, lam=1.0, eta=1.0, ymax=2.5, t_max=60, variant=1)
    a = oracle.decode(c96, y, sig, p, seed=39, trace=True)
    b = oracle.decode(c96, (y * sign).astype(np.float32), sig, p, seed=39, trace=True)
    assert (a.trace == b.trace).all() and (a.iters == b.iters).all()
    assert (oracle.unpack_bits(a.bits, c96.n) ^ cw == oracle.unpack_bits(b.bits, c96.n)).all()
    for f in range(150):
        tr = oracle.unpack_bits(a.trace[f], c96.n)
        it = int(a.iters[f])
        assert (tr[:it].sum(axis=1) == 1).all()
        assert tr[it:].sum() == 0


# ---------------------------------------------------------------- mode switching

def test_mode_switching_turns_single_bit_after_the_first_decrease(oracle_lib, c96):
    """Sec. III-B: mu starts at 1 (multi-bit rounds); the first round whose
    decision has a lower objective than the previous one sets mu = 0, and every
    later round flips exactly the best single bit (w = 1, eta = 0)."""
    h = c96.dense().astype(np.int64)
    sig = channel.sigma_from_ebn0(2.5, c96.rate)
    F = 120
    y = channel.bpsk_awgn(F, c96.n, sig, seed=40)
    ysat = np.clip(y, -2.5, 2.5)
    p = oracle.Params(w=1.0, theta=-0.6, lam=1.0, eta=0.0, ymax=2.5, t_max=40, variant=2)
    r = oracle.decode(c96, y, sig, p, seed=41, trace=True)
    switched = multi_rounds = 0
    for f in range(F):
        xs, tr = _replay(c96, y, r, f)
        bits = ((1 - xs) / 2).astype(np.uint8)
        packed = np.packbits(bits, axis=1, bitorder="little")
        Fx = oracle.objective(c96, np.repeat(y[f:f + 1], len(xs), axis=0), 2.5, packed)
        drops = [t for t in range(1, len(xs)) if Fx[t] < Fx[t - 1]]
        t_sw = drops[0] if drops else None
        for t in range(int(r.iters[f])):
            if t_sw is not None and t >= t_sw:
                assert tr[t].sum() == 1, (f, t)
                x = xs[t]
                base = _dense_objective(h, ysat[f:f + 1].astype(np.float64), x[None])[0]
                flipped = np.repeat(x[None], c96.n, axis=0) * (1 - 2 * np.eye(c96.n))
                gains = _dense_objective(h, np.repeat(ysat[f:f + 1].astype(np.float64), c96.n, axis=0),
                                         flipped) - base
                assert gains[int(np.nonzero(tr[t])[0][0])] >= gains.max() - 1e-5
            elif tr[t].sum() > 1:
                multi_rounds += 1
        switched += t_sw is not None and t_sw < int(r.iters[f])
    assert switched > 10 and multi_rounds > 10


# ---------------------------------------------------------------- quantized

@pytest.mark.parametrize("q,reuse", [(3, 0), (4, 1), (5, 1)])
def test_quantized_codeword_symmetry(oracle_lib, c96, q, reuse):
    """g is odd (g(-v) = -g(v)), so decoding (1-2c) y for a codeword c shifts
    the whole quantized trajectory by c (Sec. IV-E, V-A, V-B)."""
    h = c96.dense()
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(200, c96.n, sig, seed=42)
    cw = gf2.random_codewords(h, 200, seed=43)
    sign = (1.0 - 2.0 * cw).astype(np.float32)
    p = oracle.Params(w=0.75, theta=-0.7, lam=0.98, eta=0.9, ymax=1.75, t_max=100,
                      smooth_window=64, quant_bits=q, noise_reuse=reuse)
    a = oracle.decode(c96, y, sig, p, seed=44, trace=True)
    b = oracle.decode(c96, (y * sign).astype(np.float32), sig, p, seed=44, trace=True)
    assert (a.iters == b.iters).all() and (a.trace == b.trace).all()
    assert (oracle.unpack_bits(a.bits, c96.n) ^ cw == oracle.unpack_bits(b.bits, c96.n)).all()


def test_quantized_noiseless_and_eta_zero(oracle_lib, c96):
    """Noiseless input stops at round 0; with eta = 0 the quantized decoder
    is deterministic (g(0) = 0), with eta > 0 the seed matters."""
    p = oracle.Params(w=0.75, theta=-0.7, lam=0.98, eta=0.0, ymax=1.75, t_max=50, quant_bits=4)
    y0 = np.ones((5, c96.n), dtype=np.float32)
    r0 = oracle.decode(c96, y0, 0.7, p, seed=1)
    assert (r0.iters == 0).all() and (r0.bits == 0).all()
    sig = channel.sigma_from_ebn0(3.0, c96.rate)
    y = channel.bpsk_awgn(200, c96.n, sig, seed=45)
    a = oracle.decode(c96, y, sig, p, seed=1)
    b = oracle.decode(c96, y, sig, p, seed=2)
    assert (a.iters == b.iters).all() and (a.bits == b.bits).all()
    pn = oracle.Params(**{**p.__dict__, "eta": 0.9, "noise_reuse": 1})
    c = oracle.decode(c96, y, sig, pn, seed=1)
    d = oracle.decode(c96, y, sig, pn, seed=2)
    assert not (c.iters == d.iters).all()


def test_quantized_decoder_tracks_fp32_statistically(oracle_lib):
    """Sec. IV-E reports quantized SM-NGDBF close to unquantized at Q = 4;
    here only as a sanity range: FER within a factor of 3 either way."""
    code = codes.named_code("C1008")
    sig = channel.sigma_from_ebn0(3.5, code.rate)
    y = channel.bpsk_awgn(600, code.n, sig, seed=46)
    pf = oracle.Params(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)
    pq = oracle.Params(w=0.75, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75, t_max=300, smooth_window=64,
                       quant_bits=4, noise_reuse=1)
    a = oracle.decode(code, y, sig, pf, seed=47, threads=8)
    b = oracle.decode(code, y, sig, pq, seed=47, threads=8)
    fa = oracle.unpack_bits(a.bits, code.n).any(axis=1).mean()
    fb = oracle.unpack_bits(b.bits, code.n).any(axis=1).mean()
    assert fb <= 3 * fa + 0.02 and fa <= 3 * fb + 0.02


def test_invalid_variant_combinations_are_rejected(oracle_lib, c96):
    y = np.ones((1, c96.n), dtype=np.float32)
    for bad in (dict(variant=3), dict(quant_bits=9), dict(quant_bits=3, ymax=0.0),
                dict(quant_bits=3, variant=2), dict(noise_reuse=2)):
        p = oracle.Params(**{**oracle.Params().__dict__, **bad})
        with pytest.raises(ValueError):
            oracle.decode(c96, y, 0.5, p, seed=1)
