"""The device channel (Sec. III-A) against the oracle's channel, sample for
sample, and the device Monte Carlo counters against their definition
computed on the host from the same decoded frames."""
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


@pytest.mark.parametrize("n,frames,fmt,per_frame,cw", [
    (96, 3000, "f32", False, False), (1008, 500, "f32", True, True), (2048, 300, "i8", True, False),
    (103, 777, "f32", True, True), (4000, 64, "i8", False, True), (5, 1000, "i8", True, True)])
def test_channel_equals_oracle(torch_dev, n, frames, fmt, per_frame, cw):
    torch = torch_dev
    rng = np.random.Generator(np.random.PCG64(n + frames))
    sig = channel.frame_sigmas(frames, 2.0, 5.0, 0.5, seed=n) if per_frame else np.float32(0.7)
    if per_frame:
        sig[::7] = 0.0
    words = rng.integers(0, 256, size=(frames, (n + 7) // 8), dtype=np.uint8) if cw else None
    fb = 2 ** 33 + 5
    say("channel", n, frames, fmt)
    y = ng.channel(n, frames, torch.from_numpy(sig).cuda() if per_frame else float(sig), seed=n + 1,
                   frame_base=fb, codewords=torch.from_numpy(words).cuda() if cw else None,
                   int8=fmt == "i8")
    torch.cuda.synchronize()
    ref = oracle.channel(n, frames, sig, seed=n + 1, frame_base=fb, codewords=words, int8=fmt == "i8")
    got = y.cpu().numpy()
    if fmt == "f32":
        assert (got.view(np.uint32) == ref.view(np.uint32)).all()
    else:
        assert (got == ref).all()


def test_channel_full_size_sampled(torch_dev):
    """2^20 frames of C1008 at 3.5 dB in one call: sampled frames equal the
    oracle's, and the hard-decision error rate is Phi(-1/sigma)."""
    torch = torch_dev
    from scipy import stats

    F, n = 1 << 20, 1008
    sig = float(np.float32(channel.sigma_from_ebn0(3.5, 0.5)))
    y = ng.channel(n, F, sig, seed=2035)
    torch.cuda.synchronize()
    for start in (0, F // 2 + 7, F - 16):
        ref = oracle.channel(n, 16, sig, seed=2035, frame_base=start)
        assert (y[start:start + 16].cpu().numpy().view(np.uint32) == ref.view(np.uint32)).all()
    p = stats.norm.cdf(-1.0 / sig)
    k = int((y < 0).sum().item())
    N = F * n
    assert abs(k / N - p) < 4 * np.sqrt(p * (1 - p) / N)
    del y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,t_max,cw", [("C96", 100, False), ("C1008", 300, True), ("C2048", 300, False)])
def test_frame_stats_equal_host_counts(torch_dev, name, t_max, cw):
    torch = torch_dev
    c = codes.named_code(name)
    dc = ng.Code.from_ldpc(c)
    F = 5000
    s = torch.from_numpy(channel.frame_sigmas(F, 2.0, 4.0, c.rate, seed=91)).cuda()
    y = ng.channel(c.n, F, s, seed=92)
    p = ng.Params(w=0.75, theta=-0.9, lam=0.98, eta=0.95, ymax=2.5, t_max=t_max, smooth_window=64)
    out = ng.decode(dc, y, s, p, 93)
    rng = np.random.Generator(np.random.PCG64(94))
    words = rng.integers(0, 256, size=(F, (c.n + 7) // 8), dtype=np.uint8) if cw else None
    acc = torch.zeros(7 + t_max, dtype=torch.int64, device="cuda")
    say("frame stats", name)
    ng.frame_stats(dc, out, t_max, codewords=torch.from_numpy(words).cuda() if cw else None, acc=acc)
    ng.frame_stats(dc, out, t_max, codewords=torch.from_numpy(words).cuda() if cw else None, acc=acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy() // 2  # two calls add up
    assert (acc.cpu().numpy() % 2 == 0).all()
    bits = out.bits.cpu().numpy()
    sent = words if cw else np.zeros_like(bits)
    e = oracle.unpack_bits(bits ^ sent, c.n).sum(1).astype(np.int64)
    it = out.iters.cpu().numpy().astype(np.int64)
    conv = out.converged.cpu().numpy()
    assert got[0] == e.sum() and got[1] == (e * e).sum() and got[2] == (e > 0).sum()
    assert got[3] == ((e > 0) & (conv == 1)).sum()
    assert got[4] == it.sum() and got[5] == (conv == 0).sum()
    assert (got[6:] == np.bincount(it, minlength=t_max + 1)).all()
    dc.close()
