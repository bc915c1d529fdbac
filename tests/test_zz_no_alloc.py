"""The allocation-free decode (ngdbf_decode_noalloc, for callers that cannot
allocate device memory) against ngdbf_decode, through the C ABI: identical
decoded words, iteration counts and flags on two calls in a row, the second
with fewer frames (the shared scratch queue must start clean each time), on
the base decoder and on an extended one."""
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
    return torch


CASES = {
    # SM-NGDBF (adaptive threshold, smoothing), the base decoder
    "C1008_sm": ("C1008", 3.5, dict(w=0.75, theta=-0.9, lam=0.97, eta=0.95, ymax=2.5, t_max=300,
                                    smooth_window=64)),
    # quantized with noise reuse, the packed decoder
    "C96_q4_reuse": ("C96", 3.0, dict(w=0.75, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75, t_max=100,
                                      smooth_window=64, quant_bits=4, noise_reuse=1)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_noalloc_equals_decode_on_two_calls(torch_dev, case):
    torch = torch_dev
    name, ebn0, params = CASES[case]
    c = codes.named_code(name)
    dc = ng.Code.from_ldpc(c)
    p = ng.Params(**params)
    pc = p.c(ng.NGDBF_Y_F32)
    stream = torch.cuda.current_stream()
    for call, (frames, seed, fb) in enumerate([(20000, 401, 0), (777, 402, 12345)]):
        sig = channel.frame_sigmas(frames, ebn0 - 0.5, ebn0 + 0.5, c.rate, seed=seed)
        s_dev = torch.from_numpy(sig).cuda()
        y = channel.bpsk_awgn_device(frames, c.n, s_dev, seed=seed + 10)
        ref = ng.alloc_outputs(dc, frames, "cuda")
        out = ng.alloc_outputs(dc, frames, "cuda")
        out.iters.fill_(-1)
        out.bits.fill_(0xA5)
        out.converged.fill_(7)
        say("noalloc", case, "call", call, "frames", frames)
        ng.ngdbf_decode(dc.handle, y, frames, s_dev, 0.0, pc, seed, fb, ref.bits, ref.iters,
                        ref.converged, stream)
        ng.ngdbf_decode_noalloc(dc.handle, y, frames, s_dev, 0.0, pc, seed, fb, out.bits, out.iters,
                                out.converged, stream)
        torch.cuda.synchronize()
        assert torch.equal(out.iters, ref.iters), f"call {call}: iteration counts differ"
        assert torch.equal(out.bits, ref.bits), f"call {call}: decoded words differ"
        assert torch.equal(out.converged, ref.converged), f"call {call}: flags differ"
        assert out.iters.min().item() >= 0
        # and a few frames against the oracle
        r = oracle.decode(c, y[:16].cpu().numpy(), sig[:16], oracle.Params(**params), seed,
                          frame_base=fb, threads=8)
        assert (out.iters[:16].cpu().numpy() == r.iters).all()
        assert (out.bits[:16].cpu().numpy() == r.bits).all()
    dc.close()


def test_noalloc_rejects_bad_arguments_like_decode(torch_dev):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="code is NULL"):
        ng.ngdbf_decode_noalloc(None, None, 4, None, 0.5, p, 1, 0, None, None, None, None)
    q = ng.Params(lam=2.0).c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="lambda"):
        ng.ngdbf_decode_noalloc(None, None, 4, None, 0.5, q, 1, 0, None, None, None, None)
