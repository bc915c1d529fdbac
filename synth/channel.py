"""Seeded BPSK-AWGN channel samples (inputs to the decoder).

Sec. III-A: y = c_hat + z with bipolar c_hat in {-1,+1}^n and z i.i.d.
Gaussian of variance N0/2.  With unit-energy BPSK symbols and design rate
R = 1 - m/n, Eb/N0 = 1/(2 R sigma^2), so sigma = (2 R 10^(EbN0_dB/10))^-1/2.
(The paper's Sec. VII example pairs sigma = 0.668 with 3.50 dB for a rate-1/2
code, which this convention reproduces.)

All workloads transmit the all-zero codeword (c_hat = +1) unless a test
supplies another codeword.  Samples come from numpy's PCG64 generator on the
host, or from torch's generator on the device for large batches; neither is
part of the decoder.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Union

import numpy as np

INT8_SCALE = 16.0  # int8 storage: y_q = clamp(rint(16 y), -127, 127)


def sigma_from_ebn0(ebn0_db: float, rate: float) -> float:
    """Channel standard deviation for Eb/N0 in dB at code rate R (float64)."""
    return 1.0 / math.sqrt(2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def ebn0_from_sigma(sigma: float, rate: float) -> float:
    return 10.0 * math.log10(1.0 / (2.0 * rate * sigma * sigma))


def bpsk_awgn(n_frames: int, n: int, sigma: Union[float, Sequence[float], np.ndarray],
              seed: int, codewords: Optional[np.ndarray] = None) -> np.ndarray:
    """float32 [n_frames, n] received samples y = c_hat + sigma * z (host).

    sigma is a scalar or one value per frame.  codewords, if given, is a
    uint8 [n_frames, n] array of code bits c (c_hat = 1 - 2c); default all-zero.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n_frames, n))
    sig = np.asarray(sigma, dtype=np.float64)
    if sig.ndim == 1:
        sig = sig[:, None]
    chat = np.ones((n_frames, n)) if codewords is None else 1.0 - 2.0 * codewords.astype(np.float64)
    return (chat + sig * z).astype(np.float32)


def bpsk_awgn_device(n_frames: int, n: int, sigma, seed: int, device="cuda"):
    """float32 [n_frames, n] all-zero-codeword samples generated on the device
    with torch's generator (for batches too large to build on the host).

    sigma is a float or a float32 tensor of one value per frame."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    y = torch.randn((n_frames, n), generator=g, device=device, dtype=torch.float32)
    if isinstance(sigma, torch.Tensor):
        y.mul_(sigma.to(device=device, dtype=torch.float32).view(-1, 1))
    else:
        y.mul_(float(sigma))
    y.add_(1.0)
    return y


def quantize_int8(y):
    """int8 storage of samples: y_q = clamp(rint(16 y), -127, 127), round half
    to even, symmetric saturation.  Works on numpy arrays and torch tensors."""
    if isinstance(y, np.ndarray):
        return np.clip(np.rint(y.astype(np.float64) * INT8_SCALE), -127, 127).astype(np.int8)
    import torch

    return torch.clamp(torch.round(y * INT8_SCALE), -127, 127).to(torch.int8)


def frame_sigmas(n_frames: int, ebn0_lo: float, ebn0_hi: float, rate: float, seed: int) -> np.ndarray:
    """Per-frame sigma for Eb/N0 drawn uniformly in [lo, hi] dB (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eb = rng.uniform(ebn0_lo, ebn0_hi, size=n_frames)
    return (1.0 / np.sqrt(2.0 * rate * 10.0 ** (eb / 10.0))).astype(np.float32)
