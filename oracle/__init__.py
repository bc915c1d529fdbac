"""Python binding of the plain CPU oracle (``ngdbf_oracle.c``).

TEST INFRASTRUCTURE ONLY: the HIP decoder never imports this package.  Only
the test suite, the smoke entry point and the benchmark's CPU baseline leg
use it.  The oracle follows the paper (Sundararajan, Winstead, Boutillon,
IEEE TCOM 2014) Sec. III step by step; see ``ngdbf_oracle.c``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ngdbf_oracle.c")
_LIB = os.path.join(_HERE, "libngdbf_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fusion of a*b+c by the compiler)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm", "-pthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("w", ctypes.c_float), ("theta", ctypes.c_float),
                ("lam", ctypes.c_float), ("eta", ctypes.c_float),
                ("ymax", ctypes.c_float), ("t_max", ctypes.c_int32),
                ("smooth_window", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("quant_bits", ctypes.c_int32), ("noise_reuse", ctypes.c_int32)]


@dataclasses.dataclass
class Params:
    """Decoder parameters, paper notation (Sec. III-B..E, IV-A, IV-E, V).

    variant: 0 multi-bit (Step 3b), 1 single-bit argmin (Step 3a), 2 mode
    switching; quant_bits: 0 binary32, Q > 0 the Q-bit quantized decoder;
    noise_reuse: 1 for the shift-register chain of Sec. V-B."""

    w: float = 0.75
    theta: float = -0.6
    lam: float = 1.0
    eta: float = 0.9
    ymax: float = 2.5
    t_max: int = 100
    smooth_window: int = 0
    variant: int = 0
    quant_bits: int = 0
    noise_reuse: int = 0

    def c(self) -> _Params:
        return _Params(self.w, self.theta, self.lam, self.eta, self.ymax,
                       self.t_max, self.smooth_window, self.variant,
                       self.quant_bits, self.noise_reuse)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.ngdbf_ref_philox4x32_10.argtypes = [P, P, P]
        L.ngdbf_ref_rho.argtypes = [ctypes.c_uint32]
        L.ngdbf_ref_rho.restype = ctypes.c_float
        L.ngdbf_ref_sincos2pi.argtypes = [ctypes.c_uint32, P, P]
        L.ngdbf_ref_gauss_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P]
        L.ngdbf_ref_noise_quad.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint32, ctypes.c_uint32, P]
        L.ngdbf_ref_noise_block.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, P]
        L.ngdbf_ref_rho_range.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P]
        L.ngdbf_ref_sincos_range.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P, P]
        L.ngdbf_ref_decode.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P,
                                       ctypes.c_int32, ctypes.c_int64, P,
                                       ctypes.c_float, ctypes.POINTER(_Params),
                                       ctypes.c_uint64, ctypes.c_uint64, P, P, P,
                                       P, ctypes.c_int32]
        L.ngdbf_ref_decode.restype = ctypes.c_int
        L.ngdbf_ref_decode_f64.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P,
                                           P, ctypes.c_int64, P, ctypes.c_float,
                                           ctypes.POINTER(_Params), ctypes.c_uint64,
                                           ctypes.c_uint64, P, P, P, ctypes.c_int32]
        L.ngdbf_ref_decode_f64.restype = ctypes.c_int
        L.ngdbf_ref_quant_half.argtypes = [ctypes.c_float, ctypes.c_int32, ctypes.c_float]
        L.ngdbf_ref_quant_half.restype = ctypes.c_float
        L.ngdbf_ref_threshold_events.argtypes = [ctypes.c_float, ctypes.c_float,
                                                 ctypes.c_float, ctypes.c_int32,
                                                 ctypes.c_int32, P, P, ctypes.c_int32]
        L.ngdbf_ref_threshold_events.restype = ctypes.c_int32
        L.ngdbf_ref_reuse_sample.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                             ctypes.c_uint32, ctypes.c_int32]
        L.ngdbf_ref_reuse_sample.restype = ctypes.c_float
        L.ngdbf_ref_objective.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P,
                                          ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                          P, P]
        L.ngdbf_ref_objective.restype = ctypes.c_int
        L.ngdbf_ref_channel.argtypes = [ctypes.c_int32, ctypes.c_int64, P, ctypes.c_float,
                                        ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_int32, P]
        L.ngdbf_ref_channel.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ngdbf_ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def rho(m: int) -> float:
    return float(lib().ngdbf_ref_rho(m))


def rho_range(m0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float32)
    lib().ngdbf_ref_rho_range(m0, count, _ptr(out))
    return out


def sincos_range(i0: int, count: int) -> Tuple[np.ndarray, np.ndarray]:
    c = np.empty(count, dtype=np.float32)
    s = np.empty(count, dtype=np.float32)
    lib().ngdbf_ref_sincos_range(i0, count, _ptr(c), _ptr(s))
    return c, s


def gauss_pair(a: int, b: int) -> np.ndarray:
    z = np.zeros(2, dtype=np.float32)
    lib().ngdbf_ref_gauss_pair(a, b, _ptr(z))
    return z


def noise_quad(seed: int, frame: int, t: int, quad: int) -> np.ndarray:
    z = np.zeros(4, dtype=np.float32)
    lib().ngdbf_ref_noise_quad(seed, frame, t, quad, _ptr(z))
    return z


def noise_block(seed: int, frame: int, t: int, quad0: int, n_quads: int) -> np.ndarray:
    """float32 [4 * n_quads]: draws of bits 4*quad0 .. 4*(quad0+n_quads)-1."""
    z = np.zeros(4 * n_quads, dtype=np.float32)
    lib().ngdbf_ref_noise_block(seed, frame, t, quad0, n_quads, _ptr(z))
    return z


def quant_scale(q_bits: int, ymax: float) -> float:
    """fl32(N_Q / (2 Y_max)), the quantizer's input scale."""
    return float(np.float32(1 << q_bits) / (np.float32(2.0) * np.float32(ymax)))


def quant_half(v: float, q_bits: int, ymax: float) -> float:
    """g(v) of Sec. IV-E in units of half a quantization step (an odd integer)."""
    return float(lib().ngdbf_ref_quant_half(v, q_bits, quant_scale(q_bits, ymax)))


def threshold_events(theta: float, lam: float, ymax: float, q_bits: int, t_max: int):
    """[(theta~_i, tau~_i)] of Sec. V-A: quantized threshold values in channel
    units and the non-flip count at which each becomes active."""
    cap = 64
    vals = np.zeros(cap, dtype=np.float64)
    taus = np.zeros(cap, dtype=np.int32)
    k = lib().ngdbf_ref_threshold_events(theta, lam, ymax, q_bits, t_max, _ptr(vals),
                                         _ptr(taus), cap)
    return [(float(vals[i]), int(taus[i])) for i in range(min(k, cap))]


def reuse_sample(seed: int, frame: int, n: int, t: int, k: int) -> float:
    """The standard-normal sample of bit k in round t under noise reuse."""
    return float(lib().ngdbf_ref_reuse_sample(seed, frame, n, t, k))


def objective(code, y: np.ndarray, ymax: float, bits: np.ndarray) -> np.ndarray:
    """int64 [F]: the GDBF objective of the decisions in bits, fixed point 2^-20."""
    y = np.ascontiguousarray(y)
    y_format = 1 if y.dtype == np.int8 else 0
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    F = y.shape[0]
    out = np.zeros(F, dtype=np.int64)
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    rc = lib().ngdbf_ref_objective(code.n, code.m, _ptr(rp), _ptr(ci), _ptr(y), y_format, F,
                                   ymax, _ptr(bits), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def channel(n: int, n_frames: int, sigma, seed: int, frame_base: int = 0,
            codewords: Optional[np.ndarray] = None, int8: bool = False) -> np.ndarray:
    """Received samples of the synthetic channel (Sec. III-A), [F, n] float32
    (or int8 codes y_q = clamp(rint(16 y), -127, 127) with int8=True)."""
    sig_arr, sig_scalar = None, 0.0
    if np.ndim(sigma) == 0:
        sig_scalar = float(np.float32(sigma))
    else:
        sig_arr = np.ascontiguousarray(sigma, dtype=np.float32)
        if sig_arr.shape != (n_frames,):
            raise ValueError("sigma must be a scalar or one value per frame")
    cw = None if codewords is None else np.ascontiguousarray(codewords, dtype=np.uint8)
    y = np.zeros((n_frames, n), dtype=np.int8 if int8 else np.float32)
    rc = lib().ngdbf_ref_channel(n, n_frames, _ptr(sig_arr), sig_scalar, seed, frame_base,
                                 _ptr(cw), 1 if int8 else 0, _ptr(y))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return y


@dataclasses.dataclass
class DecodeResult:
    bits: np.ndarray       # uint8 [F, ceil(n/8)], c_k = (1 - x_k)/2, LSB first
    iters: np.ndarray      # int32 [F]
    converged: np.ndarray  # uint8 [F]
    trace: Optional[np.ndarray] = None  # uint8 [F, T, ceil(n/8)] flip masks


def decode(code, y: np.ndarray, sigma, params: Params, seed: int,
           frame_base: int = 0, trace: bool = False, threads: int = 1,
           f64: bool = False) -> DecodeResult:
    """Decode the frames of y ([F, n] float32, or int8 codes y_q = 16 y)."""
    y = np.ascontiguousarray(y)
    if y.ndim != 2 or y.shape[1] != code.n:
        raise ValueError("y must be [frames, n]")
    y_format = 1 if y.dtype == np.int8 else 0
    if y_format == 0 and y.dtype != np.float32:
        raise ValueError("y must be float32 or int8")
    F = y.shape[0]
    nb = (code.n + 7) // 8
    sig_arr = None
    sig_scalar = 0.0
    if np.ndim(sigma) == 0:
        sig_scalar = float(np.float32(sigma))
    else:
        sig_arr = np.ascontiguousarray(sigma, dtype=np.float32)
        if sig_arr.shape != (F,):
            raise ValueError("sigma must be a scalar or one value per frame")
    bits = np.zeros((F, nb), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    conv = np.zeros(F, dtype=np.uint8)
    tr = np.zeros((F, params.t_max, nb), dtype=np.uint8) if trace else None
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    p = params.c()
    if f64:
        if y_format != 0 or trace:
            raise ValueError("the f64 decoder takes float32 y and has no trace")
        rc = lib().ngdbf_ref_decode_f64(code.n, code.m, _ptr(rp), _ptr(ci), _ptr(y), F,
                                        _ptr(sig_arr), sig_scalar, ctypes.byref(p),
                                        seed, frame_base, _ptr(bits), _ptr(iters),
                                        _ptr(conv), threads)
    else:
        rc = lib().ngdbf_ref_decode(code.n, code.m, _ptr(rp), _ptr(ci), _ptr(y), y_format,
                                    F, _ptr(sig_arr), sig_scalar, ctypes.byref(p), seed,
                                    frame_base, _ptr(bits), _ptr(iters), _ptr(conv),
                                    _ptr(tr), threads)
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return DecodeResult(bits, iters, conv, tr)


def unpack_bits(bits: np.ndarray, n: int) -> np.ndarray:
    """uint8 [F, ceil(n/8)] LSB-first -> uint8 [F, n] of 0/1."""
    return np.unpackbits(bits, axis=-1, bitorder="little")[..., :n]
