"""NGDBF LDPC decoding on AMD Instinct MI355X (gfx950).

Python binding of ``libngdbf.so``, whose C ABI is declared in
``include/ngdbf.h``: Noisy Gradient-Descent Bit-Flip decoding (Sundararajan,
Winstead, Boutillon, IEEE TCOM 2014, Sec. III) of many frames per call.
The functions named ``ngdbf_*`` mirror the C entry points one to one and only
marshal arguments; every step of decoding runs in the library's HIP kernels.
PyTorch provides device memory and streams.  There is no CPU fallback:
without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libngdbf.so")

NGDBF_Y_F32 = 0
NGDBF_Y_I8 = 1

#: names of the C entry points (include/ngdbf.h)
ABI_FUNCTIONS = ("ngdbf_create_code", "ngdbf_destroy_code", "ngdbf_code_info", "ngdbf_decode",
                 "ngdbf_decode_trace", "ngdbf_decode_noalloc", "ngdbf_noise_probe", "ngdbf_code_set_shape",
                 "ngdbf_code_get_shape", "ngdbf_code_set_stats", "ngdbf_autotune", "ngdbf_decode_batch",
                 "ngdbf_decode_segments", "ngdbf_server_create", "ngdbf_server_destroy",
                 "ngdbf_server_pools", "ngdbf_server_admit", "ngdbf_server_commit",
                 "ngdbf_server_pump", "ngdbf_server_poll", "ngdbf_server_release",
                 "ngdbf_objective", "ngdbf_channel", "ngdbf_frame_stats", "ngdbf_issue_probe",
                 "ngdbf_last_error")


NGDBF_MULTI, NGDBF_SINGLE, NGDBF_MODE_SWITCH = 0, 1, 2

#: ngdbf_status values
NGDBF_OK, NGDBF_EINVAL, NGDBF_ENOMEM, NGDBF_EDEVICE, NGDBF_EUNSUPPORTED, NGDBF_EBUSY = 0, -1, -2, -3, -4, -5


class NgdbfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ngdbf status {status}: {message}")
        self.status = status


class ngdbf_params(ctypes.Structure):
    _fields_ = [("w", ctypes.c_float), ("theta", ctypes.c_float), ("lam", ctypes.c_float),
                ("eta", ctypes.c_float), ("ymax", ctypes.c_float), ("t_max", ctypes.c_int32),
                ("smooth_window", ctypes.c_int32), ("y_format", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("quant_bits", ctypes.c_int32),
                ("noise_reuse", ctypes.c_int32)]


class ngdbf_job(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n_frames", ctypes.c_int64),
                ("sigma", ctypes.c_void_p), ("sigma_scalar", ctypes.c_float),
                ("params", ngdbf_params), ("seed", ctypes.c_uint64),
                ("frame_base", ctypes.c_uint64), ("out_bits", ctypes.c_void_p),
                ("out_iters", ctypes.c_void_p), ("out_converged", ctypes.c_void_p)]


class ngdbf_segment(ctypes.Structure):
    _fields_ = [("first_slot", ctypes.c_int64), ("frame_offset", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("frame_base", ctypes.c_uint64)]


@dataclasses.dataclass
class Params:
    """Decoder parameters in the paper's notation (Sec. III-B..E, IV-A, IV-E, V).

    variant: NGDBF_MULTI, NGDBF_SINGLE or NGDBF_MODE_SWITCH; quant_bits: 0 for
    binary32, Q for the Q-bit quantized decoder; noise_reuse: 1 for the
    shift-register noise chain."""

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

    def c(self, y_format: int) -> ngdbf_params:
        return ngdbf_params(self.w, self.theta, self.lam, self.eta, self.ymax, self.t_max,
                            self.smooth_window, y_format, self.variant, self.quant_bits,
                            self.noise_reuse)


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_1402_2773_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, U32, U64, F = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float)
        L.ngdbf_create_code.argtypes = [I32, I32, I64, P, P, ctypes.POINTER(ctypes.c_void_p)]
        L.ngdbf_destroy_code.argtypes = [P]
        L.ngdbf_code_info.argtypes = [P, P, P, P]
        L.ngdbf_decode.argtypes = [P, P, I64, P, F, ctypes.POINTER(ngdbf_params), U64, U64,
                                   P, P, P, P]
        L.ngdbf_decode_trace.argtypes = [P, P, I64, P, F, ctypes.POINTER(ngdbf_params), U64,
                                         U64, P, P, P, P, P]
        L.ngdbf_decode_noalloc.argtypes = [P, P, I64, P, F, ctypes.POINTER(ngdbf_params), U64, U64,
                                           P, P, P, P]
        L.ngdbf_noise_probe.argtypes = [I32, U32, U32, U64, U64, U32, P, P, P]
        L.ngdbf_code_set_shape.argtypes = [P, I32, I32, I32]
        L.ngdbf_code_get_shape.argtypes = [P, ctypes.POINTER(ngdbf_params), P]
        L.ngdbf_code_set_stats.argtypes = [P, P]
        L.ngdbf_autotune.argtypes = [P, P, I64, P, F, ctypes.POINTER(ngdbf_params), U64, P, P, P]
        L.ngdbf_decode_batch.argtypes = [ctypes.POINTER(ngdbf_job), I32, P]
        L.ngdbf_decode_segments.argtypes = [P, P, P, F, I64, ctypes.POINTER(ngdbf_params), P,
                                            I32, I64, P, P, P, P]
        L.ngdbf_server_create.argtypes = [I32, P, ctypes.POINTER(ngdbf_params), P, I32, I32, I32,
                                          ctypes.POINTER(ctypes.c_void_p)]
        L.ngdbf_server_destroy.argtypes = [P]
        L.ngdbf_server_pools.argtypes = [P, I32, P, P, P, P, P]
        L.ngdbf_server_admit.argtypes = [P, I32, P, P, P, P, P, P, P]
        L.ngdbf_server_commit.argtypes = [P, I32, P, P]
        L.ngdbf_server_pump.argtypes = [P, P]
        L.ngdbf_server_poll.argtypes = [P, I32, P, P]
        L.ngdbf_server_release.argtypes = [P, I32, P]
        L.ngdbf_objective.argtypes = [P, P, I32, I64, F, P, P, P]
        L.ngdbf_issue_probe.argtypes = [I32, I32, I32, P, P]
        L.ngdbf_channel.argtypes = [I32, I64, P, F, U64, U64, P, I32, P, P]
        L.ngdbf_frame_stats.argtypes = [I32, I64, P, P, P, P, I32, P, P]
        L.ngdbf_last_error.argtypes = []
        L.ngdbf_last_error.restype = ctypes.c_char_p
        for name in ABI_FUNCTIONS:
            if name != "ngdbf_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise NgdbfError(status, lib().ngdbf_last_error().decode())


def _addr(x) -> Optional[int]:
    """Device/host address of a torch tensor or numpy array, an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ------------------------------------------------------------- C entry points

def ngdbf_create_code(n: int, m: int, row_ptr, col_idx, nnz: Optional[int] = None) -> ctypes.c_void_p:
    """nnz defaults to len(col_idx) (the library checks it against row_ptr[m])."""
    import numpy as np

    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().ngdbf_create_code(n, m, len(ci) if nnz is None else nnz, rp.ctypes.data,
                                   ci.ctypes.data, ctypes.byref(h)))
    return h


def ngdbf_destroy_code(code) -> None:
    _check(lib().ngdbf_destroy_code(code))


def ngdbf_code_info(code):
    n, m, nnz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ngdbf_code_info(code, ctypes.byref(n), ctypes.byref(m), ctypes.byref(nnz)))
    return n.value, m.value, nnz.value


def ngdbf_decode(code, y, n_frames: int, sigma, sigma_scalar: float, params: ngdbf_params,
                 seed: int, frame_base: int, out_bits, out_iters, out_converged, stream) -> None:
    _check(lib().ngdbf_decode(code, _addr(y), n_frames, _addr(sigma), sigma_scalar,
                              ctypes.byref(params), seed, frame_base, _addr(out_bits),
                              _addr(out_iters), _addr(out_converged), _stream(stream)))


def ngdbf_decode_trace(code, y, n_frames: int, sigma, sigma_scalar: float, params: ngdbf_params,
                       seed: int, frame_base: int, out_bits, out_iters, out_converged,
                       flip_masks, stream) -> None:
    _check(lib().ngdbf_decode_trace(code, _addr(y), n_frames, _addr(sigma), sigma_scalar,
                                    ctypes.byref(params), seed, frame_base, _addr(out_bits),
                                    _addr(out_iters), _addr(out_converged), _addr(flip_masks),
                                    _stream(stream)))


def ngdbf_decode_noalloc(code, y, n_frames: int, sigma, sigma_scalar: float, params: ngdbf_params,
                         seed: int, frame_base: int, out_bits, out_iters, out_converged, stream) -> None:
    _check(lib().ngdbf_decode_noalloc(code, _addr(y), n_frames, _addr(sigma), sigma_scalar,
                                      ctypes.byref(params), seed, frame_base, _addr(out_bits),
                                      _addr(out_iters), _addr(out_converged), _stream(stream)))


def ngdbf_noise_probe(kind: int, start: int, count: int, seed: int, frame: int, iteration: int,
                      out0, out1, stream) -> None:
    _check(lib().ngdbf_noise_probe(kind, start, count, seed, frame, iteration, _addr(out0),
                                   _addr(out1), _stream(stream)))


def ngdbf_code_set_shape(code, waves_per_frame: int, quads_per_lane: int,
                         frames_per_block: int) -> None:
    _check(lib().ngdbf_code_set_shape(code, waves_per_frame, quads_per_lane, frames_per_block))


def ngdbf_code_get_shape(code, params: Optional[ngdbf_params] = None):
    shape = (ctypes.c_int32 * 3)()
    _check(lib().ngdbf_code_get_shape(code, ctypes.byref(params) if params is not None else None,
                                      shape))
    return tuple(shape)


def ngdbf_code_set_stats(code, counters) -> None:
    """Attach a device uint64 [2] tensor (or None) as the settle-test counters."""
    _check(lib().ngdbf_code_set_stats(code, _addr(counters)))


def ngdbf_autotune(code, y, n_frames: int, sigma, sigma_scalar: float, params: ngdbf_params,
                   seed: int, stream):
    best = (ctypes.c_int32 * 3)()
    ms = ctypes.c_float()
    _check(lib().ngdbf_autotune(code, _addr(y), n_frames, _addr(sigma), sigma_scalar,
                                ctypes.byref(params), seed, best, ctypes.byref(ms),
                                _stream(stream)))
    return tuple(best), ms.value


def ngdbf_decode_batch(jobs, stream) -> None:
    arr = (ngdbf_job * len(jobs))(*jobs)
    _check(lib().ngdbf_decode_batch(arr, len(jobs), _stream(stream)))


def ngdbf_decode_segments(code, y_pool, sigma_pool, sigma_scalar: float, pool_frames: int,
                          params: ngdbf_params, segments, n_segments: int, n_frames: int,
                          bits_pool, iters_pool, conv_pool, stream) -> None:
    _check(lib().ngdbf_decode_segments(code, _addr(y_pool), _addr(sigma_pool), sigma_scalar,
                                       pool_frames, ctypes.byref(params), _addr(segments),
                                       n_segments, n_frames, _addr(bits_pool),
                                       _addr(iters_pool), _addr(conv_pool), _stream(stream)))


def ngdbf_server_create(codes, params, pool_frames, n_streams: int,
                        max_requests_per_launch: int, launches_per_stream: int) -> ctypes.c_void_p:
    k = len(codes)
    c_codes = (ctypes.c_void_p * k)(*[c.value if isinstance(c, ctypes.c_void_p) else c
                                      for c in codes])
    c_params = (ngdbf_params * k)(*params)
    c_pool = (ctypes.c_int64 * k)(*pool_frames)
    out = ctypes.c_void_p()
    _check(lib().ngdbf_server_create(k, c_codes, c_params, c_pool, n_streams,
                                     max_requests_per_launch, launches_per_stream,
                                     ctypes.byref(out)))
    return out


def ngdbf_server_destroy(server) -> None:
    _check(lib().ngdbf_server_destroy(server))


def ngdbf_server_pools(server, code_index: int):
    """(y, sigma, bits, iters, converged) device addresses of one code's pool."""
    ptrs = [ctypes.c_void_p() for _ in range(5)]
    _check(lib().ngdbf_server_pools(server, code_index, *[ctypes.byref(q) for q in ptrs]))
    return tuple(q.value for q in ptrs)


def ngdbf_server_admit(server, code_index, n_frames, seed, frame_base):
    """Admit requests in order while their pools have room.

    Returns (tickets, first_slots) of the admitted prefix."""
    import numpy as np

    k = len(code_index)
    ci = np.ascontiguousarray(code_index, dtype=np.int32)
    nf = np.ascontiguousarray(n_frames, dtype=np.int64)
    sd = np.ascontiguousarray(seed, dtype=np.uint64)
    fb = np.ascontiguousarray(frame_base, dtype=np.uint64)
    tickets = np.zeros(k, dtype=np.uint64)
    first = np.zeros(k, dtype=np.int64)
    n_adm = ctypes.c_int32()
    _check(lib().ngdbf_server_admit(server, k, _addr(ci), _addr(nf), _addr(sd), _addr(fb),
                                    _addr(tickets), _addr(first), ctypes.byref(n_adm)))
    return tickets[:n_adm.value], first[:n_adm.value]


def ngdbf_server_commit(server, tickets, stream) -> None:
    import numpy as np

    t = np.ascontiguousarray(tickets, dtype=np.uint64)
    _check(lib().ngdbf_server_commit(server, len(t), _addr(t), _stream(stream)))


def ngdbf_server_pump(server) -> int:
    n = ctypes.c_int32()
    _check(lib().ngdbf_server_pump(server, ctypes.byref(n)))
    return n.value


def ngdbf_server_poll(server, capacity: int = 1 << 16):
    import numpy as np

    t = np.zeros(capacity, dtype=np.uint64)
    n = ctypes.c_int32()
    _check(lib().ngdbf_server_poll(server, capacity, _addr(t), ctypes.byref(n)))
    return t[:n.value]


def ngdbf_server_release(server, tickets) -> None:
    import numpy as np

    t = np.ascontiguousarray(tickets, dtype=np.uint64)
    _check(lib().ngdbf_server_release(server, len(t), _addr(t)))


def ngdbf_objective(code, y, y_format: int, n_frames: int, ymax: float, bits, out, stream) -> None:
    _check(lib().ngdbf_objective(code, _addr(y), y_format, n_frames, ymax, _addr(bits),
                                 _addr(out), _stream(stream)))


def ngdbf_channel(n: int, n_frames: int, sigma, sigma_scalar: float, seed: int, frame_base: int,
                  codewords, y_format: int, y, stream) -> None:
    _check(lib().ngdbf_channel(n, n_frames, _addr(sigma), sigma_scalar, seed, frame_base,
                               _addr(codewords), y_format, _addr(y), _stream(stream)))


def ngdbf_frame_stats(n: int, n_frames: int, bits, codewords, iters, converged, t_max: int, out,
                      stream) -> None:
    _check(lib().ngdbf_frame_stats(n, n_frames, _addr(bits), _addr(codewords), _addr(iters),
                                   _addr(converged), t_max, _addr(out), _stream(stream)))


def ngdbf_issue_probe(kind: int, blocks: int, iters: int, out, stream) -> None:
    status = lib().ngdbf_issue_probe(kind, blocks, iters, _addr(out), _stream(stream))
    if status != 0:
        raise NgdbfError(status, "issue probe rejected its arguments or failed to launch")


def ngdbf_last_error() -> str:
    return lib().ngdbf_last_error().decode()


# ------------------------------------------------------------- conveniences

class Code:
    """A parity-check matrix resident on the current device (owns the handle)."""

    def __init__(self, n: int, m: int, row_ptr, col_idx):
        self.n, self.m = int(n), int(m)
        self.handle = ngdbf_create_code(self.n, self.m, row_ptr, col_idx)

    @classmethod
    def from_ldpc(cls, code) -> "Code":
        return cls(code.n, code.m, code.row_ptr, code.col_idx)

    @property
    def nbytes_row(self) -> int:
        return (self.n + 7) // 8

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            ngdbf_destroy_code(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Outputs:
    bits: "object"       # torch.uint8 [F, ceil(n/8)]
    iters: "object"      # torch.int32 [F]
    converged: "object"  # torch.uint8 [F]
    trace: "object" = None  # torch.uint8 [F, T, ceil(n/8)]


def _y_format(y) -> int:
    import torch

    if y.dtype == torch.float32:
        return NGDBF_Y_F32
    if y.dtype == torch.int8:
        return NGDBF_Y_I8
    raise ValueError("y must be float32 or int8")


def alloc_outputs(code: Code, n_frames: int, device) -> Outputs:
    import torch

    return Outputs(torch.empty((n_frames, code.nbytes_row), dtype=torch.uint8, device=device),
                   torch.empty(n_frames, dtype=torch.int32, device=device),
                   torch.empty(n_frames, dtype=torch.uint8, device=device))


def job(code: Code, y, sigma, params: Params, seed: int, out: Outputs,
        frame_base: int = 0) -> ngdbf_job:
    """One entry of a batch (the tensors must stay alive until it has run)."""
    import torch

    sig_t, sig_s = (sigma, 0.0) if isinstance(sigma, torch.Tensor) else (None, float(sigma))
    return ngdbf_job(code.handle.value, _addr(y), y.shape[0], _addr(sig_t), sig_s,
                     params.c(_y_format(y)), seed, frame_base, _addr(out.bits),
                     _addr(out.iters), _addr(out.converged))


def autotune(code: Code, y, sigma, params: Params, seed: int, stream=None):
    """Time every launch shape on the sample y and keep the fastest on the code."""
    import torch

    sig_t, sig_s = (sigma, 0.0) if isinstance(sigma, torch.Tensor) else (None, float(sigma))
    return ngdbf_autotune(code.handle, y, y.shape[0], sig_t, sig_s, params.c(_y_format(y)), seed,
                          stream)


def decode(code: Code, y, sigma, params: Params, seed: int, frame_base: int = 0,
           trace: bool = False, stream=None, out: Optional[Outputs] = None) -> Outputs:
    """Decode the frames of y (torch [F, n] float32 or int8 on the device).

    sigma: a float, or a torch float32 [F] tensor on the device.  Outputs
    are allocated on y's device unless ``out`` is given."""
    import torch

    if y.dim() != 2 or y.shape[1] != code.n:
        raise ValueError("y must be [frames, n]")
    if not y.is_contiguous():
        raise ValueError("y must be contiguous")
    fmt = _y_format(y)
    F = y.shape[0]
    if out is None:
        out = alloc_outputs(code, F, y.device)
        if trace:
            out.trace = torch.empty((F, params.t_max, code.nbytes_row), dtype=torch.uint8,
                                    device=y.device)
    sig_t, sig_s = (sigma, 0.0) if isinstance(sigma, torch.Tensor) else (None, float(sigma))
    if sig_t is not None and (sig_t.dtype != torch.float32 or sig_t.numel() != F
                              or not sig_t.is_contiguous()):
        raise ValueError("sigma must be a contiguous float32 tensor with one value per frame")
    p = params.c(fmt)
    if trace:
        ngdbf_decode_trace(code.handle, y, F, sig_t, sig_s, p, seed, frame_base, out.bits,
                           out.iters, out.converged, out.trace, stream)
    else:
        ngdbf_decode(code.handle, y, F, sig_t, sig_s, p, seed, frame_base, out.bits, out.iters,
                     out.converged, stream)
    return out


class Server:
    """Continuous-batching runtime: one resident slot pool per code.

    The pools are torch views of the library's device buffers; a request is
    admitted (slots reserved), its samples and sigma written into its slots,
    committed on a stream, launched by ``pump`` together with every other
    committed request of its code, reported by ``poll`` and released."""

    def __init__(self, codes, params, pool_frames, n_streams: int = 4,
                 max_requests_per_launch: int = 32768, launches_per_stream: int = 1):
        import torch

        self.codes = list(codes)
        self.params = list(params)
        self.handle = ngdbf_server_create([c.handle for c in self.codes],
                                          [p.c(NGDBF_Y_F32) for p in self.params],
                                          list(pool_frames), n_streams,
                                          max_requests_per_launch, launches_per_stream)
        self.pools = []
        dev = torch.device("cuda", torch.cuda.current_device())
        for i, (code, F) in enumerate(zip(self.codes, pool_frames)):
            y, sg, b, it, cv = ngdbf_server_pools(self.handle, i)
            self.pools.append(Outputs(_wrap(b, (F, code.nbytes_row), torch.uint8, dev),
                                      _wrap(it, (F,), torch.int32, dev),
                                      _wrap(cv, (F,), torch.uint8, dev)))
            self.pools[-1].y = _wrap(y, (F, code.n), torch.float32, dev)
            self.pools[-1].sigma = _wrap(sg, (F,), torch.float32, dev)

    def admit(self, code_index, n_frames, seed, frame_base):
        return ngdbf_server_admit(self.handle, code_index, n_frames, seed, frame_base)

    def commit(self, tickets, stream=None) -> None:
        ngdbf_server_commit(self.handle, tickets, stream)

    def pump(self) -> int:
        return ngdbf_server_pump(self.handle)

    def poll(self, capacity: int = 1 << 16):
        return ngdbf_server_poll(self.handle, capacity)

    def release(self, tickets) -> None:
        ngdbf_server_release(self.handle, tickets)

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            ngdbf_server_destroy(self.handle)
        self.handle = None
        self.pools = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceBuffer:
    """__cuda_array_interface__ view of library-owned device memory."""

    def __init__(self, addr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (addr, False), "version": 3, "strides": None}


def _wrap(addr: int, shape, dtype, device):
    import torch

    typestr = {torch.uint8: "|u1", torch.int32: "<i4", torch.float32: "<f4"}[dtype]
    return torch.as_tensor(_DeviceBuffer(addr, shape, typestr), device=device)


def channel(n: int, n_frames: int, sigma, seed: int, frame_base: int = 0, codewords=None,
            int8: bool = False, device="cuda", stream=None, out=None):
    """Received samples of the synthetic channel (Sec. III-A) generated on the
    device: torch [F, n] float32 (int8 codes with int8=True).  sigma: a float
    or a device float32 [F] tensor."""
    import torch

    if out is None:
        out = torch.empty((n_frames, n), dtype=torch.int8 if int8 else torch.float32, device=device)
    sig_t, sig_s = (sigma, 0.0) if isinstance(sigma, torch.Tensor) else (None, float(sigma))
    ngdbf_channel(n, n_frames, sig_t, sig_s, seed, frame_base, codewords,
                  NGDBF_Y_I8 if int8 else NGDBF_Y_F32, out, stream)
    return out


def frame_stats(code: Code, out: Outputs, t_max: int, codewords=None, stream=None, acc=None):
    """int64 [7 + t_max] device counters of decoded frames (ngdbf_frame_stats),
    added to acc if given."""
    import torch

    if acc is None:
        acc = torch.zeros(7 + t_max, dtype=torch.int64, device=out.bits.device)
    ngdbf_frame_stats(code.n, out.bits.shape[0], out.bits, codewords, out.iters, out.converged,
                      t_max, acc, stream)
    return acc


def objective(code: Code, y, ymax: float, bits, stream=None):
    """int64 [F] on the device: f(x) of Sec. III-B for the decisions in bits,
    in fixed point 2^-20 (ngdbf_objective)."""
    import torch

    out = torch.empty(y.shape[0], dtype=torch.int64, device=y.device)
    ngdbf_objective(code.handle, y, _y_format(y), y.shape[0], ymax, bits, out, stream)
    return out
