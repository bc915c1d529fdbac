// host.h -- launch of the decode kernel (host code shared by the translation
// units that instantiate its variants).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernel.h"

namespace ngdbf_host {

// Report a failure through ngdbf_last_error (decode.hip).
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// Compute units of a device (decode.hip).
int device_cus(int dev);

// Launch shape: waves per frame, bit quads per lane, frames per workgroup.
struct Shape {
  int wpf, qpl, fpb;
  int block() const { return 64 * wpf * fpb; }
};

// (waves per frame, quads per lane) pairs with built kernels
#define NGDBF_SHAPES(X) \
  X(1, 1) X(1, 2) X(1, 4) X(2, 2) X(2, 4) X(4, 1) X(4, 2) X(4, 4) X(8, 1) X(8, 2) X(16, 1)

template <int WPF, int QPL, int YFMT, bool TRACE, bool REG, int EXT>
int launch(const ngdbf::DecodeArgs &a, const Shape &sh, size_t lds_bytes, int dev, hipStream_t s) {
  auto kern = ngdbf::decode_kernel<WPF, QPL, YFMT, TRACE, REG, EXT>;
  if (lds_bytes > 64 * 1024 &&
      hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds_bytes) != hipSuccess)
    return fail(NGDBF_EUNSUPPORTED, "cannot raise the LDS limit to %zu bytes", lds_bytes);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, sh.block(), lds_bytes) !=
          hipSuccess ||
      per_cu <= 0)
    return fail(NGDBF_EUNSUPPORTED, "kernel does not fit a compute unit (block %d, LDS %zu B)",
                sh.block(), lds_bytes);
  const int cus = std::max(device_cus(dev), 1);
  const int64_t blocks_needed = (a.n_frames + sh.fpb - 1) / sh.fpb;
  // persistent grid: the resident capacity, or fewer blocks for small batches
  const int64_t grid = std::min<int64_t>((int64_t)per_cu * cus, blocks_needed);
  // frames per queue update: 1, or about 1/256 of a taker's share for very
  // large batches (at most 16)
  ngdbf::DecodeArgs args = a;
  const int64_t takers = grid * (WPF == 1 ? sh.fpb : 1);
  args.queue_chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, a.n_frames / (takers * 256)));
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.block()), lds_bytes, s, args);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return NGDBF_OK;
}

template <int YFMT, bool TRACE, int EXT>
int dispatch(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev, hipStream_t s) {
#define NGDBF_CASE(W_, Q_)                                                       \
  if (sh.wpf == W_ && sh.qpl == Q_)                                              \
    return a.dv ? launch<W_, Q_, YFMT, TRACE, true, EXT>(a, sh, lds, dev, s)     \
                : launch<W_, Q_, YFMT, TRACE, false, EXT>(a, sh, lds, dev, s);
  NGDBF_SHAPES(NGDBF_CASE)
#undef NGDBF_CASE
  return fail(NGDBF_EUNSUPPORTED, "no kernel for %d waves x %d quads", sh.wpf, sh.qpl);
}

// The extended decoders, instantiated in decode_ext.hip (one object per
// family).
int dispatch_ext_multi(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev,
                       hipStream_t s, int y_format, bool trace);
int dispatch_ext_single(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev,
                        hipStream_t s, int y_format, bool trace);
int dispatch_ext_switch(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev,
                        hipStream_t s, int y_format, bool trace);
int dispatch_ext_packed(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev,
                        hipStream_t s, int y_format, bool trace);

// Instances of one family for every y format and trace setting.
#define NGDBF_DISPATCH_FAMILY(NAME, EXT_)                                                    \
  int NAME(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev, hipStream_t s, \
           int y_format, bool trace) {                                                      \
    if (y_format == NGDBF_Y_I8)                                                             \
      return trace ? dispatch<NGDBF_Y_I8, true, EXT_>(sh, a, lds, dev, s)                   \
                   : dispatch<NGDBF_Y_I8, false, EXT_>(sh, a, lds, dev, s);                 \
    return trace ? dispatch<NGDBF_Y_F32, true, EXT_>(sh, a, lds, dev, s)                    \
                 : dispatch<NGDBF_Y_F32, false, EXT_>(sh, a, lds, dev, s);                  \
  }

}  // namespace ngdbf_host
