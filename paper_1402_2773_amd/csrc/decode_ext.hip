// decode_ext.hip -- instantiations of the extended decode kernels: single-bit
// and mode-switching flips (Sec. III-B), the quantized decoder (Sec. IV-E,
// V-A) and shift-register noise reuse (Sec. V-B).  They live in their own
// translation unit so that the two halves of the kernel set compile in
// parallel.
#include "host.h"

namespace ngdbf_host {

int dispatch_ext(const Shape &sh, const ngdbf::DecodeArgs &a, size_t lds, int dev, hipStream_t s,
                 int y_format, bool trace) {
  if (y_format == NGDBF_Y_I8) {
    return trace ? dispatch<NGDBF_Y_I8, true, true>(sh, a, lds, dev, s)
                 : dispatch<NGDBF_Y_I8, false, true>(sh, a, lds, dev, s);
  }
  return trace ? dispatch<NGDBF_Y_F32, true, true>(sh, a, lds, dev, s)
               : dispatch<NGDBF_Y_F32, false, true>(sh, a, lds, dev, s);
}

}  // namespace ngdbf_host
