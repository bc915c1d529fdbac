// decode_ext_packed.hip -- decode kernel instances for the quantized
// multi-bit decoder with the shift-register noise chain (Sec. IV-E, V-A,
// V-B) in packed signed 16-bit lanes: E~_k, theta~(u_k) and the non-flip
// counters of two bits per register.
#include "host.h"

namespace ngdbf_host {

NGDBF_DISPATCH_FAMILY(dispatch_ext_packed, ngdbf::kExtQuantReuse)

}  // namespace ngdbf_host
