// decode_ext_multi.hip -- decode kernel instances for the multi-bit rule (Step 3b) with the quantized arithmetic of Sec.
// IV-E / V-A and/or the shift-register noise chain of Sec. V-B.
// Each decoder family is a translation unit of its own so that the kernel
// set compiles in parallel.
#include "host.h"

namespace ngdbf_host {

NGDBF_DISPATCH_FAMILY(dispatch_ext_multi, ngdbf::kExtMulti)

}  // namespace ngdbf_host
