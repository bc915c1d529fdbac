// decode_ext_single.hip -- decode kernel instances for single-bit flips of argmin E_k (Sec. III-B Step 3a): S-NGDBF and
// S-GDBF, binary32 or quantized, with or without noise reuse.
// Each decoder family is a translation unit of its own so that the kernel
// set compiles in parallel.
#include "host.h"

namespace ngdbf_host {

NGDBF_DISPATCH_FAMILY(dispatch_ext_single, ngdbf::kExtSingle)

}  // namespace ngdbf_host
