// decode_ext_switch.hip -- decode kernel instances for mode switching (Sec. III-B): multi-bit rounds until the objective
// first decreases, single-bit rounds after.
// Each decoder family is a translation unit of its own so that the kernel
// set compiles in parallel.
#include "host.h"

namespace ngdbf_host {

NGDBF_DISPATCH_FAMILY(dispatch_ext_switch, ngdbf::kExtSwitch)

}  // namespace ngdbf_host
