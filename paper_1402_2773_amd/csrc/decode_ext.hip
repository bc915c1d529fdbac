// decode_ext.hip -- decode kernel instances of the extended decoder families:
//   0  dispatch_ext_multi:  the multi-bit rule (Sec. III-B Step 3b) with the
//      quantized arithmetic of Sec. IV-E / V-A and/or the shift-register
//      noise chain of Sec. V-B;
//   1  dispatch_ext_single: single-bit flips of argmin E_k (Step 3a):
//      S-NGDBF and S-GDBF, binary32 or quantized, with or without noise reuse;
//   2  dispatch_ext_switch: mode switching (Sec. III-B), multi-bit rounds
//      until the objective first decreases, single-bit rounds after;
//   3  dispatch_ext_packed: the quantized multi-bit decoder with the noise
//      chain in packed signed 16-bit lanes (E~_k, theta~(u_k) and the
//      non-flip counters of two bits per register).
// Each family is a large set of kernel instances (every launch shape, y
// format and trace setting): the build compiles this file once per family
// (-DNGDBF_EXT_FAMILY=0..3) so that the sets compile in parallel; compiled
// without the define, one object holds all four.
#include "host.h"

namespace ngdbf_host {

#if !defined(NGDBF_EXT_FAMILY) || NGDBF_EXT_FAMILY == 0
NGDBF_DISPATCH_FAMILY(dispatch_ext_multi, ngdbf::kExtMulti)
#endif
#if !defined(NGDBF_EXT_FAMILY) || NGDBF_EXT_FAMILY == 1
NGDBF_DISPATCH_FAMILY(dispatch_ext_single, ngdbf::kExtSingle)
#endif
#if !defined(NGDBF_EXT_FAMILY) || NGDBF_EXT_FAMILY == 2
NGDBF_DISPATCH_FAMILY(dispatch_ext_switch, ngdbf::kExtSwitch)
#endif
#if !defined(NGDBF_EXT_FAMILY) || NGDBF_EXT_FAMILY == 3
NGDBF_DISPATCH_FAMILY(dispatch_ext_packed, ngdbf::kExtQuantReuse)
#endif

}  // namespace ngdbf_host
