// probe.hip -- vector-ALU issue-rate probe (device code and its C entry).
//
// The decoder is bound by vector-ALU issue, and on gfx950 the issue time of a
// wave64 instruction depends on its class: 32-bit integer, bitwise, shift,
// conversion and 64-bit-product instructions hold a SIMD for four clocks,
// binary32 fma / mul / add for two, transcendental ones (sqrt, rcp, log)
// for eight.  This probe runs long unrolled chains of one class so that the
// benchmark can measure those issue times on the machine it runs on and
// weight the hardware counters of each class by them.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ngdbf.h"

namespace ngdbf {

constexpr int kProbeChains = 8;
constexpr int kProbeUnroll = 16;

template <int KIND>
__global__ void __launch_bounds__(256) issue_probe_kernel(uint32_t *out, int iters) {
  uint32_t v[kProbeChains];
  float f[kProbeChains];
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    v[c] = gid * 2654435761u + 97u * (uint32_t)c;
    f[c] = 1.0f + (float)(v[c] & 1023u) * 0.001f;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) {
        if (KIND == 0) {  // 32-bit integer: (v ^ k) + u, one v_xad_u32
          v[c] = (v[c] ^ 0x9E3779B9u) + (uint32_t)u;
        } else if (KIND == 1) {  // 64-bit product (v_mad_u64_u32) and a xor
          const uint64_t p = (uint64_t)0xD2511F53u * v[c];
          v[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
        } else if (KIND == 2) {  // binary32 fma
          f[c] = __builtin_fmaf(f[c], 0.999f, 0.001f);
        } else if (KIND == 3) {  // binary32 multiply
          f[c] = f[c] * 0.999f;
        } else {  // transcendental: hardware square root
          f[c] = __builtin_amdgcn_sqrtf(f[c]);
        }
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc ^= v[c] ^ __float_as_uint(f[c]);
  out[gid] = acc;
}

}  // namespace ngdbf

extern "C" ngdbf_status ngdbf_issue_probe(int32_t kind, int32_t blocks, int32_t iters,
                                          uint32_t *out, void *stream) {
  if (kind < 0 || kind > 4 || blocks < 1 || iters < 1 || !out) return NGDBF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const dim3 g((unsigned)blocks), b(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(ngdbf::issue_probe_kernel<0>, g, b, 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(ngdbf::issue_probe_kernel<1>, g, b, 0, s, out, iters); break;
    case 2: hipLaunchKernelGGL(ngdbf::issue_probe_kernel<2>, g, b, 0, s, out, iters); break;
    case 3: hipLaunchKernelGGL(ngdbf::issue_probe_kernel<3>, g, b, 0, s, out, iters); break;
    default: hipLaunchKernelGGL(ngdbf::issue_probe_kernel<4>, g, b, 0, s, out, iters); break;
  }
  return hipGetLastError() == hipSuccess ? NGDBF_OK : NGDBF_EDEVICE;
}
