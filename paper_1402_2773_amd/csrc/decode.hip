// decode.hip -- NGDBF decode kernels for gfx950 and the C ABI of ngdbf.h.
//
// Data layout.
//   HBM: y frame-major [F][n] (float32 or int8), sigma [F], outputs
//        out_bits [F][ceil(n/8)], out_iters [F], out_converged [F].
//   Code tables (library-owned, uploaded once): one blob of uint16 arrays
//        row_ptr[m+1] | col_idx[nnz] | col_ptr[n+1] | row_idx[nnz]
//        i.e. N(i) in CSR and M(k) in CSC (Sec. III-A), staged into LDS once
//        per workgroup and reused for every frame the workgroup decodes.
//   LDS per workgroup: the table blob, the decisions x (one byte per bit,
//        1 = x_k is -1) and the syndrome s (one byte per check, 1 = s_i is -1).
//   Registers: each lane owns QPL bit quads (bits 4j .. 4j+3, j = lane +
//        blockDim * r) and keeps their saturated y_k, thresholds theta_k and
//        smoothing counters X_k; the quad is also the unit of one Philox call.
//
// One workgroup decodes one frame at a time and loops over frames with a
// grid stride (persistent grid sized to the resident capacity).  Per round:
//   phase A  every lane forms the syndromes of its checks from LDS x,
//            a workgroup OR gives the stop test (Sec. III-B Steps 1, 4);
//   phase B  every lane forms S_k = sum_{i in M(k)} s_i for its bits from LDS
//            s, draws its quad's four Gaussians, evaluates E_k and applies
//            the flip / threshold update (Steps 2, 3b; Sec. III-C, III-D).
// HBM is touched once per frame (y in, bits out); all rounds run on chip.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdarg>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/ngdbf.h"
#include "noise.h"

namespace ngdbf {

struct DecodeArgs {
  const uint32_t *tables;  // code blob (dwords)
  int32_t n, m, nnz;
  int32_t blob_words;      // dwords in the blob
  int32_t off_col, off_colptr, off_row;  // uint16 offsets (row_ptr at 0)
  const void *y;
  int64_t n_frames;
  const float *sigma;
  float sigma_scalar;
  float w, theta, lambda, eta, ymax;
  int32_t t_max, smooth_window;
  uint32_t key0, key1;
  uint64_t frame_base;
  uint8_t *out_bits;
  int32_t *out_iters;
  uint8_t *out_conv;
  uint8_t *trace;
};

template <int YFMT>
__device__ __forceinline__ float load_sample(const void *y, int64_t idx) {
  if (YFMT == NGDBF_Y_I8) {
    // int8 code y_q; y = y_q / 16 exactly
    return (float)((const int8_t *)y)[idx] * 0.0625f;
  } else {
    return ((const float *)y)[idx];
  }
}

// Saturation at Y_max (Sec. IV-A); ymax <= 0 disables it.  Written as two
// comparisons so that a NaN sample passes through unchanged.
__device__ __forceinline__ float saturate(float v, float ymax) {
  if (ymax > 0.0f) {
    v = (v < -ymax) ? -ymax : v;
    v = (v > ymax) ? ymax : v;
  }
  return v;
}

template <int QPL, int YFMT, bool TRACE>
__global__ void __launch_bounds__(1024) decode_kernel(DecodeArgs a) {
  extern __shared__ uint32_t lds[];
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const int n = a.n, m = a.m;
  const int nq = (n + 3) >> 2;
  const int nbytes = (n + 7) >> 3;
  const int T = a.t_max, W = a.smooth_window;

  // stage the code tables once per workgroup
  for (int i = tid; i < a.blob_words; i += B) lds[i] = a.tables[i];
  const uint16_t *t16 = (const uint16_t *)lds;
  const uint16_t *row_ptr = t16;
  const uint16_t *col_idx = t16 + a.off_col;
  const uint16_t *col_ptr = t16 + a.off_colptr;
  const uint16_t *row_idx = t16 + a.off_row;
  uint8_t *xb = (uint8_t *)(lds + a.blob_words);          // [n]  1 = x_k is -1
  uint8_t *sb = xb + ((n + 3) & ~3);                        // [m]  1 = s_i is -1
  uint8_t *fb = sb + ((m + 3) & ~3);                        // [n]  flips (trace)
  __syncthreads();

  for (int64_t f = blockIdx.x; f < a.n_frames; f += gridDim.x) {
    const uint64_t frame = a.frame_base + (uint64_t)f;
    const float sigma_f = a.sigma ? a.sigma[f] : a.sigma_scalar;
    const float qs = a.eta * sigma_f;  // perturbation std (Sec. III-C)

    // Step 0 and x(0) = sign(y): -1 iff the saturated sample is < 0
    float yv[QPL * 4], thr[QPL * 4];
    int X[QPL * 4];
    uint32_t xneg = 0;  // bit 4r+b: x of bit 4(tid+B r)+b is -1
#pragma unroll
    for (int r = 0; r < QPL; ++r) {
      const int j = tid + B * r;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 4 * j + b;
        float v = 0.0f;
        if (j < nq && k < n) v = saturate(load_sample<YFMT>(a.y, f * (int64_t)n + k), a.ymax);
        yv[4 * r + b] = v;
        thr[4 * r + b] = a.theta;
        X[4 * r + b] = 0;
        const uint32_t neg = (v < 0.0f) ? 1u : 0u;
        xneg |= neg << (4 * r + b);
        if (j < nq && k < n) xb[k] = (uint8_t)neg;
      }
    }
    __syncthreads();

    int t = 0;
    int converged = 0;
    for (;; ++t) {
      // phase A: s_i = prod_{j in N(i)} x_j  (XOR of the -1 flags)
      int unsat = 0;
      for (int i = tid; i < m; i += B) {
        uint32_t v = 0;
        const int e1 = row_ptr[i + 1];
        for (int e = row_ptr[i]; e < e1; ++e) v ^= xb[col_idx[e]];
        sb[i] = (uint8_t)v;
        unsat |= (int)v;
      }
      // smoothing window t = T-W .. T (Sec. III-E)
      if (W > 0 && t >= T - W) {
#pragma unroll
        for (int q = 0; q < QPL * 4; ++q) X[q] += ((xneg >> q) & 1u) ? -1 : 1;
      }
      unsat = __syncthreads_or(unsat);
      if (!unsat) {
        converged = 1;
        break;
      }
      if (t == T) break;

      // phase B: E_k and the flip / adaptation of every owned bit
#pragma unroll
      for (int r = 0; r < QPL; ++r) {
        const int j = tid + B * r;
        if (j < nq) {
          const Draw4 d = draw_quad((uint32_t)j, (uint32_t)t, frame, a.key0, a.key1);
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int k = 4 * j + b;
            const int q = 4 * r + b;
            if (k < n) {
              int S = 0;
              const int e1 = col_ptr[k + 1];
              for (int e = col_ptr[k]; e < e1; ++e) S += sb[row_idx[e]] ? -1 : 1;
              const float xk = ((xneg >> q) & 1u) ? -1.0f : 1.0f;
              const float av = __builtin_fmaf(a.w, (float)S, xk * yv[q]);
              const float E = __builtin_fmaf(qs, d.z[b], av);
              const bool flip = E < thr[q];
              if (flip) {
                xneg ^= 1u << q;
                xb[k] = (uint8_t)((xneg >> q) & 1u);
              } else {
                thr[q] = thr[q] * a.lambda;
              }
              if (TRACE) fb[k] = flip ? 1 : 0;
            }
          }
        }
      }
      __syncthreads();
      if (TRACE) {
        uint8_t *row = a.trace + ((size_t)f * (size_t)T + (size_t)t) * (size_t)nbytes;
        for (int bb = tid; bb < nbytes; bb += B) {
          uint32_t v = 0;
          for (int i = 0; i < 8; ++i) {
            const int k = 8 * bb + i;
            if (k < n) v |= (uint32_t)fb[k] << i;
          }
          row[bb] = (uint8_t)v;
        }
      }
    }

    // output: x, or sign(X) when T was reached with smoothing on
    if (!converged && W > 0) {
#pragma unroll
      for (int r = 0; r < QPL; ++r) {
        const int j = tid + B * r;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int k = 4 * j + b;
          if (j < nq && k < n) xb[k] = (uint8_t)(X[4 * r + b] < 0 ? 1 : 0);
        }
      }
    }
    __syncthreads();
    uint8_t *ob = a.out_bits + (size_t)f * (size_t)nbytes;
    for (int bb = tid; bb < nbytes; bb += B) {
      uint32_t v = 0;
      for (int i = 0; i < 8; ++i) {
        const int k = 8 * bb + i;
        if (k < n) v |= (uint32_t)xb[k] << i;
      }
      ob[bb] = (uint8_t)v;
    }
    if (tid == 0) {
      a.out_iters[f] = t;
      if (a.out_conv) a.out_conv[f] = (uint8_t)converged;
    }
    __syncthreads();  // xb is rewritten by the next frame
  }
}

// ---------------------------------------------------------------- probes

__global__ void probe_radius_kernel(uint32_t start, uint32_t count, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) out[j] = bm_radius(start + j);
}

__global__ void probe_turn_kernel(uint32_t start, uint32_t count, float *co, float *si) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    float c, s;
    bm_turn(start + j, c, s);
    co[j] = c;
    si[j] = s;
  }
}

__global__ void probe_quad_kernel(uint32_t start, uint32_t count, uint64_t frame, uint32_t iter,
                                  uint32_t k0, uint32_t k1, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    const Draw4 d = draw_quad(start + j, iter, frame, k0, k1);
    for (int b = 0; b < 4; ++b) out[4 * (size_t)j + b] = d.z[b];
  }
}

}  // namespace ngdbf

// ==================================================================== host

struct ngdbf_code {
  int32_t n, m, nnz;
  int device;
  uint32_t *d_blob;
  int32_t blob_words;
  int32_t off_col, off_colptr, off_row;
  int32_t max_col_deg, max_row_deg;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return NGDBF_OK;
}

struct DeviceInfo {
  int cus = 0;
  size_t lds_max = 0;
};

DeviceInfo device_info(int dev) {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  std::lock_guard<std::mutex> g(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  if (cache[dev].cus == 0) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
      cache[dev].cus = p.multiProcessorCount;
      cache[dev].lds_max = p.sharedMemPerBlock;
    }
  }
  return cache[dev];
}

template <int QPL, int YFMT, bool TRACE>
int launch(const ngdbf::DecodeArgs &a, int block, size_t lds_bytes, int dev, hipStream_t s) {
  auto kern = ngdbf::decode_kernel<QPL, YFMT, TRACE>;
  if (lds_bytes > 64 * 1024) {
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes) != hipSuccess)
      return fail(NGDBF_EDEVICE, "cannot raise the LDS limit to %zu bytes", lds_bytes);
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds_bytes) != hipSuccess ||
      per_cu <= 0)
    return fail(NGDBF_EUNSUPPORTED, "kernel does not fit a compute unit (block %d, LDS %zu B)",
                block, lds_bytes);
  const DeviceInfo di = device_info(dev);
  int64_t grid = (int64_t)per_cu * std::max(di.cus, 1);
  grid = std::min<int64_t>(grid, a.n_frames);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(block), lds_bytes, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

template <int YFMT, bool TRACE>
int dispatch_qpl(int qpl, const ngdbf::DecodeArgs &a, int block, size_t lds, int dev,
                 hipStream_t s) {
  switch (qpl) {
    case 1: return launch<1, YFMT, TRACE>(a, block, lds, dev, s);
    case 2: return launch<2, YFMT, TRACE>(a, block, lds, dev, s);
    case 4: return launch<4, YFMT, TRACE>(a, block, lds, dev, s);
    default: return fail(NGDBF_EUNSUPPORTED, "no kernel for %d quads per lane", qpl);
  }
}

int check_params(const ngdbf_params *p) {
  if (!p) return fail(NGDBF_EINVAL, "params is NULL");
  if (!(p->w > 0.0f) || !std::isfinite(p->w)) return fail(NGDBF_EINVAL, "w must be finite and > 0");
  if (!std::isfinite(p->theta)) return fail(NGDBF_EINVAL, "theta must be finite");
  if (!(p->lambda > 0.0f && p->lambda <= 1.0f))
    return fail(NGDBF_EINVAL, "lambda must be in (0, 1]");
  if (!(p->eta >= 0.0f) || !std::isfinite(p->eta)) return fail(NGDBF_EINVAL, "eta must be finite and >= 0");
  if (std::isnan(p->ymax)) return fail(NGDBF_EINVAL, "ymax is NaN");
  if (p->t_max < 0 || p->t_max > 65535) return fail(NGDBF_EINVAL, "t_max must be in [0, 65535]");
  if (p->smooth_window < 0) return fail(NGDBF_EINVAL, "smooth_window must be >= 0");
  if (p->y_format != NGDBF_Y_F32 && p->y_format != NGDBF_Y_I8)
    return fail(NGDBF_EINVAL, "unknown y_format %d", p->y_format);
  return NGDBF_OK;
}

int decode_common(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                  float sigma_scalar, const ngdbf_params *p, uint64_t seed, uint64_t frame_base,
                  uint8_t *out_bits, int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
                  void *stream) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (n_frames < 0) return fail(NGDBF_EINVAL, "n_frames < 0");
  if (n_frames > 0 && (!y || !out_bits || !out_iters))
    return fail(NGDBF_EINVAL, "y, out_bits and out_iters are required");
  if (!sigma && (!(sigma_scalar >= 0.0f) || !std::isfinite(sigma_scalar)))
    return fail(NGDBF_EINVAL, "sigma_scalar must be finite and >= 0");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  if (dev != code->device)
    return fail(NGDBF_EINVAL, "code lives on device %d, current device is %d", code->device, dev);
  // report an earlier asynchronous fault before queueing more work
  const hipError_t pending = hipGetLastError();
  if (pending != hipSuccess)
    return fail(NGDBF_EDEVICE, "earlier HIP error: %s", hipGetErrorString(pending));
  hipStream_t s = (hipStream_t)stream;
  const int n = code->n, m = code->m;
  const int nbytes = (n + 7) / 8;
  if (trace && n_frames > 0 && p->t_max > 0) {
    const size_t tb = (size_t)n_frames * (size_t)p->t_max * (size_t)nbytes;
    if (hipMemsetAsync(trace, 0, tb, s) != hipSuccess)
      return fail(NGDBF_EDEVICE, "trace clear failed");
  }
  if (n_frames == 0) return ok();

  ngdbf::DecodeArgs a;
  a.tables = code->d_blob;
  a.n = n;
  a.m = m;
  a.nnz = code->nnz;
  a.blob_words = code->blob_words;
  a.off_col = code->off_col;
  a.off_colptr = code->off_colptr;
  a.off_row = code->off_row;
  a.y = y;
  a.n_frames = n_frames;
  a.sigma = sigma;
  a.sigma_scalar = sigma_scalar;
  a.w = p->w;
  a.theta = p->theta;
  a.lambda = p->lambda;
  a.eta = p->eta;
  a.ymax = p->ymax;
  a.t_max = p->t_max;
  a.smooth_window = p->smooth_window;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.frame_base = frame_base;
  a.out_bits = out_bits;
  a.out_iters = out_iters;
  a.out_conv = out_conv;
  a.trace = trace;

  // one lane per bit quad where possible: block = next power of two >= quads
  const int nq = (n + 3) / 4;
  int block = 64;
  while (block < nq && block < 1024) block *= 2;
  int qpl = (nq + block - 1) / block;
  if (qpl == 3) qpl = 4;
  const size_t lds = (size_t)code->blob_words * 4 + (size_t)((n + 3) & ~3) +
                     (size_t)((m + 3) & ~3) + (size_t)((n + 3) & ~3);
  const DeviceInfo di = device_info(dev);
  if (di.lds_max && lds > 160 * 1024)
    return fail(NGDBF_EUNSUPPORTED, "code needs %zu B of LDS", lds);
  if (p->y_format == NGDBF_Y_I8) {
    return trace ? dispatch_qpl<NGDBF_Y_I8, true>(qpl, a, block, lds, dev, s)
                 : dispatch_qpl<NGDBF_Y_I8, false>(qpl, a, block, lds, dev, s);
  }
  return trace ? dispatch_qpl<NGDBF_Y_F32, true>(qpl, a, block, lds, dev, s)
               : dispatch_qpl<NGDBF_Y_F32, false>(qpl, a, block, lds, dev, s);
}

}  // namespace

extern "C" {

const char *ngdbf_last_error(void) { return g_err; }

int ngdbf_create_code(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col_idx,
                      ngdbf_code **out) {
  if (!out) return fail(NGDBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!row_ptr || !col_idx) return fail(NGDBF_EINVAL, "row_ptr and col_idx are required");
  if (m < 1 || n <= m || n > 65535) return fail(NGDBF_EINVAL, "need 1 <= m < n <= 65535");
  if (row_ptr[0] != 0) return fail(NGDBF_EINVAL, "row_ptr[0] must be 0");
  for (int i = 0; i < m; ++i) {
    if (row_ptr[i + 1] <= row_ptr[i]) return fail(NGDBF_EINVAL, "row %d is empty or row_ptr decreases", i);
  }
  const int64_t nnz = row_ptr[m];
  if (nnz > 65535) return fail(NGDBF_EUNSUPPORTED, "nnz %lld exceeds 65535", (long long)nnz);
  std::vector<int32_t> colcnt(n + 1, 0);
  for (int i = 0; i < m; ++i) {
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int c = col_idx[e];
      if (c < 0 || c >= n) return fail(NGDBF_EINVAL, "col_idx[%d] = %d out of range", e, c);
      for (int e2 = row_ptr[i]; e2 < e; ++e2)
        if (col_idx[e2] == c) return fail(NGDBF_EINVAL, "row %d repeats column %d", i, c);
      colcnt[c + 1]++;
    }
  }
  for (int k = 0; k < n; ++k)
    if (colcnt[k + 1] == 0) return fail(NGDBF_EINVAL, "column %d is empty", k);
  std::vector<int32_t> colptr(n + 1, 0);
  for (int k = 0; k < n; ++k) colptr[k + 1] = colptr[k] + colcnt[k + 1];
  std::vector<int32_t> rowidx(nnz), fill(colptr.begin(), colptr.end() - 1);
  for (int i = 0; i < m; ++i)
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) rowidx[fill[col_idx[e]]++] = i;

  // blob of uint16: row_ptr[m+1] | col_idx[nnz] | col_ptr[n+1] | row_idx[nnz]
  const int off_col = m + 1;
  const int off_colptr = off_col + (int)nnz;
  const int off_row = off_colptr + n + 1;
  const int total16 = off_row + (int)nnz;
  const int words = (total16 + 1) / 2;
  std::vector<uint16_t> blob((size_t)words * 2, 0);
  int maxr = 0, maxc = 0;
  for (int i = 0; i <= m; ++i) blob[i] = (uint16_t)row_ptr[i];
  for (int64_t e = 0; e < nnz; ++e) blob[off_col + e] = (uint16_t)col_idx[e];
  for (int k = 0; k <= n; ++k) blob[off_colptr + k] = (uint16_t)colptr[k];
  for (int64_t e = 0; e < nnz; ++e) blob[off_row + e] = (uint16_t)rowidx[e];
  for (int i = 0; i < m; ++i) maxr = std::max(maxr, row_ptr[i + 1] - row_ptr[i]);
  for (int k = 0; k < n; ++k) maxc = std::max(maxc, colptr[k + 1] - colptr[k]);

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  ngdbf_code *c = (ngdbf_code *)calloc(1, sizeof(ngdbf_code));
  if (!c) return fail(NGDBF_ENOMEM, "host allocation failed");
  c->n = n;
  c->m = m;
  c->nnz = (int32_t)nnz;
  c->device = dev;
  c->blob_words = words;
  c->off_col = off_col;
  c->off_colptr = off_colptr;
  c->off_row = off_row;
  c->max_row_deg = maxr;
  c->max_col_deg = maxc;
  if (hipMalloc((void **)&c->d_blob, (size_t)words * 4) != hipSuccess) {
    free(c);
    return fail(NGDBF_ENOMEM, "device allocation of %d words failed", words);
  }
  if (hipMemcpy(c->d_blob, blob.data(), (size_t)words * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->d_blob);
    free(c);
    return fail(NGDBF_EDEVICE, "upload of the code tables failed");
  }
  *out = c;
  return ok();
}

int ngdbf_destroy_code(ngdbf_code *code) {
  if (!code) return ok();
  const hipError_t e = hipFree(code->d_blob);
  free(code);
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "hipFree failed: %s", hipGetErrorString(e));
  return ok();
}

int ngdbf_code_info(const ngdbf_code *code, int32_t *n, int32_t *m, int32_t *nnz) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n) *n = code->n;
  if (m) *m = code->m;
  if (nnz) *nnz = code->nnz;
  return ok();
}

int ngdbf_decode(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                 float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                 uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                 uint8_t *out_converged, void *stream) {
  return decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                       out_iters, out_converged, nullptr, stream);
}

int ngdbf_decode_trace(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                       float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                       uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                       uint8_t *out_converged, uint8_t *flip_masks, void *stream) {
  if (n_frames > 0 && params && params->t_max > 0 && !flip_masks)
    return fail(NGDBF_EINVAL, "flip_masks is required");
  return decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                       out_iters, out_converged, flip_masks ? flip_masks : nullptr, stream);
}

int ngdbf_noise_probe(int32_t kind, uint32_t start, uint32_t count, uint64_t seed, uint64_t frame,
                      uint32_t iter, float *out0, float *out1, void *stream) {
  if (count == 0) return ok();
  if (!out0) return fail(NGDBF_EINVAL, "out0 is NULL");
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (count + 255) / 256;
  if (kind == 0) {
    if (start < 1 || (uint64_t)start + count - 1 > (1ull << 24))
      return fail(NGDBF_EINVAL, "radius probe range must lie in [1, 2^24]");
    hipLaunchKernelGGL(ngdbf::probe_radius_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0);
  } else if (kind == 1) {
    if (!out1) return fail(NGDBF_EINVAL, "out1 is NULL");
    if ((uint64_t)start + count > (1ull << 24))
      return fail(NGDBF_EINVAL, "angle probe range must lie in [0, 2^24)");
    hipLaunchKernelGGL(ngdbf::probe_turn_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0,
                       out1);
  } else if (kind == 2) {
    hipLaunchKernelGGL(ngdbf::probe_quad_kernel, dim3(blocks), dim3(256), 0, s, start, count, frame,
                       iter, (uint32_t)seed, (uint32_t)(seed >> 32), out0);
  } else {
    return fail(NGDBF_EINVAL, "unknown probe kind %d", kind);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "probe launch failed: %s", hipGetErrorString(e));
  return ok();
}

}  // extern "C"
