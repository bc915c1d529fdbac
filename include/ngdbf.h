/*
 * ngdbf.h -- C ABI of the MI355X (gfx950) NGDBF decoder.
 *
 * Noisy Gradient-Descent Bit-Flip decoding of binary LDPC codes
 * (Sundararajan, Winstead, Boutillon, IEEE TCOM 2014).  One decode call runs
 * the multi-bit NGDBF iteration of Sec. III on many received frames at once:
 *
 *   Step 0 / III-A : y_k saturated at Y_max (Sec. IV-A), x_k(0) = sign(y_k),
 *                    theta_k = theta
 *   Step 1         : s_i = prod_{j in N(i)} x_j; stop when every s_i = +1
 *   Step 2 (III-C) : E_k = x_k y_k + w sum_{i in M(k)} s_i + q_k,
 *                    q_k ~ N(0, (eta sigma)^2)
 *   Step 3b (III-D): flip x_k if E_k < theta_k, else theta_k <- lambda theta_k
 *   III-E          : optional smoothing, output sign(sum of x_k(t) over the
 *                    last W+1 states) when T is reached unconverged
 *
 * Arithmetic is IEEE binary32 with a fixed fma order and a counter-based
 * Gaussian source, so that results are reproducible bit for bit:
 *   a_k = fmaf(w, (float)S_k, x_k * y_k),  E_k = fmaf(fl(eta*sigma), z_k, a_k)
 *   z_k: Philox4x32-10 (Salmon et al., SC'11) with key = seed and counter
 *        (k >> 2, t, frame & 0xffffffff, frame >> 32), frame = frame_base + f;
 *        the four output words feed two Box-Muller pairs (bits 4j .. 4j+3).
 *
 * Conventions for every entry point:
 *  - All functions return an ngdbf_status; on failure ngdbf_last_error()
 *    returns a message for the calling thread.  Argument errors are detected
 *    on the host before any device work is queued.
 *  - "dev" pointers are device memory of the current HIP device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns code handles and their device tables.
 *  - stream is a hipStream_t (NULL = the null stream).  Decode calls are
 *    asynchronous: outputs are valid once the stream has been synchronised.
 *    A device fault surfaces as NGDBF_EDEVICE from a later call.
 */
#ifndef NGDBF_H
#define NGDBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NGDBF_OK = 0,
    NGDBF_EINVAL = -1,       /* invalid argument                              */
    NGDBF_ENOMEM = -2,       /* device or host allocation failed             */
    NGDBF_EDEVICE = -3,      /* HIP runtime error                             */
    NGDBF_EUNSUPPORTED = -4  /* valid, but outside what the kernels support  */
} ngdbf_status;

/* Opaque handle: a parity-check matrix H resident on one device. */
typedef struct ngdbf_code ngdbf_code;

/* y storage formats */
#define NGDBF_Y_F32 0        /* float32 samples                               */
#define NGDBF_Y_I8 1         /* int8 codes y_q; the decoder uses y = y_q/16    */

/* Decoder parameters (paper notation; Sec. III-B..E, IV-A). */
typedef struct {
    float w;              /* syndrome weight w > 0 (Sec. III-C Step 2)          */
    float theta;          /* initial threshold theta (Step 0 / 3b), finite      */
    float lambda;         /* adaptation factor, 0 < lambda <= 1; 1 = plain      */
    float eta;            /* perturbation scale eta >= 0; 0 = GDBF (no noise)   */
    float ymax;           /* saturation Y_max (Sec. IV-A); <= 0 disables it     */
    int32_t t_max;        /* iteration limit T, 0 <= T <= 65535 (Step 4)         */
    int32_t smooth_window;/* 0 = off; W > 0: smoothing over t = T-W .. T (III-E) */
    int32_t y_format;     /* NGDBF_Y_F32 or NGDBF_Y_I8                           */
} ngdbf_params;

/*
 * ngdbf_create_code -- upload H (Sec. III-A: N(i) row supports, M(k) column
 * supports) to the current device.
 *   n, m     : bits (columns) and checks (rows), 1 <= m < n <= 65535.
 *   row_ptr  : host, int32 [m+1], row_ptr[0] = 0, non-decreasing.
 *   col_idx  : host, int32 [row_ptr[m]], N(i) = col_idx[row_ptr[i] ..
 *              row_ptr[i+1]-1], each in [0, n), no repeats within a row.
 *   out      : receives the handle.
 * The arrays are copied; the column supports M(k) are built here.
 * Errors: NGDBF_EINVAL (bad sizes, indices, empty row or column),
 * NGDBF_EUNSUPPORTED (a column degree above 15, an irregular code with more
 * than 65535 edges), NGDBF_ENOMEM, NGDBF_EDEVICE.  A code whose tables do not
 * fit the LDS of any launch shape is refused by the decode calls.
 */
int ngdbf_create_code(int32_t n, int32_t m, const int32_t *row_ptr,
                      const int32_t *col_idx, ngdbf_code **out);

/* Release a handle and its device tables (NULL is accepted). The caller must
 * ensure no decode using it is still running. */
int ngdbf_destroy_code(ngdbf_code *code);

/* Sizes of a handle: n, m, nnz (any output pointer may be NULL). */
int ngdbf_code_info(const ngdbf_code *code, int32_t *n, int32_t *m,
                    int32_t *nnz);

/*
 * ngdbf_decode -- decode n_frames received frames (Sec. III, all steps).
 *   y          : dev, frame-major [n_frames][n], float32 or int8 (params->y_format).
 *   n_frames   : >= 0 (0 queues nothing).
 *   sigma      : dev float32 [n_frames] channel std per frame, or NULL to use
 *                sigma_scalar for every frame; the perturbation std is
 *                fl(eta * sigma) (Sec. III-C).  sigma must be >= 0 and finite.
 *   params     : host.
 *   seed       : Philox key.  frame_base: global index of frame 0 (noise
 *                counter), so a split or resumed run reproduces per-frame results.
 *   out_bits   : dev uint8 [n_frames][ceil(n/8)], c_k = (1 - x_k)/2 of the
 *                returned decision, bit k of byte k/8 (LSB first).
 *   out_iters  : dev int32 [n_frames]: completed flip rounds, in [0, T].
 *   out_converged : dev uint8 [n_frames] (may be NULL): 1 if the stop test
 *                (every s_i = +1) ended decoding, 0 if T was reached.
 *   stream     : hipStream_t.
 * Errors: NGDBF_EINVAL (NULL pointers with n_frames > 0, parameters out of
 * range), NGDBF_EDEVICE (launch failure, or an earlier fault reported now).
 */
int ngdbf_decode(const ngdbf_code *code, const void *y, int64_t n_frames,
                 const float *sigma, float sigma_scalar,
                 const ngdbf_params *params, uint64_t seed, uint64_t frame_base,
                 uint8_t *out_bits, int32_t *out_iters, uint8_t *out_converged,
                 void *stream);

/*
 * ngdbf_decode_trace -- ngdbf_decode that also records every flip decision
 * (Sec. III-B Step 3b) for parity checks of whole trajectories.
 *   flip_masks : dev uint8 [n_frames][T][ceil(n/8)]; bit k of row t is set
 *                iff x_k was flipped in round t.  Rows of rounds that did not
 *                run are written as zero.
 * Other arguments and errors as ngdbf_decode.  Slower; for verification.
 */
int ngdbf_decode_trace(const ngdbf_code *code, const void *y, int64_t n_frames,
                       const float *sigma, float sigma_scalar,
                       const ngdbf_params *params, uint64_t seed,
                       uint64_t frame_base, uint8_t *out_bits,
                       int32_t *out_iters, uint8_t *out_converged,
                       uint8_t *flip_masks, void *stream);

/*
 * ngdbf_noise_probe -- evaluate the decoder's own Gaussian-source pieces on
 * the device, for exhaustive comparison with an independent implementation.
 *   kind 0: out0[j] = rho(m) = sqrt(-2 ln(m 2^-24)) for m = start + j
 *           (start >= 1, start + count - 1 <= 2^24).
 *   kind 1: out0[j], out1[j] = cos, sin of 2 pi i 2^-24 for i = start + j
 *           (start + count <= 2^24).
 *   kind 2: out0[4j .. 4j+3] = the four N(0,1) draws of bit quad start + j
 *           of frame `frame` at iteration `iter` under key `seed`.
 *   out0/out1: dev float32 (out1 only for kind 1).  count >= 0.
 * Errors: NGDBF_EINVAL (kind or range), NGDBF_EDEVICE.
 */
int ngdbf_noise_probe(int32_t kind, uint32_t start, uint32_t count,
                      uint64_t seed, uint64_t frame, uint32_t iter,
                      float *out0, float *out1, void *stream);

/*
 * Launch shape of a code's decode kernel (all shapes give identical results):
 *   waves_per_frame : wavefronts cooperating on one frame (1, 2, 4, 8, 16);
 *   quads_per_lane  : bit quads each lane owns (1, 2, 4); a frame holds at most
 *                     64 * waves_per_frame * quads_per_lane quads (4 bits each);
 *   frames_per_block: frames per workgroup (1 unless waves_per_frame == 1, then
 *                     2, 4, 8 or 16).
 * ngdbf_code_set_shape fixes the shape used by later decodes of this code
 * (NGDBF_EINVAL if it does not fit the code, NGDBF_EUNSUPPORTED if it was not
 * built or exceeds the LDS); all-zero arguments restore the default choice.
 * ngdbf_code_get_shape reports the shape in use (host int32 [3]).
 * Not thread-safe against concurrent decodes of the same code.
 */
int ngdbf_code_set_shape(ngdbf_code *code, int32_t waves_per_frame,
                         int32_t quads_per_lane, int32_t frames_per_block);
int ngdbf_code_get_shape(const ngdbf_code *code, int32_t shape[3]);

/*
 * ngdbf_autotune -- time every built launch shape that fits the code on the
 * given sample (same arguments as ngdbf_decode; outputs go to scratch the
 * call allocates and frees) and keep the fastest on the code handle.  The
 * sample should hold several times the frames the GPU keeps resident (tens of
 * thousands): on a small sample the shapes that shorten one frame's latency
 * win, on a large batch those that maximise throughput.
 *   best : host int32 [3] (may be NULL), receives the chosen shape.
 *   elapsed_ms : host float (may be NULL), its time on the sample.
 * Synchronises the stream.  Errors as ngdbf_decode, NGDBF_ENOMEM.
 */
int ngdbf_autotune(ngdbf_code *code, const void *y, int64_t n_frames,
                   const float *sigma, float sigma_scalar,
                   const ngdbf_params *params, uint64_t seed, int32_t best[3],
                   float *elapsed_ms, void *stream);

/* One independent decode of a batch (fields as the ngdbf_decode arguments). */
typedef struct {
    const ngdbf_code *code;
    const void *y;
    int64_t n_frames;
    const float *sigma;
    float sigma_scalar;
    ngdbf_params params;
    uint64_t seed;
    uint64_t frame_base;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_converged;
} ngdbf_job;

/*
 * ngdbf_decode_batch -- decode several jobs (frames of different codes,
 * parameters and SNRs, Sec. III for each) as one unit of work on `stream`:
 * the jobs run concurrently on library-owned streams forked from and joined
 * back to `stream` with events, so the whole batch is one node group when
 * the caller captures `stream` into a hipGraph.  Every job is validated
 * before any work is queued.  Results equal those of ngdbf_decode per job.
 * jobs: host array [n_jobs]; all codes on the current device.
 * Errors: NGDBF_EINVAL (any job invalid, n_jobs < 0), NGDBF_EDEVICE.
 */
int ngdbf_decode_batch(const ngdbf_job *jobs, int32_t n_jobs, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *ngdbf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
