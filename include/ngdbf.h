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
    NGDBF_EUNSUPPORTED = -4, /* valid, but outside what the kernels support  */
    NGDBF_EBUSY = -5         /* every frame queue a launch could take is
                                held by a launch in flight (see ngdbf_decode) */
} ngdbf_status;

/* Opaque handle: a parity-check matrix H resident on one device. */
typedef struct ngdbf_code ngdbf_code;

/* y storage formats */
#define NGDBF_Y_F32 0        /* float32 samples                               */
#define NGDBF_Y_I8 1         /* int8 codes y_q; the decoder uses y = y_q/16    */

/* Bit-flip rules (Sec. III-B Step 3) */
#define NGDBF_MULTI 0        /* flip every bit with E_k < theta_k (Step 3b)     */
#define NGDBF_SINGLE 1       /* flip the one bit of least E_k, ties to the
                                lowest index (Step 3a): S-NGDBF, S-GDBF         */
#define NGDBF_MODE_SWITCH 2  /* Step 3b until the objective f(x) = sum x_k y_k +
                                sum s_i first decreases from one round to the
                                next, Step 3a from then on (mode switching)     */

/* Decoder parameters (paper notation; Sec. III-B..E, IV-A, IV-E, V-A, V-B). */
typedef struct {
    float w;              /* syndrome weight w > 0 (Sec. III-C Step 2)          */
    float theta;          /* initial threshold theta (Step 0 / 3b), finite      */
    float lambda;         /* adaptation factor, 0 < lambda <= 1; 1 = plain      */
    float eta;            /* perturbation scale eta >= 0; 0 = GDBF (no noise)   */
    float ymax;           /* saturation Y_max (Sec. IV-A); <= 0 disables it     */
    int32_t t_max;        /* iteration limit T, 0 <= T <= 65535 (Step 4)         */
    int32_t smooth_window;/* 0 = off; W > 0: smoothing over t = T-W .. T (III-E) */
    int32_t y_format;     /* NGDBF_Y_F32 or NGDBF_Y_I8                           */
    int32_t variant;      /* NGDBF_MULTI, NGDBF_SINGLE or NGDBF_MODE_SWITCH      */
    int32_t quant_bits;   /* 0: binary32 arithmetic.  Q in [1, 8]: the quantized
                             decoder of Sec. IV-E: y_k, w, q_k and theta_k pass
                             through g(v) = sign(v) (floor(|v| N_Q / 2Y_max) +
                             1/2) 2Y_max / N_Q, N_Q = 2^Q (levels capped at
                             N_Q/2 - 1, g(0) = 0), thresholds theta_k(u_k) =
                             g(theta lambda^u_k) with u_k the non-flip count
                             (Sec. V-A).  Needs ymax > 0; not with mode
                             switching.                                         */
    int32_t noise_reuse;  /* 0: a fresh q_k per bit and round.  1: the shift-
                             register chain of Sec. V-B, q_k(t) = q_{k-1}(t-1),
                             one new sample per round: bit k takes element
                             n - 1 + t - k of the frame's stream, whose element
                             j is draw j & 3 of Philox quad j >> 2 under the
                             iteration word 0xFFFFFFFF.  Needs LDS for
                             n + T - 1 samples per frame.                       */
} ngdbf_params;

/*
 * ngdbf_create_code -- upload H (Sec. III-A: N(i) row supports, M(k) column
 * supports) to the current device.
 *   n, m     : bits (columns) and checks (rows), 1 <= m < n <= 65535.
 *   nnz      : edges of H (ones in the matrix), = row_ptr[m], at most 2^24.
 *   row_ptr  : host, int32 [m+1], row_ptr[0] = 0, strictly increasing (no
 *              empty row).
 *   col_idx  : host, int32 [nnz], N(i) = col_idx[row_ptr[i] ..
 *              row_ptr[i+1]-1], each in [0, n), no repeats within a row.
 *   out      : receives the handle.
 * The arrays are copied; the column supports M(k) are built here.  The first
 * code on a device also allocates and clears that device's frame queues
 * (2 x 1024 queues of 9 cache-line-padded counters, 2.4 MB, kept until the
 * process ends; every decode launch takes one queue, see ngdbf_decode), so create codes outside a stream
 * capture.
 * Errors: NGDBF_EINVAL (bad sizes, indices, empty row or column),
 * NGDBF_EUNSUPPORTED (a column degree above 15, an irregular code with more
 * than 65535 edges), NGDBF_ENOMEM, NGDBF_EDEVICE.  A code whose tables do not
 * fit the LDS of any launch shape is refused by the decode calls.
 */
ngdbf_status ngdbf_create_code(int32_t n, int32_t m, int64_t nnz,
                               const int32_t *row_ptr, const int32_t *col_idx,
                               ngdbf_code **out);

/* Release a handle and its device tables (NULL is accepted). The caller must
 * ensure no decode using it is still running. */
ngdbf_status ngdbf_destroy_code(ngdbf_code *code);

/* Sizes of a handle: n, m, nnz (any output pointer may be NULL). */
ngdbf_status ngdbf_code_info(const ngdbf_code *code, int32_t *n, int32_t *m,
                             int32_t *nnz);

/*
 * ngdbf_decode -- decode n_frames received frames (Sec. III, all steps).
 *   y          : dev, frame-major [n_frames][n], float32 or int8 (params->y_format).
 *   n_frames   : >= 0 (0 queues nothing).
 *   sigma      : dev float32 [n_frames] channel std per frame, or NULL to use
 *                sigma_scalar for every frame; the perturbation std is
 *                fl(eta * sigma) (Sec. III-C).  sigma_scalar must be >= 0 and
 *                finite; per-frame values are used as given (a negative value
 *                draws fl(eta * sigma) z_k exactly as the definition says, and
 *                the exact noise skip bounds its magnitude).
 *   params     : host.
 *   seed       : Philox key.  frame_base: global index of frame 0 (noise
 *                counter), so a split or resumed run reproduces per-frame results.
 *   out_bits   : dev uint8 [n_frames][ceil(n/8)], c_k = (1 - x_k)/2 of the
 *                returned decision, bit k of byte k/8 (LSB first).
 *   out_iters  : dev int32 [n_frames]: completed flip rounds, in [0, T].
 *   out_converged : dev uint8 [n_frames] (may be NULL): 1 if the stop test
 *                (every s_i = +1) ended decoding, 0 if T was reached.
 *   stream     : hipStream_t.
 * The launch's waves take frames as they need them from a queue (8 device
 * counters of frame runs plus a count of finished waves, reset by the launch
 * itself when it ends).  Direct launches take queues from one ring of 1024,
 * launches recorded under stream capture from another ring of 1024, so a
 * graph's launches never share a queue with direct launches.  An event
 * recorded after each direct launch marks its queue free again; a direct
 * launch takes the next free queue of its ring (passing over those still
 * held, e.g. by one long launch while many short ones come and go on other
 * streams) and returns NGDBF_EBUSY, launching nothing, only when all 1024
 * are held by launches queued on streams and not yet finished.  At most 1024 recorded launches may belong to graphs
 * replayed at the same time; a captured graph must not be replayed on two
 * streams at the same time.  With trace rows, the rows
 * are cleared by a kernel on `stream` before the decode (no memset node
 * under capture).
 * Errors: NGDBF_EINVAL (NULL pointers with n_frames > 0, parameters out of
 * range), NGDBF_EBUSY (every queue held, see above),
 * NGDBF_EDEVICE (launch failure, or an earlier fault reported now).
 */
ngdbf_status ngdbf_decode(const ngdbf_code *code, const void *y, int64_t n_frames,
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
ngdbf_status ngdbf_decode_trace(const ngdbf_code *code, const void *y, int64_t n_frames,
                       const float *sigma, float sigma_scalar,
                       const ngdbf_params *params, uint64_t seed,
                       uint64_t frame_base, uint8_t *out_bits,
                       int32_t *out_iters, uint8_t *out_converged,
                       uint8_t *flip_masks, void *stream);

/*
 * ngdbf_decode_noalloc -- ngdbf_decode for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same decode, bit for bit, with the launch's
 * frame queue in a static device array of the library (`scratch`, one queue
 * of 9 cache-line-padded counters, 1152 bytes, held by every device the
 * library runs on until the process ends) instead of the per-device ring.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine; the code handle, y and the outputs are the caller's) and queues
 * two kernels on `stream`: one that zeroes the scratch queue, then the decode.
 * Arguments, layouts and errors as ngdbf_decode; no input size needs more
 * scratch than the array holds, and a build whose launch would need more
 * refuses with NGDBF_EUNSUPPORTED.  Every call on one device shares the same
 * scratch queue: calls that overlap on one device (on different streams, or
 * replays of a captured call beside another) race on it and may skip or
 * repeat frames, so serialise them.
 */
ngdbf_status ngdbf_decode_noalloc(const ngdbf_code *code, const void *y, int64_t n_frames,
                                  const float *sigma, float sigma_scalar,
                                  const ngdbf_params *params, uint64_t seed,
                                  uint64_t frame_base, uint8_t *out_bits,
                                  int32_t *out_iters, uint8_t *out_converged,
                                  void *stream);

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
ngdbf_status ngdbf_noise_probe(int32_t kind, uint32_t start, uint32_t count,
                      uint64_t seed, uint64_t frame, uint32_t iter,
                      float *out0, float *out1, void *stream);

/*
 * Launch shape of a code's decode kernel (all shapes give identical results):
 *   waves_per_frame : wavefronts cooperating on one frame (1, 2, 4, 8, 16);
 *   quads_per_lane  : bit quads each lane owns (1, 2, 4); a frame holds at most
 *                     64 * waves_per_frame * quads_per_lane quads (4 bits each);
 *   frames_per_block: frames per workgroup: 1 when waves_per_frame > 1, else
 *                     1 .. 16 (the default takes the first of 16, 12, 8, 4,
 *                     2, 1 that the LDS holds).
 * ngdbf_code_set_shape fixes the shape used by later decodes of this code
 * (NGDBF_EINVAL if it does not fit the code, NGDBF_EUNSUPPORTED if it was not
 * built or exceeds the LDS); all-zero arguments restore the default choice.
 * ngdbf_code_get_shape reports the shape that decodes with `params` use (host
 * int32 [3]); params may be NULL (the multi-bit binary32 decoder).  The
 * default differs between decoders: the extended ones (quantized, noise
 * reuse, single-bit with noise reuse, mode switching) take at most two quads
 * per lane (more waves per frame); the base decoder, the packed quantized
 * decoder with noise reuse and the single-bit decoder with per-bit draws take
 * one wave per frame whenever the code fits in 1024 bits; longer codes take
 * the fewest waves that hold them (the base decoder: two waves of four quads
 * up to 2048 bits, then four waves of four quads; its frames of two or more
 * waves read the code tables from global memory instead of the LDS).
 * Not thread-safe against concurrent decodes of the same code.
 */
ngdbf_status ngdbf_code_set_shape(ngdbf_code *code, int32_t waves_per_frame,
                         int32_t quads_per_lane, int32_t frames_per_block);
ngdbf_status ngdbf_code_get_shape(const ngdbf_code *code, const ngdbf_params *params,
                         int32_t shape[3]);

/*
 * ngdbf_code_set_stats -- attach (or, with NULL, detach) device counters to a
 * code for instrumentation of the exact noise skip of the multi-bit binary32
 * decoder (Sec. III-C draws every q_k; a pair of bits whose decision the bound
 * on the Box-Muller radius fixes needs no transform).
 *   counters : dev uint64 [2], or NULL.  While attached, every decode of this
 *              code by that decoder adds to counters[0] the bit pairs it
 *              evaluated (ceil(n / 2) per frame and round) and to counters[1]
 *              the pairs it transformed; the caller zeroes them.  Other
 *              decoders leave them unchanged.
 * While attached, every wave updates the counters once per round (slower: for
 * instrumentation, not for timed runs); results are unchanged.  Not
 * thread-safe against concurrent decodes of the same code.
 * Errors: NGDBF_EINVAL (code is NULL).
 */
ngdbf_status ngdbf_code_set_stats(ngdbf_code *code, uint64_t *counters);

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
ngdbf_status ngdbf_autotune(ngdbf_code *code, const void *y, int64_t n_frames,
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
 * jobs of fewer than 65536 frames run concurrently on library-owned streams
 * forked from and joined back to `stream` with events; larger jobs, each of
 * which fills the device, run one after another on `stream` beside them.  The
 * whole batch is one node group when the caller captures `stream` into a
 * hipGraph.  Every job is validated before any work is queued.  Results equal
 * those of ngdbf_decode per job.  Each job takes its own frame queue (see
 * ngdbf_decode), so a batch holds at most 1024 jobs.
 * jobs: host array [n_jobs]; all codes on the current device.
 * Errors: NGDBF_EINVAL (any job invalid, n_jobs < 0 or above 1024),
 * NGDBF_EBUSY (no free queue for a job, see ngdbf_decode), NGDBF_EDEVICE.
 */
ngdbf_status ngdbf_decode_batch(const ngdbf_job *jobs, int32_t n_jobs, void *stream);

/*
 * Segmented decoding: frames scattered over slot ranges of resident pools.
 * Segment s covers launch frames [frame_offset_s, frame_offset_{s+1}) (the last
 * one up to n_frames); its frames live at pool slots first_slot_s, ... and are
 * keyed for the noise as (seed_s, frame_base_s + i).  A frame therefore
 * decodes exactly as ngdbf_decode would decode it with that seed and frame
 * index, whatever else shares the launch.
 */
typedef struct {
    int64_t first_slot;    /* pool slot of the segment's first frame              */
    int64_t frame_offset;  /* launch index of that frame; 0 for the first segment,
                              strictly increasing                                  */
    uint64_t seed;         /* Philox key of the segment                            */
    uint64_t frame_base;   /* noise frame index of the segment's first frame       */
} ngdbf_segment;

/*
 * ngdbf_decode_segments -- decode n_frames frames given as segments.
 *   y_pool, sigma_pool : dev [pool_frames][n] float32 / int8 and [pool_frames]
 *                        (sigma_pool may be NULL: sigma_scalar for all).
 *   segments           : dev ngdbf_segment [n_segments], n_segments >= 1.
 *   bits_pool, iters_pool, conv_pool : dev pools indexed by slot like y_pool
 *                        (conv_pool may be NULL).
 * The caller guarantees that every segment's slots lie in [0, pool_frames);
 * a frame whose slot falls outside is skipped (nothing is read or written).
 * Errors as ngdbf_decode.
 */
ngdbf_status ngdbf_decode_segments(const ngdbf_code *code, const void *y_pool,
                          const float *sigma_pool, float sigma_scalar,
                          int64_t pool_frames, const ngdbf_params *params,
                          const ngdbf_segment *segments, int32_t n_segments,
                          int64_t n_frames, uint8_t *bits_pool,
                          int32_t *iters_pool, uint8_t *conv_pool, void *stream);

/*
 * Serving runtime: continuous batching of decode requests (Sec. III per
 * frame) over pools of frame slots kept resident in HBM.  A request is a run
 * of frames of one code with its own noise key (seed, frame_base); its results
 * equal those of a standalone ngdbf_decode of its frames with that key,
 * whatever it shares a launch with.  All calls on one server are serialised
 * internally; the server, its pools and streams belong to the device current
 * at creation.  Errors: NGDBF_EINVAL (bad argument, unknown or wrong-state
 * ticket), NGDBF_ENOMEM (pools do not fit), NGDBF_EDEVICE (HIP failure, or a
 * launch that failed on the device, reported by poll).
 */
typedef struct ngdbf_server ngdbf_server;

/*
 * ngdbf_server_create -- one slot pool per code: y float32 [pool_frames_i][n_i],
 * sigma float32 [pool_frames_i], bits [pool_frames_i][ceil(n_i/8)], iterations
 * int32 and converged uint8 [pool_frames_i], all owned by the server.
 *   codes, params, pool_frames : host arrays [n_codes]; params[i].y_format must
 *                                be NGDBF_Y_F32; the codes must outlive the server.
 *   n_streams                  : library streams the launches rotate over, [1, 16].
 *   max_requests_per_launch    : [1, 32768]; 1 gives one launch per request (the
 *                                unbatched baseline), larger values batch.
 *   launches_per_stream        : launches in flight per stream, >= 1, with
 *                                n_streams * launches_per_stream <= 32.  With 1,
 *                                requests committed while every stream is busy
 *                                wait and join the next launch of their code.
 *   out                        : receives the handle (NULL on failure).
 */
ngdbf_status ngdbf_server_create(int32_t n_codes, ngdbf_code *const *codes,
                        const ngdbf_params *params, const int64_t *pool_frames,
                        int32_t n_streams, int32_t max_requests_per_launch,
                        int32_t launches_per_stream, ngdbf_server **out);
/* Waits for launches in flight, then frees everything the server owns. */
ngdbf_status ngdbf_server_destroy(ngdbf_server *server);
/*
 * ngdbf_server_pools -- device addresses of code `code_index`'s pools (any
 * output pointer may be NULL).  The client writes y and sigma of a request's
 * slots before committing it and reads its outputs once poll has reported it.
 */
ngdbf_status ngdbf_server_pools(ngdbf_server *server, int32_t code_index, float **y,
                       float **sigma, uint8_t **bits, int32_t **iters,
                       uint8_t **converged);
/*
 * ngdbf_server_admit -- reserve a contiguous slot range for each request, in
 * order, stopping at the first one whose pool has no free range of its size
 * (admission by free HBM).  Host arrays [n_requests]: code_index, n_frames
 * (1 .. pool size), seed, frame_base in; tickets, first_slots out for the
 * admitted prefix of *n_admitted requests.  A request larger than its pool is
 * NGDBF_EINVAL.
 */
ngdbf_status ngdbf_server_admit(ngdbf_server *server, int32_t n_requests,
                       const int32_t *code_index, const int64_t *n_frames,
                       const uint64_t *seed, const uint64_t *frame_base,
                       uint64_t *tickets, int64_t *first_slots,
                       int32_t *n_admitted);
/*
 * ngdbf_server_commit -- the admitted requests' inputs are complete once the
 * work queued so far on `stream` has run; their launch waits for it.
 */
ngdbf_status ngdbf_server_commit(ngdbf_server *server, int32_t n, const uint64_t *tickets,
                        void *stream);
/*
 * ngdbf_server_pump -- launch committed requests while a stream has room:
 * each launch takes, from the code whose oldest committed request is oldest,
 * up to max_requests_per_launch requests as one segmented launch on the least
 * loaded stream.  What does not fit waits for a later pump.  Never blocks on
 * the device.
 */
ngdbf_status ngdbf_server_pump(ngdbf_server *server, int32_t *n_launched);
/*
 * ngdbf_server_poll -- non-blocking: writes to tickets[0 .. *n_done) the
 * requests whose launch has finished, in launch order, at most `capacity`.
 */
ngdbf_status ngdbf_server_poll(ngdbf_server *server, int32_t capacity, uint64_t *tickets,
                      int32_t *n_done);
/*
 * ngdbf_server_release -- return finished requests' slots to their pools.  The
 * client's reads of the outputs must be complete, or queued on the stream it
 * commits later requests on.
 */
ngdbf_status ngdbf_server_release(ngdbf_server *server, int32_t n, const uint64_t *tickets);

/*
 * ngdbf_objective -- the GDBF objective of Sec. III-B, f(x) = sum_k x_k y_k +
 * sum_i s_i, of given decisions, for the convergence error of Sec. VI
 * (average of f(x(T)) - f(c) over frames, with c the sent codeword).
 * Evaluated exactly in fixed point: out[f] = sum_k x_k Y_k + 2^20 sum_i s_i,
 * Y_k = rint(2^20 y_k) with y_k saturated at ymax as in decoding (ymax <= 0:
 * none), clamped to +-2^40, NaN counted as 0.
 *   y         : dev [n_frames][n], float32 (y_format 0) or int8 (1, y = y_q/16).
 *   bits      : dev [n_frames][ceil(n/8)], decisions c_k = (1 - x_k)/2 LSB first.
 *   out       : dev int64 [n_frames].
 * Errors: NGDBF_EINVAL (NULL code or buffers, n_frames < 0, bad y_format).
 */
ngdbf_status ngdbf_objective(const ngdbf_code *code, const void *y, int32_t y_format,
                    int64_t n_frames, float ymax, const uint8_t *bits, int64_t *out,
                    void *stream);

/*
 * ngdbf_channel -- the synthetic channel of Sec. III-A on the device: BPSK
 * symbols c_hat_k = 1 - 2 c_k plus Gaussian noise of std sigma,
 *   y_k = fmaf(sigma_f, z_k, c_hat_k),
 * with z_k the standard-normal draw of bit k that the decoder's generator
 * gives under the iteration word 0xFFFFFFFE (Philox4x32-10 counter (k >> 2,
 * 0xFFFFFFFE, frame lo, frame hi), key = seed, Box-Muller as for the
 * perturbations; no decoding round and not the noise-reuse stream uses that
 * word), frame = frame_base + f.  A CPU implementation can regenerate every
 * sample bit for bit.
 *   n, n_frames : code length (1 .. 65535) and frames (>= 0).
 *   sigma       : dev float32 [n_frames] or NULL (sigma_scalar, finite >= 0).
 *   codewords   : dev uint8 [n_frames][ceil(n/8)] sent bits c_k, LSB first,
 *                 or NULL for the all-zero codeword.
 *   y_format    : NGDBF_Y_F32 (y float32 [n_frames][n]) or NGDBF_Y_I8 (int8
 *                 codes y_q = clamp(rint(16 y), -127, 127), ties to even).
 *   y           : dev output, owned by the caller.
 * Errors: NGDBF_EINVAL, NGDBF_EDEVICE.
 */
ngdbf_status ngdbf_channel(int32_t n, int64_t n_frames, const float *sigma, float sigma_scalar,
                           uint64_t seed, uint64_t frame_base, const uint8_t *codewords,
                           int32_t y_format, void *y, void *stream);

/*
 * ngdbf_frame_stats -- Monte Carlo counters of decoded frames (the BER, FER
 * and iteration statistics of Sec. IV-A/B), accumulated into out (the caller
 * zeroes it; several calls add up):
 *   out[0] bit errors sum_f e_f, with e_f the bits of the decision that
 *          differ from the sent word (all of the frame's n code bits);
 *   out[1] sum_f e_f^2 (for bit-error intervals clustered by frame);
 *   out[2] frame errors (e_f > 0);  out[3] undetected errors (e_f > 0 on a
 *          frame whose stop test ended decoding; 0 if converged is NULL);
 *   out[4] sum of iteration counts;  out[5] unconverged frames (0 if
 *          converged is NULL);  out[6 + t] frames that took t rounds,
 *          t = 0 .. t_max (counts above t_max land in the last bin).
 *   bits      : dev [n_frames][ceil(n/8)] decisions (ngdbf_decode's out_bits).
 *   codewords : dev sent bits in the same layout, or NULL (all-zero word).
 *   iters     : dev int32 [n_frames]; converged: dev uint8 [n_frames] or NULL.
 *   out       : dev int64 [7 + t_max], t_max in [0, 65535].
 * Errors: NGDBF_EINVAL, NGDBF_EDEVICE.
 */
ngdbf_status ngdbf_frame_stats(int32_t n, int64_t n_frames, const uint8_t *bits,
                               const uint8_t *codewords, const int32_t *iters,
                               const uint8_t *converged, int32_t t_max, int64_t *out,
                               void *stream);

/*
 * ngdbf_issue_probe -- instrumentation: a kernel of long unrolled chains of
 * one vector-ALU instruction class, for measuring how many clocks a wave64
 * instruction of that class holds a SIMD (the decoder is bound by vector-ALU
 * issue; the benchmark weights each class's hardware counter by this time).
 *   kind   : 0 32-bit integer (v_xad_u32), 1 64-bit product plus xor
 *            (v_mad_u64_u32, v_xor_b32), 2 binary32 fma, 3 binary32 multiply,
 *            4 transcendental (v_sqrt_f32), 5..27 one instruction each:
 *            v_xor_b32, v_lshlrev_b32, v_mad_u64_u32, v_bitop3_b32,
 *            v_and_b32, v_or_b32, v_mov_b32, v_cndmask_b32, v_add_u32,
 *            v_lshrrev_b32, v_bfe_u32, v_cmp_eq_u32, v_cmp_lt_f32,
 *            v_readlane_b32, v_writelane_b32, v_mbcnt_lo_u32_b32,
 *            v_ffbh_u32, v_lshl_add_u64, v_add3_u32, v_mad_u32_u24,
 *            v_lshl_add_u32, v_or3_b32, v_mul_u32_u24; every chain step is
 *            one instruction (kind 1: two).
 *   blocks : workgroups of 256 threads; iters >= 1 outer iterations of 16 x 8
 *            chain steps per thread.
 *   out    : dev uint32 [blocks * 256], receives a value per thread.
 * Errors: NGDBF_EINVAL (kind, sizes or NULL out), NGDBF_EDEVICE.  Does not set
 * ngdbf_last_error.
 */
ngdbf_status ngdbf_issue_probe(int32_t kind, int32_t blocks, int32_t iters, uint32_t *out,
                               void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *ngdbf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
