/*
 * pbvd.h -- C ABI of the MI355X parallel block-based Viterbi decoder.
 *
 * The decoder implements the parallel block-based Viterbi decoder (PBVD) of
 * Peng, Liu, Hou and Zhao, "A Gb/s Parallel Block-based Viterbi Decoder for
 * Convolutional Codes on GPU" (arXiv 1608.00066):
 *   - the problem (Sec. II, Sec. III-A): a stream of rate-1/R, constraint
 *     length K convolutional-code symbols received over AWGN is decoded into
 *     its information bits;
 *   - the block decomposition (Sec. III-A, Fig. 1 and 2, M = L): the stream
 *     is cut into parallel blocks (PBs) of D decoded bits, each extended by L
 *     stages on both sides; PBs are decoded independently;
 *   - per PB, a forward add-compare-select pass (Eq. 1) over the 2^(K-1)
 *     states with branch metrics shared per butterfly group (Eq. 2-6) and
 *     bit-packed survivor decisions (Sec. IV-B), then a traceback from a fixed
 *     start state that emits the D decoded bits (Alg. 1, Kernel 2), packed
 *     eight per byte (Sec. IV-C).
 *
 * Conventions fixed by this library where the paper is silent:
 *   - gen[r] bit k is g_k^(r) of Eq. 2 (octal 171 = 1111001); bit K-1 taps
 *     the current input bit; state d = (D_{K-2} ... D_0)_2 with D_{K-2} the
 *     newest input (the butterfly of Sec. III-B);
 *   - the R symbols of one stage are stored consecutively in generator order;
 *   - soft input: one int8 per symbol, q >= 0 reads as code bit 0, |q| is the
 *     cost of disagreeing with it; hard input: one byte per symbol, bit =
 *     byte & 1 (Hamming distance);
 *   - ties in add-compare-select keep the branch from S_2j;
 *   - a PB whose forward range starts at stage 0 starts from the known
 *     encoder state 0; every other PB starts from all-zero metrics (Sec.
 *     III-A);
 *   - traceback starts from state 0 (Sec. III-A, Alg. 1); at the end of an
 *     unterminated stream it starts from the state of least metric (lowest
 *     index on ties), as full-frame Viterbi does (Sec. II);
 *   - PB b covers forward stages [max(0, bD-L), min(T, bD+D+L)) and decodes
 *     bits [bD, min(n, bD+D)); T = n + (K-1) if the stream is terminated
 *     with K-1 zero bits, else T = n; there are ceil(n/D) PBs;
 *   - decoded bit i is bit (i & 7) of byte (i >> 3) (least significant bit
 *     first); unused high bits of the last byte are written as 0.
 *
 * Memory: every pointer named d_* is a device (HBM) pointer owned by the
 * caller.  The plan owns its own device workspace (survivor buffers), which
 * it allocates and grows on demand during decode and frees in pbvd_destroy.
 *
 * Concurrency: decode calls are asynchronous on the given HIP stream (NULL =
 * the null stream).  A plan holds one workspace: do not run two decodes of
 * the same plan concurrently (use one plan per stream).
 *
 * Errors: arguments are validated before anything is launched; on a
 * negative status nothing has been written to the output buffers.  No C++
 * exception crosses this interface.  pbvd_last_error() gives a
 * human-readable detail of the last failure of the calling thread.
 */
#ifndef PBVD_H
#define PBVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbvd_plan pbvd_plan;

typedef enum {
    PBVD_OK = 0,
    PBVD_EINVAL = -1,   /* invalid argument */
    PBVD_ENOTSUP = -2,  /* valid code, but no kernel compiled for it */
    PBVD_ENOMEM = -3,   /* device workspace allocation failed */
    PBVD_EHIP = -4,     /* HIP runtime error (detail in pbvd_last_error) */
    PBVD_EAGAIN = -5    /* server: request not finished yet, or queue full */
} pbvd_status;

enum {
    PBVD_SOFT_I8 = 0,   /* int8 soft value per code symbol */
    PBVD_HARD_U8 = 1    /* uint8 per code symbol, bit = byte & 1 */
};

/* How a PB's trellis (Sec. III-B) is spread over GPU lanes (Sec. IV-A).
 *   PBVD_MAP_LANES: the register kernel; all 2^(K-1) path metrics of a PB in
 *     the registers of lanes_per_pb lanes (1, 2, 4, 8), the code compiled in
 *     (the generator sets of the library's registry); the fastest mapping for
 *     long streams and large batches.
 *   PBVD_MAP_WAVE: the state-parallel kernel; one wave per PB, one lane per
 *     state (two or four for K = 8, 9), metrics exchanged between lanes every
 *     stage, generators taken at run time: any code of the ranges below, and
 *     the lowest latency per PB (short streams, single frames).
 *   PBVD_MAP_GROUP: the paper's group mapping (Sec. III-B Eq. 3-6, Sec. IV-A,
 *     Alg. 1): the butterflies fall into N_c = 2^R groups by their code word
 *     alpha; a workgroup of N_c waves decodes 64 PBs, wave w the butterflies
 *     of group w (four branch metrics per stage), lane l PB l, the metrics
 *     exchanged through LDS each stage; generators at run time.  Takes codes
 *     with K - 2 - R >= 0, 2^(K-2-R) <= 16 and groups of one size (the alpha
 *     map of full rank R; PBVD_ENOTSUP otherwise) and D + 2L <= 2^20;
 *     lanes_per_pb 0 or 2^R; no survivor export (pbvd_debug_survivors).
 *   PBVD_MAP_AUTO: the wave kernel for codes outside the registry and for
 *     calls with few PBs, the register kernel otherwise.
 * Every mapping gives the same bits and metrics. */
enum { PBVD_MAP_AUTO = 0, PBVD_MAP_LANES = 1, PBVD_MAP_WAVE = 2, PBVD_MAP_GROUP = 3 };

/* Code and block parameters (Sec. III-A, Sec. III-B). */
typedef struct {
    int32_t K;          /* constraint length, 3..9 (N = 2^(K-1) states) */
    int32_t R;          /* 1/R code rate, 2..4 */
    uint32_t gen[4];    /* generators gen[0..R-1] (bit k = g_k); at least one
                           has bit K-1 set; all < 2^K */
    int32_t D;          /* decoded bits per PB, >= 1 */
    int32_t L;          /* overlap on each side (M = L), >= 0; D + 2L < 2^30 */
    int32_t terminated; /* 1: the stream carries K-1 zero tail stages after n */
    int32_t input_kind; /* PBVD_SOFT_I8 or PBVD_HARD_U8 */
    int32_t pm_bits;    /* path-metric width, 16 or 32 (32 needs K <= 8);
                           results are identical, only the kernel differs */
    int32_t lanes_per_pb; /* GPU lanes sharing one PB's trellis: 1, 2, 4 or
                           8 (the register kernel), 64 (a whole wave, one lane
                           per state: the state-parallel kernel), or 0 to let
                           the library choose per call.  2, 4 and 8 need
                           pm_bits = 16 and K >= 7 (2), K >= 8 (4) or K = 9
                           (8).  More lanes per PB cut a PB's latency and let
                           short streams fill more of the GPU; results are
                           identical, only the kernel differs; with
                           PBVD_MAP_GROUP 0 or 2^R */
    int32_t mapping;    /* PBVD_MAP_AUTO, PBVD_MAP_LANES, PBVD_MAP_WAVE or PBVD_MAP_GROUP */
} pbvd_code;

/* Validate `code` (the code of Eq. 2 and the blocks of Sec. III-A) and pick
 * the kernels.  *out receives a new plan (no device memory is allocated yet).
 * Any generator set within the ranges above decodes (the wave mapping takes
 * the generators at run time); PBVD_ENOTSUP when the register kernel is
 * asked for (PBVD_MAP_LANES, or lanes_per_pb of 1..8) and no register
 * kernel is compiled for this generator set, or for a metric width it does
 * not support.  PBVD_EINVAL for out-of-range fields (callers must zero
 * fields they do not set, e.g. mapping). */
pbvd_status pbvd_create(const pbvd_code *code, pbvd_plan **out);

/* Decode a whole stream: the problem of Sec. II solved by the parallel
 * blocks of Sec. III-A (Fig. 2), each a forward pass (Eq. 1) and a traceback
 * (Alg. 1, Kernel 2).
 *   d_syms     : device, (n_bits + terminated*(K-1)) * R bytes, stage-major
 *   n_bits     : information bits, >= 1
 *   d_out_bits : device, ceil(n_bits/8) bytes, written completely
 *   hip_stream : hipStream_t or NULL
 * Asynchronous; equivalent to pbvd_decode_ex over all PBs.  Errors as for
 * pbvd_decode_ex. */
pbvd_status pbvd_decode(pbvd_plan *p, const void *d_syms, int64_t n_bits, uint8_t *d_out_bits,
                        void *hip_stream);

/* Decode PBs [pb_first, pb_first + pb_count) of a stream of n_bits bits
 * (resume, sharding, verification): the PBs of Sec. III-A are independent,
 * so any sub-range decodes to the same bits as inside the whole stream.
 *   d_out_bits : device, receives decoded bits [pb_first*D, min(n, (pb_first
 *                + pb_count)*D)) of the stream starting at its bit 0;
 *                ceil(that count / 8) bytes, written completely
 *   d_final_pm : device int32 [pb_count][2^(K-1)] or NULL: path metrics at the
 *                end of each PB's forward range minus their minimum
 * pb_count may be 0 (nothing is written).  Asynchronous.  PBVD_EINVAL for a
 * NULL plan or buffer, n_bits < 1 or a PB range outside [0, ceil(n_bits/D));
 * PBVD_ENOMEM when the plan's survivor workspace cannot grow; PBVD_EHIP on a
 * launch failure.  On an error nothing has been written. */
pbvd_status pbvd_decode_ex(pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                           int64_t pb_count, uint8_t *d_out_bits, int32_t *d_final_pm,
                           void *hip_stream);

/* pbvd_decode_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc while
 * decoding.  It calls no hipMalloc, hipFree or allocating library routine:
 * the survivor rows and the output staging of the call live in a static
 * device array of the library (PBVD_STATIC_SCRATCH_BYTES), which every
 * device the library runs on holds from the moment the library's code
 * object is loaded until the process ends (its address is looked up once
 * per device, by pbvd_create or by the first call).  Arguments, layout,
 * bits and final metrics are those of pbvd_decode_ex; a stream whose
 * survivors do not fit one launch is decoded in several launches that reuse
 * the array.  PBVD_EINVAL (nothing decoded) when the output staging -- 4
 * bytes per 32 decoded bits plus 8, only when D % 32 != 0 or d_out_bits is
 * not 4-byte aligned -- together with the survivors of one wave (one PB for
 * the wave mapping) exceeds the array.  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (other streams, other threads, other plans) race and must be
 * serialized by the caller. */
#define PBVD_STATIC_SCRATCH_BYTES (64u << 20)
pbvd_status pbvd_decode_ex_noalloc(pbvd_plan *p, const void *d_syms, int64_t n_bits, int64_t pb_first,
                                   int64_t pb_count, uint8_t *d_out_bits, int32_t *d_final_pm,
                                   void *hip_stream);

/* pbvd_decode_host flag: both host buffers are page-locked (e.g. from
 * hipHostMalloc), so chunks are copied by DMA straight from and to them. */
#define PBVD_HOST_PINNED 1u

/* Decode a whole stream held in host memory, overlapping transfers with
 * decoding (Sec. IV-C, Eq. 7).  The PBs are cut into chunks of chunk_pbs PBs
 * (0: about 2 chunks per stream); chunk c goes to the device (its symbols
 * with the L-stage overlap on both sides), is decoded, and its bits come
 * back on stream c mod n_streams, so the copies of one chunk overlap the
 * decoding of others.  Bits equal pbvd_decode of the same stream.
 *   h_syms    : host, (n_bits + terminated*(K-1))*R bytes, stage-major
 *   h_out     : host, ceil(n_bits/8) bytes, written completely
 *   n_streams : 1..8 HIP streams (owned by the plan, created on first use)
 *   chunk_pbs : >= 0; chunk_pbs * D must be a multiple of 8
 *   flags     : PBVD_HOST_PINNED, or 0 for pageable buffers, which are staged
 *               through pinned buffers the plan allocates
 * Synchronous: returns when h_out is complete.  Device buffers of the chunks
 * are owned by the plan and freed by pbvd_destroy. */
pbvd_status pbvd_decode_host(pbvd_plan *p, const void *h_syms, int64_t n_bits, uint8_t *h_out,
                             int32_t n_streams, int64_t chunk_pbs, uint32_t flags);

/* Lanes per PB (1, 2, 4, 8, 64 for the wave mapping, 2^R for the group
 * mapping) that pbvd_decode_ex
 * of PBs [pb_first, pb_first + pb_count) of an n_bits-bit stream uses: the
 * plan's mapping and lanes_per_pb, or the library's choice: the wave
 * mapping for codes outside the registry and for calls of fewer PBs than a
 * threshold (PBVD_WAVE_MAX_PBS overrides it); else one lane for K <= 7 when
 * that gives 4096 waves of 64 PBs, else pairs of lanes where the code allows
 * them when that gives 1024 waves, else the largest group the code allows.
 * 0 on invalid arguments. */
int32_t pbvd_call_lanes(const pbvd_plan *p, int64_t n_bits, int64_t pb_first, int64_t pb_count);

/* Number of parallel blocks of a stream: ceil(n_bits / D); 0 if n_bits < 1. */
int64_t pbvd_num_blocks(const pbvd_plan *p, int64_t n_bits);

/* Host-side block geometry (Sec. III-A): for PBs [pb_first, pb_first +
 * pb_count) of a stream of n_bits bits writes 4 values per PB to the host
 * array out: forward range start f0, end f1, decoded range start d0, end d1.
 * Returns PBVD_EINVAL for a range outside [0, pbvd_num_blocks). */
pbvd_status pbvd_block_geometry(const pbvd_plan *p, int64_t n_bits, int64_t pb_first,
                                int64_t pb_count, int64_t *out);

/* Verification hook for the survivor layout: decodes PBs [pb_first,
 * pb_first + pb_count) like pbvd_decode_ex and then expands the packed
 * survivor decisions they stored into d_dec, a device uint8 array
 * [pb_count][D+L][2^(K-1)]: row s - b*D holds the decision (1 = lower
 * branch, from S_2j+1) of every state at stage s for s in [b*D, f1); other
 * rows are zero.  d_out_bits as in pbvd_decode_ex.  Synchronizes the stream.
 * Returns PBVD_EINVAL when the range does not fit the workspace of a single
 * launch. */
pbvd_status pbvd_debug_survivors(pbvd_plan *p, const void *d_syms, int64_t n_bits,
                                 int64_t pb_first, int64_t pb_count, uint8_t *d_out_bits,
                                 uint8_t *d_dec, void *hip_stream);

/* Verification hook for the branch metrics: for stages [0, n_stages) of
 * d_syms writes the 2^R code-word metrics the forward kernel computes into
 * the device int32 array d_bm [n_stages][2^R] (code word c has c^(1) as its
 * most significant bit).  These equal the Sec. II distances minus a
 * per-stage constant shared by all code words.  Asynchronous. */
pbvd_status pbvd_debug_branch_metrics(pbvd_plan *p, const void *d_syms, int64_t n_stages,
                                      int32_t *d_bm, void *hip_stream);

/* Verification hook for the group mapping (host only, no device work): the
 * classification of Sec. III-B (Eq. 3-6, Table II) the library derives from
 * `code`'s generators.  alpha[j] (N/2 entries) receives the group of
 * butterfly j, its code word alpha = c(S_2j, 0) with c^(1) as the most
 * significant bit; masks[4 * a + t] (2^R x 4 entries) the code words of
 * group a's four branches, t = 0..3 for alpha, beta = c(S_2j, 1),
 * gamma = c(S_2j+1, 0), theta = c(S_2j+1, 1), in the same bit order.  Both
 * arrays are caller-owned host memory.  PBVD_ENOTSUP when the mapping does
 * not take the code (see PBVD_MAP_GROUP), PBVD_EINVAL for an invalid code. */
pbvd_status pbvd_debug_group_table(const pbvd_code *code, int32_t *alpha, int32_t *masks);

/* Free the plan and its device workspace (synchronizes the device). */
void pbvd_destroy(pbvd_plan *p);

/* ---- Batched decoding: many independent frames, several codes ----------
 *
 * A batch decodes many frames (each a separate stream in the sense of
 * Sec. III-A: its own PBs, its own start and end).  The PBs of all frames
 * are packed regardless of frame boundaries, so thousands of short frames
 * fill the GPU as well as one long stream does; per code mapping:
 *   register kernel (PBVD_MAP_LANES / AUTO): tiles of 64 >> lb PBs of one
 *     code, one launch per code, except that the two codes of a pair the
 *     library registers (K=7 (171,133) with (133,171,165)) share one launch
 *     when they have the same lanes per PB, 16-bit metrics and input kind
 *     (each tile decoded with its own code);
 *   state-parallel kernel (PBVD_MAP_WAVE): the PBs of every such code of one
 *     K in ONE persistent launch, longest first, waves taking PBs from work
 *     counters (one per XCD) that a fill kernel zeroes at the start of each
 *     decode;
 *   group mapping (PBVD_MAP_GROUP): tiles of 64 PBs, one launch per code.
 * The launches run on forked streams.  Every frame's output is identical to
 * decoding that frame alone with pbvd_decode and the same code parameters.
 * Decodes of one batch must not overlap each other (they share the survivor
 * area and the work counters): issue them on one stream. */

typedef struct pbvd_batch pbvd_batch;

typedef struct {
    int64_t sym_offset; /* byte offset in d_syms of the frame's first symbol;
                           the frame has (n_bits + terminated*(K-1)) * R bytes */
    int64_t n_bits;     /* information bits of the frame, >= 1 */
    int64_t out_offset; /* byte offset in d_out of the frame's ceil(n_bits/8)
                           output bytes (same bit order as pbvd_decode) */
    int32_t code;       /* index into the codes given to pbvd_batch_create */
    int32_t reserved;   /* must be 0 */
} pbvd_frame;

/* Create a batch decoder for n_codes (1..16) code/block parameter sets.
 * Each must be valid for pbvd_create and have D % 8 == 0 (decoded blocks
 * start on byte boundaries). */
pbvd_status pbvd_batch_create(const pbvd_code *codes, int32_t n_codes, pbvd_batch **out);

/* Describe the frames (host array) of the next decodes: builds the work list
 * (PBs of all frames, grouped by code, longest first, 64 per wave), uploads
 * it and sizes the device workspace.  sym_bytes / out_bytes are the sizes of
 * the device buffers later passed to pbvd_batch_decode; every frame must lie
 * inside them and output ranges must not overlap.  Synchronous: first waits
 * for this batch's earlier decodes (those launched outside graph capture;
 * nothing else on the device is waited for), then uploads.  A graph captured
 * from pbvd_batch_decode refers to the work list of its capture: it must
 * have finished before, and must not be replayed after, the next call.
 * PBVD_EINVAL on a bad frame (nothing is changed); after any other failure
 * the batch holds no frames (decodes write nothing) until a call succeeds. */
pbvd_status pbvd_batch_set_frames(pbvd_batch *b, const pbvd_frame *frames, int64_t n_frames,
                                  int64_t sym_bytes, int64_t out_bytes);

/* Decode the frames last given to pbvd_batch_set_frames (Sec. III-A per
 * frame): the launches above, asynchronous on hip_stream.  It allocates
 * nothing, copies nothing from the host and records no memset (the work
 * counters are reset by a kernel), so it can be captured in a HIP graph and
 * replayed.  Bytes of d_out outside the frames' output ranges are not
 * written.  PBVD_EINVAL for NULL buffers, PBVD_EHIP for a failed launch. */
pbvd_status pbvd_batch_decode(pbvd_batch *b, const void *d_syms, uint8_t *d_out, void *hip_stream);

/* Work-list statistics of the current frames: tiles (waves), parallel blocks,
 * forward stages summed over PBs, and device workspace bytes; any pointer may
 * be NULL. */
pbvd_status pbvd_batch_info(const pbvd_batch *b, int64_t *n_tiles, int64_t *n_blocks,
                            int64_t *n_forward_stages, int64_t *workspace_bytes);

/* Free the batch and its device memory (synchronizes the device). */
void pbvd_batch_destroy(pbvd_batch *b);

/* ---- Request server: continuous batching of decode requests -------------
 *
 * A server decodes independent requests (one frame each, host memory in and
 * out) as they arrive.  A worker thread keeps up to max_inflight batches on
 * the device at once, each in its own part of a fixed device-memory budget
 * with its own streams: whenever a part is free and requests wait, it admits
 * the waiting requests that fit (first come, first served), copies their
 * symbols and work list to the device in one transfer, runs the batched
 * kernels of pbvd_batch_decode and copies the bits back.  Requests arriving
 * while batches run are admitted as parts free up, so their work overlaps on
 * the device.  Each request's bits equal pbvd_decode of its frame alone with
 * the same code parameters, whatever it was batched with. */

typedef struct pbvd_server pbvd_server;

typedef struct {
    int64_t device_bytes;     /* device memory of all batches in flight: inputs,
                                 outputs, work lists and survivor rows; split
                                 evenly between max_inflight batches; at least
                                 1 MiB per batch */
    int32_t max_inflight;     /* batches on the device at once, 1..8 */
    int32_t max_batch_frames; /* requests per batch, >= 1 */
    int64_t max_queued;       /* requests waiting for admission, >= 1; beyond it
                                 pbvd_server_submit returns PBVD_EAGAIN */
} pbvd_server_config;

typedef struct {
    int64_t submit_ns;    /* steady-clock time of pbvd_server_submit */
    int64_t start_ns;     /* when the batch carrying it was launched */
    int64_t done_ns;      /* when its bits were in the caller's buffer */
    int32_t batch_frames; /* requests in that batch */
    int32_t status;       /* PBVD_OK, or the failure of its batch */
} pbvd_request_info;

/* Create a server for n_codes (1..16) code/block parameter sets (each valid
 * for pbvd_batch_create) on the current device.  Codes that leave the mapping
 * to the library (PBVD_MAP_AUTO, lanes_per_pb 0) decode on the wave mapping,
 * the lowest latency per request; PBVD_ENOTSUP for PBVD_MAP_GROUP.  Allocates the device budget and pinned
 * staging buffers and starts the worker thread (which polls for 2 ms after
 * its last work before it sleeps, to admit requests quickly). */
pbvd_status pbvd_server_create(const pbvd_code *codes, int32_t n_codes, const pbvd_server_config *cfg,
                               pbvd_server **out);

/* Queue one request: frame of n_bits information bits of code index `code`,
 * host symbols (layout of pbvd_decode; copied before the call returns) and a
 * host output buffer of ceil(n_bits/8) bytes that must stay valid until the
 * request is waited for.  *ticket identifies it.  PBVD_EINVAL if the request
 * alone exceeds one batch's part of the budget, PBVD_EAGAIN if the queue is
 * full.  Thread-safe. */
pbvd_status pbvd_server_submit(pbvd_server *s, int32_t code, const void *syms, int64_t n_bits,
                               uint8_t *out_bits, int64_t *ticket);

/* Wait for a request (timeout_us < 0: without limit).  On return with
 * PBVD_OK its bits are in the output buffer; info (may be NULL) receives its
 * timing.  The ticket is released by a return other than PBVD_EAGAIN
 * (timeout).  Thread-safe. */
pbvd_status pbvd_server_wait(pbvd_server *s, int64_t ticket, int64_t timeout_us, pbvd_request_info *info);

/* Batches launched, requests finished and the largest number of batches that
 * were in flight at once; any pointer may be NULL. */
pbvd_status pbvd_server_counters(pbvd_server *s, int64_t *batches, int64_t *requests_done,
                                 int64_t *peak_inflight);

/* Finish every queued request, stop the worker and free the server. */
void pbvd_server_destroy(pbvd_server *s);

/* Static description of a status code. */
const char *pbvd_strerror(pbvd_status s);

/* Detail of the last failed call on this thread ("" if none). */
const char *pbvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PBVD_H */
