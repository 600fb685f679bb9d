/*
 * szi.h -- C ABI of libszi, an MI355X (gfx950) implementation of the G-Interp
 * error-bounded lossy compressor of cuSZ-i (arXiv 2312.05492).
 *
 * The compression pipeline is the one of Fig. overview (Sec. IV):
 *   prediction-quantisation by multi-level spline interpolation with
 *   anchor points (Sec. V-A, V-B), auto-tuned by data profiling
 *   (Sec. V-C), then a quant-code histogram and coarse-grained Huffman
 *   encoding with outliers gathered by stream compaction (Sec. VI-A).
 * Decompression decodes the quant-codes and replays the same predictions
 * (Sec. V-B.1).  The closed de-redundancy pass of Sec. VI-B is not part of
 * this library.
 *
 * Conventions
 *  - Every call returns sz_status: 0 on success, a negative code on error.
 *    On error outputs are left untouched and sz_last_error(ctx) returns a
 *    message.  Nothing aborts the process.
 *  - Fields are FP32, C-order.  sz_dims.n[0] is the FASTEST dimension (x);
 *    n[ndim-1] the slowest.  A numpy array of shape (nz, ny, nx) has
 *    n = {nx, ny, nz}.
 *  - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *    default stream).  Work is enqueued on that stream.
 *  - Device pointers must belong to the context's device.  The caller owns
 *    every input and output buffer it passes; the library never writes to an
 *    input.  Buffers inside sz_result belong to the context until
 *    sz_result_free.
 *  - A context may be used by one host thread at a time.  Independent
 *    contexts on the same device may run concurrently on different streams.
 *  - Limits: ndim in {2, 3}; 1 <= total points < 2^32; radius R in
 *    [2, 1024]; Huffman chunk in {256, 512, 1024, 2048}; anchor stride and
 *    window fixed to the defaults below.
 */
#ifndef SZI_H
#define SZI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SZ_OK = 0,
    SZ_ERR_INVALID_ARG = -1,  /* bad pointer, size, shape or parameter */
    SZ_ERR_NONFINITE = -2,    /* the input field holds NaN or Inf */
    SZ_ERR_OOM = -3,          /* device allocation failed or budget exceeded */
    SZ_ERR_DEVICE = -4,       /* a HIP runtime call failed */
    SZ_ERR_CORRUPT = -5,      /* a blob failed its size or CRC-32 checks */
    SZ_ERR_UNSUPPORTED = -6,  /* a valid option this build does not implement */
    SZ_ERR_CAPACITY = -7      /* a caller buffer is too small */
} sz_status;

/* Error-bound mode (Sec. V-C.1): an absolute bound, or one relative to the
 * value range (the relative bound times the range is the absolute one). */
typedef enum { SZ_EB_ABS = 0, SZ_EB_REL = 1 } sz_eb_mode;

/* Spline per dimension (Sec. V-B.1).  LINEAR uses the linear spline even
 * where four neighbours exist; the cubic modes use the quadratic splines
 * where only three exist.  AUTO picks the cubic with the lower profiled
 * error (Sec. V-C.2). */
typedef enum {
    SZ_INTERP_LINEAR = 0,
    SZ_INTERP_CUBIC_NAK = 1,      /* not-a-knot: (-1, 9, 9, -1)/16 */
    SZ_INTERP_CUBIC_NATURAL = 2,  /* natural: (-3, 23, 23, -3)/40 */
    SZ_INTERP_CUBIC_AUTO = 3
} sz_interp;

typedef struct {
    uint32_t ndim;      /* 2 or 3 */
    uint32_t reserved;  /* 0 */
    uint64_t n[3];      /* n[0] fastest; entries >= ndim ignored */
} sz_dims;

typedef struct {
    int32_t eb_mode;        /* sz_eb_mode */
    int32_t reserved0;      /* 0 */
    double eb;              /* >= 0, finite */
    int32_t interp[3];      /* sz_interp per dimension index (0 = fastest) */
    int32_t order[3];       /* order[k] = dimension index of the k-th pass at
                               every level; order[0] < 0 = auto (least smooth
                               first, Sec. V-C.2) */
    double alpha;           /* level-bound reduction factor (Sec. V-B.2);
                               <= 0 = Eq. 1; 1 = the same bound everywhere */
    uint32_t radius;        /* R: codes q+R in 1..2R-1, 0 = outlier; 0 = 512 */
    uint32_t huff_chunk;    /* symbols per Huffman chunk; 0 = 1024 */
    uint32_t anchor_stride; /* 0 = default: 8 in 3D, 16 in 2D (Sec. V-A) */
    uint32_t window[3];     /* 0 = default: (32, 8, 8) in 3D, (64, 16) in 2D,
                               i.e. four basic blocks along x (Sec. V-D) */
} sz_params;

/* A compressed field.  Device pointers are owned by the context until
 * sz_result_free.  codes and hist are kept for inspection; they are not
 * part of the serialized blob. */
typedef struct {
    float* anchors;          /* lattice points, C-order, lossless */
    uint64_t n_anchors;
    uint16_t* codes;         /* n quant-codes: q+R; 0 = outlier; R at anchors */
    uint64_t n;
    uint32_t* outlier_idx;   /* ascending linear indices */
    float* outlier_val;      /* original values at those indices */
    uint64_t n_outliers;
    uint32_t* words;         /* Huffman bitstream */
    uint64_t n_words;
    uint16_t* chunk_bits;    /* bit count of every chunk */
    uint64_t n_chunks;
    uint32_t* hist;          /* 2R symbol counts */
    uint8_t* code_len;       /* 2R canonical code lengths (device) */
    uint64_t compressed_bytes;  /* size of the serialized blob */
    uint8_t header[256];     /* blob header (host copy), layout below */
    void* internal;          /* library bookkeeping; do not touch */
} sz_result;

typedef struct sz_ctx sz_ctx;

/* Fill p with the defaults: REL 1e-3, AUTO splines and order, Eq. 1 alpha,
 * R = 512, chunk 1024, default stride and window. */
void sz_params_default(sz_params* p);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * device memory the context may hold (0 = no cap). */
sz_status sz_ctx_create(sz_ctx** out, int device, uint64_t hbm_budget_bytes);
sz_status sz_ctx_destroy(sz_ctx* ctx);
const char* sz_last_error(const sz_ctx* ctx);
/* Device bytes held by the context now (pools included). */
uint64_t sz_ctx_bytes_in_use(const sz_ctx* ctx);

/* Launch shape of the persistent interpolation kernels: workgroups per
 * compute unit (1..64), or 0 (the default) for as many as are resident at
 * once.  Arithmetic-neutral: every setting gives byte-identical results; it
 * only trades occupancy against tail effects. */
sz_status sz_ctx_set_grid(sz_ctx* ctx, int workgroups_per_cu);
/* Launch-shape tuner for the interpolation kernels (compression, kind 0)
 * and the replay (kind 1), the batched launches of Sec. V-D included.  A
 * shape is a kernel variant (0: compiled for three waves per SIMD; 1: for
 * four, 2D only) and a grid (workgroups per compute unit, 0 = resident
 * capacity).  Every shape gives byte-identical results.
 *
 * sz_ctx_set_tuning(ctx, 1): a plain (non-graph) call that meets a
 * (kind, ndim, radius) with no shape yet times each candidate shape on its
 * own data, keeps the fastest for the context and uses it from then on;
 * the call's results do not change.  sz_ctx_set_grid(ctx, n > 0) takes
 * precedence over the tuner's grid and turns tuning off.
 * sz_ctx_set_shape pins a shape for a key (SZ_ERR_INVALID_ARG for a
 * variant that does not exist for ndim).  sz_ctx_get_shape reports the
 * shape in use for a key and whether one was tuned or pinned (*known). */
sz_status sz_ctx_set_tuning(sz_ctx* ctx, int on);
sz_status sz_ctx_set_shape(sz_ctx* ctx, int kind, int ndim, int radius, int variant,
                           int workgroups_per_cu);
sz_status sz_ctx_get_shape(sz_ctx* ctx, int kind, int ndim, int radius, int* variant,
                           int* workgroups_per_cu, int* known);
/* Graph mode (default off): the device work of a call is captured into a HIP
 * graph once per launch signature (number of fields, their grids, the
 * Huffman grouping, the launch shape) and replayed afterwards, on a stream of
 * the context that first waits for the caller's stream; the call still
 * returns after its work has finished.  Compression runs as two graphs
 * around the host codebook step, decompression as one.  The kernel
 * arguments of a graph live in a context-owned device arena filled from a
 * pinned mirror by the graph's first node.  Results are identical to the
 * default mode; per-stage timing is not recorded inside graphs. */
sz_status sz_ctx_set_graphs(sz_ctx* ctx, int enable);

/* Per-stage device timing.  When enabled, the context records a HIP event
 * pair around every kernel launch (on the stream the kernel runs on) and
 * accumulates the elapsed times once the call has synchronized.  Stages: */
typedef enum {
    SZ_STAGE_RANGE = 0,     /* value range, Sec. V-C.1 */
    SZ_STAGE_PROFILE = 1,   /* sampled spline errors, Sec. V-C.1 */
    SZ_STAGE_PLAN = 2,      /* alpha, level bounds, splines, order */
    SZ_STAGE_INTERP = 3,    /* interpolation predictor-quantiser + histogram */
    SZ_STAGE_CODEBOOK = 4,  /* histogram read-back, host codebook, upload */
    SZ_STAGE_HUFF_STATS = 5,
    SZ_STAGE_SCAN = 6,
    SZ_STAGE_ENCODE = 7,    /* Huffman packing + outlier compaction */
    SZ_STAGE_DECODE = 8,    /* Huffman decode */
    SZ_STAGE_SCATTER = 9,   /* outliers into the output */
    SZ_STAGE_REPLAY = 10,   /* interpolation replay (decompression) */
    SZ_STAGE_ELIDE = 11,    /* zero-word elision of the Huffman words (and its restore) */
    SZ_STAGE_COUNT = 12
} sz_stage;
/* enable != 0 turns timing on (and clears the totals). */
sz_status sz_ctx_set_timing(sz_ctx* ctx, int enable);
/* ms[SZ_STAGE_COUNT] receive accumulated milliseconds, launches[] the
 * number of timed intervals per stage (either may be NULL); reset != 0
 * clears the totals afterwards. */
sz_status sz_ctx_read_timing(sz_ctx* ctx, double* ms, uint64_t* launches, int reset);

/* Compress the device field d_in (n[0]*n[1]*n[2] floats, 4-byte aligned as
 * any float array is; INVALID_ARG otherwise, no 16-byte alignment needed:
 * the kernels take a faster path where rows start on 16 bytes).  Runs the whole
 * pipeline on `stream`: range and profiling (Sec. V-C.1), auto-tuning
 * (Sec. V-C.2, Eq. 1), level bounds (Sec. V-B.2), the interpolation
 * predictor-quantiser with a fused histogram (Sec. V-A/B/D, VI-A), the host
 * codebook (Sec. VI-A), Huffman encoding and outlier compaction.  Returns
 * when *out is complete (the call synchronizes the stream).
 * Errors: INVALID_ARG, NONFINITE, OOM, DEVICE, UNSUPPORTED. */
sz_status sz_compress(sz_ctx* ctx, const float* d_in, const sz_dims* dims,
                      const sz_params* params, void* stream, sz_result* out);

/* Compress nfields fields in one pass of batched launches: one persistent
 * interpolation launch over every window of every field, one batched
 * encode.  d_in[i], dims[i], params[i] describe field i; outs[i] receives
 * its result, byte-identical to what sz_compress returns for it alone.
 * A batch of four or more fields builds its host code books on worker
 * threads that the context starts on first use (seven) and keeps until
 * sz_ctx_destroy. */
sz_status sz_compress_batch(sz_ctx* ctx, uint32_t nfields, const float* const* d_in,
                            const sz_dims* dims, const sz_params* params, void* stream,
                            sz_result* outs);

/* Compress with a code book the caller gives instead of one built from this
 * field's histogram (Sec. VI-A builds it on the host between the histogram
 * and the encoding; reusing one, e.g. across the time steps of a
 * simulation, removes that host round trip).  code_len: host array of 2R
 * canonical code lengths, every symbol 1..24 bits with Kraft sum <= 1, so
 * that any quant-code can be encoded (sz_code_lengths makes one from a
 * histogram).  The pipeline is enqueued at once and the call waits once,
 * at the end; the result's histogram is this field's, its code lengths the
 * given ones, and the blob decodes like any other.  The Huffman words are
 * allocated for 24 bits per point, the outlier lists for a guess that the
 * call enlarges (running the encode again) when the field has more.
 * Errors: as sz_compress; INVALID_ARG for a code book that misses a symbol,
 * exceeds 24 bits or breaks the Kraft inequality. */
sz_status sz_compress_with_code(sz_ctx* ctx, const float* d_in, const sz_dims* dims,
                                const sz_params* params, const uint8_t* code_len, void* stream,
                                sz_result* out);

/* sz_compress_batch with a given code book per field (code_len[i]: host
 * array of 2R_i lengths, as for sz_compress_with_code): the whole batch is
 * enqueued at once, with no host round trip between the histograms and the
 * encoding, and in graph mode (sz_ctx_set_graphs) both of its graphs run
 * back to back.  Each result equals sz_compress_with_code's for its field.
 * Errors: as sz_compress_batch and sz_compress_with_code. */
sz_status sz_compress_batch_with_code(sz_ctx* ctx, uint32_t nfields, const float* const* d_in,
                                      const sz_dims* dims, const sz_params* params,
                                      const uint8_t* const* code_len, void* stream,
                                      sz_result* outs);

/* Code lengths for sz_compress_with_code from a histogram of nsym = 2R
 * bins (host memory): the length-limited Huffman lengths of the counts
 * plus one, so that every symbol gets a code.  Host only, no context.
 * Errors: INVALID_ARG (null pointer, nsym outside 2..2048). */
sz_status sz_code_lengths(const uint32_t* hist, uint32_t nsym, uint8_t* code_len);

/* Decompress a device-resident result into d_out (n floats, 4-byte aligned;
 * INVALID_ARG otherwise), replaying the predictions (Sec. V-B.1).  Returns
 * after the stream has completed.
 * Errors: INVALID_ARG, OOM, DEVICE, CORRUPT. */
sz_status sz_decompress(sz_ctx* ctx, const sz_result* res, float* d_out, void* stream);

/* Decompress several results in batched launches (one decode launch, one
 * replay launch over all windows of all fields). */
sz_status sz_decompress_batch(sz_ctx* ctx, uint32_t nfields, const sz_result* res,
                              float* const* d_out, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): sz_decompress
 * of one field without any allocation.  All of its scratch (the decoded
 * quant-codes, 2 bytes per point, and the launch descriptors) lives in a
 * static device workspace of the library, one per GPU, of
 * 2^26 + 2^20 bytes; fields of more than 2^25 points are refused with
 * UNSUPPORTED.  The call only enqueues work on the stream and returns: the
 * caller synchronises before reading d_out.  The workspace keeps the last
 * call's contents; calls on one GPU that overlap in time (other streams,
 * other host threads, other contexts) race on it and must be serialised by
 * the caller.  The output equals sz_decompress's bit for bit.
 * Errors: INVALID_ARG, CORRUPT, UNSUPPORTED, DEVICE. */
sz_status sz_decompress_noalloc(sz_ctx* ctx, const sz_result* res, float* d_out, void* stream);

/* Write the blob of res to host memory host_dst (capacity cap bytes).
 * *written receives res->compressed_bytes.  CAPACITY if cap is too small. */
sz_status sz_serialize(sz_ctx* ctx, const sz_result* res, void* host_dst, uint64_t cap,
                       uint64_t* written);

/* Parse a host blob (checking sizes and every CRC-32), copy it to the
 * device and fill *out so that sz_decompress can run on it.
 * Errors: CORRUPT, UNSUPPORTED (other version), OOM, DEVICE. */
sz_status sz_upload(sz_ctx* ctx, const void* host_blob, uint64_t bytes, void* stream,
                    sz_result* out);

/* Release the device buffers of a result (safe on a zeroed result). */
sz_status sz_result_free(sz_ctx* ctx, sz_result* res);

/* Copy one section of a result to host memory (for inspection and tests).
 * *written receives the section size in bytes. */
typedef enum {
    SZ_SEC_ANCHORS = 0, SZ_SEC_CODES = 1, SZ_SEC_OUTLIER_IDX = 2, SZ_SEC_OUTLIER_VAL = 3,
    SZ_SEC_WORDS = 4, SZ_SEC_CHUNK_BITS = 5, SZ_SEC_HIST = 6, SZ_SEC_CODE_LEN = 7
} sz_section;
sz_status sz_result_read(sz_ctx* ctx, const sz_result* res, int32_t section, void* host_dst,
                         uint64_t cap, uint64_t* written);

/*
 * Blob layout, little-endian; each section zero-padded to 8 bytes.
 *   off  size  field
 *     0     4  magic "SZI1"
 *     4     4  u32 version = 1
 *     8     4  u32 ndim
 *    12     4  u32 anchor stride S
 *    16    24  u64 n[3]           (unused dimensions 0)
 *    40    12  u32 window[3]      (unused dimensions 0)
 *    52     4  u32 radius R
 *    56     4  u32 Huffman length limit (24)
 *    60     4  u32 Huffman chunk C
 *    64     4  u32 eb_mode
 *    68     4  u32 levels L = log2 S
 *    72     8  f64 eb as given
 *    80     8  f64 alpha used
 *    88    12  f32 vmin, vmax, e (absolute bound, rounded down to FP32)
 *   100    12  i32 spline per dimension (0 linear, 1 NAK, 2 natural)
 *   112    12  i32 order (unused -1)
 *   124     4  u32 flags: bit 0 = words section zero-elided (below); other bits 0
 *   128    64  f32 e_l for l = 1..16 (l = 1 is stride 1; unused 0)
 *   192    32  u64 n_anchors, n_chunks, n_words, n_outliers
 *   224    24  u32 CRC-32 of each section (unpadded)
 *   248     4  reserved 0
 *   252     4  u32 CRC-32 of bytes 0..251
 *   256        anchors f32[n_anchors], code_len u8[2R], chunk_bits u16[n_chunks],
 *              words u32[n_words], outlier_idx u32[n_outliers],
 *              outlier_val f32[n_outliers]
 * Huffman: canonical codes from the lengths; chunk j covers symbols
 * [jC, min((j+1)C, n)), its codewords packed most-significant bit first
 * from bit 31 of its first word, zero-padded to a word; chunks follow each
 * other word-aligned.
 * Zero-word elision (the de-redundancy step after Huffman coding, in the
 * role Sec. VI-B gives a closed library): when it is shorter than the
 * n_words words, the words section holds instead a bitmap of
 * ceil(n_words / 32) u32 (bit k % 32 of bitmap word k / 32 set when word k
 * is non-zero) followed by the non-zero words in order, and flags bit 0 is
 * set.  n_words still counts all words.
 */

/* ------------------------------------------------------------ serving
 * A request server for a stream of compress and decompress jobs of uneven
 * sizes (continuous batching).  It has `slots` workers, each with its own
 * context (resident buffer pool) and HIP stream.  Requests wait in arrival
 * order; a free worker admits the oldest one whose device-memory estimate
 * fits what the HBM budget leaves, runs it as a plain sz_compress or
 * sz_decompress on its stream, and posts a completion.  Requests in
 * different slots overlap on the device, and the host codebook step of one
 * compression overlaps other requests' kernels.  A request's result depends
 * only on the request: the same as a plain call, alone or in any mix.
 *
 * The budget counts, for every running request, an upper bound of the
 * device memory it can take, and for every compression result not yet freed
 * its actual size.  Compression: with W = 3 n + 4 (n / 256 + 10) bytes for
 * the words of n points (kLmax = 24 bits a point, a word a chunk, slack),
 * 2 n + W + (W + W / 32 + 4) + 8 n + n / 16 + 2 MiB (codes, words, their
 * elided section while it is built, outliers, scratch, metadata);
 * decompression: 2 n + 1 MiB (codes).  0 = no limit.  With a budget, the
 * device memory of all workers together (what they hold and the blocks they
 * cache for reuse) stays within it: a worker returns cached blocks to the
 * device, its own first, then every worker's, before an allocation would
 * pass the budget.  The caller's input and output buffers are not counted.
 *
 * Resident code books (Sec. VI-A builds the code book on the host between
 * the histogram and the encoding; a stream of similar fields, such as the
 * time steps of a simulation, can keep one).  A compression request with
 * book = k > 0 uses the server's book k when it holds one for the request's
 * radius, as sz_compress_with_code does, with no host round trip; otherwise
 * it builds its own as sz_compress does and leaves sz_code_lengths of its
 * histogram as book k.  Such a result's blob may then differ from a plain
 * call's in its code lengths and words, never in its reconstruction.  The
 * books live until sz_server_destroy.
 *
 * The server may be called from any host thread.  Inputs (the field of a
 * compression, the result and output buffer of a decompression) must stay
 * valid until the request's completion has been polled; a result must not be
 * freed while a decompression of it is queued or running. */
typedef struct sz_server sz_server;

typedef enum { SZ_REQ_COMPRESS = 0, SZ_REQ_DECOMPRESS = 1 } sz_req_kind;

typedef struct {
    int32_t kind;            /* sz_req_kind */
    int32_t book;            /* compression: 0, or a resident code book k > 0 (below) */
    uint64_t tag;            /* the caller's id, echoed in the completion */
    const float* d_in;       /* compression: the field (device) */
    sz_dims dims;            /* compression: its shape */
    sz_params params;        /* compression: its parameters */
    const sz_result* src;    /* decompression: a result of this server or of any
                                context on the same device */
    float* d_out;            /* decompression: the output field (device) */
} sz_request;

typedef struct {
    uint64_t tag;
    int32_t status;          /* sz_status of the request */
    int32_t slot;            /* the worker that ran it */
    double t_submit;         /* seconds since the server was created: */
    double t_start;          /*   submitted, admitted, finished (its stream */
    double t_done;           /*   drained) */
    sz_result result;        /* compression: free with sz_server_result_free */
} sz_completion;

/* Create a server with 1..64 worker slots on a device. */
sz_status sz_server_create(sz_server** out, int device, int slots, uint64_t hbm_budget_bytes);
/* Enqueue a copy of *req.  SZ_ERR_OOM if the request alone exceeds the
 * budget; SZ_ERR_INVALID_ARG for a malformed request.  Errors of the work
 * itself are reported in the completion's status. */
sz_status sz_server_submit(sz_server* s, const sz_request* req);
/* Move up to cap completions, oldest first, into out; *n receives the count.
 * With wait != 0, block until at least one is available, or until nothing
 * runs and nothing queued can be admitted (then *n = 0). */
sz_status sz_server_poll(sz_server* s, sz_completion* out, uint32_t cap, uint32_t* n, int wait);
/* Free a compression result of this server and return its bytes to the
 * budget. */
sz_status sz_server_result_free(sz_server* s, sz_result* res);
/* Bytes charged against the budget, queued requests, running requests. */
sz_status sz_server_stats(sz_server* s, uint64_t* charged, uint64_t* queued, uint64_t* running);
const char* sz_server_last_error(const sz_server* s);
/* Cancel queued requests, wait for running ones, release everything,
 * including results not yet freed (their sz_result values become invalid). */
sz_status sz_server_destroy(sz_server* s);

#ifdef __cplusplus
}
#endif

#endif /* SZI_H */
