/*
 * dqz.h -- C ABI of libdqz, an error-bounded lossy compressor for fp32
 * fields on AMD MI355X (gfx950), implementing the dual-quantization +
 * Huffman method of cuSZ (Tian et al., PACT'20).
 *
 * Compression (Sec. 3.1-3.2 of the paper):
 *   value-range-relative error bound (footnote in Sec. 3.2.2)
 *   -> prequantization d° = round(d / 2eb) (Sec. 3.1.2, Algorithm 2)
 *   -> 1-layer Lorenzo prediction inside zero-padded blocks of 32 (1D),
 *      16x16 (2D) or 8x8x8 (3D) points (Sec. 3.1.1)
 *   -> postquantization delta = d° - p° with a cap of +-radius; values
 *      outside the cap are outliers stored verbatim (Algorithm 2)
 *   -> histogram of quantization codes (Sec. 3.2.1)
 *   -> Huffman code lengths + canonical codebook (Sec. 3.2.2-3.2.3)
 *   -> encode + deflate into one bit-dense stream (Sec. 3.2.4).
 * Decompression (Sec. 3.3): inflate, then reversed dual-quantization.
 *
 * Guarantee (the error-bounded problem statement of Sec. 2): every finite
 * input element comes back within eb_abs, |x - x'| <= eb_abs evaluated in
 * double precision; non-finite elements come back bit-exact.  Elements whose
 * fp32 reconstruction would miss the bound are stored verbatim ("patches",
 * the rehearsal/watchdog idea of Algorithm 1 applied to the final fp32
 * value).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers on the context's GPU; h_* are
 *     host pointers.  The caller owns all of them; the library never frees
 *     caller memory and never writes outside [ptr, ptr + capacity).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     stream-ordered.  dqz_compress / dqz_decompress wait for their own work
 *     at the end (to read back size and status, a few hundred bytes); the
 *     _async variants return after enqueueing and write the same facts into
 *     a caller-provided dqz_result, so a sequence of them can be captured in
 *     a HIP graph.
 *   - Device memory: a context owns one device workspace, allocated by
 *     dqz_ctx_create / dqz_ctx_reserve only.  dqz_compress, dqz_decompress
 *     and their _async variants never allocate or free memory; a call that
 *     needs more workspace than the context holds fails with DQZ_ENOMEM and
 *     dqz_ctx_workspace then reports the size that would have sufficed.
 *   - Calls on one context must not overlap (they share its workspace);
 *     separate contexts are independent.
 *   - Every function returns DQZ_OK (0) or a negative dqz_status; no C++
 *     exception crosses this boundary.  On error, output buffers hold
 *     unspecified bytes and the context stays usable.
 *
 * Archive layout (little-endian), fixed 128-byte header followed by
 *   lengths   u8[2R]                          Huffman code length per code
 *   chunks    u64[n_chunks]                   stream bit offset of each chunk
 *   subchunks u16[n_sub]                      stream bits of each subchunk
 *   exceptions {u32 key, u32 payload}[n_out + n_patch], ascending key,
 *             key = 2*position + kind; kind 0: outlier, payload = delta
 *             (int32); kind 1: patch, payload = raw fp32 bits of the input
 *   stream    u32[ceil(total_bits / 32)]      codewords MSB-first; stream
 *             bit i is bit (31 - i % 32) of word i / 32
 * Positions are indices in the padded block-major order: blocks in
 * row-major order of block coordinates, points row-major inside a full-size
 * block (points outside the field are skipped by the stream).  A subchunk is
 * `sub_size` consecutive positions, a chunk `chunk_subs` subchunks.  The
 * lengths and chunk sections start 8-byte aligned (after padding), as does
 * the exception section.
 */
#ifndef DQZ_H
#define DQZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dqz_status;

#define DQZ_OK 0
#define DQZ_EINVAL (-1)       /* bad argument: shape, eb, radius, sizes, null pointer */
#define DQZ_ETOOSMALL (-2)    /* archive or field capacity too small */
#define DQZ_ENOMEM (-3)       /* workspace too small, or a device / pinned host allocation failed */
#define DQZ_ECORRUPT (-4)     /* archive fails validation */
#define DQZ_EUNSUPPORTED (-5) /* valid request outside this build's limits */
#define DQZ_EHIP (-6)         /* a HIP runtime call failed (message in dqz_ctx_last_error) */
#define DQZ_EINTERNAL (-7)    /* a device-side ordering wait timed out (kernels exited; retry) */
/* DQZ_EAGAIN (-8): see dqz_server_wait */

#define DQZ_EB_ABS 0     /* eb is the absolute bound */
#define DQZ_EB_VALREL 1  /* eb is relative to (max - min) of the finite values */

#define DQZ_HEADER_BYTES 128

/* Field shape: ndim in {1,2,3}; dims[0..ndim-1] slowest -> fastest (C
 * row-major); entries past ndim are ignored.  An extent of 0 is an empty
 * field.  The padded position count (blocks * block volume) must stay below
 * 2^31. */
typedef struct {
    uint32_t ndim;
    uint32_t reserved;
    uint64_t dims[3];
} dqz_shape;

/* Compression parameters.  Zero fields take the defaults noted. */
typedef struct {
    double eb;           /* error bound, finite and > 0 */
    int32_t eb_mode;     /* DQZ_EB_ABS or DQZ_EB_VALREL */
    uint32_t radius;     /* code cap R: power of two in [1, 1024]; 2R quantization bins (default 512) */
    uint32_t sub_size;   /* positions per subchunk: power of two in [32, 1024] (default 128) */
    uint32_t chunk_subs; /* subchunks per chunk: power of two in [1, 65536] (default 64) */
    uint32_t layers;     /* Lorenzo predictor layers, 1 or 2 (default 1): the generalized
                            predictor with binomial coefficients of Sec. 3.1.2; recorded in
                            the archive header (byte 117 = layers - 1) */
    uint32_t reserved;   /* must be 0 */
} dqz_params;

/* What an _async call reports, written by its kernels into device-visible
 * memory (device memory, or mapped pinned host memory), 8-byte aligned:
 *   status          dqz_status of the device-side work (DQZ_OK, DQZ_ETOOSMALL,
 *                   DQZ_ENOMEM, DQZ_ECORRUPT, DQZ_EUNSUPPORTED, DQZ_EINVAL,
 *                   DQZ_EINTERNAL)
 *   archive_bytes   compression: the archive size (also with DQZ_ETOOSMALL);
 *                   decompression: the archive size read from its header
 *   workspace_need  with DQZ_ENOMEM: the workspace bytes that would have sufficed
 *   header          compression: the archive's 128-byte header
 * The fields are final once the stream has passed the call's work. */
typedef struct {
    uint32_t flags;      /* device status flags (diagnostic) */
    int32_t status;
    uint64_t archive_bytes;
    uint64_t workspace_need;
    uint64_t reserved;
    uint8_t header[DQZ_HEADER_BYTES];
} dqz_result;

typedef struct dqz_ctx dqz_ctx;

/* Create a context on HIP device `device` holding `workspace_cap` bytes of
 * device workspace (0: none yet; reserve before the first call).  The
 * workspace holds every intermediate of a call (control block, histogram,
 * codebook, scan states, staged exception records, code array, decoding
 * tables) and stays resident across calls.  DQZ_ENOMEM if it cannot be
 * allocated.  Supports the paper's GPU-resident pipeline (Sec. 3, data kept
 * on the device, Sec. 4.2.1). */
dqz_status dqz_ctx_create(int device, uint64_t workspace_cap, dqz_ctx **out);
void dqz_ctx_destroy(dqz_ctx *ctx);

/* Grow the context's workspace to at least `workspace_bytes` (no-op if it is
 * already that large).  The only place besides dqz_ctx_create that allocates
 * device memory; must not overlap a call on this context.  DQZ_ENOMEM on
 * failure (the old workspace is kept). */
dqz_status dqz_ctx_reserve(dqz_ctx *ctx, uint64_t workspace_bytes);

/* Host-only: the workspace the context holds, and the workspace the most
 * recent call on it needed (after DQZ_ENOMEM: the size that would have
 * sufficed).  Either output may be NULL. */
dqz_status dqz_ctx_workspace(const dqz_ctx *ctx, uint64_t *workspace_bytes, uint64_t *last_need);

/* Host-only: worst-case archive size for this shape and parameters (every
 * element an outlier and a patch, longest codes) and the workspace with
 * which dqz_compress never fails with DQZ_ENOMEM (a typical field needs
 * about 3 bytes per element of it; exception records past a tile's staging
 * slot take the rest).  Either output pointer may be NULL.  Sizes follow
 * the archive layout above (Sec. 3.2.4 deflate output plus tables). */
dqz_status dqz_compress_bound(const dqz_shape *shape, const dqz_params *params,
                              uint64_t *archive_max, uint64_t *workspace_bytes);

/* Host-only: the workspace dqz_decompress needs for the archive whose
 * 128-byte header is at h_header.  DQZ_ECORRUPT for a bad header. */
dqz_status dqz_decompress_bound(const void *h_header, uint64_t header_bytes, uint64_t *workspace_bytes);

/* Compress the fp32 field at d_field (row-major, `shape`) into d_archive
 * (capacity archive_cap bytes): the whole of Sec. 3.1-3.2 (range and error
 * bound, dual-quantization with outliers, histogram, codebook, encode +
 * deflate).  On success *archive_bytes holds the archive size; if h_header
 * is non-NULL the 128-byte header is copied there too.  If the archive does
 * not fit, returns DQZ_ETOOSMALL and *archive_bytes holds the size that
 * would have been needed when it is known (0 otherwise).  DQZ_ENOMEM when
 * the workspace is too small (dqz_ctx_workspace tells how much is needed). */
dqz_status dqz_compress(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape,
                        const dqz_params *params, void *d_archive, uint64_t archive_cap,
                        uint64_t *archive_bytes, void *h_header, void *stream);

/* dqz_compress without waiting: enqueues the same kernels on `stream` and
 * returns; status, archive size and header arrive in *d_result (see
 * dqz_result).  The return value covers only the host-side checks (arguments,
 * workspace size).  Nothing in it synchronizes, allocates or sets memory, so
 * a stream capture of it is a valid HIP graph; field, archive, result and
 * the context's workspace must stay valid while the work runs. */
dqz_status dqz_compress_async(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape,
                              const dqz_params *params, void *d_archive, uint64_t archive_cap,
                              dqz_result *d_result, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dqz_compress_async without a context.  The workspace is a fixed 128 MiB
 * device array inside the library (one copy per GPU, resident until the
 * process ends; its address is looked up on the first call on each device),
 * so nothing is allocated, freed or set on the host side.  Runs on the
 * calling thread's current HIP device; status, archive size and header
 * arrive in *d_result as for dqz_compress_async.  DQZ_EUNSUPPORTED, before
 * anything is enqueued, when the field's workspace (dqz_compress_bound's
 * workspace less the exception overflow pool: about 3 bytes per element)
 * exceeds the array -- fields of up to about 40 million elements fit;
 * exception records past the tiles' staging slots use the rest of the array,
 * and when they do not fit the device reports DQZ_ENOMEM in d_result.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams or threads, or with dqz_compress_async_static work
 * still running) race and must be serialized by the caller.  The kernels
 * clear what must start at zero themselves. */
dqz_status dqz_compress_async_static(const float *d_field, const dqz_shape *shape, const dqz_params *params,
                                     void *d_archive, uint64_t archive_cap, dqz_result *d_result, void *stream);

/* Host-only: parse and validate a 128-byte header.  Any output may be NULL.
 * field_elems = product of the dims. */
dqz_status dqz_archive_info(const void *h_header, uint64_t header_bytes, dqz_shape *shape,
                            dqz_params *params, uint64_t *field_elems, uint64_t *archive_bytes);

/* Decompress the archive at d_archive (archive_bytes long) into d_field
 * (capacity field_cap_elems floats, row-major): inflate and reversed
 * dual-quantization (Sec. 3.3, the decompression half of Algorithm 2).
 * h_header may point to a host copy of the archive's 128-byte header (skips
 * a device->host read); NULL reads it from d_archive.  Returns DQZ_ECORRUPT
 * for an archive that fails validation (the field then holds unspecified
 * values), DQZ_ENOMEM when the workspace is too small. */
dqz_status dqz_decompress(dqz_ctx *ctx, const void *d_archive, uint64_t archive_bytes,
                          const void *h_header, float *d_field, uint64_t field_cap_elems,
                          void *stream);

/* dqz_decompress without waiting (h_header is required); the device-side
 * status arrives in d_result->status.  Graph-capturable like
 * dqz_compress_async. */
dqz_status dqz_decompress_async(dqz_ctx *ctx, const void *d_archive, uint64_t archive_bytes,
                                const void *h_header, float *d_field, uint64_t field_cap_elems,
                                dqz_result *d_result, void *stream);

/* Batched calls: many fields in one call (the paper compresses one field per
 * launch sequence, Sec. 3; batching spreads a batch over concurrent lanes).
 * dqz_ctx_set_lanes gives the context `lanes` concurrent lanes (HIP streams of
 * default priority, 1..DQZ_MAX_LANES; 1 runs a batch on the caller's stream)
 * and with DQZ_LANES_GRAPH captures each batch into a HIP graph, replayed with
 * one launch while the same call (same pointers, shapes, parameters) repeats.
 * It synchronizes the device and may create streams, events and graphs:
 * call it at set-up, not while a batch of this context is in flight. */
#define DQZ_MAX_LANES 8
#define DQZ_LANES_GRAPH 1u
dqz_status dqz_ctx_set_lanes(dqz_ctx *ctx, uint32_t lanes, uint32_t flags);

/* Host-only: the workspace a batch of these fields needs on a context with
 * `lanes` lanes (each lane holds the largest fixed layout among the fields
 * assigned to it; what the context holds beyond the sum is split among the
 * lanes as their exception overflow pools). */
dqz_status dqz_batch_workspace(uint32_t n, const dqz_shape *shapes, const dqz_params *params, uint32_t lanes,
                               uint64_t *workspace_bytes);

/* Compress n fields: field i (d_fields[i], shapes[i], params[i]) into
 * d_archives[i] (capacity archive_caps[i]); status, size and header of field
 * i arrive in d_results[i] (device-visible memory, n entries, 8-byte
 * aligned) as for dqz_compress_async.  Enqueues on `stream` and returns (the
 * lanes fork from and join back into it).  Fields are assigned to lanes
 * longest first, each to the least loaded lane; every archive is byte for
 * byte the one dqz_compress writes for that field alone.  DQZ_ENOMEM when
 * the workspace is below dqz_batch_workspace (dqz_ctx_workspace reports the
 * need).  Host-side argument errors name the field in dqz_ctx_last_error. */
dqz_status dqz_compress_batch(dqz_ctx *ctx, uint32_t n, const float *const *d_fields, const dqz_shape *shapes,
                              const dqz_params *params, void *const *d_archives, const uint64_t *archive_caps,
                              dqz_result *d_results, void *stream);

/* Decompress n archives (Sec. 3.3 for each): archive i (d_archives[i],
 * archive_bytes[i], its 128-byte header at h_headers + 128 i on the host)
 * into d_fields[i] (capacity field_caps[i] floats); per-archive status in
 * d_results[i].  Lanes and graphs as for dqz_compress_batch; each lane needs
 * the largest dqz_decompress_bound among its archives. */
dqz_status dqz_decompress_batch(dqz_ctx *ctx, uint32_t n, const void *const *d_archives,
                                const uint64_t *archive_bytes, const void *h_headers, float *const *d_fields,
                                const uint64_t *field_caps, dqz_result *d_results, void *stream);

/* Autotuner for the deflate/inflate chunking (the paper sweeps the chunk
 * size per dataset, Sec. 4.2 / its chunk-size table): for the shape class of
 * this field (ndim, size octave, eb mode and decade, radius) pick sub_size in
 * {128, 256, 512} and chunk_subs in {16, 64, 256} by compressing and
 * decompressing the field with each (decompression timed with HIP events):
 * the smallest archive among the candidates that decompress within
 * (1 + tolerance) of the fastest.  The bit stream does not depend on the
 * choice.  The choice is cached on the context; a later call for the same
 * class returns it without measuring unless flags has DQZ_TUNE_FORCE.
 * *out = base with sub_size and chunk_subs set.  Synchronizes `stream`; the
 * workspace must hold the field's compression layout plus an archive bound,
 * the field and 64 MiB (DQZ_ENOMEM otherwise). */
#define DQZ_TUNE_FORCE 1u
dqz_status dqz_tune(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape, const dqz_params *base,
                    double tolerance, uint32_t flags, dqz_params *out, void *stream);

/* Serving: continuous batching of compression and decompression requests on
 * one GPU (the paper's kernels, Sec. 3, run per request; a served request's
 * output is byte for byte what dqz_compress / dqz_decompress write for it).
 * A server owns `slots` concurrent slots (each a HIP stream of default
 * priority, an event and a pinned status block) and one resident device
 * arena of `workspace_bytes` from which each admitted request gets its
 * workspace; all of it is allocated by dqz_server_create, nothing per
 * request.  One dispatcher thread admits requests in arrival order as soon as
 * a slot is free and the request's footprint (input bytes + output capacity +
 * workspace) fits `hbm_budget` beside the running requests' footprints (the
 * head of the queue waits until it fits; a request runs alone if it exceeds
 * the budget by itself), enqueues its kernels on the slot's stream and polls
 * the slots' completion events, so requests that arrive while others run
 * start as soon as a slot and memory free up and their kernels overlap the
 * running ones.  A compression gets its fixed workspace layout plus room for
 * one exception record per element; one whose records overflow that runs
 * again first in line with the size the device reported.
 * The caller owns every input and output buffer and keeps it valid until the
 * request's completion has been collected with dqz_server_wait. */
typedef struct dqz_server dqz_server;
typedef struct {
    uint32_t slots;            /* concurrent requests on the device, 1..DQZ_MAX_LANES */
    uint32_t reserved;
    uint64_t workspace_bytes;  /* resident device arena for the requests' workspaces */
    uint64_t hbm_budget;       /* cap on the summed footprints of the running requests */
} dqz_server_config;
#define DQZ_REQ_COMPRESS 0u
#define DQZ_REQ_DECOMPRESS 1u
typedef struct {
    uint32_t kind;             /* DQZ_REQ_COMPRESS or DQZ_REQ_DECOMPRESS */
    uint32_t reserved;
    const void *d_input;       /* compression: fp32 field; decompression: archive */
    uint64_t input_bytes;      /* decompression: archive bytes */
    void *d_output;            /* compression: archive buffer; decompression: field buffer */
    uint64_t output_capacity;  /* bytes */
    dqz_shape shape;           /* compression */
    dqz_params params;         /* compression */
    uint8_t header[DQZ_HEADER_BYTES];   /* decompression: host copy of the archive's header */
} dqz_request;
typedef struct {
    int32_t status;            /* the request's dqz_status */
    uint32_t reserved;
    uint64_t output_bytes;     /* archive bytes (with DQZ_ETOOSMALL: the size needed) or field bytes */
    uint64_t footprint;        /* device bytes it was admitted with */
    double t_submit_us, t_admit_us, t_done_us;   /* server clock: submitted, admitted, completion seen */
    uint8_t header[DQZ_HEADER_BYTES];   /* compression: the archive's header */
} dqz_completion;
typedef struct {
    uint64_t submitted, admitted, completed, failed, retried;
    uint64_t max_running;          /* most requests on the device at once */
    uint64_t max_in_flight_bytes;  /* largest summed footprint of running requests */
} dqz_server_stats;
#define DQZ_EAGAIN (-8)   /* dqz_server_wait: not completed within the timeout */
dqz_status dqz_server_create(int device, const dqz_server_config *cfg, dqz_server **out);
/* Waits for every submitted request to complete, then frees the server. */
void dqz_server_destroy(dqz_server *server);
/* Validate (host only) and queue a request; *ticket names it.  DQZ_ENOMEM if
 * its workspace exceeds the arena (it could never run); argument errors as
 * for the single-field calls.  Thread-safe. */
dqz_status dqz_server_submit(dqz_server *server, const dqz_request *req, uint64_t *ticket);
/* Wait up to timeout_us (negative: without limit) for a request's completion
 * and collect it (once per ticket); DQZ_EAGAIN on timeout.  Thread-safe. */
dqz_status dqz_server_wait(dqz_server *server, uint64_t ticket, int64_t timeout_us, dqz_completion *out);
dqz_status dqz_server_get_stats(dqz_server *server, dqz_server_stats *out);

/* Host path.  The paper's overall throughput counts the archive's trip to
 * host memory (Sec. 4.2, its overall figures), and a field larger than the
 * device memory is compressed block by block (the prediction blocks of
 * Sec. 3.1.1 are independent).  dqz_stream_compress reads a field from host
 * memory (pinned memory lets the copies overlap the kernels) in slabs: runs
 * of the slowest axis about slab_bytes long whose extent is a multiple of the
 * prediction block edge along it (32 in 1D, 16 in 2D, 8 in 3D), so every
 * block lies in one slab.  Each slab becomes an ordinary archive compressed
 * with an absolute bound (in the value-range-relative mode: eb times the
 * whole field's finite range, found in a first pass over the slabs), written
 * into h_container after a 128-byte container header and the slab offsets.
 * The decompressed field is bit for bit what dqz_decompress gives for a
 * whole-field archive compressed with that absolute bound.  Uploads, kernels
 * and downloads of consecutive slabs overlap on three streams (`stream` and
 * the context's two copy streams).  The workspace holds two slabs of input
 * and archive plus one slab's compression workspace with one exception
 * record per element (dqz_stream_workspace); DQZ_ENOMEM if smaller.
 * Synchronous: returns when the container is complete in host memory. */
dqz_status dqz_stream_workspace(const dqz_shape *shape, const dqz_params *params, uint64_t slab_bytes,
                                uint64_t *workspace_bytes, uint64_t *container_max);
dqz_status dqz_stream_compress(dqz_ctx *ctx, const float *h_field, const dqz_shape *shape, const dqz_params *params,
                               uint64_t slab_bytes, void *h_container, uint64_t container_cap,
                               uint64_t *container_bytes, void *stream);
/* Host-only: parse and validate a container (and its slabs' headers): shape,
 * slab count, the absolute bound, and the workspace dqz_stream_decompress
 * needs.  Any output may be NULL.  DQZ_ECORRUPT for a bad container. */
dqz_status dqz_stream_info(const void *h_container, uint64_t bytes, dqz_shape *shape, uint32_t *n_slabs,
                           double *eb_abs, uint64_t *workspace_bytes);
/* Decompress a container from host memory into the host field (capacity
 * field_cap_elems floats), slab by slab with the copies overlapping the
 * kernels (Sec. 3.3 per slab).  Synchronous. */
dqz_status dqz_stream_decompress(dqz_ctx *ctx, const void *h_container, uint64_t bytes, float *h_field,
                                 uint64_t field_cap_elems, void *stream);

const char *dqz_status_str(dqz_status status);
/* Text of the last error on this context ("" if none); with ctx == NULL, why
 * the most recent dqz_ctx_create on the calling thread failed. */
const char *dqz_ctx_last_error(const dqz_ctx *ctx);

/* Per-stage timing (the paper's per-kernel breakdown, Sec. 4.2).  `level` 0
 * turns it off.  At level 1 every dqz_compress / dqz_decompress on this
 * context records HIP events on its stream between its kernels (a small
 * per-call cost, about a microsecond per event); level 2 also sums per-wave
 * phase durations inside the decoding kernel (DQZ_DBG_PHASES), which costs a
 * few same-address atomics per wave and slows that kernel noticeably.
 * DQZ_TIMING_STAGE(which, stage) records only the two events around one
 * stage of one call kind (the other stages read 0).  dqz_stage_times
 * returns the elapsed microseconds of each stage of the most recent call of
 * that kind:
 *   compress   (which = 0): [0] scratch clearing (absolute mode; in the
 *              value-range-relative mode the range kernel clears it and this
 *              stage is 0), [1] value range + eb (0 in absolute mode), [2] dual-quantization + histogram + exceptions, [3] their
 *              tile scan (and the histogram sum), [4] codebook + header,
 *              [5] encode + deflate (widths, tile offsets, packing, one pass)
 *   decompress (which = 1): [0] decoding tables (and, for 128-position
 *              subchunks, the exception index), [1] inflate (other subchunk
 *              sizes: inflate + reconstruct), [2] reconstruct (128-position
 *              subchunks; 0 otherwise)
 * `us` must hold DQZ_MAX_STAGES doubles; *n_stages receives the count. */
#define DQZ_MAX_STAGES 8
#define DQZ_TIMING_STAGE(which, stage) (0x100 | ((which) << 4) | (stage))
dqz_status dqz_ctx_set_timing(dqz_ctx *ctx, int level);
dqz_status dqz_stage_times(dqz_ctx *ctx, int which, double *us, int *n_stages);

/* Stage dumps for parity testing (the intermediates of Sec. 3.1-3.2): copy a
 * buffer of the most recent dqz_compress on this context to host memory
 * (DQZ_EINVAL after a decompression or a workspace reallocation, which
 * overwrite them).
 *   DQZ_DBG_CODES      u16 per padded position (0xFFFF outside the field)
 *   DQZ_DBG_HISTOGRAM  u32[2R]
 *   DQZ_DBG_CODEBOOK   u64[2R], (length << 56) | canonical code
 *   DQZ_DBG_PHASES     u64[32], phase timestamps of the one-workgroup kernels and
 *                      decoding-wave durations (recorded at timing level 2);
 *                      also readable after a dqz_decompress (until a
 *                      reallocation or a batched or streaming call), the
 *                      entries of the other kind of call then meaningless
 * `bytes` must equal the buffer's size. */
#define DQZ_DBG_CODES 1
#define DQZ_DBG_HISTOGRAM 2
#define DQZ_DBG_CODEBOOK 3
#define DQZ_DBG_PHASES 4     /* u64[32], wall clock at 100 MHz: marks inside the codebook
                                kernel [0..15] and the decoding-table kernel [16..18];
                                first decoding-wave start [24], last decoding-wave end
                                [25], phase durations summed over the decoding waves
                                [26..31]: for 128-position subchunks (inflate kernel)
                                tables + stream window, inflate; otherwise tables,
                                stream window + exception search, inflate, outlier
                                marks, reconstruct, patches */
dqz_status dqz_debug_copy(dqz_ctx *ctx, int what, void *h_dst, uint64_t bytes);

/* Test hook for failure handling: with what = DQZ_INJECT_ALLOC_FAIL the next
 * `count` workspace allocations of this context (dqz_ctx_reserve) fail with
 * DQZ_ENOMEM as if the device were out of memory; 0 clears it. */
#define DQZ_INJECT_ALLOC_FAIL 1
dqz_status dqz_debug_inject(dqz_ctx *ctx, int what, int count);

#ifdef __cplusplus
}
#endif

#endif /* DQZ_H */
