// dqz_capi.cpp -- the C ABI of libdqz: argument validation, geometry and
// archive layout, the context's device workspace, and the stream-ordered
// launch sequence.
//
// Compression:   [clear scratch | range + eb (valrel)] -> quantize -> tile
//                scan -> codebook + header -> encode + deflate -> readback
//                (status, size, header) through a small block the kernels
//                write into host-visible memory.
// Decompression: decoding tables -> inflate -> reconstruct -> readback.
//
// The workspace is allocated when the context is created or reserved,
// never inside dqz_compress / dqz_decompress: a call whose layout does not
// fit returns DQZ_ENOMEM and reports the size that would have sufficed.
#include "../../include/dqz.h"
#include "dqz_internal.h"
#include "dqz_host.h"

#include <hip/hip_runtime.h>

#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

using namespace dqz;
using namespace dqz::host;

static_assert(sizeof(dqz_result) == sizeof(Readback), "dqz_result mirrors the kernels' readback block");
static_assert(offsetof(dqz_result, status) == offsetof(Readback, code), "dqz_result layout");
static_assert(offsetof(dqz_result, archive_bytes) == offsetof(Readback, archive_bytes), "dqz_result layout");
static_assert(offsetof(dqz_result, workspace_need) == offsetof(Readback, workspace_need), "dqz_result layout");
static_assert(offsetof(dqz_result, header) == offsetof(Readback, header), "dqz_result layout");

namespace dqz {
namespace host {

constexpr uint32_t kDefaultRadius = 512;
constexpr uint32_t kDefaultSub = 128;
constexpr uint32_t kDefaultChunkSubs = 64;

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }
uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
uint32_t log2u(uint32_t v) {
    uint32_t s = 0;
    while ((1u << s) < v) s++;
    return s;
}

dqz_status fail(dqz_ctx *ctx, dqz_status st, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return st;
}

dqz_status hip_fail(dqz_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, DQZ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}



dqz_status make_geom(const dqz_shape *s, Geom &g, std::string &why) {
    if (!s) { why = "shape is NULL"; return DQZ_EINVAL; }
    if (s->ndim < 1 || s->ndim > 3) { why = "ndim must be 1, 2 or 3"; return DQZ_EINVAL; }
    uint64_t n3[3] = {1, 1, 1};
    for (uint32_t i = 0; i < s->ndim; i++) n3[3 - s->ndim + i] = s->dims[i];
    for (int a = 0; a < 3; a++)
        if (n3[a] >= (1ull << 31)) { why = "extent too large"; return DQZ_EUNSUPPORTED; }
    const uint32_t b3[3][3] = {{1, 1, 32}, {1, 16, 16}, {8, 8, 8}};
    uint64_t nblocks = 1, nelem = 1;
    for (int a = 0; a < 3; a++) {
        g.n[a] = (uint32_t)n3[a];
        g.b[a] = b3[s->ndim - 1][a];
        g.nb[a] = (uint32_t)((n3[a] + g.b[a] - 1) / g.b[a]);
        nblocks *= g.nb[a];
        nelem *= n3[a];
    }
    g.bvol = g.b[0] * g.b[1] * g.b[2];
    g.ndim = s->ndim;
    g.nelem = nelem;
    const uint64_t padded = nblocks * g.bvol;
    if (padded >= (1ull << 31)) { why = "field too large: padded positions must stay below 2^31"; return DQZ_EUNSUPPORTED; }
    g.padded = (uint32_t)padded;
    return DQZ_OK;
}

dqz_status make_layout(const Geom &g, uint32_t radius, uint32_t sub, uint32_t csubs, Layout &L, std::string &why) {
    if (!is_pow2(radius) || radius > 4096) { why = "radius must be a power of two <= 4096"; return DQZ_EINVAL; }
    if (radius > kMaxRadius) { why = "radius above 1024 is not supported by this build"; return DQZ_EUNSUPPORTED; }
    if (!is_pow2(sub) || sub < 32 || sub > 1024) { why = "sub_size must be a power of two in [32, 1024]"; return DQZ_EINVAL; }
    if (!is_pow2(csubs) || csubs > 65536) { why = "chunk_subs must be a power of two <= 65536"; return DQZ_EINVAL; }
    L.radius = radius;
    L.nsym = 2 * radius;
    L.sub_size = sub;
    L.sub_shift = log2u(sub);
    L.chunk_subs = csubs;
    const uint64_t n_sub = (g.padded + (uint64_t)sub - 1) / sub;
    const uint64_t n_chunks = (n_sub + csubs - 1) / csubs;
    L.n_sub = (uint32_t)n_sub;
    L.n_chunks = (uint32_t)n_chunks;
    L.off_len = kHeaderBytes;
    L.off_chunk = align_up(L.off_len + L.nsym, 8);
    L.off_sub = L.off_chunk + 8 * n_chunks;
    L.off_exc = align_up(L.off_sub + 2 * n_sub, 8);
    L.cap = 0;
    L.layers = 1;
    L.ws_fixed = 0;
    return DQZ_OK;
}

dqz_status set_layers(const dqz_params *p, Layout &L, std::string &why) {
    const uint32_t layers = p->layers ? p->layers : 1u;
    if (layers > kMaxLayers || p->reserved) {
        why = "layers must be 1 or 2 (and reserved 0)";
        return DQZ_EINVAL;
    }
    L.layers = layers;
    return DQZ_OK;
}

void fill_params(const dqz_params *p, uint32_t &radius, uint32_t &sub, uint32_t &csubs) {
    radius = p->radius ? p->radius : kDefaultRadius;
    sub = p->sub_size ? p->sub_size : kDefaultSub;
    csubs = p->chunk_subs ? p->chunk_subs : kDefaultChunkSubs;
}

// Wait for the stream: poll for up to a millisecond (the end of each call is
// on the critical path, and a polling wait returns sooner than a blocking
// one), then block so that a long call does not hold a host core.
hipError_t wait_stream(hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipStreamQuery(s);
        if (e != hipErrorNotReady) return e;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(1000)) return hipStreamSynchronize(s);
    }
}

// why the most recent dqz_ctx_create on this thread failed
thread_local std::string g_create_error;
dqz_status create_fail(dqz_status st, const std::string &why) {
    g_create_error = why;
    return st;
}

// readback status before the codebook kernel has written the block
constexpr uint32_t kNoReadback = 0xFFFFFFFFu;

// Workspace layout.  Compression: control block, decoding tables, the zeroed
// region (histogram replicas and their sum, encoder look-back states), the
// codebooks, range partials, the quantize tiles' scan arrays and overflow
// bases, the per-tile exception slots, the code array, then (from
// `fixed`) the exception overflow pool, which takes the rest of the
// workspace.  Decompression: control block, tables, the decoded code array
// and the per-unit exception index (over the compression buffers).

WsLayout ws_layout(const Plan &P, bool compress) {
    WsLayout w;
    memset(&w, 0, sizeof(w));
    auto take = [](uint64_t &cur, uint64_t bytes) {
        const uint64_t at = align_up(cur, 256);
        cur = at + bytes;
        return at;
    };
    w.n_segs_q = (P.tiles_q + kSegTiles - 1) / kSegTiles;
    uint64_t cur = 0;
    w.ctl = take(cur, sizeof(Ctl));
    w.tab = take(cur, sizeof(DecodeTables));
    if (!compress) {
        // 128-position subchunks: decoded codes, 256 bytes per subchunk for
        // whole waves of 64 subchunks, and the exception index per unit
        w.qws = P.L.sub_size == 128 ? take(cur, 256ull * ((P.L.n_sub + 63) / 64 * 64)) : 0;
        w.unit_exc = P.L.sub_size == 128 ? take(cur, 4ull * (recon_units(P.g) + 1)) : 0;
        w.total = w.fixed = align_up(cur, 256);
        return w;
    }
    w.hist = take(cur, 4ull * kHistReplicas * P.L.nsym);
    w.hist_sum = take(cur, 4ull * P.L.nsym);   // zeroed too: an empty field never writes it
    w.eflag = take(cur, 128ull * P.tiles_e);    // encode look-back states (one line each) start at zero
    w.zero_end = align_up(cur, 256);
    w.book = take(cur, 8ull * P.L.nsym);
    w.book32 = take(cur, 4ull * P.L.nsym);
    w.parts = take(cur, 8ull * kMinmaxMaxBlocks);
    for (int k = 0; k < 2; k++) {
        w.qval[k] = take(cur, 4ull * P.tiles_q);
        w.qexcl[k] = take(cur, 4ull * P.tiles_q);
        w.qseg_total[k] = take(cur, 8ull * w.n_segs_q);
    }
    w.ovf_base = take(cur, 4ull * P.tiles_q);
    w.stage = take(cur, 8ull * kExcCap * P.tiles_q);
    w.codes = take(cur, 2ull * P.g.padded);
    w.fixed = align_up(cur, 256);
    // worst case: every element an outlier and a patch, all past the slots
    w.total = w.fixed + 16ull * P.g.nelem;
    return w;
}

// stage marks: mark(ctx, which, i) records event i of call kind `which`
void mark(dqz_ctx *ctx, int which, int i, hipStream_t s) {
    if (!ctx || !ctx->timing) return;
    if (i == 0)
        for (int k = 0; k <= DQZ_MAX_STAGES; k++) ctx->ev_rec[which][k] = false;
    const int only = ctx->only_stage[which];
    if (only == -1 || i == only || i == only + 1) {
        (void)hipEventRecord(ctx->ev[which][i], s);
        ctx->ev_rec[which][i] = true;
    }
    ctx->n_ev[which] = i + 1;
}

const char *status_message(dqz_status st) {
    switch (st) {
        case DQZ_EINTERNAL: return "internal consistency check failed";
        case DQZ_EINVAL: return "error bound out of range for this field";
        case DQZ_ENOMEM: return "workspace too small for this field's exception records";
        case DQZ_EUNSUPPORTED: return "code length above 64 bits";
        case DQZ_ECORRUPT: return "archive failed validation";
        case DQZ_ETOOSMALL: return "archive capacity too small";
        default: return "";
    }
}

uint32_t rd_u32(const uint8_t *p, int off) {
    uint32_t v;
    memcpy(&v, p + off, 4);
    return v;
}
uint64_t rd_u64(const uint8_t *p, int off) {
    uint64_t v;
    memcpy(&v, p + off, 8);
    return v;
}

// Parse and validate a header; fills the plan (with the archive-dependent
// counts) when `P` is non-NULL.

dqz_status parse_header(const uint8_t *hb, uint64_t n, HeaderInfo &hi, Plan *P, std::string &why) {
    if (!hb || n < kHeaderBytes) { why = "header too short"; return DQZ_ECORRUPT; }
    if (rd_u32(hb, 0) != kMagic || (hb[4] | (hb[5] << 8)) != (int)kVersion) { why = "bad magic or version"; return DQZ_ECORRUPT; }
    const uint32_t ndim = hb[6], mode = hb[7];
    if (ndim < 1 || ndim > 3 || mode > 1) { why = "bad ndim or eb mode"; return DQZ_ECORRUPT; }
    memset(&hi, 0, sizeof(hi));
    hi.shape.ndim = ndim;
    const uint64_t n3[3] = {rd_u64(hb, 8), rd_u64(hb, 16), rd_u64(hb, 24)};
    for (uint32_t a = 0; a < 3 - ndim; a++)
        if (n3[a] != 1) { why = "bad dims"; return DQZ_ECORRUPT; }
    for (uint32_t i = 0; i < ndim; i++) hi.shape.dims[i] = n3[3 - ndim + i];
    Plan local;
    Plan &pl = P ? *P : local;
    std::string w2;
    if (make_geom(&hi.shape, pl.g, w2) != DQZ_OK) { why = "bad dims: " + w2; return DQZ_ECORRUPT; }
    for (int a = 0; a < 3; a++)
        if (rd_u32(hb, 32 + 4 * a) != pl.g.b[a]) { why = "bad block dims"; return DQZ_ECORRUPT; }
    const uint32_t radius = rd_u32(hb, 44), sub = rd_u32(hb, 104), csubs = rd_u32(hb, 108);
    if (make_layout(pl.g, radius, sub, csubs, pl.L, w2) != DQZ_OK) { why = "bad parameters: " + w2; return DQZ_ECORRUPT; }
    double ebp;
    memcpy(&ebp, hb + 48, 8);
    hi.params.eb = ebp;
    hi.params.eb_mode = (int32_t)mode;
    hi.params.radius = radius;
    hi.params.sub_size = sub;
    hi.params.chunk_subs = csubs;
    if (hb[117] + 1u > kMaxLayers || hb[118] || hb[119]) { why = "bad predictor layers"; return DQZ_ECORRUPT; }
    pl.L.layers = hb[117] + 1u;
    hi.params.layers = pl.L.layers;
    hi.nelem = rd_u64(hb, 80);
    if (hi.nelem != pl.g.nelem) { why = "element count mismatch"; return DQZ_ECORRUPT; }
    const uint64_t n_out = rd_u32(hb, 88), n_patch = rd_u32(hb, 92);
    if (n_out > hi.nelem || n_patch > hi.nelem) { why = "bad exception counts"; return DQZ_ECORRUPT; }
    hi.n_exc = n_out + n_patch;
    hi.total_bits = rd_u64(hb, 96);
    if (hi.total_bits > 64ull * hi.nelem) { why = "bad stream length"; return DQZ_ECORRUPT; }
    if (rd_u32(hb, 112) != pl.L.n_chunks) { why = "chunk count mismatch"; return DQZ_ECORRUPT; }
    hi.max_len = hb[116];
    if (hi.max_len > 63 || (hi.nelem > 0 && hi.max_len == 0)) { why = "bad max code length"; return DQZ_ECORRUPT; }
    hi.n_words = (hi.total_bits + 31) / 32;
    hi.off_str = pl.L.off_exc + 8 * hi.n_exc;
    const uint64_t end = hi.off_str + 4 * hi.n_words;
    hi.archive_bytes = rd_u64(hb, 120);
    if (hi.archive_bytes != end) { why = "archive size mismatch"; return DQZ_ECORRUPT; }
    uint32_t hbits = rd_u32(hb, 64);
    memcpy(&hi.h, &hbits, 4);
    if (!std::isfinite(hi.h) || !(hi.h > 0.0f)) { why = "bad quantization step"; return DQZ_ECORRUPT; }
    return DQZ_OK;
}

dqz_status alloc_workspace(dqz_ctx *ctx, uint64_t bytes) {
    if (ctx->inject_alloc_fail > 0) {
        ctx->inject_alloc_fail--;
        return fail(ctx, DQZ_ENOMEM, "device workspace allocation failed (injected)");
    }
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, DQZ_ENOMEM, "device workspace allocation failed");
    }
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    ctx->last_valid = false;
    ctx->phases_valid = false;
    return DQZ_OK;
}

// Validate the arguments of a compression and plan it (host only); the
// workspace size check is the caller's.
dqz_status plan_compress_args(const float *d_field, const dqz_shape *shape, const dqz_params *params,
                              const void *d_archive, uint64_t archive_cap, Plan &P, WsLayout &W, std::string &why) {
    if (!params || !d_archive) { why = "null argument"; return DQZ_EINVAL; }
    if (!(params->eb > 0.0) || !std::isfinite(params->eb)) { why = "eb must be finite and > 0"; return DQZ_EINVAL; }
    if (params->eb_mode != DQZ_EB_ABS && params->eb_mode != DQZ_EB_VALREL) { why = "bad eb_mode"; return DQZ_EINVAL; }
    dqz_status st = make_geom(shape, P.g, why);
    if (st != DQZ_OK) return st;
    if (P.g.nelem && !d_field) { why = "null field"; return DQZ_EINVAL; }
    uint32_t radius, sub, csubs;
    fill_params(params, radius, sub, csubs);
    if ((st = make_layout(P.g, radius, sub, csubs, P.L, why)) != DQZ_OK) return st;
    if ((st = set_layers(params, P.L, why)) != DQZ_OK) return st;
    if (params->eb_mode == DQZ_EB_ABS) {
        const double e = params->eb;
        const float h = (float)(2.0 * e), r = (float)(1.0 / (2.0 * e));
        if (e < (double)FLT_MIN || !std::isfinite(h) || !(r >= FLT_MIN) || !std::isfinite(r)) {
            why = "eb out of the fp32 range";
            return DQZ_EINVAL;
        }
    }
    P.L.cap = archive_cap;
    if (archive_cap < P.L.off_exc) { why = "archive capacity below the fixed sections"; return DQZ_ETOOSMALL; }
    P.tiles_q = quantize_tiles(P.g);
    P.tiles_e = encode_tiles(P.g);
    W = ws_layout(P, true);
    P.L.ws_fixed = W.fixed;
    return DQZ_OK;
}

dqz_status plan_compress(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape, const dqz_params *params,
                         const void *d_archive, uint64_t archive_cap, Plan &P, WsLayout &W) {
    std::string why;
    const dqz_status st = plan_compress_args(d_field, shape, params, d_archive, archive_cap, P, W, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    ctx->last_need = W.fixed;
    if (ctx->ws_bytes < W.fixed)
        return fail(ctx, DQZ_ENOMEM, "workspace too small: this field needs at least " + std::to_string(W.fixed) +
                                          " bytes (dqz_ctx_reserve)");
    return DQZ_OK;
}

// Enqueue the compression kernels; they write status, size and header to rb.
// The workspace is [ws, ws + ws_bytes) on the stream's device (ws_bytes >=
// W.fixed); `ctx` (may be NULL) takes the timing marks and the stage-dump
// pointers.
void enqueue_compress(dqz_ctx *ctx, uint8_t *ws, uint64_t ws_bytes, int ncu, const float *d_field,
                      const dqz_params *params, uint8_t *arc, const Plan &P, const WsLayout &W, Readback *rb,
                      hipStream_t s) {
    Ctl *ctl = reinterpret_cast<Ctl *>(ws + W.ctl);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + W.hist);
    uint64_t *book = reinterpret_cast<uint64_t *>(ws + W.book);
    uint32_t *book32 = reinterpret_cast<uint32_t *>(ws + W.book32);
    uint32_t *parts = reinterpret_cast<uint32_t *>(ws + W.parts);
    uint16_t *codes = reinterpret_cast<uint16_t *>(ws + W.codes);
    QuantBufs qb;
    qb.codes = codes;
    qb.hist = hist;
    qb.hist_sum = reinterpret_cast<uint32_t *>(ws + W.hist_sum);
    qb.stage = reinterpret_cast<uint2 *>(ws + W.stage);
    qb.cap = kExcCap;
    qb.pool = reinterpret_cast<uint2 *>(ws + W.fixed);
    qb.pool_cap = (ws_bytes - W.fixed) / 8;
    qb.ovf_base = reinterpret_cast<uint32_t *>(ws + W.ovf_base);
    TileScan &qs = qb.scan;
    for (int k = 0; k < 2; k++) {
        qs.val[k] = reinterpret_cast<uint32_t *>(ws + W.qval[k]);
        qs.excl[k] = reinterpret_cast<uint32_t *>(ws + W.qexcl[k]);
        qs.seg_total[k] = reinterpret_cast<uint64_t *>(ws + W.qseg_total[k]);
    }
    qs.n_tiles = P.tiles_q;
    qs.n_segs = W.n_segs_q;
    qs.nvals = 2;
    EncodeBufs eb;
    eb.codes = codes;
    eb.book = book;
    eb.book32 = book32;
    eb.stage = qb.stage;
    eb.cap = kExcCap;
    eb.pool = qb.pool;
    eb.ovf_base = qb.ovf_base;
    eb.qscan = qs;
    eb.n_tiles_q = P.tiles_q;
    eb.eflag = reinterpret_cast<uint64_t *>(ws + W.eflag);

    if (ctx) ctx->ev_ready[0] = false;
    mark(ctx, 0, 0, s);
    // value-range-relative mode: the range kernel also clears the scratch
    if (params->eb_mode != DQZ_EB_VALREL) launch_init(s, ctl, ws + W.hist, W.zero_end - W.hist, params->eb_mode, params->eb);
    mark(ctx, 0, 1, s);
    if (params->eb_mode == DQZ_EB_VALREL)
        launch_minmax(s, d_field, P.g.nelem, ctl, parts, params->eb, ncu, ws + W.hist, W.zero_end - W.hist);
    mark(ctx, 0, 2, s);
    launch_quantize(s, d_field, P.g, P.L, ctl, qb);
    mark(ctx, 0, 3, s);
    launch_quantize_scan(s, P.g, P.L, qb);
    mark(ctx, 0, 4, s);
    launch_codebook(s, P.g, P.L, ctl, qb.hist_sum, book, book32, arc, params->eb_mode, params->eb, qs, rb);
    mark(ctx, 0, 5, s);
    launch_encode(s, P.g, P.L, ctl, rb, eb, arc, ncu);
    mark(ctx, 0, 6, s);
    if (!ctx) return;
    ctx->last_valid = true;
    ctx->phases_valid = true;
    ctx->last_codes = codes;
    ctx->last_hist = hist;
    ctx->last_book = book;
    ctx->last_ctl = ctl;
    ctx->last_tab = reinterpret_cast<DecodeTables *>(ws + W.tab);
    ctx->last_padded = P.g.padded;
    ctx->last_nsym = P.L.nsym;
}

// Validate a decompression and plan it (host only); the workspace size check
// is the caller's.
dqz_status plan_decompress_args(const uint8_t *hb, uint64_t archive_bytes, float *d_field, uint64_t field_cap_elems,
                                HeaderInfo &hi, Plan &P, WsLayout &W, std::string &why) {
    dqz_status st = parse_header(hb, kHeaderBytes, hi, &P, why);
    if (st != DQZ_OK) return st;
    if (hi.archive_bytes != archive_bytes) { why = "archive length differs from its header"; return DQZ_ECORRUPT; }
    if (field_cap_elems < hi.nelem) { why = "field capacity too small"; return DQZ_ETOOSMALL; }
    if (hi.nelem && !d_field) { why = "null field"; return DQZ_EINVAL; }
    W = ws_layout(P, false);
    return DQZ_OK;
}

dqz_status plan_decompress(dqz_ctx *ctx, const void *d_archive, uint64_t archive_bytes, const uint8_t *hb,
                           float *d_field, uint64_t field_cap_elems, HeaderInfo &hi, Plan &P, WsLayout &W) {
    std::string why;
    (void)d_archive;
    const dqz_status st = plan_decompress_args(hb, archive_bytes, d_field, field_cap_elems, hi, P, W, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    ctx->last_need = hi.nelem ? W.total : 0;
    if (hi.nelem && ctx->ws_bytes < W.total)
        return fail(ctx, DQZ_ENOMEM, "workspace too small: this archive needs " + std::to_string(W.total) +
                                          " bytes (dqz_ctx_reserve)");
    return DQZ_OK;
}

void enqueue_decompress(dqz_ctx *ctx, uint8_t *ws, int ncu, const uint8_t *arc, float *d_field, const HeaderInfo &hi,
                        const Plan &P, const WsLayout &W, Readback *rb, hipStream_t s) {
    DecodeTables *tab = reinterpret_cast<DecodeTables *>(ws + W.tab);
    const bool trace = ctx && ctx->trace;
    if (ctx) {
        ctx->last_valid = false;   // the decompression scratch overlaps the compression's
        ctx->phases_valid = true;
        ctx->last_ctl = reinterpret_cast<Ctl *>(ws + W.ctl);
        ctx->last_tab = tab;
        ctx->ev_ready[1] = false;
    }
    mark(ctx, 1, 0, s);
    const bool two_pass = P.L.sub_size == 128;
    uint4 *qws = two_pass ? reinterpret_cast<uint4 *>(ws + W.qws) : nullptr;
    uint32_t *unit_exc = two_pass ? reinterpret_cast<uint32_t *>(ws + W.unit_exc) : nullptr;
    launch_decode_tables(s, P.L, arc, hi.max_len, tab, rb, (uint32_t)hi.n_exc, unit_exc, recon_units(P.g));
    mark(ctx, 1, 1, s);
    launch_decode(s, P.g, P.L, arc, hi.off_str, hi.n_words, (uint32_t)hi.n_exc, hi.h, tab, d_field, trace, qws, rb,
                  ncu);
    mark(ctx, 1, 2, s);
    if (two_pass) launch_recon(s, P.g, P.L, arc, (uint32_t)hi.n_exc, hi.h, tab, qws, unit_exc, d_field, rb);
    mark(ctx, 1, 3, s);
}

}  // namespace host

dqz_status compress_on_workspace(uint8_t *ws, uint64_t ws_bytes, int ncu, const float *d_field,
                                 const dqz_shape *shape, const dqz_params *params, void *d_archive,
                                 uint64_t archive_cap, Readback *d_result, hipStream_t stream, uint64_t *need) {
    Plan P;
    WsLayout W;
    std::string why;
    *need = 0;
    const dqz_status st = plan_compress_args(d_field, shape, params, d_archive, archive_cap, P, W, why);
    if (st != DQZ_OK) return st;
    *need = W.fixed;
    if (ws_bytes < W.fixed) return DQZ_EUNSUPPORTED;
    enqueue_compress(nullptr, ws, ws_bytes, ncu, d_field, params, reinterpret_cast<uint8_t *>(d_archive), P, W,
                     d_result, stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? DQZ_OK : DQZ_EHIP;
}

}  // namespace dqz

extern "C" {

const char *dqz_status_str(dqz_status s) {
    switch (s) {
        case DQZ_OK: return "ok";
        case DQZ_EINVAL: return "invalid argument";
        case DQZ_ETOOSMALL: return "buffer too small";
        case DQZ_ENOMEM: return "out of memory";
        case DQZ_ECORRUPT: return "corrupt archive";
        case DQZ_EUNSUPPORTED: return "unsupported";
        case DQZ_EHIP: return "HIP runtime error";
        case DQZ_EINTERNAL: return "internal device error";
        case DQZ_EAGAIN: return "not completed yet";
        default: return "unknown status";
    }
}

const char *dqz_ctx_last_error(const dqz_ctx *ctx) { return ctx ? ctx->last_error.c_str() : g_create_error.c_str(); }

dqz_status dqz_ctx_create(int device, uint64_t workspace_cap, dqz_ctx **out) {
    g_create_error.clear();
    if (!out) return create_fail(DQZ_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return create_fail(DQZ_EHIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    }
    if (device < 0 || device >= count) return create_fail(DQZ_EINVAL, "no such device");
    dqz_ctx *ctx = new (std::nothrow) dqz_ctx;
    if (!ctx) return create_fail(DQZ_ENOMEM, "host allocation failed");
    ctx->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete ctx;
        return create_fail(DQZ_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->ncu = ncu;
    if ((e = decode_kernel_attributes()) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return create_fail(DQZ_EHIP, std::string("decoding kernels' LDS attributes: ") + hipGetErrorString(e));
    }
    if ((e = hipHostMalloc((void **)&ctx->h_rb, 3 * sizeof(Readback), hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return create_fail(DQZ_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    if ((e = hipHostGetDevicePointer((void **)&ctx->d_rb, ctx->h_rb, 0)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(ctx->h_rb);
        delete ctx;
        return create_fail(DQZ_EHIP, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
    }
    if ((e = hipStreamCreateWithFlags(&ctx->copy_in, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&ctx->copy_out, hipStreamNonBlocking)) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->copy_in) (void)hipStreamDestroy(ctx->copy_in);
        (void)hipHostFree(ctx->h_rb);
        delete ctx;
        return create_fail(DQZ_EHIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
    }
    if (workspace_cap && alloc_workspace(ctx, workspace_cap) != DQZ_OK) {
        const std::string why = ctx->last_error;
        (void)hipStreamDestroy(ctx->copy_in);
        (void)hipStreamDestroy(ctx->copy_out);
        (void)hipHostFree(ctx->h_rb);
        delete ctx;
        return create_fail(DQZ_ENOMEM, why);
    }
    *out = ctx;
    return DQZ_OK;
}

void dqz_ctx_destroy(dqz_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (!ctx->lanes.empty() || ctx->capture) (void)hipDeviceSynchronize();
    for (int k = 0; k < 2; k++) {
        if (ctx->graphs[k].exec) (void)hipGraphExecDestroy(ctx->graphs[k].exec);
        if (ctx->graphs[k].graph) (void)hipGraphDestroy(ctx->graphs[k].graph);
    }
    for (auto &ln : ctx->lanes) {
        (void)hipEventDestroy(ln.done);
        (void)hipStreamDestroy(ln.stream);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->copy_in) (void)hipStreamSynchronize(ctx->copy_in);
    if (ctx->copy_out) (void)hipStreamSynchronize(ctx->copy_out);
    if (ctx->copy_in) (void)hipStreamDestroy(ctx->copy_in);
    if (ctx->copy_out) (void)hipStreamDestroy(ctx->copy_out);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->h_rb) (void)hipHostFree(ctx->h_rb);
    for (int k = 0; k < 2; k++)
        for (int i = 0; i <= DQZ_MAX_STAGES; i++)
            if (ctx->ev[k][i]) (void)hipEventDestroy(ctx->ev[k][i]);
    delete ctx;
}

dqz_status dqz_ctx_reserve(dqz_ctx *ctx, uint64_t workspace_bytes) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (workspace_bytes <= ctx->ws_bytes) return DQZ_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return alloc_workspace(ctx, workspace_bytes);
}

dqz_status dqz_ctx_workspace(const dqz_ctx *ctx, uint64_t *workspace_bytes, uint64_t *last_need) {
    if (!ctx) return DQZ_EINVAL;
    if (workspace_bytes) *workspace_bytes = ctx->ws_bytes;
    if (last_need) *last_need = ctx->last_need;
    return DQZ_OK;
}

dqz_status dqz_compress_bound(const dqz_shape *shape, const dqz_params *params, uint64_t *archive_max,
                              uint64_t *workspace_bytes) {
    if (!params) return DQZ_EINVAL;
    Plan P;
    std::string why;
    dqz_status st = make_geom(shape, P.g, why);
    if (st != DQZ_OK) return st;
    uint32_t radius, sub, csubs;
    fill_params(params, radius, sub, csubs);
    if ((st = make_layout(P.g, radius, sub, csubs, P.L, why)) != DQZ_OK) return st;
    if ((st = set_layers(params, P.L, why)) != DQZ_OK) return st;
    P.tiles_q = quantize_tiles(P.g);
    P.tiles_e = encode_tiles(P.g);
    // every element an outlier and a patch (16 bytes) and a 64-bit code
    if (archive_max) *archive_max = P.L.off_exc + 16ull * P.g.nelem + 8ull * P.g.nelem + 8;
    if (workspace_bytes) *workspace_bytes = ws_layout(P, true).total;
    return DQZ_OK;
}

dqz_status dqz_decompress_bound(const void *h_header, uint64_t header_bytes, uint64_t *workspace_bytes) {
    HeaderInfo hi;
    Plan P;
    std::string why;
    dqz_status st = parse_header(reinterpret_cast<const uint8_t *>(h_header), header_bytes, hi, &P, why);
    if (st != DQZ_OK) return st;
    if (workspace_bytes) *workspace_bytes = hi.nelem ? ws_layout(P, false).total : 0;
    return DQZ_OK;
}

dqz_status dqz_compress(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape, const dqz_params *params,
                        void *d_archive, uint64_t archive_cap, uint64_t *archive_bytes, void *h_header,
                        void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!archive_bytes) return fail(ctx, DQZ_EINVAL, "null argument");
    *archive_bytes = 0;
    Plan P;
    WsLayout W;
    dqz_status st = plan_compress(ctx, d_field, shape, params, d_archive, archive_cap, P, W);
    if (st != DQZ_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->h_rb->bits = kNoReadback;   // the codebook kernel overwrites it
    ctx->h_rb->code = 0;
    enqueue_compress(ctx, reinterpret_cast<uint8_t *>(ctx->ws), ctx->ws_bytes, ctx->ncu, d_field, params,
                     reinterpret_cast<uint8_t *>(d_archive), P, W, ctx->d_rb, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, wait_stream(s));
    ctx->ev_ready[0] = ctx->timing;
    const Readback &rb = *ctx->h_rb;
    if (rb.bits == kNoReadback) return fail(ctx, DQZ_EINTERNAL, "the codebook kernel did not report");
    st = (dqz_status)rb.code;
    if (st == DQZ_ETOOSMALL) *archive_bytes = rb.archive_bytes;
    if (st == DQZ_ENOMEM) ctx->last_need = rb.workspace_need;
    if (st != DQZ_OK) {
        std::string msg = status_message(st);
        if (st == DQZ_ENOMEM) msg += ": needs " + std::to_string(rb.workspace_need) + " bytes (dqz_ctx_reserve)";
        return fail(ctx, st, msg);
    }
    *archive_bytes = rb.archive_bytes;
    if (h_header) memcpy(h_header, rb.header, kHeaderBytes);
    return DQZ_OK;
}

dqz_status dqz_compress_async(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape, const dqz_params *params,
                              void *d_archive, uint64_t archive_cap, dqz_result *d_result, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!d_result || (reinterpret_cast<uintptr_t>(d_result) & 7u)) return fail(ctx, DQZ_EINVAL, "result must be 8-byte aligned");
    Plan P;
    WsLayout W;
    dqz_status st = plan_compress(ctx, d_field, shape, params, d_archive, archive_cap, P, W);
    if (st != DQZ_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    enqueue_compress(ctx, reinterpret_cast<uint8_t *>(ctx->ws), ctx->ws_bytes, ctx->ncu, d_field, params,
                     reinterpret_cast<uint8_t *>(d_archive), P, W, reinterpret_cast<Readback *>(d_result), s);
    HIP_TRY(ctx, hipGetLastError());
    ctx->ev_ready[0] = false;
    return DQZ_OK;
}

dqz_status dqz_archive_info(const void *h_header, uint64_t header_bytes, dqz_shape *shape, dqz_params *params,
                            uint64_t *field_elems, uint64_t *archive_bytes) {
    HeaderInfo hi;
    std::string why;
    dqz_status st = parse_header(reinterpret_cast<const uint8_t *>(h_header), header_bytes, hi, nullptr, why);
    if (st != DQZ_OK) return st;
    if (shape) *shape = hi.shape;
    if (params) *params = hi.params;
    if (field_elems) *field_elems = hi.nelem;
    if (archive_bytes) *archive_bytes = hi.archive_bytes;
    return DQZ_OK;
}

dqz_status dqz_decompress(dqz_ctx *ctx, const void *d_archive, uint64_t archive_bytes, const void *h_header,
                          float *d_field, uint64_t field_cap_elems, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!d_archive) return fail(ctx, DQZ_EINVAL, "null archive");
    if (archive_bytes < kHeaderBytes) return fail(ctx, DQZ_ECORRUPT, "archive shorter than its header");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t hb[kHeaderBytes];
    if (h_header) {
        memcpy(hb, h_header, kHeaderBytes);
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->h_rb->header, d_archive, kHeaderBytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        memcpy(hb, ctx->h_rb->header, kHeaderBytes);
    }
    HeaderInfo hi;
    Plan P;
    WsLayout W;
    dqz_status st = plan_decompress(ctx, d_archive, archive_bytes, hb, d_field, field_cap_elems, hi, P, W);
    if (st != DQZ_OK) return st;
    if (hi.nelem == 0) return DQZ_OK;
    ctx->h_rb->bits = 0;   // the decoding kernels set it on damage
    ctx->h_rb->code = 0;
    enqueue_decompress(ctx, reinterpret_cast<uint8_t *>(ctx->ws), ctx->ncu, reinterpret_cast<const uint8_t *>(d_archive),
                       d_field, hi, P, W, ctx->d_rb, s);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, wait_stream(s));
    ctx->ev_ready[1] = ctx->timing;
    st = (dqz_status)ctx->h_rb->code;
    return st == DQZ_OK ? DQZ_OK : fail(ctx, st, status_message(st));
}

dqz_status dqz_decompress_async(dqz_ctx *ctx, const void *d_archive, uint64_t archive_bytes, const void *h_header,
                                float *d_field, uint64_t field_cap_elems, dqz_result *d_result, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!d_archive || !h_header) return fail(ctx, DQZ_EINVAL, "null archive or header");
    if (!d_result || (reinterpret_cast<uintptr_t>(d_result) & 7u)) return fail(ctx, DQZ_EINVAL, "result must be 8-byte aligned");
    if (archive_bytes < kHeaderBytes) return fail(ctx, DQZ_ECORRUPT, "archive shorter than its header");
    HeaderInfo hi;
    Plan P;
    WsLayout W;
    dqz_status st = plan_decompress(ctx, d_archive, archive_bytes, reinterpret_cast<const uint8_t *>(h_header),
                                    d_field, field_cap_elems, hi, P, W);
    if (st != DQZ_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Readback *rb = reinterpret_cast<Readback *>(d_result);
    launch_publish(s, rb, 0u, hi.archive_bytes);   // the decoding kernels overwrite it on damage
    if (hi.nelem)
        enqueue_decompress(ctx, reinterpret_cast<uint8_t *>(ctx->ws), ctx->ncu, reinterpret_cast<const uint8_t *>(d_archive),
                           d_field, hi, P, W, rb, s);
    HIP_TRY(ctx, hipGetLastError());
    ctx->ev_ready[1] = false;
    return DQZ_OK;
}

dqz_status dqz_ctx_set_timing(dqz_ctx *ctx, int level) {
    if (!ctx) return DQZ_EINVAL;
    int only[2] = {-1, -1};
    if (level >= 0x100) {
        const int which = (level >> 4) & 0xF, stage = level & 0xF;
        if (level > 0x1FF || which > 1 || stage >= DQZ_MAX_STAGES)
            return fail(ctx, DQZ_EINVAL, "DQZ_TIMING_STAGE: which must be 0 or 1 and stage below DQZ_MAX_STAGES");
        only[which] = stage;
        only[1 - which] = -2;
    } else if (level < 0 || level > 2) {
        return fail(ctx, DQZ_EINVAL, "timing level must be 0, 1, 2 or DQZ_TIMING_STAGE(which, stage)");
    }
    const bool enable = level > 0;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (enable && !ctx->ev[0][0]) {
        for (int k = 0; k < 2; k++)
            for (int i = 0; i <= DQZ_MAX_STAGES; i++) HIP_TRY(ctx, hipEventCreate(&ctx->ev[k][i]));
    }
    ctx->timing = enable;
    ctx->trace = level == 2;
    ctx->only_stage[0] = only[0];
    ctx->only_stage[1] = only[1];
    ctx->ev_ready[0] = ctx->ev_ready[1] = false;
    return DQZ_OK;
}

dqz_status dqz_stage_times(dqz_ctx *ctx, int which, double *us, int *n_stages) {
    if (!ctx || !us || !n_stages || which < 0 || which > 1) return DQZ_EINVAL;
    *n_stages = 0;
    if (!ctx->ev_ready[which]) return fail(ctx, DQZ_EINVAL, "no timed call of this kind on this context");
    const int n = ctx->n_ev[which] - 1;
    for (int i = 0; i < n; i++) {
        float ms = 0.0f;
        if (ctx->ev_rec[which][i] && ctx->ev_rec[which][i + 1])
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev[which][i], ctx->ev[which][i + 1]));
        us[i] = 1000.0 * ms;
    }
    *n_stages = n;
    return DQZ_OK;
}

dqz_status dqz_debug_copy(dqz_ctx *ctx, int what, void *h_dst, uint64_t bytes) {
    if (!ctx || !h_dst) return DQZ_EINVAL;
    if (what == DQZ_DBG_PHASES && !ctx->phases_valid)
        return fail(ctx, DQZ_EINVAL, "no call on this context since its last reallocation or batched call");
    if (what != DQZ_DBG_PHASES && !ctx->last_valid)
        return fail(ctx, DQZ_EINVAL, "no compression on this context since its last decompression or reallocation");
    const void *src = nullptr;
    uint64_t need = 0;
    switch (what) {
        case DQZ_DBG_CODES: src = ctx->last_codes; need = 2 * ctx->last_padded; break;
        case DQZ_DBG_HISTOGRAM: {
            // the kernels keep kHistReplicas partial copies; return their sum
            need = 4ull * ctx->last_nsym;
            if (bytes != need) return fail(ctx, DQZ_EINVAL, "size mismatch");
            std::string buf(4ull * kHistReplicas * ctx->last_nsym, '\0');
            HIP_TRY(ctx, hipSetDevice(ctx->device));
            HIP_TRY(ctx, hipMemcpy(&buf[0], ctx->last_hist, buf.size(), hipMemcpyDeviceToHost));
            const uint32_t *parts = reinterpret_cast<const uint32_t *>(buf.data());
            uint32_t *dst = reinterpret_cast<uint32_t *>(h_dst);
            for (uint32_t i = 0; i < ctx->last_nsym; i++) {
                uint32_t v = 0;
                for (uint32_t r = 0; r < kHistReplicas; r++) v += parts[r * ctx->last_nsym + i];
                dst[i] = v;
            }
            return DQZ_OK;
        }
        case DQZ_DBG_CODEBOOK: src = ctx->last_book; need = 8ull * ctx->last_nsym; break;
        case DQZ_DBG_PHASES: {
            if (bytes != 8 * 32) return fail(ctx, DQZ_EINVAL, "size mismatch");
            HIP_TRY(ctx, hipSetDevice(ctx->device));
            uint64_t *dst = reinterpret_cast<uint64_t *>(h_dst);
            HIP_TRY(ctx, hipMemcpy(dst, ctx->last_ctl->phase, 8 * 16, hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(dst + 16, ctx->last_tab->phase, 8 * 16, hipMemcpyDeviceToHost));
            return DQZ_OK;
        }
        default: return fail(ctx, DQZ_EINVAL, "unknown stage");
    }
    if (bytes != need) return fail(ctx, DQZ_EINVAL, "size mismatch");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpy(h_dst, src, bytes, hipMemcpyDeviceToHost));
    return DQZ_OK;
}

dqz_status dqz_debug_inject(dqz_ctx *ctx, int what, int count) {
    if (!ctx || count < 0) return DQZ_EINVAL;
    if (what != DQZ_INJECT_ALLOC_FAIL) return fail(ctx, DQZ_EINVAL, "unknown injection");
    ctx->inject_alloc_fail = count;
    return DQZ_OK;
}

}  // extern "C"
