// dqz_stream.cpp -- the host path: fields in host memory, compressed slab by
// slab (so a field may exceed the device's memory, as the paper's host-side
// SZ does with its block-by-block processing, Sec. 4.1) into a container of
// ordinary archives, with the host<->device copies overlapped with the
// kernels; and its inverse.
//
// A slab is a run of the field's slowest axis whose extent is a multiple of
// the prediction block edge along that axis (32 in 1D, 16 in 2D, 8 in 3D),
// so every prediction block lies in one slab and the blocks, their Lorenzo
// deltas, outliers and patches are exactly those of the whole field; only
// the Huffman coding (a codebook per slab) differs.  In the value-range-
// relative mode a first pass streams every slab through the range kernels
// and folds the slabs' ranges on the device; every slab is then compressed
// with the resulting absolute bound, so the decompressed field is bit for bit
// the one a whole-field compression with that bound gives.
//
// Pipeline: three streams (host-to-device copies, kernels, device-to-host
// copies) and two buffers of each kind, so slab k's upload and slab k - 1's
// archive download run beside slab k's (or k - 1's) kernels.
//
// Container (little-endian): 128-byte header
//   0 magic 'DQZS', 4 version u16, 6 ndim u8, 7 eb mode u8 (as given),
//   8 dims u64[3] (slowest first, leading 1s for fewer dims), 32 slab extent
//   u64 (along the slowest axis of the field), 40 slab count u32, 44 radius
//   u32, 48 eb as given f64, 56 absolute bound f64, 64 min f32, 68 max f32
//   (value-range-relative mode), 72 elements u64, 80 container bytes u64,
//   88 subchunk size u32, 92 chunk subchunks u32;
// then (slabs + 1) u64 byte offsets of the slab archives (the last one is
// the container's end), then the archives, each starting 8-byte aligned.
#include "dqz_host.h"

#include <cfloat>
#include <cmath>
#include <cstring>

using namespace dqz;
using namespace dqz::host;

namespace {

constexpr uint32_t kStreamMagic = 0x535A5144u;   // 'D' 'Q' 'Z' 'S'
constexpr uint32_t kStreamVersion = 1;
constexpr uint64_t kStreamHeader = 128;

uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }
uint64_t align8(uint64_t v) { return (v + 7) / 8 * 8; }

struct StreamGeom {
    dqz_shape shape;          // the whole field
    uint64_t row_elems = 1;   // elements per index of the slowest axis
    uint64_t extent = 0;      // slab extent along the slowest axis
    uint32_t n_slabs = 0;
    uint64_t nelem = 0;
};

uint32_t block_edge(uint32_t ndim) { return ndim == 1 ? 32u : (ndim == 2 ? 16u : 8u); }

dqz_status stream_geom(const dqz_shape *shape, uint64_t slab_bytes, StreamGeom &sg, std::string &why) {
    Geom g;
    dqz_status st = make_geom(shape, g, why);
    if (st != DQZ_OK) return st;
    sg.shape = *shape;
    sg.nelem = g.nelem;
    sg.row_elems = 1;
    for (uint32_t a = 1; a < shape->ndim; a++) sg.row_elems *= shape->dims[a];
    const uint64_t n0 = shape->dims[0];
    const uint32_t e = block_edge(shape->ndim);
    uint64_t rows = sg.row_elems ? slab_bytes / (4 * sg.row_elems) : n0;
    rows = rows / e * e;
    if (rows < e) rows = e;
    if (rows > n0) rows = n0;
    sg.extent = rows;
    sg.n_slabs = n0 == 0 || sg.row_elems == 0 ? 0u : (uint32_t)((n0 + rows - 1) / rows);
    return DQZ_OK;
}

dqz_shape slab_shape(const StreamGeom &sg, uint32_t k) {
    dqz_shape s = sg.shape;
    const uint64_t n0 = sg.shape.dims[0];
    const uint64_t lo = (uint64_t)k * sg.extent;
    s.dims[0] = (lo + sg.extent <= n0) ? sg.extent : n0 - lo;
    return s;
}

// Device buffers of a streaming compression, carved from the workspace.
struct CompressBufs {
    uint64_t ws_bytes;        // compression workspace (first in the workspace)
    uint64_t acc;             // range fold
    uint64_t in[2], arc[2];
    uint64_t arc_cap;
    uint64_t total;
};

dqz_status compress_bufs(const StreamGeom &sg, const dqz_params *params, CompressBufs &b, std::string &why) {
    memset(&b, 0, sizeof(b));
    if (!sg.n_slabs) return DQZ_OK;
    const dqz_shape s0 = slab_shape(sg, 0);   // the largest slab
    Plan P;
    WsLayout W;
    static const float kDummy = 0.0f;
    dqz_params p = *params;
    p.eb_mode = DQZ_EB_ABS;
    p.eb = 1.0;   // the layout does not depend on the bound
    dqz_status st = plan_compress_args(&kDummy, &s0, &p, &kDummy, ~0ull, P, W, why);
    if (st != DQZ_OK) return st;
    uint64_t amax = 0;
    st = dqz_compress_bound(&s0, &p, &amax, nullptr);
    if (st != DQZ_OK) return st;
    const uint64_t field = 4ull * P.g.nelem;
    // the fixed layout and one exception record per element
    b.ws_bytes = align256(W.fixed + 8ull * P.g.nelem);
    uint64_t cur = b.ws_bytes;
    b.acc = cur;
    cur += 256;
    for (int i = 0; i < 2; i++) {
        b.in[i] = cur;
        cur += align256(field);
    }
    b.arc_cap = amax;
    for (int i = 0; i < 2; i++) {
        b.arc[i] = cur;
        cur += align256(amax);
    }
    b.total = cur;
    return DQZ_OK;
}

void put64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
void put32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
uint64_t get64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }
uint32_t get32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }

struct Events {
    hipEvent_t in[2] = {}, comp[2] = {}, out[2] = {};
    ~Events() {
        for (int i = 0; i < 2; i++) {
            if (in[i]) (void)hipEventDestroy(in[i]);
            if (comp[i]) (void)hipEventDestroy(comp[i]);
            if (out[i]) (void)hipEventDestroy(out[i]);
        }
    }
    hipError_t create() {
        for (int i = 0; i < 2; i++) {
            hipError_t e = hipEventCreateWithFlags(&in[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&comp[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&out[i], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

// Parsed container: geometry, parameters, slab archive offsets.
struct Container {
    StreamGeom sg;
    uint32_t eb_mode;
    double eb_param, eb_abs;
    const uint64_t *offsets;   // n_slabs + 1 (unaligned host pointer: read with memcpy)
};

dqz_status parse_container(const uint8_t *c, uint64_t bytes, Container &ct, std::string &why) {
    if (!c || bytes < kStreamHeader) { why = "container shorter than its header"; return DQZ_ECORRUPT; }
    if (get32(c) != kStreamMagic || (c[4] | (c[5] << 8)) != (int)kStreamVersion) { why = "bad magic or version"; return DQZ_ECORRUPT; }
    dqz_shape s;
    memset(&s, 0, sizeof(s));
    s.ndim = c[6];
    if (s.ndim < 1 || s.ndim > 3 || c[7] > 1) { why = "bad ndim or eb mode"; return DQZ_ECORRUPT; }
    for (uint32_t a = 0; a < 3 - s.ndim; a++)
        if (get64(c + 8 + 8 * a) != 1) { why = "bad dims"; return DQZ_ECORRUPT; }
    for (uint32_t i = 0; i < s.ndim; i++) s.dims[i] = get64(c + 8 + 8 * (3 - s.ndim + i));
    Geom g;
    dqz_status st = make_geom(&s, g, why);
    if (st != DQZ_OK) return DQZ_ECORRUPT;
    ct.sg.shape = s;
    ct.sg.nelem = g.nelem;
    ct.sg.row_elems = 1;
    for (uint32_t a = 1; a < s.ndim; a++) ct.sg.row_elems *= s.dims[a];
    ct.sg.extent = get64(c + 32);
    ct.sg.n_slabs = get32(c + 40);
    const uint32_t e = block_edge(s.ndim);
    const uint64_t n0 = s.dims[0];
    const bool empty = n0 == 0 || ct.sg.row_elems == 0;
    if (empty ? ct.sg.n_slabs != 0
              : (ct.sg.extent == 0 || (ct.sg.extent % e && ct.sg.extent != n0) || ct.sg.extent > n0 ||
                 ct.sg.n_slabs != (n0 + ct.sg.extent - 1) / ct.sg.extent)) {
        why = "bad slab geometry";
        return DQZ_ECORRUPT;
    }
    if (get64(c + 72) != g.nelem || get64(c + 80) != bytes) { why = "element count or size mismatch"; return DQZ_ECORRUPT; }
    ct.eb_mode = c[7];
    memcpy(&ct.eb_param, c + 48, 8);
    memcpy(&ct.eb_abs, c + 56, 8);
    const uint64_t idx_end = kStreamHeader + 8ull * (ct.sg.n_slabs + 1);
    if (idx_end > bytes) { why = "index past the end"; return DQZ_ECORRUPT; }
    ct.offsets = reinterpret_cast<const uint64_t *>(c + kStreamHeader);
    uint64_t prev = align8(idx_end);
    for (uint32_t k = 0; k <= ct.sg.n_slabs; k++) {
        const uint64_t o = get64(c + kStreamHeader + 8ull * k);
        if (o < prev || o > bytes || (k < ct.sg.n_slabs && (o & 7u))) { why = "bad slab offsets"; return DQZ_ECORRUPT; }
        prev = o;
    }
    if (get64(c + kStreamHeader + 8ull * ct.sg.n_slabs) != bytes) { why = "bad container end"; return DQZ_ECORRUPT; }
    return DQZ_OK;
}

uint64_t slab_off(const Container &ct, uint32_t k) {
    uint64_t v;
    memcpy(&v, reinterpret_cast<const uint8_t *>(ct.offsets) + 8ull * k, 8);
    return v;
}

// A slab archive's header checked against the container: its plan.
dqz_status slab_plan(const uint8_t *c, const Container &ct, uint32_t k, HeaderInfo &hi, Plan &P, WsLayout &W,
                     std::string &why) {
    const uint64_t lo = slab_off(ct, k), hi_off = slab_off(ct, k + 1);
    const uint64_t bytes = hi_off - lo;
    if (bytes < kHeaderBytes) { why = "slab archive too short"; return DQZ_ECORRUPT; }
    uint64_t abytes = get64(c + lo + 120);
    if (abytes > bytes || bytes - abytes >= 8) { why = "slab archive size mismatch"; return DQZ_ECORRUPT; }
    const dqz_shape want = slab_shape(ct.sg, k);
    static float kDummy;
    dqz_status st = plan_decompress_args(c + lo, abytes, &kDummy, ~0ull, hi, P, W, why);
    if (st != DQZ_OK) return DQZ_ECORRUPT;
    if (hi.shape.ndim != want.ndim) { why = "slab shape mismatch"; return DQZ_ECORRUPT; }
    for (uint32_t a = 0; a < want.ndim; a++)
        if (hi.shape.dims[a] != want.dims[a]) { why = "slab shape mismatch"; return DQZ_ECORRUPT; }
    return DQZ_OK;
}

}  // namespace

extern "C" {

dqz_status dqz_stream_workspace(const dqz_shape *shape, const dqz_params *params, uint64_t slab_bytes,
                                uint64_t *workspace_bytes, uint64_t *container_max) {
    if (!params) return DQZ_EINVAL;
    StreamGeom sg;
    std::string why;
    dqz_status st = stream_geom(shape, slab_bytes, sg, why);
    if (st != DQZ_OK) return st;
    CompressBufs b;
    st = compress_bufs(sg, params, b, why);
    if (st != DQZ_OK) return st;
    if (workspace_bytes) *workspace_bytes = b.total;
    if (container_max) {
        uint64_t tot = align8(kStreamHeader + 8ull * (sg.n_slabs + 1));
        for (uint32_t k = 0; k < sg.n_slabs; k++) {
            const dqz_shape s = slab_shape(sg, k);
            uint64_t amax = 0;
            dqz_params p = *params;
            p.eb_mode = DQZ_EB_ABS;
            p.eb = 1.0;
            if ((st = dqz_compress_bound(&s, &p, &amax, nullptr)) != DQZ_OK) return st;
            tot += align8(amax);
        }
        *container_max = tot;
    }
    return DQZ_OK;
}

dqz_status dqz_stream_compress(dqz_ctx *ctx, const float *h_field, const dqz_shape *shape, const dqz_params *params,
                               uint64_t slab_bytes, void *h_container, uint64_t container_cap,
                               uint64_t *container_bytes, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!params || !container_bytes || !h_container) return fail(ctx, DQZ_EINVAL, "null argument");
    *container_bytes = 0;
    if (!(params->eb > 0.0) || !std::isfinite(params->eb)) return fail(ctx, DQZ_EINVAL, "eb must be finite and > 0");
    if (params->eb_mode != DQZ_EB_ABS && params->eb_mode != DQZ_EB_VALREL) return fail(ctx, DQZ_EINVAL, "bad eb_mode");
    StreamGeom sg;
    std::string why;
    dqz_status st = stream_geom(shape, slab_bytes, sg, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    if (sg.nelem && !h_field) return fail(ctx, DQZ_EINVAL, "null field");
    uint32_t radius, sub, csubs;
    fill_params(params, radius, sub, csubs);
    CompressBufs B;
    if ((st = compress_bufs(sg, params, B, why)) != DQZ_OK) return fail(ctx, st, why);
    ctx->last_need = B.total;
    if (ctx->ws_bytes < B.total)
        return fail(ctx, DQZ_ENOMEM, "workspace too small for streaming: needs " + std::to_string(B.total) +
                                         " bytes (dqz_stream_workspace, dqz_ctx_reserve)");
    const uint64_t idx_end = align8(kStreamHeader + 8ull * (sg.n_slabs + 1));
    if (container_cap < idx_end) return fail(ctx, DQZ_ETOOSMALL, "container capacity below its index");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->last_valid = false;
    ctx->phases_valid = false;
    hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(ctx->ws);
    uint8_t *out = reinterpret_cast<uint8_t *>(h_container);
    const uint8_t *src = reinterpret_cast<const uint8_t *>(h_field);
    const uint64_t row_bytes = 4ull * sg.row_elems;
    Events ev;
    HIP_TRY(ctx, ev.create());

    // value-range-relative mode: the range of the whole field, slab by slab
    double eb_abs = params->eb;
    uint32_t keys[2] = {0xFFFFFFFFu, 0u};
    if (params->eb_mode == DQZ_EB_VALREL) {
        Plan P0;
        WsLayout W0;
        dqz_params p0 = *params;
        const dqz_shape s0 = slab_shape(sg, 0);
        if (sg.n_slabs) {
            static const float kDummy = 0.0f;
            st = plan_compress_args(&kDummy, &s0, &p0, &kDummy, ~0ull, P0, W0, why);
            if (st != DQZ_OK) return fail(ctx, st, why);
        }
        Ctl *ctl = reinterpret_cast<Ctl *>(ws + W0.ctl);
        uint32_t *acc = reinterpret_cast<uint32_t *>(ws + B.acc);
        for (uint32_t k = 0; k < sg.n_slabs; k++) {
            const uint32_t b = k & 1u;
            const dqz_shape s = slab_shape(sg, k);
            const uint64_t n = s.dims[0] * sg.row_elems;
            if (k >= 2) HIP_TRY(ctx, hipEventSynchronize(ev.comp[b]));   // the buffer's previous slab is read
            HIP_TRY(ctx, hipMemcpyAsync(ws + B.in[b], src + (uint64_t)k * sg.extent * row_bytes, 4ull * n,
                                        hipMemcpyHostToDevice, ctx->copy_in));
            HIP_TRY(ctx, hipEventRecord(ev.in[b], ctx->copy_in));
            HIP_TRY(ctx, hipStreamWaitEvent(cs, ev.in[b], 0));
            launch_minmax(cs, reinterpret_cast<const float *>(ws + B.in[b]), n, ctl,
                          reinterpret_cast<uint32_t *>(ws + W0.parts), p0.eb, ctx->ncu, ws + W0.hist,
                          W0.zero_end - W0.hist);
            launch_range_fold(cs, ctl, acc, k == 0);
            HIP_TRY(ctx, hipEventRecord(ev.comp[b], cs));
        }
        if (sg.n_slabs) {
            HIP_TRY(ctx, hipMemcpyAsync(ctx->h_rb[1].header, acc, 8, hipMemcpyDeviceToHost, cs));
            HIP_TRY(ctx, hipStreamSynchronize(cs));
            memcpy(keys, ctx->h_rb[1].header, 8);
        }
        // eb_abs = valrel (max - min) over the finite values; a range of 1
        // when there is none or max == min (the range kernels' rule)
        double range = 1.0;
        if (keys[0] != 0xFFFFFFFFu) {
            float fmin, fmax;
            const uint32_t bmin = key2f(keys[0]), bmax = key2f(keys[1]);
            memcpy(&fmin, &bmin, 4);
            memcpy(&fmax, &bmax, 4);
            const double d = (double)fmax - (double)fmin;
            if (d > 0.0) range = d;
        }
        eb_abs = params->eb * range;
    }
    {
        const double two_e = 2.0 * eb_abs;
        const float h = (float)two_e, r = (float)(1.0 / two_e);
        if (!std::isfinite(eb_abs) || eb_abs < (double)FLT_MIN || !std::isfinite(h) || !std::isfinite(r) ||
            !(r >= FLT_MIN))
            return fail(ctx, DQZ_EINVAL, "error bound out of range for this field");
    }

    // the slabs, with the absolute bound
    dqz_params ps = *params;
    ps.eb_mode = DQZ_EB_ABS;
    ps.eb = eb_abs;
    ps.radius = radius;
    ps.sub_size = sub;
    ps.chunk_subs = csubs;
    uint64_t off = idx_end;
    std::vector<uint64_t> offsets(sg.n_slabs + 1, 0);
    dqz_status result = DQZ_OK;
    auto finish = [&](uint32_t j) -> dqz_status {
        const uint32_t b = j & 1u;
        HIP_TRY(ctx, hipEventSynchronize(ev.comp[b]));
        const Readback &rb = ctx->h_rb[1 + b];
        if (rb.bits == 0xFFFFFFFFu) return fail(ctx, DQZ_EINTERNAL, "a slab's codebook kernel did not report");
        if (rb.code != DQZ_OK) {
            ctx->last_need = rb.code == DQZ_ENOMEM ? rb.workspace_need : ctx->last_need;
            return fail(ctx, rb.code, "slab " + std::to_string(j) + ": " + status_message(rb.code));
        }
        const uint64_t nb = rb.archive_bytes;
        if (off + nb > container_cap) {
            *container_bytes = 0;
            return fail(ctx, DQZ_ETOOSMALL, "container capacity exceeded");
        }
        offsets[j] = off;
        HIP_TRY(ctx, hipMemcpyAsync(out + off, ws + B.arc[b], nb, hipMemcpyDeviceToHost, ctx->copy_out));
        HIP_TRY(ctx, hipEventRecord(ev.out[b], ctx->copy_out));
        const uint64_t end = off + nb;
        off = align8(end);
        if (off > end && off <= container_cap) memset(out + end, 0, off - end);
        return DQZ_OK;
    };
    for (uint32_t k = 0; k < sg.n_slabs && result == DQZ_OK; k++) {
        const uint32_t b = k & 1u;
        const dqz_shape s = slab_shape(sg, k);
        const uint64_t n = s.dims[0] * sg.row_elems;
        Plan P;
        WsLayout W;
        st = plan_compress_args(reinterpret_cast<const float *>(ws + B.in[b]), &s, &ps, ws + B.arc[b], B.arc_cap, P,
                                W, why);
        if (st != DQZ_OK) { result = fail(ctx, st, why); break; }
        if (k >= 2) HIP_TRY(ctx, hipEventSynchronize(ev.out[b]));   // slab k - 2's archive has left arc[b]
        HIP_TRY(ctx, hipMemcpyAsync(ws + B.in[b], src + (uint64_t)k * sg.extent * row_bytes, 4ull * n,
                                    hipMemcpyHostToDevice, ctx->copy_in));
        HIP_TRY(ctx, hipEventRecord(ev.in[b], ctx->copy_in));
        HIP_TRY(ctx, hipStreamWaitEvent(cs, ev.in[b], 0));
        ctx->h_rb[1 + b].bits = 0xFFFFFFFFu;
        ctx->h_rb[1 + b].code = 0;
        enqueue_compress(nullptr, ws, B.ws_bytes, ctx->ncu, reinterpret_cast<const float *>(ws + B.in[b]), &ps,
                         ws + B.arc[b], P, W, ctx->d_rb + 1 + b, cs);
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipEventRecord(ev.comp[b], cs));
        if (k >= 1) result = finish(k - 1);
    }
    if (result == DQZ_OK && sg.n_slabs) result = finish(sg.n_slabs - 1);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->copy_out));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    if (result != DQZ_OK) return result;
    offsets[sg.n_slabs] = sg.n_slabs ? off : idx_end;
    if (sg.n_slabs) {
        // the container ends at the last archive's end (no trailing pad)
        const uint64_t last_end = offsets[sg.n_slabs - 1] + ctx->h_rb[1 + ((sg.n_slabs - 1) & 1u)].archive_bytes;
        offsets[sg.n_slabs] = last_end;
    }
    const uint64_t total = offsets[sg.n_slabs];
    uint8_t *h = out;
    memset(h, 0, kStreamHeader);
    put32(h, kStreamMagic);
    h[4] = (uint8_t)kStreamVersion;
    h[5] = 0;
    h[6] = (uint8_t)sg.shape.ndim;
    h[7] = (uint8_t)params->eb_mode;
    for (uint32_t a = 0; a < 3; a++) {
        const uint32_t first = 3 - sg.shape.ndim;
        put64(h + 8 + 8 * a, a < first ? 1ull : sg.shape.dims[a - first]);
    }
    put64(h + 32, sg.extent);
    put32(h + 40, sg.n_slabs);
    put32(h + 44, radius);
    memcpy(h + 48, &params->eb, 8);
    memcpy(h + 56, &eb_abs, 8);
    if (params->eb_mode == DQZ_EB_VALREL && keys[0] != 0xFFFFFFFFu) {
        put32(h + 64, key2f(keys[0]));
        put32(h + 68, key2f(keys[1]));
    }
    put64(h + 72, sg.nelem);
    put64(h + 80, total);
    put32(h + 88, sub);
    put32(h + 92, csubs);
    for (uint32_t k = 0; k <= sg.n_slabs; k++) put64(h + kStreamHeader + 8ull * k, offsets[k]);
    for (uint64_t i = kStreamHeader + 8ull * (sg.n_slabs + 1); i < idx_end; i++) h[i] = 0;
    *container_bytes = total;
    return DQZ_OK;
}

dqz_status dqz_stream_info(const void *h_container, uint64_t bytes, dqz_shape *shape, uint32_t *n_slabs,
                           double *eb_abs, uint64_t *workspace_bytes) {
    Container ct;
    std::string why;
    const uint8_t *c = reinterpret_cast<const uint8_t *>(h_container);
    dqz_status st = parse_container(c, bytes, ct, why);
    if (st != DQZ_OK) return st;
    if (shape) *shape = ct.sg.shape;
    if (n_slabs) *n_slabs = ct.sg.n_slabs;
    if (eb_abs) *eb_abs = ct.eb_abs;
    if (workspace_bytes) {
        uint64_t ws = 0, arc = 0, field = 0;
        for (uint32_t k = 0; k < ct.sg.n_slabs; k++) {
            HeaderInfo hi;
            Plan P;
            WsLayout W;
            if ((st = slab_plan(c, ct, k, hi, P, W, why)) != DQZ_OK) return st;
            ws = W.total > ws ? W.total : ws;
            arc = hi.archive_bytes > arc ? hi.archive_bytes : arc;
            field = 4 * hi.nelem > field ? 4 * hi.nelem : field;
        }
        *workspace_bytes = ct.sg.n_slabs ? align256(ws) + 2 * align256(arc) + 2 * align256(field) : 0;
    }
    return DQZ_OK;
}

dqz_status dqz_stream_decompress(dqz_ctx *ctx, const void *h_container, uint64_t bytes, float *h_field,
                                 uint64_t field_cap_elems, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    Container ct;
    std::string why;
    const uint8_t *c = reinterpret_cast<const uint8_t *>(h_container);
    dqz_status st = parse_container(c, bytes, ct, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    if (field_cap_elems < ct.sg.nelem) return fail(ctx, DQZ_ETOOSMALL, "field capacity too small");
    if (ct.sg.nelem && !h_field) return fail(ctx, DQZ_EINVAL, "null field");
    // plans of every slab (host only) and the buffers
    std::vector<HeaderInfo> H(ct.sg.n_slabs);
    std::vector<Plan> P(ct.sg.n_slabs);
    std::vector<WsLayout> W(ct.sg.n_slabs);
    uint64_t ws_need = 0, arc_max = 0, field_max = 0;
    for (uint32_t k = 0; k < ct.sg.n_slabs; k++) {
        if ((st = slab_plan(c, ct, k, H[k], P[k], W[k], why)) != DQZ_OK)
            return fail(ctx, st, "slab " + std::to_string(k) + ": " + why);
        ws_need = W[k].total > ws_need ? W[k].total : ws_need;
        arc_max = H[k].archive_bytes > arc_max ? H[k].archive_bytes : arc_max;
        field_max = 4 * H[k].nelem > field_max ? 4 * H[k].nelem : field_max;
    }
    const uint64_t o_arc0 = align256(ws_need), o_arc1 = o_arc0 + align256(arc_max);
    const uint64_t o_out0 = o_arc1 + align256(arc_max), o_out1 = o_out0 + align256(field_max);
    const uint64_t total = ct.sg.n_slabs ? o_out1 + align256(field_max) : 0;
    ctx->last_need = total;
    if (ctx->ws_bytes < total)
        return fail(ctx, DQZ_ENOMEM, "workspace too small for streaming: needs " + std::to_string(total) +
                                         " bytes (dqz_stream_info, dqz_ctx_reserve)");
    if (!ct.sg.n_slabs) return DQZ_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->last_valid = false;
    ctx->phases_valid = false;
    hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(ctx->ws);
    const uint64_t o_arc[2] = {o_arc0, o_arc1}, o_out[2] = {o_out0, o_out1};
    uint8_t *dst = reinterpret_cast<uint8_t *>(h_field);
    const uint64_t row_bytes = 4ull * ct.sg.row_elems;
    Events ev;
    HIP_TRY(ctx, ev.create());
    dqz_status result = DQZ_OK;
    auto check = [&](uint32_t j) {
        const Readback &rb = ctx->h_rb[1 + (j & 1u)];
        if (rb.code != DQZ_OK && result == DQZ_OK)
            result = fail(ctx, rb.code, "slab " + std::to_string(j) + ": " + status_message(rb.code));
    };
    for (uint32_t k = 0; k < ct.sg.n_slabs; k++) {
        const uint32_t b = k & 1u;
        if (k >= 2) {
            HIP_TRY(ctx, hipEventSynchronize(ev.out[b]));   // slab k - 2 has left both buffers
            check(k - 2);
        }
        HIP_TRY(ctx, hipMemcpyAsync(ws + o_arc[b], c + slab_off(ct, k), H[k].archive_bytes, hipMemcpyHostToDevice,
                                    ctx->copy_in));
        HIP_TRY(ctx, hipEventRecord(ev.in[b], ctx->copy_in));
        HIP_TRY(ctx, hipStreamWaitEvent(cs, ev.in[b], 0));
        ctx->h_rb[1 + b].bits = 0;
        ctx->h_rb[1 + b].code = 0;
        if (H[k].nelem)
            enqueue_decompress(nullptr, ws, ctx->ncu, ws + o_arc[b], reinterpret_cast<float *>(ws + o_out[b]), H[k],
                               P[k], W[k], ctx->d_rb + 1 + b, cs);
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipEventRecord(ev.comp[b], cs));
        HIP_TRY(ctx, hipStreamWaitEvent(ctx->copy_out, ev.comp[b], 0));
        HIP_TRY(ctx, hipMemcpyAsync(dst + (uint64_t)k * ct.sg.extent * row_bytes, ws + o_out[b], 4 * H[k].nelem,
                                    hipMemcpyDeviceToHost, ctx->copy_out));
        HIP_TRY(ctx, hipEventRecord(ev.out[b], ctx->copy_out));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->copy_out));
    HIP_TRY(ctx, hipStreamSynchronize(cs));
    for (uint32_t j = ct.sg.n_slabs >= 2 ? ct.sg.n_slabs - 2 : 0; j < ct.sg.n_slabs; j++) check(j);
    return result;
}

}  // extern "C"
