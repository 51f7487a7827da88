// dqz_batch.cpp -- many fields in one call, and the parameter autotuner.
//
// Batching.  The fields of a batch are spread over the context's concurrent
// lanes (HIP streams of default priority, joined back to the caller's stream
// by events), longest first onto the least loaded lane, so that one field's
// latency-bound stages (tile scans, codebook, decoding tables) run while
// other fields' bandwidth-bound passes keep the HBM busy.  Each lane works in
// its own slice of the context's workspace.  In graph mode the whole batch
// (fork, every field's kernels, join) is captured once into a HIP graph and
// replayed with one launch while the same batch repeats.  Every field's
// archive is the one dqz_compress writes for it alone: lanes change when a
// field runs, never what it computes.
//
// Autotuning.  The subchunk and chunk sizes (Sec. 3.2.4 deflates and
// Sec. 3.3 inflates in chunks whose size the paper tunes per dataset) do not
// change the bit stream, only the decoding tables in the archive and how the
// decoder parallelizes.  The tuner compresses and decompresses the caller's
// field with each candidate, times the decompression with HIP events, and
// keeps the smallest archive among the candidates that decompress within a
// tolerance of the fastest; the choice is cached per shape class.
#include "dqz_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

using namespace dqz;
using namespace dqz::host;

namespace {

// Longest-processing-time assignment of fields (work = padded positions) to
// `lanes` lanes: lane_of[i] for field i.
std::vector<uint32_t> assign_lanes(const std::vector<uint64_t> &work, uint32_t lanes) {
    std::vector<uint32_t> order(work.size());
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return work[a] > work[b]; });
    std::vector<uint64_t> load(lanes, 0);
    std::vector<uint32_t> lane_of(work.size(), 0);
    for (uint32_t i : order) {
        const uint32_t k = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_of[i] = k;
        load[k] += work[i] + 1;
    }
    return lane_of;
}

struct BatchPlan {
    std::vector<Plan> P;
    std::vector<WsLayout> W;
    std::vector<HeaderInfo> H;        // decompression only
    std::vector<uint32_t> lane_of;
    std::vector<uint64_t> base, size; // per lane: workspace slice
    uint64_t need = 0;                // sum of the lanes' fixed parts
};

// Slices of the workspace: lane k gets the largest fixed layout among its
// fields plus an equal share of what is left (its exception overflow pool).
dqz_status slice_workspace(BatchPlan &B, uint32_t lanes, uint64_t ws_bytes, bool compress) {
    std::vector<uint64_t> fixed(lanes, 0);
    for (size_t i = 0; i < B.P.size(); i++) {
        const uint64_t f = compress ? B.W[i].fixed : B.W[i].total;
        fixed[B.lane_of[i]] = std::max(fixed[B.lane_of[i]], f);
    }
    B.need = 0;
    for (uint64_t f : fixed) B.need += (f + 255) / 256 * 256;
    if (B.need > ws_bytes) return DQZ_ENOMEM;
    const uint64_t extra = (ws_bytes - B.need) / lanes / 256 * 256;
    B.base.assign(lanes, 0);
    B.size.assign(lanes, 0);
    uint64_t cur = 0;
    for (uint32_t k = 0; k < lanes; k++) {
        B.base[k] = cur;
        B.size[k] = (fixed[k] + 255) / 256 * 256 + extra;
        cur += B.size[k];
    }
    return DQZ_OK;
}

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

// Enqueue `body(lane, stream)` for every used lane between a fork from and a
// join into `s`.
template <typename F>
dqz_status fork_join(dqz_ctx *ctx, hipStream_t s, uint32_t used_lanes, F body) {
    if (used_lanes <= 1) {
        body(0u, s);
        return DQZ_OK;
    }
    HIP_TRY(ctx, hipEventRecord(ctx->fork, s));
    for (uint32_t k = 0; k < used_lanes; k++) {
        Lane &ln = ctx->lanes[k];
        HIP_TRY(ctx, hipStreamWaitEvent(ln.stream, ctx->fork, 0));
        body(k, ln.stream);
        HIP_TRY(ctx, hipEventRecord(ln.done, ln.stream));
        HIP_TRY(ctx, hipStreamWaitEvent(s, ln.done, 0));
    }
    return DQZ_OK;
}

void drop_graph(BatchGraph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.key.clear();
}

// Run `enqueue(stream)` on `s`, directly or through the context's cached
// graph for this key (captured on the first call with the key).
template <typename F>
dqz_status run_batch(dqz_ctx *ctx, int which, std::vector<uint64_t> &&key, hipStream_t s, F enqueue) {
    if (!ctx->use_graph) return enqueue(s);
    BatchGraph &g = ctx->graphs[which];
    if (g.exec && g.key == key) {
        HIP_TRY(ctx, hipGraphLaunch(g.exec, s));
        return DQZ_OK;
    }
    drop_graph(g);
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    const dqz_status st = enqueue(ctx->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
    if (st != DQZ_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
    g.graph = graph;
    HIP_TRY(ctx, hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    g.key = std::move(key);
    HIP_TRY(ctx, hipGraphLaunch(g.exec, s));
    return DQZ_OK;
}

uint64_t shape_class(const Geom &g, const dqz_params *p) {
    uint64_t k = g.ndim;
    k = k * 64 + (uint64_t)(64 - __builtin_clzll(g.nelem | 1));   // size octave
    k = k * 4 + (uint64_t)p->eb_mode;
    k = k * 64 + (uint64_t)(int)(std::floor(std::log10(p->eb)) + 32);   // eb decade
    k = k * 4096 + p->radius;
    return k;
}

}  // namespace

extern "C" {

dqz_status dqz_ctx_set_lanes(dqz_ctx *ctx, uint32_t lanes, uint32_t flags) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (lanes < 1 || lanes > DQZ_MAX_LANES) return fail(ctx, DQZ_EINVAL, "lanes must be in [1, DQZ_MAX_LANES]");
    if (flags & ~(uint32_t)DQZ_LANES_GRAPH) return fail(ctx, DQZ_EINVAL, "unknown lane flags");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());   // no batch of this context may be running
    for (int k = 0; k < 2; k++) drop_graph(ctx->graphs[k]);
    while (ctx->lanes.size() > lanes) {
        Lane &ln = ctx->lanes.back();
        (void)hipEventDestroy(ln.done);
        (void)hipStreamDestroy(ln.stream);
        ctx->lanes.pop_back();
    }
    while (ctx->lanes.size() < lanes) {
        Lane ln;
        HIP_TRY(ctx, hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
        const hipError_t e = hipEventCreateWithFlags(&ln.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(ln.stream);
            return hip_fail(ctx, e, "hipEventCreateWithFlags");
        }
        ctx->lanes.push_back(ln);
    }
    if (!ctx->fork) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    if (!ctx->capture) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    ctx->use_graph = (flags & DQZ_LANES_GRAPH) != 0;
    return DQZ_OK;
}

dqz_status dqz_batch_workspace(uint32_t n, const dqz_shape *shapes, const dqz_params *params, uint32_t lanes,
                               uint64_t *workspace_bytes) {
    if (!workspace_bytes || (n && (!shapes || !params)) || lanes < 1 || lanes > DQZ_MAX_LANES) return DQZ_EINVAL;
    BatchPlan B;
    B.P.resize(n);
    B.W.resize(n);
    std::vector<uint64_t> work(n);
    for (uint32_t i = 0; i < n; i++) {
        std::string why;
        static const float kDummy = 0.0f;
        const dqz_status st = plan_compress_args(&kDummy, &shapes[i], &params[i], &kDummy, ~0ull, B.P[i], B.W[i], why);
        if (st != DQZ_OK) return st;
        work[i] = B.P[i].g.padded;
    }
    B.lane_of = assign_lanes(work, lanes);
    (void)slice_workspace(B, lanes, ~0ull, true);
    *workspace_bytes = B.need;
    return DQZ_OK;
}

dqz_status dqz_compress_batch(dqz_ctx *ctx, uint32_t n, const float *const *d_fields, const dqz_shape *shapes,
                              const dqz_params *params, void *const *d_archives, const uint64_t *archive_caps,
                              dqz_result *d_results, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (n == 0) return DQZ_OK;
    if (!d_fields || !shapes || !params || !d_archives || !archive_caps || !d_results)
        return fail(ctx, DQZ_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(d_results) & 7u) return fail(ctx, DQZ_EINVAL, "results must be 8-byte aligned");
    const uint32_t lanes = ctx->lanes.empty() ? 1u : (uint32_t)ctx->lanes.size();
    BatchPlan B;
    B.P.resize(n);
    B.W.resize(n);
    std::vector<uint64_t> work(n);
    std::vector<uint64_t> key = {0, n, lanes};
    for (uint32_t i = 0; i < n; i++) {
        std::string why;
        const dqz_status st = plan_compress_args(d_fields[i], &shapes[i], &params[i], d_archives[i], archive_caps[i],
                                                 B.P[i], B.W[i], why);
        if (st != DQZ_OK) return fail(ctx, st, "field " + std::to_string(i) + ": " + why);
        work[i] = B.P[i].g.padded;
        uint64_t h = mix(0, reinterpret_cast<uintptr_t>(d_fields[i]));
        h = mix(h, reinterpret_cast<uintptr_t>(d_archives[i]));
        h = mix(h, archive_caps[i]);
        key.push_back(h);
        uint64_t sb[4];
        memcpy(sb, &shapes[i], sizeof(sb));
        key.insert(key.end(), sb, sb + 4);
        uint64_t pb[4];
        static_assert(sizeof(dqz_params) == sizeof(pb), "params layout");
        memcpy(pb, &params[i], sizeof(pb));
        key.insert(key.end(), pb, pb + 4);
    }
    key.push_back(reinterpret_cast<uintptr_t>(d_results));
    B.lane_of = assign_lanes(work, lanes);
    if (slice_workspace(B, lanes, ctx->ws_bytes, true) != DQZ_OK) {
        ctx->last_need = B.need;
        return fail(ctx, DQZ_ENOMEM, "workspace too small for this batch: needs " + std::to_string(B.need) +
                                         " bytes (dqz_batch_workspace, dqz_ctx_reserve)");
    }
    ctx->last_need = B.need;
    key.push_back(reinterpret_cast<uintptr_t>(ctx->ws));
    key.push_back(ctx->ws_bytes);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->last_valid = false;
    ctx->phases_valid = false;
    ctx->ev_ready[0] = false;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(ctx->ws);
    Readback *rb = reinterpret_cast<Readback *>(d_results);
    const uint32_t used = std::min<uint32_t>(lanes, n);
    dqz_status st = run_batch(ctx, 0, std::move(key), s, [&](hipStream_t top) -> dqz_status {
        return fork_join(ctx, top, used, [&](uint32_t k, hipStream_t ls) {
            for (uint32_t i = 0; i < n; i++) {
                if (B.lane_of[i] != k) continue;
                enqueue_compress(nullptr, ws + B.base[k], B.size[k], ctx->ncu, d_fields[i], &params[i],
                                 reinterpret_cast<uint8_t *>(d_archives[i]), B.P[i], B.W[i], rb + i, ls);
            }
        });
    });
    if (st != DQZ_OK) return st;
    HIP_TRY(ctx, hipGetLastError());
    return DQZ_OK;
}

dqz_status dqz_decompress_batch(dqz_ctx *ctx, uint32_t n, const void *const *d_archives,
                                const uint64_t *archive_bytes, const void *h_headers, float *const *d_fields,
                                const uint64_t *field_caps, dqz_result *d_results, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (n == 0) return DQZ_OK;
    if (!d_archives || !archive_bytes || !h_headers || !d_fields || !field_caps || !d_results)
        return fail(ctx, DQZ_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(d_results) & 7u) return fail(ctx, DQZ_EINVAL, "results must be 8-byte aligned");
    const uint32_t lanes = ctx->lanes.empty() ? 1u : (uint32_t)ctx->lanes.size();
    const uint8_t *hb = reinterpret_cast<const uint8_t *>(h_headers);
    BatchPlan B;
    B.P.resize(n);
    B.W.resize(n);
    B.H.resize(n);
    std::vector<uint64_t> work(n);
    std::vector<uint64_t> key = {1, n, lanes};
    for (uint32_t i = 0; i < n; i++) {
        std::string why;
        if (!d_archives[i]) return fail(ctx, DQZ_EINVAL, "field " + std::to_string(i) + ": null archive");
        const dqz_status st = plan_decompress_args(hb + (uint64_t)kHeaderBytes * i, archive_bytes[i], d_fields[i],
                                                   field_caps[i], B.H[i], B.P[i], B.W[i], why);
        if (st != DQZ_OK) return fail(ctx, st, "archive " + std::to_string(i) + ": " + why);
        work[i] = B.P[i].g.padded;
        uint64_t h = mix(0, reinterpret_cast<uintptr_t>(d_archives[i]));
        h = mix(h, reinterpret_cast<uintptr_t>(d_fields[i]));
        h = mix(h, archive_bytes[i]);
        h = mix(h, field_caps[i]);
        key.push_back(h);
        uint64_t words[kHeaderBytes / 8];
        memcpy(words, hb + (uint64_t)kHeaderBytes * i, kHeaderBytes);
        key.insert(key.end(), words, words + kHeaderBytes / 8);
    }
    key.push_back(reinterpret_cast<uintptr_t>(d_results));
    B.lane_of = assign_lanes(work, lanes);
    if (slice_workspace(B, lanes, ctx->ws_bytes, false) != DQZ_OK) {
        ctx->last_need = B.need;
        return fail(ctx, DQZ_ENOMEM, "workspace too small for this batch: needs " + std::to_string(B.need) +
                                         " bytes (dqz_ctx_reserve)");
    }
    ctx->last_need = B.need;
    key.push_back(reinterpret_cast<uintptr_t>(ctx->ws));
    key.push_back(ctx->ws_bytes);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->last_valid = false;
    ctx->phases_valid = false;
    ctx->ev_ready[1] = false;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(ctx->ws);
    Readback *rb = reinterpret_cast<Readback *>(d_results);
    const uint32_t used = std::min<uint32_t>(lanes, n);
    dqz_status st = run_batch(ctx, 1, std::move(key), s, [&](hipStream_t top) -> dqz_status {
        return fork_join(ctx, top, used, [&](uint32_t k, hipStream_t ls) {
            for (uint32_t i = 0; i < n; i++) {
                if (B.lane_of[i] != k) continue;
                // status OK unless a decoding kernel reports damage
                launch_publish(ls, rb + i, 0u, B.H[i].archive_bytes);
                if (B.H[i].nelem)
                    enqueue_decompress(nullptr, ws + B.base[k], ctx->ncu,
                                       reinterpret_cast<const uint8_t *>(d_archives[i]), d_fields[i], B.H[i], B.P[i],
                                       B.W[i], rb + i, ls);
            }
        });
    });
    if (st != DQZ_OK) return st;
    HIP_TRY(ctx, hipGetLastError());
    return DQZ_OK;
}

dqz_status dqz_tune(dqz_ctx *ctx, const float *d_field, const dqz_shape *shape, const dqz_params *base,
                    double tolerance, uint32_t flags, dqz_params *out, void *stream) {
    if (!ctx) return DQZ_EINVAL;
    ctx->last_error.clear();
    if (!base || !out || !(tolerance >= 0.0) || (flags & ~(uint32_t)DQZ_TUNE_FORCE))
        return fail(ctx, DQZ_EINVAL, "bad argument");
    Geom g;
    std::string why;
    dqz_status st = make_geom(shape, g, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    dqz_params bp = *base;
    uint32_t radius, sub, csubs;
    fill_params(&bp, radius, sub, csubs);
    bp.radius = radius;
    const uint64_t cls = shape_class(g, &bp);
    if (!(flags & DQZ_TUNE_FORCE))
        for (const auto &e : ctx->tuned)
            if (e.first == cls) {
                *out = e.second;
                out->eb = base->eb;
                out->eb_mode = base->eb_mode;
                return DQZ_OK;
            }
    if (!g.nelem) {
        *out = bp;
        return DQZ_OK;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // candidates: subchunk sizes (table bytes against decoding parallelism)
    // and chunk sizes (offsets table against per-wave prefix work)
    static const uint32_t kSubs[] = {128, 256, 512};
    static const uint32_t kChunks[] = {16, 64, 256};
    struct Cand { uint32_t sub, csubs; uint64_t bytes; double us; };
    std::vector<Cand> cands;
    uint64_t amax = 0, wsb = 0;
    dqz_params p = bp;
    p.sub_size = 128;
    p.chunk_subs = 64;
    st = dqz_compress_bound(shape, &p, &amax, &wsb);
    if (st != DQZ_OK) return fail(ctx, st, "bound");
    // archive and field buffers for the trials come from the workspace's end:
    // the trial's own compression workspace is what precedes them
    const uint64_t field_bytes = (4 * g.nelem + 255) / 256 * 256, arc_bytes = (amax + 255) / 256 * 256;
    Plan P0;
    WsLayout W0;
    st = plan_compress_args(d_field, shape, &p, d_field, amax, P0, W0, why);
    if (st != DQZ_OK) return fail(ctx, st, why);
    const uint64_t need = W0.fixed + arc_bytes + field_bytes + (64ull << 20);
    ctx->last_need = need;
    if (ctx->ws_bytes < need)
        return fail(ctx, DQZ_ENOMEM, "workspace too small for tuning: needs " + std::to_string(need) + " bytes");
    uint8_t *ws = reinterpret_cast<uint8_t *>(ctx->ws);
    const uint64_t trial_ws = ctx->ws_bytes - arc_bytes - field_bytes;
    uint8_t *arc = ws + trial_ws;
    float *fout = reinterpret_cast<float *>(ws + trial_ws + arc_bytes);
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    dqz_status result = DQZ_OK;
    for (uint32_t sb : kSubs) {
        for (uint32_t cs : kChunks) {
            p.sub_size = sb;
            p.chunk_subs = cs;
            Plan P;
            WsLayout W;
            st = plan_compress_args(d_field, shape, &p, arc, amax, P, W, why);
            if (st != DQZ_OK) { result = fail(ctx, st, why); break; }
            ctx->h_rb->bits = 0xFFFFFFFFu;
            enqueue_compress(nullptr, ws, trial_ws, ctx->ncu, d_field, &p, arc, P, W, ctx->d_rb, s);
            hipError_t e = wait_stream(s);
            if (e != hipSuccess) { result = hip_fail(ctx, e, "tuning compression"); break; }
            if (ctx->h_rb->code != DQZ_OK) { result = fail(ctx, ctx->h_rb->code, "tuning compression failed"); break; }
            const uint64_t bytes = ctx->h_rb->archive_bytes;
            uint8_t hdr[kHeaderBytes];
            memcpy(hdr, ctx->h_rb->header, kHeaderBytes);
            HeaderInfo hi;
            Plan PD;
            WsLayout WD;
            st = plan_decompress_args(hdr, bytes, fout, g.nelem, hi, PD, WD, why);
            if (st != DQZ_OK || WD.total > trial_ws) { result = fail(ctx, DQZ_EINTERNAL, "tuning plan"); break; }
            float best = 1e30f;
            for (int rep = 0; rep < 3; rep++) {
                ctx->h_rb->bits = 0;
                ctx->h_rb->code = 0;
                (void)hipEventRecord(e0, s);
                enqueue_decompress(nullptr, ws, ctx->ncu, arc, fout, hi, PD, WD, ctx->d_rb, s);
                (void)hipEventRecord(e1, s);
                e = wait_stream(s);
                if (e != hipSuccess) break;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                best = std::min(best, ms);
            }
            if (e != hipSuccess) { result = hip_fail(ctx, e, "tuning decompression"); break; }
            if (ctx->h_rb->code != DQZ_OK) { result = fail(ctx, ctx->h_rb->code, "tuning decompression failed"); break; }
            cands.push_back({sb, cs, bytes, 1000.0 * best});
        }
        if (result != DQZ_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->last_valid = false;
    ctx->phases_valid = false;
    if (result != DQZ_OK) return result;
    double fastest = 1e300;
    for (const Cand &c : cands) fastest = std::min(fastest, c.us);
    const Cand *pick = nullptr;
    for (const Cand &c : cands)
        if (c.us <= fastest * (1.0 + tolerance) && (!pick || c.bytes < pick->bytes)) pick = &c;
    dqz_params r = bp;
    r.sub_size = pick->sub;
    r.chunk_subs = pick->csubs;
    bool found = false;
    for (auto &e : ctx->tuned)
        if (e.first == cls) { e.second = r; found = true; }
    if (!found) ctx->tuned.emplace_back(cls, r);
    *out = r;
    return DQZ_OK;
}

}  // extern "C"
