// dqz_host.h -- host-side pieces of the C ABI shared by its translation
// units: the context, the plan of one call (geometry, archive layout,
// workspace layout) and the stream-ordered launch sequences.
#pragma once

#include "../../include/dqz.h"
#include "dqz_internal.h"

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

namespace dqz {
namespace host {

struct Plan {
    Geom g;
    Layout L;
    uint32_t tiles_q = 0, tiles_e = 0;
};

// Workspace layout.  Compression: control block, decoding tables, the zeroed
// region (histogram replicas and their sum, encoder look-back states), the
// codebooks, range partials, the quantize tiles' scan arrays and overflow
// bases, the per-tile exception slots, the code array, then (from
// `fixed`) the exception overflow pool, which takes the rest of the
// workspace.  Decompression: control block, tables, the decoded code array
// and the per-unit exception index (over the compression buffers).
struct WsLayout {
    uint64_t ctl, tab, hist, zero_end;
    uint64_t hist_sum, book, book32, parts;
    uint64_t qval[2], qexcl[2], qseg_total[2];
    uint64_t ovf_base, eflag;
    uint64_t stage, codes, fixed, qws, unit_exc, total;
    uint32_t n_segs_q;
};

// What a parsed and validated 128-byte header says.
struct HeaderInfo {
    dqz_shape shape;
    dqz_params params;
    uint64_t nelem, n_exc, total_bits, archive_bytes, off_str, n_words;
    uint32_t max_len;
    float h;
};

// One concurrent lane of a context: its own HIP stream (default priority)
// and the event that joins it back to the caller's stream.
struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

// A captured batch, replayed while the same call repeats.
struct BatchGraph {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace host
}  // namespace dqz

struct dqz_ctx {
    int device = 0;
    int ncu = 256;
    void *ws = nullptr;        // device workspace
    uint64_t ws_bytes = 0;
    uint64_t last_need = 0;    // workspace the most recent call needed
    // readback blocks in pinned host memory, written by the kernels: [0] for
    // the single calls, [1], [2] for the two slabs in flight of a streaming call
    dqz::Readback *h_rb = nullptr;
    dqz::Readback *d_rb = nullptr;  // the same blocks' device address
    hipStream_t copy_in = nullptr, copy_out = nullptr;   // streaming calls' copy streams
    int inject_alloc_fail = 0; // test hook: workspace allocations that fail on purpose
    std::string last_error;
    // most recent compression, for the stage dumps (cleared by a decompression,
    // whose scratch overlaps these buffers, and by a workspace reallocation)
    bool last_valid = false;
    uint16_t *last_codes = nullptr;
    uint32_t *last_hist = nullptr;
    uint64_t *last_book = nullptr;
    uint64_t last_padded = 0;
    uint32_t last_nsym = 0;
    dqz::Ctl *last_ctl = nullptr;
    dqz::DecodeTables *last_tab = nullptr;
    // the phase marks of the most recent single call on ws (either kind) are readable
    bool phases_valid = false;
    // per-stage timing (events between kernels) and, at level 2, the decoding
    // kernel's per-wave phase sums
    bool timing = false;
    bool trace = false;
    hipEvent_t ev[2][DQZ_MAX_STAGES + 1] = {};
    int n_ev[2] = {0, 0};
    bool ev_rec[2][DQZ_MAX_STAGES + 1] = {};
    int only_stage[2] = {-1, -1};   // >= 0: events only around this stage (-2: none)
    bool ev_ready[2] = {false, false};
    // concurrent lanes for batched calls, the fork event, the capture stream
    // and the cached batch graphs (compress, decompress)
    std::vector<dqz::host::Lane> lanes;
    hipEvent_t fork = nullptr;
    hipStream_t capture = nullptr;
    bool use_graph = false;
    dqz::host::BatchGraph graphs[2];
    // tuned parameters per shape class
    std::vector<std::pair<uint64_t, dqz_params>> tuned;
};

namespace dqz {
namespace host {

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

dqz_status fail(dqz_ctx *ctx, dqz_status st, const std::string &msg);
dqz_status hip_fail(dqz_ctx *ctx, hipError_t e, const char *what);
dqz_status make_geom(const dqz_shape *s, Geom &g, std::string &why);
dqz_status make_layout(const Geom &g, uint32_t radius, uint32_t sub, uint32_t csubs, Layout &L, std::string &why);
void fill_params(const dqz_params *p, uint32_t &radius, uint32_t &sub, uint32_t &csubs);
// Lorenzo layers from the parameters into the layout (DQZ_EINVAL unless 0, 1, 2)
dqz_status set_layers(const dqz_params *p, Layout &L, std::string &why);
hipError_t wait_stream(hipStream_t s);
WsLayout ws_layout(const Plan &P, bool compress);
const char *status_message(dqz_status st);
dqz_status parse_header(const uint8_t *hb, uint64_t n, HeaderInfo &hi, Plan *P, std::string &why);
dqz_status plan_compress_args(const float *d_field, const dqz_shape *shape, const dqz_params *params,
                              const void *d_archive, uint64_t archive_cap, Plan &P, WsLayout &W, std::string &why);
// The workspace is [ws, ws + ws_bytes) on the stream's device (ws_bytes >=
// W.fixed); `ctx` (may be NULL) takes the timing marks and the stage-dump
// pointers.
void enqueue_compress(dqz_ctx *ctx, uint8_t *ws, uint64_t ws_bytes, int ncu, const float *d_field,
                      const dqz_params *params, uint8_t *arc, const Plan &P, const WsLayout &W, Readback *rb,
                      hipStream_t s);
dqz_status plan_decompress_args(const uint8_t *hb, uint64_t archive_bytes, float *d_field, uint64_t field_cap_elems,
                                HeaderInfo &hi, Plan &P, WsLayout &W, std::string &why);
// The workspace is ws (at least W.total bytes); `ctx` (may be NULL) as above.
void enqueue_decompress(dqz_ctx *ctx, uint8_t *ws, int ncu, const uint8_t *arc, float *d_field, const HeaderInfo &hi,
                        const Plan &P, const WsLayout &W, Readback *rb, hipStream_t s);

}  // namespace host
}  // namespace dqz
