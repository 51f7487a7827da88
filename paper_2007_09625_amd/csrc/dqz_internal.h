// dqz_internal.h -- device-side data structures and wave64 helpers shared by
// the libdqz kernels and the host orchestrator.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dqz.h"

namespace dqz {

constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kMagic = 0x315A5144u;   // bytes 'D' 'Q' 'Z' '1'
constexpr uint32_t kVersion = 1;
constexpr uint32_t kTile = 4096;           // padded positions per quantize / encode tile
constexpr uint32_t kLutBits = 13;          // decode table width (u16 entries: len << 11 | sym)
constexpr uint32_t kLut2Max = 3072;        // second-level decode table entries (codes longer than kLutBits)
constexpr uint32_t kUnitShift = 9;         // reconstruction unit: 512 padded positions (four 128-position subchunks)
constexpr uint32_t kHistReplicas = 16;     // global histogram copies (spreads the flush atomics)
constexpr uint32_t kExcCap = 512;          // staged exception records per quantize tile; more go to the overflow pool
constexpr uint32_t kMaxRadius = 1024;      // codebook kernel keeps 2R <= 2048 symbols in LDS
constexpr uint32_t kMaxSyms = 2 * kMaxRadius;
constexpr uint16_t kNoSymbol = 0xFFFF;     // code slot of a padded position outside the field
constexpr uint32_t kDecodeWaveSubs = 64;   // subchunks decoded by one wave (one per lane)
constexpr uint32_t kMaxLayers = 2;         // Lorenzo predictor layers the kernels implement

// Device status bits (Ctl::status); status_code maps them to a dqz_status.
enum : uint32_t {
    ST_EINVAL = 1u,        // eb / derived h, r out of range
    ST_ETOOSMALL = 2u,     // archive capacity exceeded
    ST_EUNSUPPORTED = 4u,  // code longer than 64 bits
    ST_ECORRUPT = 8u,      // archive fails validation during decode
    ST_EINTERNAL = 16u,    // internal consistency check failed
    ST_ENOMEM = 32u,       // the workspace's exception overflow pool is too small for this field
};

// Readback block: status, archive size and header of a call, written by the
// kernels into memory the host can read (pinned host memory, or the caller's
// dqz_result for the asynchronous entry points).  `bits` holds the ST_* flags,
// `code` the dqz_status they map to.
struct Readback {
    uint32_t bits;
    int32_t code;
    uint64_t archive_bytes;
    uint64_t workspace_need;   // with ST_ENOMEM: the workspace bytes that would have sufficed
    uint64_t reserved;
    uint8_t header[128];
};

// dqz_status of a set of ST_* flags (the first applicable, most severe first)
__host__ __device__ inline int32_t status_code(uint32_t b) {
    if (b & ST_EINTERNAL) return -7;
    if (b & ST_EINVAL) return -1;
    if (b & ST_ENOMEM) return -3;
    if (b & ST_EUNSUPPORTED) return -5;
    if (b & ST_ECORRUPT) return -4;
    if (b & ST_ETOOSMALL) return -2;
    return 0;
}
__device__ __forceinline__ void publish_status(Readback *rb, uint32_t bits) {
    rb->bits = bits;
    rb->code = status_code(bits);
}

// Geometry: every field is viewed as (nz, ny, nx) with block extents
// (bz, by, bx) = (1,1,32) for 1D, (1,16,16) for 2D, (8,8,8) for 3D.
struct Geom {
    uint32_t n[3];
    uint32_t b[3];
    uint32_t nb[3];
    uint32_t bvol;
    uint32_t ndim;
    uint32_t padded;   // nblocks * bvol, < 2^31
    uint64_t nelem;
};

// Section offsets of the archive that are known before any kernel runs.
struct Layout {
    uint64_t off_len, off_chunk, off_sub, off_exc;
    uint64_t cap;          // archive capacity in bytes
    uint32_t n_sub, n_chunks;
    uint32_t sub_size, chunk_subs;
    uint32_t radius, nsym;
    uint32_t sub_shift;    // log2(sub_size)
    uint32_t layers;       // Lorenzo predictor layers (1 or 2)
    uint64_t ws_fixed;     // compression workspace bytes before the exception overflow pool
};

// Control block in device scratch: the values that only the device knows.
struct Ctl {
    double eb_abs;
    float h, r;
    uint32_t vmin_key, vmax_key;   // totally ordered keys of the finite range
    uint32_t status;
    uint32_t n_out, n_patch, n_exc;
    uint32_t max_len;
    uint32_t pad0, pad1;
    uint64_t pool_used;             // overflow-pool records taken by the quantize tiles
    uint64_t exc_total, out_total;  // written by the last quantize segment
    uint64_t bits_total;            // written by the last encode-count segment
    uint64_t total_bits;
    uint64_t off_str;
    uint64_t archive_bytes;
    uint64_t n_words;
    // copy of the header as written (for the host readback)
    uint8_t header[kHeaderBytes];
    // phase timestamps (wall clock, 100 MHz) of the one-workgroup kernels
    uint64_t phase[16];
};

// Decoder tables built from the archive's code lengths.
struct DecodeTables {
    uint16_t lut[1u << kLutBits];   // (len << 11) | sym for codes of <= kLutBits bits;
                                    // 0x8000 | shortest length for a prefix of longer codes
    // Second level, flat: the top kLutBits + lut2_bits stream bits v index
    // lut2[v - (lut2_v0 << lut2_bits)] for v >= lut2_v0 << lut2_bits (the
    // long-code prefixes start at lut2_v0); entries (len << 11) | sym, 0 for
    // a code longer than kLutBits + lut2_bits or beyond the table
    uint16_t lut2[kLut2Max];
    uint32_t lut2_v0, lut2_bits, lut2_n;
    uint64_t limit[65];             // left-aligned end of the codes of length <= l
    uint64_t first_code[65];        // canonical first code of each length
    uint32_t count[65];             // codes of each length
    uint32_t first_index[65];       // index of the first such code in `sorted`
    uint16_t sorted[kMaxSyms];      // symbols in canonical order
    uint32_t max_len;
    uint32_t status;
    // [0..2] this kernel's marks; [8] first decode-wave start, [9] last
    // decode-wave end, [10..15] decode-phase durations summed over the waves
    // (tables, window + search, inflate, outlier marks, reconstruct, patches)
    uint64_t phase[16];
};

// ---------------------------------------------------------------------------
// Ordered float keys: unsigned order of the key = IEEE total order of x.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t f2key(uint32_t u) { return (u & 0x80000000u) ? ~u : (u | 0x80000000u); }
__host__ __device__ inline uint32_t key2f(uint32_t k) { return (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k; }

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below(uint32_t lane) {
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

// Value of lane (lane ^ D) within the wave: DPP quad permutes for D = 1, 2,
// row shifts for 4, a row rotate for 8, the row-pair and half-wave swaps
// for 16 and 32 (all in the VALU, no LDS round trip).
template <uint32_t D>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v, uint32_t lane) {
    static_assert(D == 1 || D == 2 || D == 4 || D == 8 || D == 16 || D == 32, "lane distance");
    if (D == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if (D == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if (D == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x104, 0xF, 0xF, false);   // row_shl:4
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
        return (lane & 4u) ? dn : up;
    }
    if (D == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);   // row_ror:8
    if (D == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16u) ? p[0] : p[1];
    }
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32u) ? p[0] : p[1];
}
template <uint32_t D>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v, uint32_t lane) {
    const uint32_t lo = xor_lane32<D>((uint32_t)v, lane), hi = xor_lane32<D>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
template <uint32_t D>
__device__ __forceinline__ uint32_t xor_lane_t(uint32_t v, uint32_t lane) { return xor_lane32<D>(v, lane); }
template <uint32_t D>
__device__ __forceinline__ uint64_t xor_lane_t(uint64_t v, uint32_t lane) { return xor_lane64<D>(v, lane); }

// Sum and maximum over the 64 lanes (32- or 64-bit), by those exchanges.
// Every wave helper here is called by whole waves (all 64 lanes active).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    const uint32_t lane = lane_id();
    v += xor_lane_t<32>(v, lane);
    v += xor_lane_t<16>(v, lane);
    v += xor_lane_t<8>(v, lane);
    v += xor_lane_t<4>(v, lane);
    v += xor_lane_t<2>(v, lane);
    v += xor_lane_t<1>(v, lane);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    const uint32_t lane = lane_id();
    T o;
    o = xor_lane_t<32>(v, lane); v = o > v ? o : v;
    o = xor_lane_t<16>(v, lane); v = o > v ? o : v;
    o = xor_lane_t<8>(v, lane); v = o > v ? o : v;
    o = xor_lane_t<4>(v, lane); v = o > v ? o : v;
    o = xor_lane_t<2>(v, lane); v = o > v ? o : v;
    o = xor_lane_t<1>(v, lane); v = o > v ? o : v;
    return v;
}

// DPP move that yields 0 where the source lane lies outside the 16-lane row
// or the destination row is masked off (CTRL: row_shr:n = 0x110 + n,
// row_bcast:15 = 0x142 (lane 15 of each row into the next row),
// row_bcast:31 = 0x143 (lane 31 into rows 2 and 3)).
template <uint32_t CTRL, uint32_t ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_zero(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
template <uint32_t CTRL, uint32_t ROWS = 0xF>
__device__ __forceinline__ uint64_t dpp_zero(uint64_t v) {
    return ((uint64_t)dpp_zero<CTRL, ROWS>((uint32_t)(v >> 32)) << 32) | dpp_zero<CTRL, ROWS>((uint32_t)v);
}

// Sum over the 64 lanes through those exchanges (no LDS round trip).
__device__ __forceinline__ uint32_t wave_sum_xor(uint32_t v) {
    const uint32_t lane = lane_id();
    v += xor_lane32<1>(v, lane);
    v += xor_lane32<2>(v, lane);
    v += xor_lane32<4>(v, lane);
    v += xor_lane32<8>(v, lane);
    v += xor_lane32<16>(v, lane);
    v += xor_lane32<32>(v, lane);
    return v;
}

// Workgroups of one launch are dispatched round-robin over the 8 XCDs, each
// with its own L2.  This bijection of [0, n) gives every XCD a contiguous run
// of tiles, so cache lines shared by neighbouring tiles stay in one L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t wg, uint32_t n) {
    const uint32_t x = wg % kXcds, k = wg / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Inclusive prefix sum over the 64 lanes (32- or 64-bit): a scan inside each
// 16-lane row by row shifts, then each row's total carried into the rows
// after it by the two row broadcasts; all in the VALU.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    v += dpp_zero<0x111>(v);
    v += dpp_zero<0x112>(v);
    v += dpp_zero<0x114>(v);
    v += dpp_zero<0x118>(v);
    v += dpp_zero<0x142, 0xA>(v);
    v += dpp_zero<0x143, 0xC>(v);
    return v;
}

// ---------------------------------------------------------------------------
// Ordered prefix over tiles, through kernel boundaries only (no spin-waits,
// no device-scope fences: on a multi-XCD part an agent-scope release writes
// back the L2).  The producer kernel stores one value per tile; k_seg_scan
// (one workgroup per segment of kSegTiles tiles) writes the exclusive prefix
// inside each segment and the segment totals; a consumer workgroup adds the
// totals of the segments before its own with one block reduction.
// ---------------------------------------------------------------------------
constexpr uint32_t kSegTiles = 256;
constexpr uint32_t kMaxSegs = 2048;   // 2^31 positions / kTile / kSegTiles

struct TileScan {
    uint32_t *val[2];        // per tile
    uint32_t *excl[2];       // per tile, exclusive inside the segment
    uint64_t *seg_total[2];  // per segment
    uint32_t n_tiles, n_segs, nvals;
};

// Exclusive scan over the 256 threads of a workgroup (u64), returns the total
// in *total.  sh: 4 u64 of LDS scratch.
__device__ __forceinline__ uint64_t block_excl_scan256(uint64_t v, uint64_t *sh, uint64_t *total) {
    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint64_t incl = wave_incl_scan<uint64_t>(v);
    __syncthreads();
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    uint64_t off = 0, tot = 0;
    for (uint32_t i = 0; i < 4; i++) {
        if (i < w) off += sh[i];
        tot += sh[i];
    }
    *total = tot;
    return off + incl - v;
}

// Sum over the 256 threads of a workgroup (u64).  sh: 4 u64 of LDS scratch.
__device__ __forceinline__ uint64_t block_sum256(uint64_t v, uint64_t *sh) {
    uint64_t tot;
    (void)block_excl_scan256(v, sh, &tot);
    return tot;
}

// Producer side: one thread records the tile's value(s).
__device__ __forceinline__ void tile_publish(const TileScan &S, uint32_t tile, uint32_t v0, uint32_t v1) {
    if (threadIdx.x == 0) {
        S.val[0][tile] = v0;
        if (S.nvals > 1) S.val[1][tile] = v1;
    }
}

// Consumer side (all 256 threads): global exclusive prefix of value k at
// `tile`.  Reads the totals of the segments before the tile's own.
__device__ __forceinline__ uint64_t tile_offset(const TileScan &S, uint32_t k, uint32_t tile, uint64_t *sh) {
    const uint32_t seg = tile / kSegTiles;
    uint64_t part = 0;
    for (uint32_t i = threadIdx.x; i < seg; i += 256) part += S.seg_total[k][i];
    return block_sum256(part, sh) + S.excl[k][tile];
}

// Grand total of value k (all 256 threads).
__device__ __forceinline__ uint64_t scan_total(const TileScan &S, uint32_t k, uint64_t *sh) {
    uint64_t part = 0;
    for (uint32_t i = threadIdx.x; i < S.n_segs; i += 256) part += S.seg_total[k][i];
    return block_sum256(part, sh);
}

// Optional side job of the quantize segment scan: sum the histogram
// replicas into the final histogram (hist_out[b] = sum of the replicas).
struct HistJob {
    const uint32_t *replicas;
    uint32_t *hist_out;
    uint32_t nsym;
};
void launch_seg_scan(hipStream_t s, const TileScan &S, const HistJob *hj = nullptr);

// ---------------------------------------------------------------------------
// Dual-quantization arithmetic (single IEEE operations, no contraction).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t prequant(float v, float r) {
    const float t = __fmul_rn(v, r);
    return (fabsf(t) < 1073741824.0f) ? (int32_t)rintf(t) : 0;
}
__device__ __forceinline__ float dequant(int32_t d, float h) { return __fmul_rn((float)d, h); }
__device__ __forceinline__ bool needs_patch(float v, int32_t d, float h, double eb) {
    const float xr = dequant(d, h);
    return !(fabs(__dsub_rn((double)v, (double)xr)) <= eb);
}
// The quantize kernels take the same decision with the double-precision test
// only where a single-precision one cannot settle it: |v - xr| rounded to
// fp32 is within 2^-24 of the exact difference, so a rounded value <= thr
// (an fp32 at most eb (1 - 2^-20)) means no patch; non-finite values fail
// that test and go on to the exact one.
__device__ __forceinline__ float patch_threshold(double eb) { return (float)(eb * (1.0 - 0x1p-20)); }

// ---------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).
// ---------------------------------------------------------------------------
void launch_init(hipStream_t s, Ctl *ctl, void *zero_base, uint64_t zero_bytes, int eb_mode, double eb);
void launch_publish(hipStream_t s, Readback *rb, uint32_t bits, uint64_t archive_bytes);
// (also clears the control block and [zero_base, +zero_bytes), as launch_init does)
void launch_minmax(hipStream_t s, const float *x, uint64_t n, Ctl *ctl, uint32_t *partials, double valrel, int ncu,
                   void *zero_base, uint64_t zero_bytes);
constexpr uint32_t kMinmaxMaxBlocks = 2048;
// fold the control block's (min key, max key) into acc[0..1] (first: set it)
void launch_range_fold(hipStream_t s, const Ctl *ctl, uint32_t *acc, bool first);
struct QuantBufs {
    uint16_t *codes;
    uint32_t *hist;        // kHistReplicas * 2R
    uint32_t *hist_sum;    // 2R, the replicas summed
    uint2 *stage;          // tiles * cap exception records
    uint32_t cap;
    uint2 *pool;           // records past a tile's cap, taken in runs by atomic reservation
    uint64_t pool_cap;     // records the pool holds
    uint32_t *ovf_base;    // per tile: first pool record of its overflow run
    TileScan scan;         // exception count (0) and outlier count (1) per tile
};
void launch_quantize(hipStream_t s, const float *x, const Geom &g, const Layout &L, Ctl *ctl, const QuantBufs &b);
void launch_quantize_scan(hipStream_t s, const Geom &g, const Layout &L, const QuantBufs &b);
uint32_t quantize_tiles(const Geom &g);
void launch_codebook(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const uint32_t *hist,
                     uint64_t *book, uint32_t *book32, uint8_t *archive, int eb_mode, double eb_param,
                     const TileScan &qscan,
                     Readback *rb);
struct EncodeBufs {
    const uint16_t *codes;
    const uint64_t *book;
    const uint32_t *book32;
    const uint2 *stage;    // quantize staging
    uint32_t cap;
    const uint2 *pool;     // quantize overflow pool
    const uint32_t *ovf_base;
    TileScan qscan;        // offsets of the staged exceptions
    uint64_t *eflag;       // per encode tile: look-back state (zeroed before the launch)
    uint32_t n_tiles_q;
};
void launch_encode(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, Readback *rb, const EncodeBufs &b,
                   uint8_t *archive, int ncu);
uint32_t encode_tiles(const Geom &g);
void launch_decode_tables(hipStream_t s, const Layout &L, const uint8_t *archive, uint32_t max_len_hdr,
                          DecodeTables *tab, Readback *rb, uint32_t n_exc, uint32_t *unit_exc,
                          uint32_t n_units);
size_t decode_lds_bytes(const Layout &L);
hipError_t decode_kernel_attributes();   // once per device, before the first decoding launch
// Subchunks of 128 positions: launch_decode inflates into `qws` (u16 per
// padded position) and launch_recon reconstructs from it; other subchunk
// sizes decode in one kernel (qws unused).
void launch_decode(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint64_t off_str,
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out, bool trace,
                   uint4 *qws, Readback *rb, int ncu);
void launch_recon(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint32_t n_exc, float h,
                  const DecodeTables *tab, const uint4 *qws, const uint32_t *unit_exc, float *out, Readback *rb);
// Compression on a caller-given workspace [ws, ws + ws_bytes) of the current
// device, status and size into d_result (dqz_compress_async without a
// context).  *need: the workspace the field needs (0 if the arguments are
// invalid); DQZ_EUNSUPPORTED when ws_bytes is below it.
dqz_status compress_on_workspace(uint8_t *ws, uint64_t ws_bytes, int ncu, const float *d_field,
                                 const dqz_shape *shape, const dqz_params *params, void *d_archive,
                                 uint64_t archive_cap, Readback *d_result, hipStream_t stream, uint64_t *need);
// reconstruction units of 512 padded positions
inline uint32_t recon_units(const Geom &g) { return (g.padded + (1u << kUnitShift) - 1) >> kUnitShift; }

}  // namespace dqz
