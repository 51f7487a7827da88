// dqz_internal.h -- device-side data structures and wave64 helpers shared by
// the libdqz kernels and the host orchestrator.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dqz {

constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kMagic = 0x315A5144u;   // bytes 'D' 'Q' 'Z' '1'
constexpr uint32_t kVersion = 1;
constexpr uint32_t kTile = 4096;           // padded positions per quantize / encode tile
constexpr uint32_t kLutBits = 13;          // decode table width (u16 entries: len << 11 | sym)
constexpr uint32_t kHistReplicas = 16;     // global histogram copies (spreads the flush atomics)
constexpr uint32_t kSpinLimit = 1u << 20;  // look-back polls before a wait is declared stuck
constexpr uint32_t kMaxRadius = 1024;      // codebook kernel keeps 2R <= 2048 symbols in LDS
constexpr uint32_t kMaxSyms = 2 * kMaxRadius;
constexpr uint16_t kNoSymbol = 0xFFFF;     // code slot of a padded position outside the field
constexpr uint32_t kDecodeWaveSubs = 64;   // subchunks decoded by one wave (one per lane)

// Device status bits (Ctl::status), mapped to dqz_status on the host.
enum : uint32_t {
    ST_EINVAL = 1u,        // eb / derived h, r out of range
    ST_ETOOSMALL = 2u,     // archive capacity exceeded
    ST_EUNSUPPORTED = 4u,  // code longer than 64 bits
    ST_ECORRUPT = 8u,      // archive fails validation during decode
    ST_EINTERNAL = 16u,    // a look-back wait exceeded its poll limit (kernel exits anyway)
};

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
    uint32_t pad;
};

// Control block in device scratch: the values that only the device knows.
struct Ctl {
    double eb_abs;
    float h, r;
    uint32_t vmin_key, vmax_key;   // totally ordered keys of the finite range
    uint32_t status;
    uint32_t ticket_q, ticket_e;   // dynamic tile tickets (quantize, encode)
    uint32_t minmax_done;
    uint32_t n_out, n_patch, n_exc;
    uint32_t max_len;
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
                                    // (min_len << 11) | 0x8000 for a prefix of longer codes
    uint64_t limit[65];             // left-aligned end of the codes of length <= l
    uint64_t first_code[65];        // canonical first code of each length
    uint32_t count[65];             // codes of each length
    uint32_t first_index[65];       // index of the first such code in `sorted`
    uint16_t sorted[kMaxSyms];      // symbols in canonical order
    uint32_t max_len;
    uint32_t status;
    uint64_t phase[8];
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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Inclusive prefix sum over the 64 lanes.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back (single-pass ordered prefix over tiles taken in ticket
// order).  One 64-bit word per tile: value << 2 | flag, flag 0 = not yet
// published, 1 = tile aggregate, 2 = inclusive prefix.  Value and flag share
// one word, so relaxed agent-scope atomics suffice.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lb_publish(uint64_t *st, uint32_t tile, uint64_t value, uint32_t flag) {
    __hip_atomic_store(st + tile, (value << 2) | flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of one wave; returns the sum of the values of all
// tiles before `tile`.
// Tiles are numbered by workgroup index; workgroups are dispatched in
// index order, so every tile a wait depends on has started.  The poll count
// is bounded anyway: a stuck wait sets ST_EINTERNAL in *err and returns.
__device__ inline uint64_t lb_exclusive(const uint64_t *st, uint32_t tile, uint32_t *err) {
    const uint32_t lane = lane_id();
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;
    uint32_t polls = 0;
    while (base >= 0) {
        if (++polls > kSpinLimit) {
            if (lane == 0) atomicOr(err, ST_EINTERNAL);
            return excl;
        }
        const int64_t j = base - (int64_t)lane;
        uint64_t s = 2;   // virtual predecessor before tile 0: inclusive, value 0
        if (j >= 0) s = __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = (uint32_t)(s & 3u);
        const uint64_t empty = __ballot(flag == 0);
        const uint64_t incl = __ballot(flag == 2);
        if (incl) {
            const uint32_t first = (uint32_t)__ffsll((unsigned long long)incl) - 1u;
            const uint64_t need = (first == 63) ? ~0ull : ((2ull << first) - 1ull);
            if (empty & need) { __builtin_amdgcn_s_sleep(1); continue; }
            excl += wave_sum<uint64_t>(lane <= first ? (s >> 2) : 0ull);
            break;
        }
        if (empty) { __builtin_amdgcn_s_sleep(1); continue; }
        excl += wave_sum<uint64_t>(s >> 2);
        base -= 64;
    }
    return excl;
}

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

// ---------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).
// ---------------------------------------------------------------------------
void launch_init(hipStream_t s, Ctl *ctl, void *zero_base, uint64_t zero_bytes, int eb_mode, double eb);
void launch_minmax(hipStream_t s, const float *x, uint64_t n, Ctl *ctl, uint32_t *partials, double valrel, int ncu);
constexpr uint32_t kMinmaxMaxBlocks = 2048;
void launch_quantize(hipStream_t s, const float *x, const Geom &g, const Layout &L, Ctl *ctl, uint16_t *codes,
                     uint32_t *hist, uint64_t *lb, uint8_t *archive);
uint32_t quantize_tiles(const Geom &g);
void launch_codebook(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const uint32_t *hist,
                     uint64_t *book, uint32_t *book32, uint8_t *archive, int eb_mode, double eb_param);
void launch_zero_stream(hipStream_t s, const Geom &g, Ctl *ctl, uint8_t *archive);
void launch_encode(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const uint16_t *codes,
                   const uint64_t *book, const uint32_t *book32, uint64_t *lb, uint8_t *archive);
uint32_t encode_tiles(const Geom &g);
void launch_decode_tables(hipStream_t s, const Layout &L, const uint8_t *archive, uint32_t max_len_hdr,
                          DecodeTables *tab);
size_t decode_lds_bytes(const Layout &L);
void launch_decode(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint64_t off_str,
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out);

}  // namespace dqz
