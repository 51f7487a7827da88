// kernels_decode.hip -- inflate + reversed dual-quantization (Sec. 3.3).
//
// One wave decodes 64 consecutive subchunks, one per lane: the lane starts
// at the subchunk's bit offset (chunk offset + prefix of subchunk bit
// counts) and decodes every point of the subchunk with a 2^13-entry LDS
// lookup table (longer codes by a second-level table or the canonical
// first-code rule).  The inverse of the Lorenzo mixed difference is a prefix
// sum along every axis (Algorithm 2's cascading reconstruction,
// reorganised), in wrapping int32; values are dequantized as
// fl32(d°) * fl32(2 eb) and written row-major, outliers take their deltas
// from the exception list and patches (verbatim values) replace values last.
//
// Subchunks of 128 positions (the default) go through two kernels: inflate
// into a code array, then one wave per 512-position unit reconstructs
// (k_inflate128, k_recon).  Other subchunk sizes decode and reconstruct in
// one kernel with an LDS code buffer (k_decode).
#include "dqz_internal.h"

namespace dqz {

// LDS-typed pointers: every access through them is a ds_* instruction (a
// generic pointer could be merged with a global one into a flat access)
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) int16_t lds_i16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

constexpr uint32_t kDecMaxWaves = 2;   // waves per workgroup (they share the lookup table)

struct DecArgs {
    Geom g;
    Layout L;
    const uint8_t *archive;
    const uint32_t *words;
    uint64_t n_words;
    uint64_t last_word;   // n_words - 1 (0 for an empty stream, whose loads read the archive header)
    const uint2 *exc;
    uint32_t n_exc;
    const DecodeTables *tab;
    uint32_t *status;
    float *out;
    float h;
    uint32_t wave_tasks;
    uint32_t qstride;   // LDS code-buffer stride per subchunk (sub_size + 2: spreads lanes over banks)
    uint32_t win_words; // LDS stream-window words per wave
    uint32_t trace;     // record phase durations into tab->phase
    uint4 *qws;         // 128-position subchunks: 16 x 16 bytes of codes per subchunk, lane-interleaved
    Readback *rb;       // the call's readback block, read by the host after the stream ends
};

// Stream word i.  Indices past the end are clamped to the last word rather
// than tested: the load is then unconditional, so its result is never merged
// through a branch, and the compiler keeps it in flight until first use.
// Bits past the end of the stream never decide a symbol of a valid stream
// (only the top `len` bits of the window select a code of length `len`);
// a damaged stream is caught by the per-subchunk bit count check.
__device__ __forceinline__ uint32_t ld_word(const DecArgs &a, uint64_t i) {
    return a.words[i < a.last_word ? i : a.last_word];
}

// LDS copy of the decoding tables
struct DecLds {
    uint64_t limit[65];
    uint64_t first_code[65];
    uint32_t first_index[65];
};

// Is padded position p inside the field?
__device__ __forceinline__ bool pos_real(const Geom &g, uint64_t p) {
    if (g.ndim == 1) return p < g.nelem;
    const uint32_t blk = (uint32_t)(p / g.bvol), in = (uint32_t)(p % g.bvol);
    const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
    const uint32_t ix = in % g.b[2], iy = (in / g.b[2]) % g.b[1], iz = in / (g.b[2] * g.b[1]);
    return Bz * g.b[0] + iz < g.n[0] && By * g.b[1] + iy < g.n[1] && Bx * g.b[2] + ix < g.n[2];
}

__device__ __forceinline__ bool block_full(const Geom &g, uint32_t blk) {
    const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
    return (Bz + 1) * g.b[0] <= g.n[0] && (By + 1) * g.b[1] <= g.n[1] && (Bx + 1) * g.b[2] <= g.n[2];
}

__device__ __forceinline__ uint64_t pos_to_index(const Geom &g, uint64_t p) {
    if (g.ndim == 1) return p;
    const uint32_t blk = (uint32_t)(p / g.bvol), in = (uint32_t)(p % g.bvol);
    const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
    const uint32_t ix = in % g.b[2], iy = (in / g.b[2]) % g.b[1], iz = in / (g.b[2] * g.b[1]);
    return ((uint64_t)(Bz * g.b[0] + iz) * g.n[1] + (By * g.b[1] + iy)) * g.n[2] + (Bx * g.b[2] + ix);
}

// Window word k sits at k + k/16: lanes read words about one subchunk apart,
// and the pad spreads those reads over the LDS banks.
__device__ __forceinline__ uint32_t win_slot(uint32_t k) { return k + (k >> 4); }

// n copies of an 8-bit row mask in consecutive bytes (n clamped to 0..4)
__device__ __forceinline__ uint32_t rows8(uint32_t rowmask, int32_t n) {
    n = n < 0 ? 0 : (n > 4 ? 4 : n);
    return n ? rowmask * (0x01010101u >> (8 * (4 - n))) : 0u;
}

// In-field mask of the 32 padded positions [p, p + 32), p a multiple of 32:
// bit k is set when position p + k lies inside the field.  Such a run lies in
// one block (8^3, 16^2 or 32 positions) and covers whole rows of it: four
// rows of 8 in 3D, two rows of 16 in 2D.
__device__ __forceinline__ uint32_t real_mask32(const Geom &g, uint32_t p) {
    if (p >= g.padded) return 0u;
    if (g.ndim == 1) {
        const uint64_t c = g.nelem > p ? g.nelem - p : 0;
        return c >= 32 ? ~0u : ((1u << c) - 1u);
    }
    if (g.ndim == 2) {
        const uint32_t blk = p >> 8, y0 = (p & 255u) >> 4;
        const uint32_t Bx = blk % g.nb[2], By = blk / g.nb[2];
        const uint32_t vx = min(16u, g.n[2] - 16 * Bx), vy = min(16u, g.n[1] - 16 * By);
        const uint32_t row = (1u << vx) - 1u;
        return (y0 < vy ? row : 0u) | (y0 + 1 < vy ? row << 16 : 0u);
    }
    const uint32_t blk = p >> 9, in = p & 511u;
    const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
    const uint32_t vx = min(8u, g.n[2] - 8 * Bx), vy = min(8u, g.n[1] - 8 * By), vz = min(8u, g.n[0] - 8 * Bz);
    if ((in >> 6) >= vz) return 0u;
    return rows8((1u << vx) - 1u, (int32_t)vy - (int32_t)((in >> 3) & 7u));
}

// Inflate the S padded positions of the subchunk starting at stream bit
// `start` (positions pa ..) into q[]; returns the number of stream bits
// consumed.  The common step has no divergent branch: the refill is a
// select, the next stream word is read from the LDS window every step, and
// the in-field test is a bit of a 32-position mask.  Codes the lookup table
// does not resolve (longer than kLutBits), invalid table entries and stream
// words outside the window take one uniform branch that is rarely entered.
__device__ __forceinline__ uint32_t inflate(const DecArgs &a, const lds_u32 *win, uint32_t nwin, uint64_t wlo,
                                            uint64_t start, uint32_t pa, uint32_t S, lds_u16 *q, const lds_u16 *lut,
                                            const DecLds &t, const lds_u16 *sorted, uint32_t max_len, bool &bad) {
    const uint64_t sw = start >> 5;   // the lane's first stream word
    // window index of word sw + kr is relw + kr; a lane outside the window
    // (only with damaged chunk offsets) misses on every read
    const uint32_t relw = (sw >= wlo && sw - wlo < nwin) ? (uint32_t)(sw - wlo) : nwin;
    const uint32_t wlast = nwin ? nwin - 1 : 0;
    auto word = [&](uint32_t kr) -> uint32_t {
        const uint32_t k = relw + kr;
        return (k < nwin) ? win[win_slot(k)] : ld_word(a, sw + kr);
    };
    const uint32_t R = a.L.radius;
    uint32_t used = 0, kr = 2;
    uint32_t o = (uint32_t)(start & 31u);
    uint64_t cur = (((uint64_t)word(0) << 32) | word(1)) << o;
    int32_t avail = 64 - (int32_t)o;
    uint32_t nxt = word(kr);
    uint32_t rmask = 0;
    for (uint32_t i = 0; i < S; i++) {
        if ((i & 31u) == 0) rmask = real_mask32(a.g, pa + i);
        // refill: the next word enters right below the valid bits
        const bool need = avail <= 32;
        const uint32_t shl = need ? (uint32_t)(32 - avail) : 0u;
        cur |= need ? ((uint64_t)nxt << shl) : 0ull;
        avail += need ? 32 : 0;
        kr += need ? 1u : 0u;
        const uint32_t k = relw + kr;
        nxt = win[win_slot(k < nwin ? k : wlast)];
        // decode
        const bool real = (rmask >> (i & 31u)) & 1u;
        const uint32_t e = lut[(uint32_t)(cur >> (64 - kLutBits))];
        uint32_t len = (e >> 11) & 15u, sym = e & 0x7FFu;
        const bool slow = real && ((e & 0x8000u) || len == 0);
        bool moved = false;
        if (__any((int)(slow || k >= nwin))) {
            if (k >= nwin) nxt = ld_word(a, sw + kr);
            if (slow && !(e & 0x8000u)) {   // no code starts with these bits
                bad = true;
                len = 1;
                sym = R;
            } else if (slow) {
                // a longer code: canonical limits from the shortest possible length
                uint32_t l = e & 63u;
                uint64_t wv = cur;
                if (max_len > 32) {
                    const uint64_t bp = start + used;
                    const uint64_t ww = bp >> 5;
                    const uint32_t ob = (uint32_t)(bp & 31u);
                    const uint64_t h2 = ((uint64_t)ld_word(a, ww) << 32) | ld_word(a, ww + 1);
                    wv = ob ? ((h2 << ob) | (ld_word(a, ww + 2) >> (32 - ob))) : h2;
                }
                while (l < max_len && wv >= t.limit[l]) l++;
                const uint64_t c = wv >> (64 - l);
                const uint64_t idx = t.first_index[l] + (c - t.first_code[l]);
                if (idx >= a.L.nsym) { bad = true; sym = R; }
                else sym = sorted[idx];
                len = l;
                if ((int32_t)l > avail) {   // a code over 32 bits: restart the reader after it
                    used += l;
                    const uint64_t bp = start + used;
                    o = (uint32_t)(bp & 31u);
                    kr = (uint32_t)((bp >> 5) - sw);
                    cur = (((uint64_t)word(kr) << 32) | word(kr + 1)) << o;
                    avail = 64 - (int32_t)o;
                    kr += 2;
                    nxt = word(kr);
                    moved = true;
                }
            }
        }
        if (!real || moved) len = 0;
        cur <<= len;
        avail -= (int32_t)len;
        used += len;
        q[i] = (uint16_t)(real ? sym : R);
    }
    return used;
}

// Wave-cooperative lower bound over the exception keys: the first index e
// with key(e) >= key (n if none).  Each round probes 64 evenly spaced keys,
// so about three dependent loads find the bracket among 2^18 entries.  On an
// unsorted (damaged) list it still returns an index in [0, n].
__device__ __forceinline__ uint32_t wave_lower_bound(const uint2 *exc, uint32_t n, uint64_t key, uint32_t lane) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 64) {
        const uint32_t span = hi - lo;
        const uint32_t idx = lo + (uint32_t)(((uint64_t)span * (lane + 1)) / 65);   // strictly increasing in lane
        const uint32_t c = (uint32_t)__popcll(__ballot((uint64_t)exc[idx].x < key));
        const uint32_t nlo = c ? (uint32_t)__shfl((int)idx, (int)c - 1, 64) + 1 : lo;
        const uint32_t nhi = c < 64 ? (uint32_t)__shfl((int)idx, (int)c, 64) : hi;
        lo = nlo;
        hi = nhi;
    }
    const uint32_t idx = lo + lane;
    return lo + (uint32_t)__popcll(__ballot(idx < hi && (uint64_t)exc[idx < hi ? idx : lo].x < key));
}

// ---- cross-lane inclusive scans of the reconstruction, on DPP row shifts
// (VALU, within 16-lane rows) and the gfx950 row/half swaps.

// A cross-lane result must be computed with every lane active: a lane that
// is off in EXEC supplies 0.  The empty asm makes the value opaque, so the
// compiler cannot turn `cond ? cross_lane(v) : 0` into a branch that runs the
// cross-lane move under a partial EXEC mask.
__device__ __forceinline__ uint32_t pinned(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// lane - K within the lane's 16-lane row (0 across the row start)
template <int K>
__device__ __forceinline__ uint32_t row_shr(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + K, 0xF, 0xF, true));
}

// value of lane - 16 for lanes of rows 1 and 3 (from rows 0 and 2);
// `even_from_odd` receives rows 1 and 3 in rows 0 and 2
__device__ __forceinline__ void row_swap16(uint32_t v, uint32_t &odd_from_even, uint32_t &even_from_odd) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    odd_from_even = pinned(r[0]);
    even_from_odd = pinned(r[1]);
}
// value of lane - 32 for lanes 32..63
__device__ __forceinline__ uint32_t half_up32(uint32_t v) {
    return pinned(__builtin_amdgcn_permlane32_swap(v, v, false, false)[0]);
}

// lane - 8 with rotation inside the 16-lane row: lane i gets lane (i + 8) mod 16
__device__ __forceinline__ uint32_t row_ror8(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, true));
}

// inclusive scan within groups of G consecutive lanes (G = 8, 16 or 32);
// every cross-lane value is taken unconditionally, then selected.  DPP row
// shifts stop at 16-lane rows, so a 32-lane group adds the lower row's total
// (lanes 15 and 47) to its upper row.
template <uint32_t G>
__device__ __forceinline__ uint32_t seg_scan(uint32_t t, uint32_t lane) {
    const uint32_t l = lane & (G - 1);
    uint32_t d = row_shr<1>(t);
    t += (l >= 1) ? d : 0u;
    d = row_shr<2>(t);
    t += (l >= 2) ? d : 0u;
    d = row_shr<4>(t);
    t += (l >= 4) ? d : 0u;
    if (G >= 16) {
        d = row_shr<8>(t);
        t += (l >= 8) ? d : 0u;
    }
    if (G >= 32) {
        const uint32_t t0 = __builtin_amdgcn_readlane(t, 15), t1 = __builtin_amdgcn_readlane(t, 47);
        t += (l >= 16) ? (lane >= 32 ? t1 : t0) : 0u;
    }
    return t;
}

// inclusive scan over the 8 lanes of equal (lane % 8), lane = 8 y + x: the
// pair (2r, 2r + 1) of y shares row r; within-row pair sums, then each row
// adds the exclusive prefix of the row totals (rows swapped by the gfx950
// row and half swaps)
__device__ __forceinline__ uint32_t stride8_scan(uint32_t t, uint32_t lane) {
    const bool odd_y = (lane >> 3) & 1u;
    const uint32_t row = lane >> 4;
    const uint32_t d8 = row_shr<8>(t);
    const uint32_t s = t + (odd_y ? d8 : 0u);           // y even: t_y; y odd: t_{y-1} + t_y
    const uint32_t r8 = row_ror8(s);
    const uint32_t T = odd_y ? s : r8;                  // the row's total at every lane
    uint32_t ofe, efo;
    row_swap16(T, ofe, efo);                            // rows 1, 3 <- rows 0, 2 and back
    const uint32_t pair = T + ((row & 1u) ? ofe : efo); // T0 + T1 in rows 0, 1; T2 + T3 in rows 2, 3
    const uint32_t low = half_up32(pair);               // rows 2, 3 <- T0 + T1
    return s + ((row & 1u) ? ofe : 0u) + (row >= 2 ? low : 0u);
}

// code buffer slot -> wrapping delta; outlier deltas come from the wave's
// LDS copy of its first kDecXp exception payloads, later ones from memory
constexpr uint32_t kDecXp = 256;
__device__ __forceinline__ uint32_t slot_delta(const DecArgs &a, uint16_t q, uint32_t e0, const lds_u32 *xp,
                                               bool &bad) {
    if (q & 0x8000u) {
        const uint32_t k = q & 0x7FFFu;
        return k < kDecXp ? xp[k] : a.exc[e0 + k].y;
    }
    if (q == 0) bad = true;
    return (uint32_t)q - a.L.radius;
}

// ---- prologue shared by both decode kernels ------------------------------

// The decoding tables into LDS: 16-byte loads, eight of a thread's in flight
// at once (the lookup table is 16 KB at offset 0 of the 256-byte aligned
// tables; the sorted symbols are 8-byte aligned, nsym a multiple of 2).
__device__ __forceinline__ void tables_to_lds(const DecArgs &a, lds_u16 *s_lut, lds_u16 *s_sorted, DecLds &t) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *src = reinterpret_cast<const u32x4 *>(a.tab->lut);
    __attribute__((address_space(3))) u32x4 *dst = (__attribute__((address_space(3))) u32x4 *)s_lut;
    constexpr uint32_t kVec = (1u << kLutBits) * 2 / 16;
    for (uint32_t i0 = threadIdx.x; i0 < kVec; i0 += 8 * blockDim.x) {
        u32x4 v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * blockDim.x;
            v[j] = src[i < kVec ? i : 0];
        }
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * blockDim.x;
            if (i < kVec) dst[i] = v[j];
        }
    }
    const uint32_t *ssrc = reinterpret_cast<const uint32_t *>(a.tab->sorted);
    lds_u32 *sdst = (lds_u32 *)s_sorted;
    for (uint32_t i = threadIdx.x; i < a.L.nsym / 2; i += blockDim.x) sdst[i] = ssrc[i];
    for (uint32_t i = threadIdx.x; i < 65; i += blockDim.x) {
        const uint64_t l = a.tab->limit[i], f = a.tab->first_code[i];
        const uint32_t x = a.tab->first_index[i];
        t.limit[i] = l;
        t.first_code[i] = f;
        t.first_index[i] = x;
    }
}

// Start bit of the lane's subchunk s = sub0 + lane (chunk offset + prefix of
// the subchunk bit counts), its bit count, and the wave's stream range copied
// into the LDS window (coalesced, unconditional loads).  Called by whole
// active waves.
struct WaveStream {
    uint64_t start, wlo;
    uint32_t bits, nwin;
    bool whole;   // the window holds every word a lane of the wave reads
};
template <bool PAD>
__device__ __forceinline__ WaveStream wave_stream(const DecArgs &a, uint64_t sub0, uint32_t lane, bool has,
                                                  lds_u32 *win) {
    WaveStream r;
    const uint64_t s = sub0 + lane;
    const uint8_t *subp = a.archive + a.L.off_sub;
    r.bits = has ? ((uint32_t)subp[2 * s] | ((uint32_t)subp[2 * s + 1] << 8)) : 0u;
    const uint32_t incl = wave_incl_scan<uint32_t>(r.bits);
    const uint32_t excl = incl - r.bits;
    const uint32_t C = a.L.chunk_subs;
    const uint64_t *chunks = reinterpret_cast<const uint64_t *>(a.archive + a.L.off_chunk);
    if (C >= 64) {
        const uint64_t cs = (sub0 / C) * C;
        uint64_t pre = 0;
        for (uint64_t j = cs + lane; j < sub0; j += 64) pre += (uint32_t)subp[2 * j] | ((uint32_t)subp[2 * j + 1] << 8);
        pre = wave_sum<uint64_t>(pre);
        r.start = chunks[sub0 / C] + pre + excl;
    } else {
        const uint64_t c = (has ? s : sub0) / C;
        const uint32_t k = (uint32_t)(c * C - sub0);
        const uint32_t at = __shfl(excl, (int)k, 64);
        r.start = chunks[c] + excl - at;
    }
    // the window starts at the first subchunk's word and covers the last
    // subchunk's end plus the two words a reader may look past it
    r.wlo = __shfl(r.start, 0, 64) >> 5;
    const uint64_t whi = wave_max<uint64_t>(has ? ((r.start + r.bits) >> 5) + 3 : 0);
    const uint32_t cap = PAD ? a.win_words / 17 * 16 : a.win_words;   // logical words whose slots fit
    r.nwin = whi > r.wlo ? (uint32_t)(whi - r.wlo < cap ? whi - r.wlo : cap) : 0u;
    r.whole = whi <= r.wlo || whi - r.wlo <= cap;
    for (uint32_t b = 0; b < r.nwin; b += 64 * 8) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) v[j] = ld_word(a, r.wlo + b + j * 64 + lane);
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t k = b + j * 64 + lane;
            if (k < r.nwin) win[PAD ? win_slot(k) : k] = v[j];
        }
    }
    return r;
}

// lane j - 1 (j - 2) of the lane's quad; quad_perm [0,0,1,2] and [0,0,0,1]
__device__ __forceinline__ uint32_t quad_shr1(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x90, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t quad_shr2(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x40, 0xF, 0xF, false));
}

__global__ __launch_bounds__(64 * kDecMaxWaves) void k_decode(DecArgs a) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ DecLds s_t;
    lds_u16 *s_lut = (lds_u16 *)s_dyn;                                              // 1 << kLutBits
    lds_u16 *s_sorted = s_lut + (1u << kLutBits);                                  // nsym
    lds_u16 *s_q = s_sorted + a.L.nsym;                                            // waves * 64 * qstride
    lds_u32 *s_win = (lds_u32 *)(s_q + (blockDim.x / 64) * 64 * a.qstride);        // waves * win_words
    if (a.tab->status) return;   // the code lengths failed validation: tables are not usable
    uint64_t tm[7];
    tm[0] = a.trace ? wall_clock64() : 0;
    tables_to_lds(a, s_lut, s_sorted, s_t);
    __syncthreads();
    if (a.trace) tm[1] = wall_clock64();

    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t gw = blockIdx.x * (blockDim.x / 64) + w;
    const bool active = gw < a.wave_tasks;
    const uint32_t S = a.L.sub_size, sh = a.L.sub_shift;
    lds_u16 *wq = s_q + w * 64 * a.qstride;
    const uint64_t sub0 = (uint64_t)gw * 64;
    const uint64_t P0 = sub0 << sh;
    const uint64_t P1 = active ? ((P0 + (64ull << sh)) < a.g.padded ? (P0 + (64ull << sh)) : a.g.padded) : P0;
    bool bad = false;
    uint32_t e0 = 0, e1 = 0;

    // ---- start bit of this lane's subchunk; the wave's stream range goes to LDS
    const uint64_t s = sub0 + lane;
    const bool has = active && s < a.L.n_sub;
    uint32_t bits_s = 0;
    uint64_t start = 0, wlo = 0;
    uint32_t nwin = 0;
    lds_u32 *win = s_win + w * a.win_words;
    lds_u32 *xp = s_win + (blockDim.x / 64) * a.win_words + w * kDecXp;   // exception payloads
    if (active) {
        const WaveStream ws = wave_stream<true>(a, sub0, lane, has, win);
        bits_s = ws.bits;
        start = ws.start;
        wlo = ws.wlo;
        nwin = ws.nwin;
        // ---- exception range of this wave
        e0 = wave_lower_bound(a.exc, a.n_exc, 2ull * P0, lane);
        e1 = wave_lower_bound(a.exc, a.n_exc, 2ull * P1, lane);
    }
    __syncthreads();
    if (a.trace) tm[2] = wall_clock64();
    // ---- inflate the subchunk into the LDS code buffer
    if (has) {
        const uint32_t pa = (uint32_t)(s << sh);
        const uint32_t max_len = a.tab->max_len < 63u ? a.tab->max_len : 63u;
        const uint32_t used = inflate(a, win, nwin, wlo, start, pa, S, wq + lane * a.qstride, s_lut, s_t, s_sorted,
                                      max_len, bad);
        // the subchunk must lie inside the stream and consume exactly its recorded bits
        if (used != bits_s || start + bits_s > 32ull * a.n_words) bad = true;
    }
    if (a.trace) tm[3] = wall_clock64();
    __syncthreads();
    if (active) {
        // ---- outliers: mark their slots with an index into the exception list
        for (uint32_t e = e0 + lane; e < e1; e += 64) {
            const uint2 r = a.exc[e];
            if (e - e0 < kDecXp) xp[e - e0] = r.y;
            if (r.x & 1u) continue;
            const uint64_t loc = (uint64_t)(r.x >> 1) - P0;
            if (loc >= P1 - P0) { bad = true; continue; }   // only in an unsorted (damaged) list
            lds_u16 *slot = wq + (loc >> sh) * a.qstride + (loc & (S - 1));
            if (*slot != 0 || e - e0 > 0x7FFFu) bad = true;
            else *slot = (uint16_t)(0x8000u | (e - e0));
        }
    }
    __syncthreads();
    if (a.trace) tm[4] = wall_clock64();
    if (active) {
        const Geom &g = a.g;
        const float h = a.h;
        const bool layers2 = a.L.layers == 2;   // each axis's prefix sum twice
        auto qat = [&](uint64_t loc) -> uint16_t { return wq[(loc >> sh) * a.qstride + (loc & (S - 1))]; };
        if (g.ndim == 3) {
            const uint32_t ly = lane / 8, lx = lane % 8;
            const uint32_t bfirst = (uint32_t)(P0 / 512), blast = (uint32_t)((P1 - 1) / 512);
            for (uint32_t blk = bfirst; blk <= blast; blk++) {
                const uint64_t base = (uint64_t)blk * 512 - P0;
                uint32_t v[8];
                uint32_t run = 0, run2 = 0;
#pragma unroll
                for (uint32_t z = 0; z < 8; z++) {
                    run += slot_delta(a, qat(base + z * 64 + lane), e0, xp, bad);
                    run2 += run;
                    v[z] = layers2 ? run2 : run;
                }
#pragma unroll
                for (uint32_t z = 0; z < 8; z++) v[z] = seg_scan<8>(stride8_scan(v[z], lane), lane);
                if (layers2) {
#pragma unroll
                    for (uint32_t z = 0; z < 8; z++) v[z] = seg_scan<8>(stride8_scan(v[z], lane), lane);
                }
                const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
                const uint32_t x = Bx * 8 + lx, y = By * 8 + ly;
#pragma unroll
                for (uint32_t z = 0; z < 8; z++) {
                    const uint32_t zz = Bz * 8 + z;
                    if (x < g.n[2] && y < g.n[1] && zz < g.n[0])
                        a.out[((uint64_t)zz * g.n[1] + y) * g.n[2] + x] = dequant((int32_t)v[z], h);
                }
            }
        } else if (g.ndim == 2) {
            const uint32_t grp = lane / 16, lx = lane % 16;
            const uint32_t bfirst = (uint32_t)(P0 / 256), blast = (uint32_t)((P1 - 1) / 256);
            for (uint32_t b4 = bfirst; b4 <= blast; b4 += 4) {
                const uint32_t blk = b4 + grp;
                const bool ok = blk <= blast;
                const uint64_t base = (uint64_t)blk * 256 - P0;
                const uint32_t Bx = blk % g.nb[2], By = blk / g.nb[2];
                const uint32_t x = Bx * 16 + lx;
                uint32_t col = 0, col2 = 0;
                for (uint32_t y = 0; y < 16; y++) {
                    if (ok) col += slot_delta(a, qat(base + y * 16 + lx), e0, xp, bad);
                    col2 += col;
                    uint32_t t = seg_scan<16>(layers2 ? col2 : col, lane);
                    if (layers2) t = seg_scan<16>(t, lane);
                    const uint32_t yy = By * 16 + y;
                    if (ok && x < g.n[2] && yy < g.n[1]) a.out[(uint64_t)yy * g.n[2] + x] = dequant((int32_t)t, h);
                }
            }
        } else {
            for (uint64_t off = 0; P0 + off < P1; off += 64) {
                const uint64_t loc = off + lane;
                const uint64_t p = P0 + loc;
                uint32_t t = seg_scan<32>((p < P1) ? slot_delta(a, qat(loc), e0, xp, bad) : 0u, lane);
                if (layers2) t = seg_scan<32>(t, lane);
                if (p < g.nelem) a.out[p] = dequant((int32_t)t, h);
            }
        }
    }
    __syncthreads();   // all regular values are stored before patches overwrite some
    if (a.trace) tm[5] = wall_clock64();
    if (active) {
        for (uint32_t e = e0 + lane; e < e1; e += 64) {
            const uint2 r = a.exc[e];
            if (!(r.x & 1u)) continue;
            const uint64_t p = r.x >> 1;
            if (!pos_real(a.g, p)) { bad = true; continue; }
            a.out[pos_to_index(a.g, p)] = __uint_as_float(r.y);
        }
    }
    if (bad) {
        atomicOr(a.status, ST_ECORRUPT);
        publish_status(a.rb, ST_ECORRUPT);
    }
    if (a.trace && active && lane == 0) {
        tm[6] = wall_clock64();
        uint64_t *ph = const_cast<uint64_t *>(a.tab->phase);
        atomicMin((unsigned long long *)&ph[8], (unsigned long long)tm[0]);
        atomicMax((unsigned long long *)&ph[9], (unsigned long long)tm[6]);
        for (int k = 0; k < 6; k++) atomicAdd((unsigned long long *)&ph[10 + k], (unsigned long long)(tm[k + 1] - tm[k]));
    }
}

// ---------------------------------------------------------------------------
// Subchunks of 128 positions (the default size) take two kernels.
//
// k_inflate128: one wave decodes 64 subchunks, one per lane, into 16-bit
// codes in a workspace array: eight codes per 16-byte group, group g of the
// wave's lane l at [(16 w + g) 64 + l] for wave w of 64 subchunks, so every
// store instruction writes 1 KiB contiguously.  The waves of a workgroup share the lookup tables in LDS, each
// with its stream window; one workgroup per CU with as many waves as spread
// the launch over all CUs (up to 14: tables plus windows fill the 160 KiB)
// keeps every wave of a large field resident at once.  Every step
// reads both table levels at once and selects, so codes of up to
// kLutBits + b2 bits take no branch; only longer codes and invalid entries
// go on to the canonical limits.
//
// k_recon<NDIM>: one wave per unit of 512 padded positions (one 8^3 block,
// two 16^2 blocks or sixteen 32-blocks).  Each lane loads eight consecutive
// codes (a piece of an x-row), takes its outliers from the unit's exception
// records, and the inverse of the Lorenzo prediction is a prefix sum along
// every axis: in-lane along x; in 3D the block then goes through LDS twice
// so that y and z are in-lane too, in 2D and 1D the other axes are scans
// across lanes.
// ---------------------------------------------------------------------------
constexpr uint32_t kInfMaxWaves = 14; // waves per inflate workgroup, at most (they share the lookup tables)
constexpr uint32_t kInfWin = 2432;    // LDS stream-window words per wave (9.5 KiB)
constexpr uint32_t kReconWaves = 8;   // units (one per wave) per reconstruction workgroup (8 measured best against 2, 4, 16)
constexpr uint32_t kScatterMin = 4;   // 1D/2D units with more records than this scatter them through LDS

// Both lookup-table levels into LDS: 16-byte copies, eight of a thread's
// loads in flight (the tables are 256-byte aligned, the second level starts
// 16 KiB in).
__device__ __forceinline__ void luts_to_lds(const DecodeTables *tab, lds_u16 *s_lut, lds_u16 *s_lut2) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(tab->lut);
    lds_u32x4 *dst = (lds_u32x4 *)s_lut;
    constexpr uint32_t kVec = (1u << kLutBits) * 2 / 16;
    for (uint32_t i0 = threadIdx.x; i0 < kVec; i0 += 8 * blockDim.x) {
        u32x4 v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * blockDim.x;
            v[j] = src[i < kVec ? i : 0];
        }
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t i = i0 + j * blockDim.x;
            if (i < kVec) dst[i] = v[j];
        }
    }
    const uint32_t n2 = tab->lut2_n ? (tab->lut2_n < kLut2Max ? (tab->lut2_n + 7) / 8 : kLut2Max / 8) : 1u;
    const u32x4 *src2 = reinterpret_cast<const u32x4 *>(tab->lut2);
    lds_u32x4 *dst2 = (lds_u32x4 *)s_lut2;
    for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) dst2[i] = src2[i];
}

// Does the 128-position subchunk at padded position pa lie inside the field?
// (It lies in one block: 32-blocks in 1D are whole subchunk quarters.)
__device__ __forceinline__ bool sub128_full(const Geom &g, uint32_t pa) {
    if (g.ndim == 1) return (uint64_t)pa + 128 <= g.nelem;
    return block_full(g, pa / g.bvol);
}

// Inflate the lane's 128 positions (padded positions pa ..) into 16 packed
// 16-byte groups dst[64 g]; returns the stream bits consumed.  ALLREAL: every
// position of the wave lies inside the field (none is tested).  WHOLE: the
// window holds every word the wave's lanes read (no bounds test per word).
// The window is unpadded: word k at win[k].
//
// The reader keeps two stream words w0, w1 and nb = 32 - b, b in [1, 32] the
// bits of w0 already consumed: the next 32 stream bits are one funnel shift,
// alignbit(w0, w1, nb).  Window word kk follows w1 (read ahead into `nxt`);
// the stream position is 32 (sw + kk - relw - 2) + b.  A code (at most
// kLutBits + b2 <= 20 bits on the common step) moves past w0 at most once.
// Both table levels are read every step, from the top kLutBits and
// kLutBits + b2 bits, and the first level's long-prefix flag selects between
// them.  Longer codes and invalid entries take one uniform branch.
template <bool ALLREAL, bool WHOLE>
__device__ __forceinline__ uint32_t inflate_codes(const DecArgs &a, const lds_u32 *win, uint32_t nwin, uint64_t wlo,
                                                  uint64_t start, uint32_t pa, uint4 *dst, const lds_u16 *lut,
                                                  const lds_u16 *lut2, uint32_t b2, uint32_t base2,
                                                  uint32_t max_len, bool &bad) {
    const uint64_t sw = start >> 5;   // the lane's first stream word
    // window index of word sw + kr is relw + kr; a lane outside the window
    // (only with damaged chunk offsets) misses on every read
    const uint32_t relw = (sw >= wlo && sw - wlo < nwin) ? (uint32_t)(sw - wlo) : nwin;
    const uint32_t wlast = nwin ? nwin - 1 : 0;
    // words read off the common step are waited for where they are read: a
    // global load left pending would make later steps wait for every vector
    // memory operation, the group stores included
    auto word = [&](uint32_t kr) -> uint32_t {
        const uint32_t k = relw + kr;
        return pinned((k < nwin) ? win[k] : ld_word(a, sw + kr));
    };
    const uint32_t R = a.L.radius;
    const uint32_t o = (uint32_t)(start & 31u);
    // b = o, or b = 32 with w0 the word before the first when o = 0
    uint32_t w0, w1, nxt, kk;
    if (o) { w0 = word(0); w1 = word(1); nxt = word(2); kk = relw + 2; }
    else { w0 = 0; w1 = word(0); nxt = word(1); kk = relw + 1; }
    const lds_u32 *wp = win + kk;   // window word kk (stepped with kk)
    const uint32_t lut2_at = (uint32_t)(size_t)lut2 - 2u * base2;   // LDS byte address of entry "prefix 0"
    uint32_t nb = (32u - o) & 31u;
    uint32_t rmask = ~0u;
    for (uint32_t g = 0; g < 16; g++) {
        if (!ALLREAL && (g & 3u) == 0) rmask = real_mask32(a.g, pa + g * 8);
        uint32_t pk[4];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const bool real = ALLREAL || ((rmask >> ((g & 3u) * 8 + j)) & 1u);
            const uint32_t peek = __builtin_amdgcn_alignbit(w0, w1, nb);
            // first level read sign-extended: its long-prefix entries
            // (0x8000 | length) come out negative
            const int32_t e1s = reinterpret_cast<const lds_i16 *>(lut)[peek >> (32 - kLutBits)];
            const uint32_t e1 = (uint32_t)e1s;
            // second level, read at every step: base2 is folded into the LDS
            // byte address, so a prefix below the long-code range (whose
            // entry is never used) reads some other LDS word, or zero past
            // the allocation; LDS reads cannot fault
            const uint32_t e2 = *reinterpret_cast<const lds_u16 *>(
                (size_t)(lut2_at + ((peek >> (32 - kLutBits - b2)) << 1)));
            const uint32_t e = e1s >= 0 ? e1 : e2;
            uint32_t len = e >> 11, sym = e & 0x7FFu;
            const bool other = real && len == 0;   // longer than the second level, or no code
            if (__builtin_expect(__any((int)other), 0)) {
                if (other && !(e1 & 0x8000u)) {   // no code starts with these bits
                    bad = true;
                    len = 1;
                    sym = R;
                } else if (other) {
                    // canonical limits from the shortest length past both levels,
                    // on 64 fresh bits at the lane's position
                    kk = (uint32_t)(wp - win);
                    const uint64_t bp = (sw << 5) + 32ull * (kk - relw - 2) + (32u - nb);
                    const uint32_t rk = (uint32_t)((bp >> 5) - sw), ob = (uint32_t)(bp & 31u);
                    const uint64_t h2 = ((uint64_t)word(rk) << 32) | word(rk + 1);
                    const uint64_t wv = ob ? ((h2 << ob) | (word(rk + 2) >> (32 - ob))) : h2;
                    const uint32_t lmin = e1 & 63u;
                    uint32_t l = lmin > kLutBits + b2 ? lmin : kLutBits + b2 + 1;
                    l = l < 63u ? l : 63u;
                    while (l < max_len && wv >= a.tab->limit[l]) l++;
                    const uint64_t c = wv >> (64 - l);
                    const uint64_t idx = a.tab->first_index[l] + (c - a.tab->first_code[l]);
                    if (idx >= a.L.nsym) { bad = true; sym = R; }
                    else sym = a.tab->sorted[idx];
                    // restart the reader after the code
                    const uint64_t np = bp + l;
                    const uint32_t kr = (uint32_t)((np >> 5) - sw), o2 = (uint32_t)(np & 31u);
                    if (o2) { w0 = word(kr); w1 = word(kr + 1); nxt = word(kr + 2); kk = relw + kr + 2; }
                    else { w1 = word(kr); nxt = word(kr + 1); kk = relw + kr + 1; }
                    wp = win + kk;
                    nb = (32u - o2) & 31u;
                    len = 0;
                }
            }
            if (!real) len = 0;
            // consume: past w0 (nb below zero) shifts the words by one
            const int32_t nn = (int32_t)nb - (int32_t)len;
            const bool adv = nn < 0;
            w0 = adv ? w1 : w0;
            w1 = adv ? nxt : w1;
            nb = (uint32_t)nn & 31u;
            wp = adv ? wp + 1 : wp;
            if (WHOLE) {
                nxt = *wp;
            } else {
                kk = (uint32_t)(wp - win);
                nxt = win[kk < nwin ? kk : wlast];
                if (__builtin_expect(__any((int)(kk >= nwin)), 0)) {
                    if (kk >= nwin) nxt = pinned(ld_word(a, sw + (kk - relw)));
                }
            }
            const uint32_t s16 = real ? sym : R;
            pk[j >> 1] = (j & 1u) ? (pk[j >> 1] | (s16 << 16)) : s16;
        }
        dst[g * 64] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    }
    kk = (uint32_t)(wp - win);
    return 32u * (kk - relw - 2) + (32u - nb) - o;
}

__global__ __launch_bounds__(64 * kInfMaxWaves) void k_inflate128(DecArgs a) {
    // static tables (their addresses fold into the instruction offsets),
    // the stream windows in dynamic LDS
    __shared__ __attribute__((aligned(16))) uint16_t s_lut_[1u << kLutBits];
    __shared__ __attribute__((aligned(16))) uint16_t s_lut2_[kLut2Max];
    extern __shared__ uint32_t s_dyn[];
    lds_u16 *s_lut = (lds_u16 *)s_lut_;
    lds_u16 *s_lut2 = (lds_u16 *)s_lut2_;
    lds_u32 *s_win = (lds_u32 *)s_dyn;   // waves * kInfWin
    if (a.tab->status) return;   // the code lengths failed validation: tables are not usable
    const uint64_t t0 = a.trace ? wall_clock64() : 0;
    luts_to_lds(a.tab, s_lut, s_lut2);
    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t gw = blockIdx.x * (blockDim.x / 64) + w;
    const bool active = gw < a.wave_tasks;
    const uint64_t sub0 = (uint64_t)gw * 64;
    const bool has = active && sub0 + lane < a.L.n_sub;
    lds_u32 *win = s_win + w * kInfWin;
    WaveStream ws = {0, 0, 0, 0};
    if (active) ws = wave_stream<false>(a, sub0, lane, has, win);
    __syncthreads();
    const uint64_t t1 = a.trace ? wall_clock64() : 0;
    bool bad = false;
    if (has) {
        const uint32_t pa = (uint32_t)((sub0 + lane) << 7);
        const uint32_t max_len = a.tab->max_len < 63u ? a.tab->max_len : 63u;
        // second level: width and first index (an empty table keeps one
        // zero entry; short codes' speculative reads land anywhere in LDS)
        const uint32_t b2 = a.tab->lut2_bits, base2 = a.tab->lut2_v0 << b2;
        uint4 *dst = a.qws + sub0 * 16 + lane;   // lane-interleaved groups
        uint32_t used;
        if (ws.whole && __all((int)sub128_full(a.g, pa)))
            used = inflate_codes<true, true>(a, win, ws.nwin, ws.wlo, ws.start, pa, dst, s_lut, s_lut2, b2, base2,
                                             max_len, bad);
        else if (ws.whole)
            used = inflate_codes<false, true>(a, win, ws.nwin, ws.wlo, ws.start, pa, dst, s_lut, s_lut2, b2, base2,
                                              max_len, bad);
        else
            used = inflate_codes<false, false>(a, win, ws.nwin, ws.wlo, ws.start, pa, dst, s_lut, s_lut2, b2, base2,
                                               max_len, bad);
        // the subchunk must lie inside the stream and consume exactly its recorded bits
        if (used != ws.bits || ws.start + ws.bits > 32ull * a.n_words) bad = true;
    }
    if (bad) {
        atomicOr(a.status, ST_ECORRUPT);
        publish_status(a.rb, ST_ECORRUPT);
    }
    if (a.trace && active && lane == 0) {
        const uint64_t t2 = wall_clock64();
        uint64_t *ph = const_cast<uint64_t *>(a.tab->phase);
        atomicMin((unsigned long long *)&ph[8], (unsigned long long)t0);
        atomicMax((unsigned long long *)&ph[9], (unsigned long long)t2);
        atomicAdd((unsigned long long *)&ph[10], (unsigned long long)(t1 - t0));
        atomicAdd((unsigned long long *)&ph[11], (unsigned long long)(t2 - t1));
    }
}

struct ReconArgs {
    Geom g;
    const uint4 *codes;         // u16 code per padded position, eight per 16 bytes
    const uint2 *exc;           // exception records {key = 2 pos + kind, payload}
    const uint32_t *unit_exc;   // first record of each 512-position unit (n_units + 1 entries)
    const DecodeTables *tab;
    float *out;
    uint32_t *status;
    Readback *rb;               // the call's readback block
    uint32_t n_exc, n_units, radius;
    float h;
};

// The lane's piece of the unit: eight consecutive positions 8 slot .. 8 slot + 7.
// 3D: lane = 8 z + y holds row y of plane z; 1D: lane = 4 b + q holds quarter q
// of block b; both in position order.  2D: lane = 32 b + 16 h + y holds half h
// of row y of block b (slot 32 b + 2 y + h), so each y-column is one 16-lane row.
template <uint32_t NDIM>
__device__ __forceinline__ uint32_t unit_slot(uint32_t lane) {
    return NDIM == 2 ? ((lane & 32u) | ((lane & 15u) << 1) | ((lane >> 4) & 1u)) : lane;
}
template <uint32_t NDIM>
__device__ __forceinline__ uint32_t slot_lane(uint32_t slot) {
    return NDIM == 2 ? ((slot & 32u) | ((slot & 1u) << 4) | ((slot >> 1) & 15u)) : slot;
}

// One unit: its lane piece d[] (deltas, outliers still 0) and code-0 mask,
// records [rs, re) of the exception list.
// The unit's records of one kind (outliers or patches) scattered into the
// wave's LDS buffer: buf[rel] their values, buf[512 ..) a bitmap of their
// positions; records load one per lane, 64 at a time.  Returns the lane's
// eight position bits (slot = the lane's piece of eight positions).
template <bool PATCH>
__device__ __forceinline__ uint32_t scatter_records(const ReconArgs &a, uint32_t rs, uint32_t re, uint32_t P0,
                                                    uint32_t lane, uint32_t slot, lds_u32 *buf, bool &bad,
                                                    uint32_t &n_kind) {
    if (lane < 16) buf[512 + lane] = 0u;   // (one wave: its LDS operations take effect in order)
    for (uint32_t base = rs; base < re; base += 64) {
        const uint32_t i = base + lane;
        if (i < re) {
            const uint2 r = a.exc[i];
            const uint32_t rel = (r.x >> 1) - P0;
            if (rel >= 512u) {
                if (!PATCH) bad = true;   // reported once
            } else if ((r.x & 1u) == (PATCH ? 1u : 0u)) {
                buf[rel] = r.y;
                __hip_atomic_fetch_or(&buf[512 + (rel >> 5)], 1u << (rel & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                n_kind++;
            }
        }
    }
    return (buf[512 + (slot >> 2)] >> ((slot & 3u) * 8u)) & 0xFFu;
}

template <uint32_t NDIM, uint32_t LAYERS>
__device__ __forceinline__ void recon_unit(const ReconArgs &a, uint32_t u, uint32_t lane, uint32_t (&d)[8],
                                           uint32_t zmask, uint32_t rs, uint32_t re, lds_u32 *buf, bool &bad) {
    const Geom &g = a.g;
    const uint32_t P0 = u << kUnitShift;
    if (rs > re || re > a.n_exc) {
        bad = true;
        rs = re = 0;
    }
    // outlier deltas; patches come last.  A unit with more than a few records
    // scatters them through the LDS buffer (records one per lane), the others
    // walk theirs as wave-uniform scalar loads
    const uint32_t slot = unit_slot<NDIM>(lane);
    const bool scatter = re - rs > kScatterMin;   // uniform
    uint32_t n_out = 0;
    if (scatter) {
        const uint32_t m = scatter_records<false>(a, rs, re, P0, lane, slot, buf, bad, n_out);
        if (m & ~zmask) bad = true;   // an outlier record on a code that is not 0
        if (m) {
#pragma unroll
            for (uint32_t k = 0; k < 8; k++)
                if ((m >> k) & 1u) d[k] = buf[8 * slot + k];
        }
        n_out = wave_sum<uint32_t>(n_out);
    } else {
        for (uint32_t i = rs; i < re; i++) {
            const uint2 r = a.exc[i];
            const uint32_t rel = (r.x >> 1) - P0;
            if (rel >= 512u) {
                bad = true;
                continue;
            }
            if (r.x & 1u) continue;
            n_out++;
            const uint32_t x = rel & 7u;
            if (lane == slot_lane<NDIM>(rel >> 3)) {
                if (!((zmask >> x) & 1u)) bad = true;
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    if (k == x) d[k] = r.y;
            }
        }
    }
    // every code 0 takes exactly one record (keys increase)
    if (wave_sum<uint32_t>(__popc(zmask)) != n_out) bad = true;

    // inverse Lorenzo prediction: inclusive prefix sums along every axis
    // (LAYERS times each), wrapping modulo 2^32 like the forward difference
#pragma unroll
    for (uint32_t l = 0; l < LAYERS; l++) {
#pragma unroll
        for (uint32_t x = 1; x < 8; x++) d[x] += d[x - 1];
        if (NDIM == 3) {
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) d[x] = seg_scan<8>(d[x], lane);
        } else if (NDIM == 2) {
            uint32_t ofe, efo;
            row_swap16(d[7], ofe, efo);   // the left half-row's total, for the right half
            const uint32_t left = ((lane >> 4) & 1u) ? ofe : 0u;
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) d[x] += left;
        } else {
            // exclusive prefix of the lane totals within the block's quad
            const uint32_t t = d[7], q4 = lane & 3u;
            const uint32_t s1 = quad_shr1(t);
            const uint32_t i1 = t + (q4 >= 1 ? s1 : 0u);
            const uint32_t s2 = quad_shr2(i1);
            const uint32_t ex = i1 + (q4 >= 2 ? s2 : 0u) - t;
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) d[x] += ex;
        }
    }
#pragma unroll
    for (uint32_t l = 0; l < LAYERS; l++) {
        if (NDIM == 3) {
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) d[x] = stride8_scan(d[x], lane);
        } else if (NDIM == 2) {
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) d[x] = seg_scan<16>(d[x], lane);
        }
    }
    float f[8];
#pragma unroll
    for (uint32_t x = 0; x < 8; x++) f[x] = dequant((int32_t)d[x], a.h);

    // output index of the lane's first position and how many of its eight lie in the field
    uint64_t o0 = 0;
    uint32_t cnt = 0;
    if (NDIM == 3) {
        const uint32_t Bx = u % g.nb[2], By = (u / g.nb[2]) % g.nb[1], Bz = u / (g.nb[2] * g.nb[1]);
        const uint32_t z = lane >> 3, y = lane & 7u;
        const uint32_t vx = min(8u, g.n[2] - 8 * Bx), vy = min(8u, g.n[1] - 8 * By), vz = min(8u, g.n[0] - 8 * Bz);
        cnt = (z < vz && y < vy) ? vx : 0u;
        o0 = ((uint64_t)(8 * Bz + z) * g.n[1] + 8 * By + y) * g.n[2] + 8 * Bx;
    } else if (NDIM == 2) {
        const uint32_t B = 2 * u + (lane >> 5), y = lane & 15u, xh = (lane >> 4) & 1u;
        if (B < g.nb[1] * g.nb[2]) {
            const uint32_t Bx = B % g.nb[2], By = B / g.nb[2];
            const uint32_t vx = min(16u, g.n[2] - 16 * Bx), vy = min(16u, g.n[1] - 16 * By);
            cnt = (y < vy && vx > 8 * xh) ? min(8u, vx - 8 * xh) : 0u;
            o0 = (uint64_t)(16 * By + y) * g.n[2] + 16 * Bx + 8 * xh;
        }
    } else {
        o0 = (uint64_t)P0 + 8 * lane;
        cnt = g.nelem > o0 ? (g.nelem - o0 < 8 ? (uint32_t)(g.nelem - o0) : 8u) : 0u;
    }
    // patches replace the lane's values before they are stored
    if (scatter) {
        uint32_t n_patch = 0;
        const uint32_t m = scatter_records<true>(a, rs, re, P0, lane, slot, buf, bad, n_patch);
        if (m >> cnt) bad = true;   // a patch outside the field
        if (m) {
#pragma unroll
            for (uint32_t k = 0; k < 8; k++)
                if ((m >> k) & 1u) f[k] = __uint_as_float(buf[8 * slot + k]);
        }
    } else {
        for (uint32_t i = rs; i < re; i++) {
            const uint2 r = a.exc[i];
            if (!(r.x & 1u)) continue;
            const uint32_t rel = (r.x >> 1) - P0;
            if (rel >= 512u) continue;   // reported above
            const uint32_t x = rel & 7u;
            if (lane == slot_lane<NDIM>(rel >> 3)) {
                if (x >= cnt) bad = true;   // a patch outside the field
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    if (k == x) f[k] = __uint_as_float(r.y);
            }
        }
    }
    float *o = a.out + o0;
    const bool vec = ((reinterpret_cast<uintptr_t>(a.out) & 15u) == 0) && (NDIM == 1 || (g.n[2] & 3u) == 0);
    if (cnt == 8 && vec) {
        reinterpret_cast<float4 *>(o)[0] = make_float4(f[0], f[1], f[2], f[3]);
        reinterpret_cast<float4 *>(o)[1] = make_float4(f[4], f[5], f[6], f[7]);
    } else {
#pragma unroll
        for (uint32_t x = 0; x < 8; x++)
            if (x < cnt) o[x] = f[x];
    }
}

// 3D units: the lane's x-row piece (x-prefix in-lane) goes through an LDS
// copy of the block twice, so that the y and then the z prefix are in-lane
// too: lane 8 z + x holds a y-column, then lane 8 y + x a z-column.  Rows of
// the copy are 9 words apart (bank spread for the column reads).
template <uint32_t LAYERS>
__device__ __forceinline__ void recon_block3(const ReconArgs &a, uint32_t u, uint32_t lane, uint32_t (&d)[8],
                                             uint32_t zmask, uint32_t rs, uint32_t re, lds_u32 *blk, bool &bad) {
    const Geom &g = a.g;
    const uint32_t P0 = u << kUnitShift;
    if (rs > re || re > a.n_exc) {
        bad = true;
        rs = re = 0;
    }
    const bool any_rec = rs < re;
    uint32_t n_out = 0;
    if (any_rec) {
        for (uint32_t i = rs; i < re; i++) {
            const uint2 r = a.exc[i];
            const uint32_t rel = (r.x >> 1) - P0;
            if (rel >= 512u) {
                bad = true;
                continue;
            }
            if (r.x & 1u) continue;
            n_out++;
            const uint32_t x = rel & 7u;
            if (lane == (rel >> 3)) {
                if (!((zmask >> x) & 1u)) bad = true;
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    if (k == x) d[k] = r.y;
            }
        }
    }
    // every code 0 takes exactly one record (keys increase)
    if (__any((int)(zmask != 0)) || any_rec) {
        uint32_t nz = 0;
#pragma unroll
        for (uint32_t x = 0; x < 8; x++) nz += (uint32_t)__popcll(__ballot((int)((zmask >> x) & 1u)));
        if (nz != n_out) bad = true;
    }
    // x in-lane (lane = 8 z + y); the sums wrap modulo 2^32 like the
    // forward difference; LAYERS prefix sums along each axis
#pragma unroll
    for (uint32_t l = 0; l < LAYERS; l++)
#pragma unroll
        for (uint32_t x = 1; x < 8; x++) d[x] += d[x - 1];
    const uint32_t hi = lane >> 3, lo = lane & 7u;
#pragma unroll
    for (uint32_t x = 0; x < 8; x++) blk[72 * hi + 9 * lo + x] = d[x];   // (z, y) = (hi, lo)
    // a wave's LDS accesses complete in order; the barriers keep the compiler
    // from moving the column reads above the other lanes' writes
    __builtin_amdgcn_wave_barrier();
    // y: lane 8 z + x reads the column (z, ., x)
#pragma unroll
    for (uint32_t y = 0; y < 8; y++) d[y] = blk[72 * hi + 9 * y + lo];
#pragma unroll
    for (uint32_t l = 0; l < LAYERS; l++)
#pragma unroll
        for (uint32_t y = 1; y < 8; y++) d[y] += d[y - 1];
#pragma unroll
    for (uint32_t y = 0; y < 8; y++) blk[72 * hi + 9 * y + lo] = d[y];
    __builtin_amdgcn_wave_barrier();
    // z: lane 8 y + x reads the column (., y, x)
#pragma unroll
    for (uint32_t z = 0; z < 8; z++) d[z] = blk[72 * z + 9 * hi + lo];
#pragma unroll
    for (uint32_t l = 0; l < LAYERS; l++)
#pragma unroll
        for (uint32_t z = 1; z < 8; z++) d[z] += d[z - 1];
    float f[8];
#pragma unroll
    for (uint32_t z = 0; z < 8; z++) f[z] = dequant((int32_t)d[z], a.h);
    // lane (y, x) = (hi, lo) holds the z-column
    const uint32_t Bx = u % g.nb[2], By = (u / g.nb[2]) % g.nb[1], Bz = u / (g.nb[2] * g.nb[1]);
    const uint32_t vx = min(8u, g.n[2] - 8 * Bx), vy = min(8u, g.n[1] - 8 * By), vz = min(8u, g.n[0] - 8 * Bz);
    const bool in_col = hi < vy && lo < vx;
    if (any_rec) {
        for (uint32_t i = rs; i < re; i++) {
            const uint2 r = a.exc[i];
            if (!(r.x & 1u)) continue;
            const uint32_t rel = (r.x >> 1) - P0;
            if (rel >= 512u) continue;   // reported above
            const uint32_t z = rel >> 6;
            if (lane == (rel & 63u)) {
                if (!in_col || z >= vz) bad = true;   // a patch outside the field
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    if (k == z) f[k] = __uint_as_float(r.y);
            }
        }
    }
    if (in_col) {
        const uint64_t plane = (uint64_t)g.n[1] * g.n[2];
        float *o = a.out + ((uint64_t)(8 * Bz) * g.n[1] + 8 * By + hi) * g.n[2] + 8 * Bx + lo;
#pragma unroll
        for (uint32_t z = 0; z < 8; z++)
            if (z < vz) o[z * plane] = f[z];
    }
}

// One unit per wave.
template <uint32_t NDIM, uint32_t LAYERS>
__global__ __launch_bounds__(64 * kReconWaves) void k_recon(ReconArgs a) {
    __shared__ uint32_t s_blk[kReconWaves][576];   // 3D: the block, rows 9 words apart; 1D/2D: the records
    if (a.tab->status) return;   // the inflate kernel did not run
    const uint32_t lane = lane_id(), w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const uint32_t u = blockIdx.x * kReconWaves + w;
    if (u >= a.n_units) return;   // whole waves
    const uint32_t slot = unit_slot<NDIM>(lane);
    // group slot % 16 of subchunk 4 u + slot / 16, lane-interleaved by wave of 64 subchunks
    const uint4 q = a.codes[((uint64_t)(u >> 4) * 16 + (slot & 15u)) * 64 + (u & 15u) * 4 + (slot >> 4)];
    // (clamped: a damaged list leaves the index meaningless, never out of range)
    const uint32_t re = min(a.unit_exc[u + 1], a.n_exc), rs = min(a.unit_exc[u], re);
    const uint32_t R = a.radius;
    const bool lv = (u << kUnitShift) + 8 * slot < a.g.padded;
    uint32_t d[8];   // wrapping deltas
    uint32_t zmask = 0;   // code 0: an outlier
    {
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (uint32_t m = 0; m < 4; m++) {
            const uint32_t c0 = w4[m] & 0xFFFFu, c1 = w4[m] >> 16;
            d[2 * m] = lv ? c0 - R : 0u;
            d[2 * m + 1] = lv ? c1 - R : 0u;
            zmask |= ((lv && c0 == 0) ? 1u : 0u) << (2 * m);
            zmask |= ((lv && c1 == 0) ? 1u : 0u) << (2 * m + 1);
        }
    }
    bool bad = false;
    if (NDIM == 3) recon_block3<LAYERS>(a, u, lane, d, zmask, rs, re, (lds_u32 *)s_blk[w], bad);
    else recon_unit<NDIM, LAYERS>(a, u, lane, d, zmask, rs, re, (lds_u32 *)s_blk[w], bad);
    if (bad) {
        atomicOr(a.status, ST_ECORRUPT);
        publish_status(a.rb, ST_ECORRUPT);
    }
}

static uint32_t decode_waves(const Layout &L) { return L.sub_size <= 256 ? kDecMaxWaves : 1u; }

constexpr size_t kDecLdsLimit = 160 * 1024;       // LDS one workgroup may allocate on gfx950
constexpr uint32_t kDecWinWordsMax = 2688;        // 10.5 KiB stream window per wave (64 subchunks of 128 at ~9.5 bits)

static size_t decode_lds_fixed(const Layout &L) {
    return sizeof(uint16_t) * ((1u << kLutBits) + L.nsym + (size_t)decode_waves(L) * 64 * (L.sub_size + 2)) +
           sizeof(uint32_t) * decode_waves(L) * kDecXp + sizeof(DecLds);
}

// stream-window words per wave: the cap, or what the LDS left over allows
static uint32_t decode_win_words(const Layout &L) {
    const size_t fixed = decode_lds_fixed(L);
    const size_t left = fixed < kDecLdsLimit ? (kDecLdsLimit - fixed) / (4 * decode_waves(L)) : 0;
    const uint32_t w = left < kDecWinWordsMax ? (uint32_t)left : kDecWinWordsMax;
    return w & ~63u;
}

size_t decode_lds_bytes(const Layout &L) {
    return decode_lds_fixed(L) - sizeof(DecLds) + 4ull * decode_waves(L) * decode_win_words(L);
}

// Dynamic LDS limits of the decoding kernels, set once per device before any
// launch (not between launches, so that a stream capture holds launches only).
hipError_t decode_kernel_attributes() {
    // the dynamic allowance is what the CU's LDS leaves beside the kernel's
    // static arrays (the LDS tables of k_inflate128, the shared block of k_decode)
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, (const void *)k_inflate128);
    if (e != hipSuccess) return e;
    const size_t inf_dyn = 4ull * kInfMaxWaves * kInfWin;
    if (fa.sharedSizeBytes + inf_dyn > kDecLdsLimit) return hipErrorInvalidConfiguration;
    e = hipFuncSetAttribute((const void *)k_inflate128, hipFuncAttributeMaxDynamicSharedMemorySize, (int)inf_dyn);
    if (e != hipSuccess) return e;
    e = hipFuncGetAttributes(&fa, (const void *)k_decode);
    if (e != hipSuccess) return e;
    if (fa.sharedSizeBytes > sizeof(DecLds)) return hipErrorInvalidConfiguration;   // decode_lds_bytes assumes it
    return hipFuncSetAttribute((const void *)k_decode, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kDecLdsLimit - fa.sharedSizeBytes));
}

void launch_decode(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint64_t off_str,
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out, bool trace,
                   uint4 *qws, Readback *rb, int ncu) {
    DecArgs a;
    a.g = g;
    a.L = L;
    a.archive = archive;
    a.words = reinterpret_cast<const uint32_t *>(n_words ? archive + off_str : archive);
    a.n_words = n_words;
    a.last_word = n_words ? n_words - 1 : 0;
    a.exc = reinterpret_cast<const uint2 *>(archive + L.off_exc);
    a.n_exc = n_exc;
    a.tab = tab;
    a.status = &tab->status;
    a.out = out;
    a.h = h;
    a.wave_tasks = (L.n_sub + 63) / 64;
    a.qstride = L.sub_size + 2;
    a.win_words = decode_win_words(L);
    a.trace = trace ? 1u : 0u;
    a.qws = qws;
    a.rb = rb;
    if (a.wave_tasks == 0) return;
    if (L.sub_size == 128 && qws) {
        // codes only; launch_recon finishes
        a.win_words = kInfWin;
        // one workgroup per CU, waves spread evenly over the CUs
        const uint32_t cus = ncu > 0 ? (uint32_t)ncu : 256u;
        uint32_t waves = (a.wave_tasks + cus - 1) / cus;
        waves = waves < 1 ? 1 : (waves > kInfMaxWaves ? kInfMaxWaves : waves);
        const uint32_t blocks = (a.wave_tasks + waves - 1) / waves;
        const size_t lds = 4ull * waves * kInfWin;   // the windows (the tables are static)
        hipLaunchKernelGGL(k_inflate128, dim3(blocks), dim3(64 * waves), lds, s, a);
        return;
    }

    const uint32_t waves = decode_waves(L);
    const uint32_t blocks = (a.wave_tasks + waves - 1) / waves;
    const size_t lds = decode_lds_bytes(L);
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(64 * waves), lds, s, a);
}

void launch_recon(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint32_t n_exc, float h,
                  const DecodeTables *tab, const uint4 *qws, const uint32_t *unit_exc, float *out, Readback *rb) {
    ReconArgs a;
    a.g = g;
    a.codes = qws;
    a.exc = reinterpret_cast<const uint2 *>(archive + L.off_exc);
    a.unit_exc = unit_exc;
    a.tab = tab;
    a.out = out;
    a.status = const_cast<uint32_t *>(&tab->status);
    a.rb = rb;
    a.n_exc = n_exc;
    a.n_units = recon_units(g);
    a.radius = L.radius;
    a.h = h;
    if (a.n_units == 0) return;
    const uint32_t blocks = (a.n_units + kReconWaves - 1) / kReconWaves;
    const dim3 grid(blocks), block(64 * kReconWaves);
    if (L.layers == 2) {
        if (g.ndim == 3) hipLaunchKernelGGL((k_recon<3, 2>), grid, block, 0, s, a);
        else if (g.ndim == 2) hipLaunchKernelGGL((k_recon<2, 2>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_recon<1, 2>), grid, block, 0, s, a);
    } else {
        if (g.ndim == 3) hipLaunchKernelGGL((k_recon<3, 1>), grid, block, 0, s, a);
        else if (g.ndim == 2) hipLaunchKernelGGL((k_recon<2, 1>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_recon<1, 1>), grid, block, 0, s, a);
    }
}

}  // namespace dqz
