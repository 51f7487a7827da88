// kernels_decode.hip -- inflate + reversed dual-quantization (Sec. 3.3).
//
// One wave decodes 64 consecutive subchunks, one per lane: the lane starts
// at the subchunk's bit offset (chunk offset + prefix of subchunk bit
// counts) and decodes every point of the subchunk with a 2^12-entry LDS
// lookup table (longer codes by the canonical first-code rule) into an LDS
// code buffer.  The wave then marks outliers in that buffer from the sorted
// exception list, and reconstructs each block: the inverse of the Lorenzo
// mixed difference is a prefix sum along every axis (Algorithm 2's cascading
// reconstruction, reorganised), done in registers along the slow axis and
// with cross-lane scans along the fast axes, in wrapping int32.  Values are
// dequantized as fl32(d°) * fl32(2 eb) and written row-major; patches
// (verbatim values) are applied last.
#include "dqz_internal.h"

namespace dqz {

// LDS-typed pointers: every access through them is a ds_* instruction (a
// generic pointer could be merged with a global one into a flat access)
typedef __attribute__((address_space(3))) uint16_t lds_u16;
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
    uint32_t *hstatus;  // status word in pinned host memory, read after the stream ends
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

// Decode one symbol from the top of `cur` (more than 32 valid bits, so every
// code of up to 32 bits is present); `used` counts the lane's consumed bits.
// Codes longer than 32 bits (possible only when max_len > 32) are read from
// a fresh 64-bit window in memory and set `reinit`: the caller then restarts
// its reader at the new position.
__device__ __forceinline__ uint32_t decode_sym(const DecArgs &a, uint64_t &cur, int32_t &avail, uint32_t &used,
                                               uint64_t start, const lds_u16 *lut, const DecLds &t,
                                               const lds_u16 *sorted, uint32_t max_len, bool &bad, bool &reinit) {
    const uint32_t e = lut[(uint32_t)(cur >> (64 - kLutBits))];
    uint32_t len, sym;
    if (!(e & 0x8000u)) {
        len = e >> 11;
        sym = e & 0x7FFu;
        if (len == 0) { bad = true; len = 1; }
    } else {
        // a longer code: canonical limits from the shortest possible length
        uint32_t l = e & 63u;
        uint64_t win = cur;
        if (max_len > 32) {
            const uint64_t bp = start + used;
            const uint64_t w = bp >> 5;
            const uint32_t o = (uint32_t)(bp & 31u);
            const uint64_t hi = ((uint64_t)ld_word(a, w) << 32) | ld_word(a, w + 1);
            win = o ? ((hi << o) | (ld_word(a, w + 2) >> (32 - o))) : hi;
        }
        while (l < max_len && win >= t.limit[l]) l++;
        const uint64_t c = win >> (64 - l);
        const uint64_t idx = t.first_index[l] + (c - t.first_code[l]);
        if (idx >= a.L.nsym) { bad = true; sym = a.L.radius; }
        else sym = sorted[idx];
        len = l;
        if ((int32_t)l > avail) {   // only possible for codes over 32 bits
            used += l;
            reinit = true;
            return sym;
        }
    }
    cur <<= len;
    avail -= (int32_t)len;
    used += len;
    return sym;
}

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
};
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
    const uint32_t cap = a.win_words / 17 * 16;   // logical words whose padded slots fit
    r.nwin = whi > r.wlo ? (uint32_t)(whi - r.wlo < cap ? whi - r.wlo : cap) : 0u;
    for (uint32_t b = 0; b < r.nwin; b += 64 * 8) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) v[j] = ld_word(a, r.wlo + b + j * 64 + lane);
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t k = b + j * 64 + lane;
            if (k < r.nwin) win[win_slot(k)] = v[j];
        }
    }
    return r;
}

// ---- reconstruction for subchunks of 128 positions, in registers ----------
//
// The lane reads back its own 128 codes.  In 3D they are two z-planes of one
// 8^3 block, and the block's four subchunks sit in one DPP quad: the 2D
// prefix sums of each plane are in-lane, the z prefix crosses the quad by two
// lane shifts.  In 2D they are 8 rows of a 16^2 block (a lane pair per block);
// in 1D four whole 32-blocks, all in-lane.

// lane j - 1 (j - 2) of the lane's quad; quad_perm [0,0,1,2] and [0,0,0,1]
__device__ __forceinline__ uint32_t quad_shr1(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x90, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t quad_shr2(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x40, 0xF, 0xF, false));
}
// lanes 1 and 3 of the quad receive lanes 0 and 2: quad_perm [0,0,2,2]
__device__ __forceinline__ uint32_t quad_pair_lo(uint32_t v) {
    return pinned((uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xA0, 0xF, 0xF, false));
}

// The lane's 128 deltas from its codes in the LDS code buffer (outlier slots
// marked with their index in the exception list).
__device__ __forceinline__ void deltas_from_lds(const DecArgs &a, const lds_u16 *wq, uint32_t lane, uint32_t e0,
                                                const lds_u32 *xp, bool has, bool &bad, int32_t (&v)[128]) {
    const uint32_t R = a.L.radius;
    // the lane's codes: 64 aligned pairs (the code-buffer stride is even)
    const lds_u32 *src = (const lds_u32 *)(wq + lane * a.qstride);
    uint32_t special = 0;
#pragma unroll
    for (uint32_t k = 0; k < 64; k++) {
        const uint32_t two = has ? src[k] : (R | (R << 16));
        const uint32_t q0 = two & 0xFFFFu, q1 = two >> 16;
        v[2 * k] = (int32_t)q0 - (int32_t)R;
        v[2 * k + 1] = (int32_t)q1 - (int32_t)R;
        // code 0 (an unmarked outlier) or a marked outlier slot
        special |= ((q0 - 1u) >= 0x7FFFu ? 1u : 0u) | ((q1 - 1u) >= 0x7FFFu ? 1u : 0u);
    }
    if (special) {
#pragma unroll
        for (uint32_t i = 0; i < 128; i++) {
            const uint32_t q = (uint32_t)(v[i] + (int32_t)R);
            if (q & 0x8000u) v[i] = (int32_t)slot_delta(a, (uint16_t)q, e0, xp, bad);
            else if (q == 0) bad = true;
        }
    }
}

// Reconstruction of the lane's 128 deltas in place, dequantization and the
// stores of its in-field values.  Called by whole active waves (the
// cross-lane steps need every lane).
template <uint32_t NDIM>
__device__ __forceinline__ void recon128(const DecArgs &a, int32_t (&v)[128], uint32_t lane, uint32_t P0, bool has) {
    const Geom &g = a.g;
    const float h = a.h;
    const uint32_t pa = P0 + lane * 128u;
    const uint32_t n1 = g.n[1], n2 = g.n[2];
    const bool vec = (n2 % 4u == 0) && ((reinterpret_cast<uintptr_t>(a.out) & 15u) == 0);
    if (NDIM == 3) {
        const uint32_t blk = pa >> 9;
        const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
        const uint32_t vx = min(8u, n2 - 8 * Bx), vy = min(8u, n1 - 8 * By), vz = min(8u, g.n[0] - 8 * Bz);
#pragma unroll
        for (uint32_t zi = 0; zi < 2; zi++) {
#pragma unroll
            for (uint32_t y = 0; y < 8; y++)
#pragma unroll
                for (uint32_t x = 1; x < 8; x++) v[zi * 64 + y * 8 + x] += v[zi * 64 + y * 8 + x - 1];
#pragma unroll
            for (uint32_t y = 1; y < 8; y++)
#pragma unroll
                for (uint32_t x = 0; x < 8; x++) v[zi * 64 + y * 8 + x] += v[zi * 64 + (y - 1) * 8 + x];
        }
        // z prefix across the quad, one row of the two planes at a time; each
        // row is stored as soon as it is final (keeps few rows live)
        const uint32_t jq = lane & 3u, z0 = 2 * jq;
        const bool okA = has && z0 < vz, okB = has && z0 + 1 < vz;
        float *oA = a.out + ((8ull * Bz + z0) * n1 + 8 * By) * n2 + 8 * Bx;
        float *oB = oA + (uint64_t)n1 * n2;
#pragma unroll
        for (uint32_t y = 0; y < 8; y++) {
#pragma unroll
            for (uint32_t x = 0; x < 8; x++) {
                const uint32_t k = y * 8 + x;
                const uint32_t b = (uint32_t)(v[64 + k] + v[k]);   // planes 2j and 2j + 1
                const uint32_t s1 = quad_shr1(b);
                const uint32_t t1 = b + (jq >= 1 ? s1 : 0u);
                const uint32_t s2 = quad_shr2(t1);
                const uint32_t t = t1 + (jq >= 2 ? s2 : 0u);       // inclusive over the quad
                v[k] += (int32_t)(t - b);
                v[64 + k] = (int32_t)t;
            }
            if (y < vy) {
#pragma unroll
                for (uint32_t zi = 0; zi < 2; zi++) {
                    if (!(zi ? okB : okA)) continue;
                    float *o = (zi ? oB : oA) + (uint64_t)y * n2;
                    const uint32_t r = zi * 64 + y * 8;
                    if (vx == 8 && vec) {
                        reinterpret_cast<float4 *>(o)[0] = make_float4(dequant(v[r], h), dequant(v[r + 1], h),
                                                                       dequant(v[r + 2], h), dequant(v[r + 3], h));
                        reinterpret_cast<float4 *>(o)[1] = make_float4(dequant(v[r + 4], h), dequant(v[r + 5], h),
                                                                       dequant(v[r + 6], h), dequant(v[r + 7], h));
                    } else {
#pragma unroll
                        for (uint32_t x = 0; x < 8; x++)
                            if (x < vx) o[x] = dequant(v[r + x], h);
                    }
                }
            }
        }
    } else if (NDIM == 2) {
        const uint32_t blk = pa >> 8;
        const uint32_t Bx = blk % g.nb[2], By = blk / g.nb[2];
        const uint32_t vx = min(16u, n2 - 16 * Bx), vy = min(16u, n1 - 16 * By);
#pragma unroll
        for (uint32_t y = 0; y < 8; y++)
#pragma unroll
            for (uint32_t x = 1; x < 16; x++) v[y * 16 + x] += v[y * 16 + x - 1];
#pragma unroll
        for (uint32_t y = 1; y < 8; y++)
#pragma unroll
            for (uint32_t x = 0; x < 16; x++) v[y * 16 + x] += v[(y - 1) * 16 + x];
        const uint32_t j2 = lane & 1u;
#pragma unroll
        for (uint32_t x = 0; x < 16; x++) {
            const uint32_t lower = quad_pair_lo((uint32_t)v[7 * 16 + x]);   // the lower half-block's column sums
            const int32_t add = j2 ? (int32_t)lower : 0;
#pragma unroll
            for (uint32_t y = 0; y < 8; y++) v[y * 16 + x] += add;
        }
        if (!has) return;
        const uint32_t y0 = 8 * j2;
#pragma unroll
        for (uint32_t y = 0; y < 8; y++) {
            if (y0 + y >= vy) continue;
            float *o = a.out + (uint64_t)(16 * By + y0 + y) * n2 + 16 * Bx;
            const uint32_t r = y * 16;
            if (vx == 16 && vec) {
#pragma unroll
                for (uint32_t qd = 0; qd < 4; qd++)
                    reinterpret_cast<float4 *>(o)[qd] =
                        make_float4(dequant(v[r + 4 * qd], h), dequant(v[r + 4 * qd + 1], h),
                                    dequant(v[r + 4 * qd + 2], h), dequant(v[r + 4 * qd + 3], h));
            } else {
#pragma unroll
                for (uint32_t x = 0; x < 16; x++)
                    if (x < vx) o[x] = dequant(v[r + x], h);
            }
        }
    } else {
#pragma unroll
        for (uint32_t i = 1; i < 128; i++)
            if (i & 31u) v[i] += v[i - 1];
        if (!has) return;
        float *o = a.out + pa;
        const uint64_t c64 = g.nelem > pa ? g.nelem - pa : 0;
        if (c64 >= 128 && ((reinterpret_cast<uintptr_t>(a.out) & 15u) == 0)) {
#pragma unroll
            for (uint32_t qd = 0; qd < 32; qd++)
                reinterpret_cast<float4 *>(o)[qd] = make_float4(dequant(v[4 * qd], h), dequant(v[4 * qd + 1], h),
                                                                dequant(v[4 * qd + 2], h), dequant(v[4 * qd + 3], h));
        } else {
            const uint32_t c = (uint32_t)c64;
#pragma unroll
            for (uint32_t i = 0; i < 128; i++)
                if (i < c) o[i] = dequant(v[i], h);
        }
    }
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
        const WaveStream ws = wave_stream(a, sub0, lane, has, win);
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
        if (used != bits_s) bad = true;
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
    if (active && S == 128) {
        int32_t v[128];
        deltas_from_lds(a, wq, lane, e0, xp, has, bad, v);
        if (a.g.ndim == 3) recon128<3>(a, v, lane, (uint32_t)P0, has);
        else if (a.g.ndim == 2) recon128<2>(a, v, lane, (uint32_t)P0, has);
        else recon128<1>(a, v, lane, (uint32_t)P0, has);
    } else if (active) {
        const Geom &g = a.g;
        const float h = a.h;
        auto qat = [&](uint64_t loc) -> uint16_t { return wq[(loc >> sh) * a.qstride + (loc & (S - 1))]; };
        if (g.ndim == 3) {
            const uint32_t ly = lane / 8, lx = lane % 8;
            const uint32_t bfirst = (uint32_t)(P0 / 512), blast = (uint32_t)((P1 - 1) / 512);
            for (uint32_t blk = bfirst; blk <= blast; blk++) {
                const uint64_t base = (uint64_t)blk * 512 - P0;
                uint32_t v[8];
                uint32_t run = 0;
#pragma unroll
                for (uint32_t z = 0; z < 8; z++) {
                    run += slot_delta(a, qat(base + z * 64 + lane), e0, xp, bad);
                    v[z] = run;
                }
#pragma unroll
                for (uint32_t z = 0; z < 8; z++) v[z] = seg_scan<8>(stride8_scan(v[z], lane), lane);
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
                uint32_t col = 0;
                for (uint32_t y = 0; y < 16; y++) {
                    if (ok) col += slot_delta(a, qat(base + y * 16 + lx), e0, xp, bad);
                    const uint32_t t = seg_scan<16>(col, lane);
                    const uint32_t yy = By * 16 + y;
                    if (ok && x < g.n[2] && yy < g.n[1]) a.out[(uint64_t)yy * g.n[2] + x] = dequant((int32_t)t, h);
                }
            }
        } else {
            for (uint64_t off = 0; P0 + off < P1; off += 64) {
                const uint64_t loc = off + lane;
                const uint64_t p = P0 + loc;
                const uint32_t t = seg_scan<32>((p < P1) ? slot_delta(a, qat(loc), e0, xp, bad) : 0u, lane);
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
        *a.hstatus = ST_ECORRUPT;
    }
    if (a.trace && active && lane == 0) {
        tm[6] = wall_clock64();
        uint64_t *ph = const_cast<uint64_t *>(a.tab->phase);
        atomicMin((unsigned long long *)&ph[8], (unsigned long long)tm[0]);
        atomicMax((unsigned long long *)&ph[9], (unsigned long long)tm[6]);
        for (int k = 0; k < 6; k++) atomicAdd((unsigned long long *)&ph[10 + k], (unsigned long long)(tm[k + 1] - tm[k]));
    }
}

constexpr uint32_t kG128Waves = 4;       // waves per workgroup (they share the lookup table)
constexpr uint32_t kG128Win = 2432;      // LDS stream-window slots per wave (9.5 KiB)
constexpr uint32_t kG128Out = 512;       // outlier records staged per wave (position u16 + delta u32)
constexpr uint32_t kG128Pat = 128;       // patch records staged per wave (position u16 + value u32)

// The lane's 128 deltas from its codes in the workspace slot; outliers (code
// 0) take their deltas from the wave's staged outlier list, or from the
// archive's exception list when the wave had more outliers than were staged.
// Every outlier record must be used exactly once.
__device__ __forceinline__ void deltas_from_slot(const DecArgs &a, const uint4 *qslot, uint32_t lane, uint32_t P0,
                                                 uint32_t e0, uint32_t e1, uint32_t n_out, const lds_u16 *opos,
                                                 const lds_u32 *oval, uint32_t cap, bool has, bool &bad,
                                                 int32_t (&v)[128]) {
    const uint32_t R = a.L.radius;
    uint32_t zero = 0;
    if (has) {
        // all sixteen loads issue before any is used
        uint4 q[16];
#pragma unroll
        for (uint32_t g = 0; g < 16; g++) q[g] = qslot[g * 64];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t g = 0; g < 16; g++) {
            const uint4 q4 = q[g];
            const uint32_t u[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t q0 = u[k] & 0xFFFFu, q1 = u[k] >> 16;
                v[8 * g + 2 * k] = (int32_t)q0 - (int32_t)R;
                v[8 * g + 2 * k + 1] = (int32_t)q1 - (int32_t)R;
                zero |= (q0 == 0 ? 1u : 0u) | (q1 == 0 ? 1u : 0u);
            }
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < 128; i++) v[i] = 0;
    }
    uint32_t hits = 0;
    if (zero) {
        const uint32_t rel0 = lane * 128u;
        const bool ovf = n_out > cap;
        uint32_t oc;
        {
            uint32_t lo = ovf ? e0 : 0u, hi = ovf ? e1 : n_out;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                const bool below = ovf ? ((uint64_t)a.exc[mid].x < 2ull * (P0 + rel0)) : (opos[mid] < rel0);
                if (below) lo = mid + 1; else hi = mid;
            }
            oc = lo;
        }
#pragma unroll
        for (uint32_t i = 0; i < 128; i++) {
            if (v[i] != -(int32_t)R) continue;   // code 0 marks an outlier
            int32_t d = 0;
            if (!ovf) {
                if (oc < n_out && opos[oc] == rel0 + i) d = (int32_t)oval[oc];
                else bad = true;
            } else {
                while (oc < e1 && (a.exc[oc].x & 1u)) oc++;
                if (oc < e1 && (a.exc[oc].x >> 1) == P0 + rel0 + i) d = (int32_t)a.exc[oc].y;
                else bad = true;
            }
            v[i] = d;
            oc++;
            hits++;
        }
    }
    if (wave_sum<uint32_t>(hits) != n_out) bad = true;
}

template <uint32_t NDIM>
__device__ __forceinline__ void recon128g(const DecArgs &a, const uint4 *qslot, uint32_t lane, uint32_t P0, uint32_t e0,
                                          uint32_t e1, uint32_t n_out, const lds_u16 *opos, const lds_u32 *oval,
                                          bool has, bool &bad) {
    int32_t v[128];
    deltas_from_slot(a, qslot, lane, P0, e0, e1, n_out, opos, oval, kG128Out, has, bad, v);
    recon128<NDIM>(a, v, lane, P0, has);
}

// ---------------------------------------------------------------------------
// Decoder for subchunks of 128 positions (the default S) without an LDS code
// buffer.  Each lane's codes go to a per-subchunk slot of a workspace array
// (eight codes per 16-byte store) and come back to the same lane for the
// register reconstruction, which also substitutes the lane's outliers from
// the wave's staged outlier list.  Only the lookup tables, the stream window
// and the staged outliers stay in LDS, so workgroups of four waves fit two
// per CU (two waves per SIMD).
// ---------------------------------------------------------------------------

// Inflate the lane's 128 positions into 16 packed 16-byte groups dst[64 g].
// Same steps as inflate(); the inner loop over a group of eight positions is
// unrolled so that the codes pack into registers.
__device__ __forceinline__ uint32_t inflate128(const DecArgs &a, const lds_u32 *win, uint32_t nwin, uint64_t wlo,
                                               uint64_t start, uint32_t pa, uint4 *dst, const lds_u16 *lut,
                                               const DecLds &t, const lds_u16 *sorted, uint32_t max_len, bool &bad) {
    const uint64_t sw = start >> 5;
    const uint32_t relw = (sw >= wlo && sw - wlo < nwin) ? (uint32_t)(sw - wlo) : nwin;
    const uint32_t wlast = nwin ? nwin - 1 : 0;
    // Words read off the fast path are waited for where they are read: a
    // global load left pending into the loop would make every step wait for
    // all vector memory traffic, the previous group's store included.
    auto word = [&](uint32_t kr) -> uint32_t {
        const uint32_t k = relw + kr;
        return pinned((k < nwin) ? win[win_slot(k)] : ld_word(a, sw + kr));
    };
    auto gword = [&](uint64_t i) -> uint32_t { return pinned(ld_word(a, i)); };
    const uint32_t R = a.L.radius;
    uint32_t used = 0, kr = 2;
    uint32_t o = (uint32_t)(start & 31u);
    uint64_t cur = (((uint64_t)word(0) << 32) | word(1)) << o;
    int32_t avail = 64 - (int32_t)o;
    uint32_t nxt = word(kr);
    uint32_t rmask = 0;
    for (uint32_t g = 0; g < 16; g++) {
        if ((g & 3u) == 0) rmask = real_mask32(a.g, pa + g * 8);
        uint32_t pk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const bool need = avail <= 32;
            const uint32_t shl = need ? (uint32_t)(32 - avail) : 0u;
            cur |= need ? ((uint64_t)nxt << shl) : 0ull;
            avail += need ? 32 : 0;
            kr += need ? 1u : 0u;
            const uint32_t k = relw + kr;
            nxt = win[win_slot(k < nwin ? k : wlast)];
            const bool real = (rmask >> ((g & 3u) * 8 + j)) & 1u;
            const uint32_t e = lut[(uint32_t)(cur >> (64 - kLutBits))];
            uint32_t len = (e >> 11) & 15u, sym = e & 0x7FFu;
            const bool slow = real && ((e & 0x8000u) || len == 0);
            bool moved = false;
            if (__any((int)(slow || k >= nwin))) {
                if (k >= nwin) nxt = gword(sw + kr);
                if (slow && !(e & 0x8000u)) {   // no code starts with these bits
                    bad = true;
                    len = 1;
                    sym = R;
                } else if (slow) {
                    uint32_t l = e & 63u;
                    uint64_t wv = cur;
                    if (max_len > 32) {
                        const uint64_t bp = start + used;
                        const uint64_t ww = bp >> 5;
                        const uint32_t ob = (uint32_t)(bp & 31u);
                        const uint64_t h2 = ((uint64_t)gword(ww) << 32) | gword(ww + 1);
                        wv = ob ? ((h2 << ob) | (gword(ww + 2) >> (32 - ob))) : h2;
                    }
                    while (l < max_len && wv >= t.limit[l]) l++;
                    const uint64_t c = wv >> (64 - l);
                    const uint64_t idx = t.first_index[l] + (c - t.first_code[l]);
                    if (idx >= a.L.nsym) { bad = true; sym = R; }
                    else sym = sorted[idx];
                    len = l;
                    if ((int32_t)l > avail) {
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
            pk[j >> 1] |= (real ? sym : R) << (16 * (j & 1u));
        }
        dst[g * 64] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    }
    return used;
}

template <uint32_t NDIM>
__global__ __launch_bounds__(64 * kG128Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_decode_g128(DecArgs a) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ DecLds s_t;
    lds_u16 *s_lut = (lds_u16 *)s_dyn;                                 // 1 << kLutBits
    lds_u16 *s_sorted = s_lut + (1u << kLutBits);                     // nsym
    lds_u32 *s_win = (lds_u32 *)(s_sorted + a.L.nsym);                // waves * win_words
    lds_u32 *s_oval = s_win + kG128Waves * a.win_words;               // waves * kG128Out
    lds_u16 *s_opos = (lds_u16 *)(s_oval + kG128Waves * kG128Out);    // waves * kG128Out
    lds_u32 *s_pval = (lds_u32 *)(s_opos + kG128Waves * kG128Out);    // waves * kG128Pat
    lds_u16 *s_ppos = (lds_u16 *)(s_pval + kG128Waves * kG128Pat);    // waves * kG128Pat
    if (a.tab->status) return;   // the code lengths failed validation: tables are not usable
    uint64_t tm[9];
    tm[0] = a.trace ? wall_clock64() : 0;
    tables_to_lds(a, s_lut, s_sorted, s_t);
    __syncthreads();
    if (a.trace) tm[1] = wall_clock64();

    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t gw = blockIdx.x * kG128Waves + w;
    const bool active = gw < a.wave_tasks;
    const uint64_t sub0 = (uint64_t)gw * 64;
    const uint32_t P0 = (uint32_t)(sub0 << 7);                        // padded positions are < 2^31
    const uint32_t P1 = active ? (a.g.padded - P0 < 8192u ? a.g.padded : P0 + 8192u) : P0;
    const bool has = active && sub0 + lane < a.L.n_sub;
    lds_u32 *win = s_win + w * a.win_words;
    lds_u32 *oval = s_oval + w * kG128Out;
    lds_u16 *opos = s_opos + w * kG128Out;
    lds_u32 *pval = s_pval + w * kG128Pat;
    lds_u16 *ppos = s_ppos + w * kG128Pat;
    bool bad = false;
    WaveStream ws = {0, 0, 0, 0};
    uint32_t e0 = 0, e1 = 0, n_out = 0, n_pat = 0;
    if (active) {
        ws = wave_stream(a, sub0, lane, has, win);
        e0 = wave_lower_bound(a.exc, a.n_exc, 2ull * P0, lane);
        e1 = wave_lower_bound(a.exc, a.n_exc, 2ull * P1, lane);
        // the wave's outlier and patch records, each kind compacted in
        // position order (positions relative to the wave's first)
        for (uint32_t eb = e0; eb < e1; eb += 64) {
            const uint32_t e = eb + lane;
            uint2 r = make_uint2(0u, 0u);
            if (e < e1) r = a.exc[e];
            const bool is_out = e < e1 && !(r.x & 1u), is_pat = e < e1 && (r.x & 1u);
            const uint64_t mo = __ballot(is_out), mp = __ballot(is_pat);
            const uint32_t ko = n_out + (uint32_t)__popcll(mo & lanes_below(lane));
            const uint32_t kp = n_pat + (uint32_t)__popcll(mp & lanes_below(lane));
            const uint32_t rp = (r.x >> 1) - P0;   // wraps for keys below the range (damaged list)
            if ((is_out || is_pat) && rp >= P1 - P0) bad = true;
            else if (is_out && ko < kG128Out) { opos[ko] = (uint16_t)rp; oval[ko] = r.y; }
            else if (is_pat && kp < kG128Pat) { ppos[kp] = (uint16_t)rp; pval[kp] = r.y; }
            n_out += (uint32_t)__popcll(mo);
            n_pat += (uint32_t)__popcll(mp);
        }
    }
    __syncthreads();
    if (a.trace) tm[2] = wall_clock64();

    // the wave's 64 x 16 groups, lane-interleaved: group g of lane l at
    // [16 sub0 + 64 g + l], so each store and load covers 1 KB contiguously
    uint4 *qslot = a.qws + sub0 * 16 + lane;
    if (has) {
        const uint32_t max_len = a.tab->max_len < 63u ? a.tab->max_len : 63u;
        const uint32_t used = inflate128(a, win, ws.nwin, ws.wlo, ws.start, P0 + lane * 128u, qslot, s_lut, s_t,
                                         s_sorted, max_len, bad);
        if (used != ws.bits) bad = true;
    }
    if (a.trace) tm[3] = wall_clock64();
    if (active) {
        int32_t v[128];
        deltas_from_slot(a, qslot, lane, P0, e0, e1, n_out, opos, oval, kG128Out, has, bad, v);
        if (a.trace) tm[4] = wall_clock64();
        recon128<NDIM>(a, v, lane, P0, has);
    } else if (a.trace) {
        tm[4] = wall_clock64();
    }
    if (a.trace) tm[5] = wall_clock64();
    if (a.trace) tm[6] = tm[5];
    // patches of the lane's own positions, after its regular stores (program
    // order of one thread: no barrier needed)
    if (has && n_pat) {
        const uint32_t rel0 = lane * 128u;
        if (n_pat <= kG128Pat) {
            uint32_t lo = 0, hi = n_pat;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (ppos[mid] < rel0) lo = mid + 1; else hi = mid;
            }
            for (uint32_t k = lo; k < n_pat && ppos[k] < rel0 + 128u; k++) {
                const uint64_t p = P0 + ppos[k];
                if (!pos_real(a.g, p)) { bad = true; continue; }
                a.out[pos_to_index(a.g, p)] = __uint_as_float(pval[k]);
            }
        } else {
            uint32_t lo = e0, hi = e1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if ((uint64_t)a.exc[mid].x < 2ull * (P0 + rel0)) lo = mid + 1; else hi = mid;
            }
            for (uint32_t e = lo; e < e1; e++) {
                const uint2 r = a.exc[e];
                if ((r.x >> 1) >= P0 + rel0 + 128u) break;
                if (!(r.x & 1u)) continue;
                const uint64_t p = r.x >> 1;
                if (!pos_real(a.g, p)) { bad = true; continue; }
                a.out[pos_to_index(a.g, p)] = __uint_as_float(r.y);
            }
        }
    }
    if (bad) {
        atomicOr(a.status, ST_ECORRUPT);
        *a.hstatus = ST_ECORRUPT;
    }
    if (a.trace && active && lane == 0) {
        tm[7] = wall_clock64();
        uint64_t *ph = const_cast<uint64_t *>(a.tab->phase);
        atomicMin((unsigned long long *)&ph[8], (unsigned long long)tm[0]);
        atomicMax((unsigned long long *)&ph[9], (unsigned long long)tm[7]);
        // tables, window + search, inflate, code read-back, reconstruction +
        // stores, barrier, patches
        const int slot[7] = {10, 11, 12, 13, 14, 15, 3};
        for (int k = 0; k < 7; k++)
            atomicAdd((unsigned long long *)&ph[slot[k]], (unsigned long long)(tm[k + 1] - tm[k]));
    }
}

static size_t decode_g128_lds_bytes(const Layout &L) {
    return sizeof(uint16_t) * ((1u << kLutBits) + L.nsym) +
           (size_t)kG128Waves * (4 * kG128Win + 6 * kG128Out + 6 * kG128Pat);
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

void launch_decode(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint64_t off_str,
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out, bool trace,
                   uint4 *qws, uint32_t *hstatus) {
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
    a.hstatus = hstatus;
    if (a.wave_tasks == 0) return;
    if (L.sub_size == 128 && qws) {
        a.win_words = kG128Win;
        const uint32_t blocks = (a.wave_tasks + kG128Waves - 1) / kG128Waves;
        const size_t lds = decode_g128_lds_bytes(L);
        const void *fn = g.ndim == 3 ? (const void *)k_decode_g128<3>
                                     : (g.ndim == 2 ? (const void *)k_decode_g128<2> : (const void *)k_decode_g128<1>);
        if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (g.ndim == 3) hipLaunchKernelGGL(k_decode_g128<3>, dim3(blocks), dim3(64 * kG128Waves), lds, s, a);
        else if (g.ndim == 2) hipLaunchKernelGGL(k_decode_g128<2>, dim3(blocks), dim3(64 * kG128Waves), lds, s, a);
        else hipLaunchKernelGGL(k_decode_g128<1>, dim3(blocks), dim3(64 * kG128Waves), lds, s, a);
        return;
    }

    const uint32_t waves = decode_waves(L);
    const uint32_t blocks = (a.wave_tasks + waves - 1) / waves;
    const size_t lds = decode_lds_bytes(L);
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k_decode, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(64 * waves), lds, s, a);
}

}  // namespace dqz
