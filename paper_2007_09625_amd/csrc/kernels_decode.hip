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
// code of up to 32 bits is present).  Codes longer than 32 bits (possible
// only when max_len > 32) are read from a fresh 64-bit window in memory and
// set `reinit`: the caller then restarts its reader at the new position.
__device__ __forceinline__ uint32_t decode_sym(const DecArgs &a, uint64_t &cur, int32_t &avail, uint64_t &bp,
                                               const uint16_t *lut, const DecLds &t, const uint16_t *sorted,
                                               uint32_t max_len, bool &bad, bool &reinit) {
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
            bp += l;
            reinit = true;
            return sym;
        }
    }
    cur <<= len;
    avail -= (int32_t)len;
    bp += len;
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

// Stream word i from the wave's LDS window [wlo, wlo + nwin), else from
// memory (only for stream ranges the window cannot hold).  Window word k
// sits at k + k/16: lanes read words about one subchunk apart, and the pad
// spreads those reads over the LDS banks.
__device__ __forceinline__ uint32_t win_slot(uint32_t k) { return k + (k >> 4); }

__device__ __forceinline__ uint32_t win_word(const DecArgs &a, const uint32_t *win, uint64_t wlo, uint32_t nwin,
                                             uint64_t i) {
    const uint64_t k = i - wlo;   // wraps for i < wlo
    if (__builtin_expect(k < nwin, 1)) return win[win_slot((uint32_t)k)];
    return ld_word(a, i);
}

// Inflate `cnt` padded positions starting at stream bit `start` into q[];
// returns the stream position after the last code.  `cur` holds the next
// stream bits MSB-first (more than 32 of them before each decode); `nxt` is
// the following stream word, read one refill ahead.
// Which positions of a partly filled block lie inside the field.  Block
// edges are powers of two (8^3, 16^2), so a position's in-block
// coordinates are bit fields; the block's valid extents are recomputed only
// when the position enters a new block.
struct RealTest {
    uint32_t xs, ys, bshift;        // log2 of the block's x and y edges and of its volume
    uint32_t cur_blk = ~0u, vx = 0, vy = 0, vz = 0;
    __device__ __forceinline__ bool operator()(const Geom &g, uint32_t p) {
        if (g.ndim == 1) return p < g.nelem;
        const uint32_t blk = p >> bshift;
        if (blk != cur_blk) {
            cur_blk = blk;
            const uint32_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
            vx = g.n[2] - Bx * g.b[2];
            vy = g.n[1] - By * g.b[1];
            vz = g.n[0] - Bz * g.b[0];
        }
        const uint32_t in = p & ((1u << bshift) - 1u);
        return (in & (g.b[2] - 1u)) < vx && ((in >> xs) & (g.b[1] - 1u)) < vy && (in >> (xs + ys)) < vz;
    }
};

template <bool FULL>
__device__ __forceinline__ uint64_t inflate_run(const DecArgs &a, const uint32_t *win, uint64_t wlo, uint32_t nwin,
                                                uint64_t start, uint32_t pa, uint32_t cnt, uint16_t *q,
                                                const uint16_t *lut, const DecLds &t, const uint16_t *sorted,
                                                uint32_t max_len, bool &bad) {
    RealTest real;
    real.xs = __builtin_ctz(a.g.b[2]);
    real.ys = __builtin_ctz(a.g.b[1]);
    real.bshift = __builtin_ctz(a.g.bvol);
    uint64_t bp = start;
    uint64_t wi = (bp >> 5) + 2;
    uint64_t cur = (((uint64_t)win_word(a, win, wlo, nwin, bp >> 5) << 32) | win_word(a, win, wlo, nwin, (bp >> 5) + 1))
                   << (bp & 31u);
    int32_t avail = 64 - (int32_t)(bp & 31u);
    uint32_t nxt = win_word(a, win, wlo, nwin, wi);
    for (uint32_t i = 0; i < cnt; i++) {
        if (avail <= 32) {
            cur |= (uint64_t)nxt << (32 - avail);
            avail += 32;
            nxt = win_word(a, win, wlo, nwin, ++wi);
        }
        uint32_t sym = a.L.radius;
        if (FULL || real(a.g, pa + i)) {
            bool reinit = false;
            sym = decode_sym(a, cur, avail, bp, lut, t, sorted, max_len, bad, reinit);
            if (reinit) {   // after a code over 32 bits: restart the reader at bp
                wi = (bp >> 5) + 2;
                cur = (((uint64_t)win_word(a, win, wlo, nwin, bp >> 5) << 32) |
                       win_word(a, win, wlo, nwin, (bp >> 5) + 1)) << (bp & 31u);
                avail = 64 - (int32_t)(bp & 31u);
                nxt = win_word(a, win, wlo, nwin, wi);
            }
        }
        q[i] = (uint16_t)sym;
    }
    return bp;
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

// code buffer slot -> wrapping delta
__device__ __forceinline__ uint32_t slot_delta(const DecArgs &a, uint16_t q, uint32_t e0, bool &bad) {
    if (q & 0x8000u) return a.exc[e0 + (q & 0x7FFFu)].y;
    if (q == 0) bad = true;
    return (uint32_t)q - a.L.radius;
}

__global__ __launch_bounds__(64 * kDecMaxWaves) void k_decode(DecArgs a) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ DecLds s_t;
    uint16_t *s_lut = reinterpret_cast<uint16_t *>(s_dyn);                       // 1 << kLutBits
    uint16_t *s_sorted = s_lut + (1u << kLutBits);                               // nsym
    uint16_t *s_q = s_sorted + a.L.nsym;                                         // waves * 64 * qstride
    uint32_t *s_win = reinterpret_cast<uint32_t *>(s_q + (uint64_t)(blockDim.x / 64) * 64 * a.qstride);  // waves * win_words
    if (a.tab->status) return;   // the code lengths failed validation: tables are not usable
    uint64_t tm[7];
    tm[0] = a.trace ? wall_clock64() : 0;
    {
        // tables into LDS: 16-byte loads, eight of a thread's in flight at once
        // (the lookup table is 16 KB at offset 0 of the 256-byte aligned tables;
        // the sorted symbols are 8-byte aligned, nsym a multiple of 2)
        const uint4 *src = reinterpret_cast<const uint4 *>(a.tab->lut);
        uint4 *dst = reinterpret_cast<uint4 *>(s_lut);
        constexpr uint32_t kVec = (1u << kLutBits) * 2 / 16;
        for (uint32_t i0 = threadIdx.x; i0 < kVec; i0 += 8 * blockDim.x) {
            uint4 v[8];
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
        uint32_t *sdst = reinterpret_cast<uint32_t *>(s_sorted);
        for (uint32_t i = threadIdx.x; i < a.L.nsym / 2; i += blockDim.x) sdst[i] = ssrc[i];
        for (uint32_t i = threadIdx.x; i < 65; i += blockDim.x) {
            const uint64_t l = a.tab->limit[i], f = a.tab->first_code[i];
            const uint32_t x = a.tab->first_index[i];
            s_t.limit[i] = l;
            s_t.first_code[i] = f;
            s_t.first_index[i] = x;
        }
    }
    __syncthreads();
    if (a.trace) tm[1] = wall_clock64();

    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t gw = blockIdx.x * (blockDim.x / 64) + w;
    const bool active = gw < a.wave_tasks;
    const uint32_t S = a.L.sub_size, sh = a.L.sub_shift;
    uint16_t *wq = s_q + (uint64_t)w * 64 * a.qstride;
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
    uint32_t *win = s_win + (uint64_t)w * a.win_words;
    if (active) {
        const uint8_t *subp = a.archive + a.L.off_sub;
        bits_s = has ? ((uint32_t)subp[2 * s] | ((uint32_t)subp[2 * s + 1] << 8)) : 0u;
        const uint32_t incl = wave_incl_scan<uint32_t>(bits_s);
        const uint32_t excl = incl - bits_s;
        const uint32_t C = a.L.chunk_subs;
        const uint64_t *chunks = reinterpret_cast<const uint64_t *>(a.archive + a.L.off_chunk);
        if (C >= 64) {
            const uint64_t cs = (sub0 / C) * C;
            uint64_t pre = 0;
            for (uint64_t j = cs + lane; j < sub0; j += 64) pre += (uint32_t)subp[2 * j] | ((uint32_t)subp[2 * j + 1] << 8);
            pre = wave_sum<uint64_t>(pre);
            start = chunks[sub0 / C] + pre + excl;
        } else {
            const uint64_t c = (has ? s : sub0) / C;
            const uint32_t k = (uint32_t)(c * C - sub0);
            const uint32_t at = __shfl(excl, (int)k, 64);
            start = chunks[c] + excl - at;
        }
        // the window starts at the first subchunk's word and covers the last
        // subchunk's end plus the two words a reader may look past it
        wlo = __shfl(start, 0, 64) >> 5;
        const uint64_t whi = wave_max<uint64_t>(has ? ((start + bits_s) >> 5) + 3 : 0);
        const uint32_t cap = a.win_words / 17 * 16;   // logical words whose padded slots fit
        nwin = whi > wlo ? (uint32_t)(whi - wlo < cap ? whi - wlo : cap) : 0u;
        for (uint32_t b = 0; b < nwin; b += 64 * 8) {
            uint32_t v[8];
#pragma unroll
            for (uint32_t j = 0; j < 8; j++) v[j] = ld_word(a, wlo + b + j * 64 + lane);
#pragma unroll
            for (uint32_t j = 0; j < 8; j++) {
                const uint32_t k = b + j * 64 + lane;
                if (k < nwin) win[win_slot(k)] = v[j];
            }
        }
        // ---- exception range of this wave
        e0 = wave_lower_bound(a.exc, a.n_exc, 2ull * P0, lane);
        e1 = wave_lower_bound(a.exc, a.n_exc, 2ull * P1, lane);
    }
    __syncthreads();
    if (a.trace) tm[2] = wall_clock64();
    // ---- inflate the subchunk into the LDS code buffer
    if (has) {
        const uint32_t pa = (uint32_t)(s << sh);
        const uint32_t pb = (pa + S) < a.g.padded ? (pa + S) : a.g.padded;
        uint16_t *myq = wq + lane * a.qstride;
        bool full;
        if (a.g.ndim == 1) {
            full = pb <= a.g.nelem;
        } else {
            full = true;
            for (uint32_t blk = (uint32_t)(pa / a.g.bvol); blk <= (uint32_t)((pb - 1) / a.g.bvol); blk++)
                full = full && block_full(a.g, blk);
        }
        const uint32_t max_len = a.tab->max_len < 63u ? a.tab->max_len : 63u;
        const uint32_t cnt = (uint32_t)(pb - pa);
        const uint64_t end =
            full ? inflate_run<true>(a, win, wlo, nwin, start, pa, cnt, myq, s_lut, s_t, s_sorted, max_len, bad)
                 : inflate_run<false>(a, win, wlo, nwin, start, pa, cnt, myq, s_lut, s_t, s_sorted, max_len, bad);
        if (end - start != bits_s) bad = true;
    }
    if (a.trace) tm[3] = wall_clock64();
    __syncthreads();
    if (active) {
        // ---- outliers: mark their slots with an index into the exception list
        for (uint32_t e = e0 + lane; e < e1; e += 64) {
            const uint32_t key = a.exc[e].x;
            if (key & 1u) continue;
            const uint64_t loc = (uint64_t)(key >> 1) - P0;
            if (loc >= P1 - P0) { bad = true; continue; }   // only in an unsorted (damaged) list
            uint16_t *slot = wq + (loc >> sh) * a.qstride + (loc & (S - 1));
            if (*slot != 0 || e - e0 > 0x7FFFu) bad = true;
            else *slot = (uint16_t)(0x8000u | (e - e0));
        }
    }
    __syncthreads();
    if (a.trace) tm[4] = wall_clock64();
    if (active) {
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
                    run += slot_delta(a, qat(base + z * 64 + lane), e0, bad);
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
                    if (ok) col += slot_delta(a, qat(base + y * 16 + lx), e0, bad);
                    const uint32_t t = seg_scan<16>(col, lane);
                    const uint32_t yy = By * 16 + y;
                    if (ok && x < g.n[2] && yy < g.n[1]) a.out[(uint64_t)yy * g.n[2] + x] = dequant((int32_t)t, h);
                }
            }
        } else {
            for (uint64_t off = 0; P0 + off < P1; off += 64) {
                const uint64_t loc = off + lane;
                const uint64_t p = P0 + loc;
                const uint32_t t = seg_scan<32>((p < P1) ? slot_delta(a, qat(loc), e0, bad) : 0u, lane);
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
    if (bad) atomicOr(a.status, ST_ECORRUPT);
    if (a.trace && active && lane == 0) {
        tm[6] = wall_clock64();
        uint64_t *ph = const_cast<uint64_t *>(a.tab->phase);
        atomicMin((unsigned long long *)&ph[8], (unsigned long long)tm[0]);
        atomicMax((unsigned long long *)&ph[9], (unsigned long long)tm[6]);
        for (int k = 0; k < 6; k++) atomicAdd((unsigned long long *)&ph[10 + k], (unsigned long long)(tm[k + 1] - tm[k]));
    }
}

static uint32_t decode_waves(const Layout &L) { return L.sub_size <= 256 ? kDecMaxWaves : 1u; }

constexpr size_t kDecLdsLimit = 160 * 1024;       // LDS one workgroup may allocate on gfx950
constexpr uint32_t kDecWinWordsMax = 2688;        // 10.5 KiB stream window per wave (64 subchunks of 128 at ~9.5 bits)

static size_t decode_lds_fixed(const Layout &L) {
    return sizeof(uint16_t) * ((1u << kLutBits) + L.nsym + (size_t)decode_waves(L) * 64 * (L.sub_size + 2)) +
           sizeof(DecLds);
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
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out, bool trace) {
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
    if (a.wave_tasks == 0) return;
    const uint32_t waves = decode_waves(L);
    const uint32_t blocks = (a.wave_tasks + waves - 1) / waves;
    const size_t lds = decode_lds_bytes(L);
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k_decode, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(64 * waves), lds, s, a);
}

}  // namespace dqz
