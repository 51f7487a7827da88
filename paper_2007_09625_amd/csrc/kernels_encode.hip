// kernels_encode.hip -- Huffman encode + deflate (Sec. 3.2.4).
//
// The paper encodes each symbol to a fixed-length (code, width) word in one
// fine-grained pass and then concatenates the words chunk by chunk with one
// thread per chunk.  Here one launch, k_enc_stream, produces the bit-dense
// stream in a single pass over the code array (tile = kTile padded
// positions, one workgroup per tile):
//
//   - workgroup b codes tile b.  Workgroups go to the XCDs round-robin and
//     each XCD starts its own in order, so the lowest unfinished tile always
//     holds a slot and waits on nothing unfinished: the look-back below
//     always ends (its polls are bounded all the same, an overrun being
//     reported as an internal error).  A shared tile counter would cost a
//     same-address atomic per tile, and those serialize across the chip;
//   - code widths from an LDS copy of the codebook (32-bit codewords when
//     every code fits in 24 bits, the paper's adaptive representation, else
//     64-bit) give the subchunk bit counts (written to the archive) and the
//     tile's bit count;
//   - the tile's stream offset comes from a decoupled look-back over one
//     64-bit word per tile holding (state, value): the tile publishes its
//     own count at once, then adds the counts of its predecessors back to
//     the nearest one that has published its inclusive prefix, and
//     publishes its own inclusive prefix.  The words are read and written
//     with device-scope atomics only (no fences), so nothing else in
//     memory has to become visible early;
//   - the codewords are ORed into an LDS word buffer and leave as one
//     contiguous run.  A stream word belongs to the tile in which its first
//     bit lies: the tile leaves out a first word begun by an earlier tile and
//     completes its last word with the first bits of the stream after it
//     (encoded from the following codes), so every word is written once,
//     whole, and the stream needs no clearing.
//
// The same launch copies the quantize tiles' staged exception records to
// their final place and writes the chunk offsets.
#include "dqz_internal.h"

namespace dqz {

struct EncArgs {
    Geom g;
    Layout L;
    Ctl *ctl;
    Readback *rb;     // the call's readback block: errors found here are reported there too
    EncodeBufs b;
    uint8_t *archive;
    uint32_t n_tiles_e;
};

constexpr uint32_t kEncPer = kTile / 256;              // positions per thread

// The control-block fields the encoder reads, loaded once at the start (the
// codebook kernel wrote them; nothing in this launch changes them).
struct EncCtl {
    uint32_t status, max_len;
    uint64_t total_bits, off_str, n_words;
};
__device__ __forceinline__ EncCtl load_enc_ctl(const Ctl *ctl) {
    EncCtl c;
    c.status = ctl->status;
    c.max_len = ctl->max_len;
    c.total_bits = ctl->total_bits;
    c.off_str = ctl->off_str;
    c.n_words = ctl->n_words;
    return c;
}
constexpr uint32_t kBadStatus = ST_EINVAL | ST_ETOOSMALL | ST_EUNSUPPORTED | ST_EINTERNAL | ST_ENOMEM;

template <bool WIDE> struct Codeword;
template <> struct Codeword<false> {
    typedef uint32_t T;
    static __device__ __forceinline__ uint32_t len(uint32_t e) { return e >> 24; }
    static __device__ __forceinline__ uint64_t code(uint32_t e) { return e & 0xFFFFFFu; }
};
template <> struct Codeword<true> {
    typedef uint64_t T;
    static __device__ __forceinline__ uint32_t len(uint64_t e) { return (uint32_t)(e >> 56); }
    static __device__ __forceinline__ uint64_t code(uint64_t e) { return e & 0x00FFFFFFFFFFFFFFull; }
};

// N consecutive codes of this thread from padded position my0 (padding ->
// kNoSymbol); N a multiple of 8, or 4
template <uint32_t N>
__device__ __forceinline__ void load_codes(const EncArgs &a, uint64_t my0, uint16_t (&q)[N]) {
    static_assert(N % 8 == 0 || N == 4, "codes per thread");
    const uint32_t padded = a.g.padded;
    if (my0 + N <= padded) {
        uint32_t u[N / 2];
        if (N % 8 == 0) {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.b.codes + my0);
#pragma unroll
            for (uint32_t v = 0; v < N / 8; v++) {
                const uint4 u4 = src[v];
                u[4 * v] = u4.x;
                u[4 * v + 1] = u4.y;
                u[4 * v + 2] = u4.z;
                u[4 * v + 3] = u4.w;
            }
        } else {
            const uint2 u2 = *reinterpret_cast<const uint2 *>(a.b.codes + my0);
            u[0] = u2.x;
            u[1] = u2.y;
        }
#pragma unroll
        for (uint32_t i = 0; i < N / 2; i++) {
            q[2 * i] = (uint16_t)(u[i] & 0xFFFF);
            q[2 * i + 1] = (uint16_t)(u[i] >> 16);
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < N; i++) q[i] = (my0 + i < padded) ? a.b.codes[my0 + i] : kNoSymbol;
    }
}

// ---------------------------------------------------------------------------
// tile prefix states: one u64 per tile (zeroed before the launch), the top
// two bits say what the low 62 hold
// ---------------------------------------------------------------------------
constexpr uint64_t kAggregate = 1ull << 62;   // the tile's own bit count
constexpr uint64_t kInclusive = 2ull << 62;   // bits of all tiles up to and including this one
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 20;     // polls before a missing predecessor is an internal error
constexpr uint32_t kFlagStride = 16;          // u64 per tile state: one 128-byte line each

__device__ __forceinline__ uint64_t flag_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void report_internal(const EncArgs &a) {
    atomicOr(&a.ctl->status, ST_EINTERNAL);
    publish_status(a.rb, a.ctl->status | ST_EINTERNAL);
}

// Stream bit offset of tile t > 0 (one whole wave): predecessors are read 64
// at a time, nearest first; their counts are summed back to the nearest one
// with an inclusive prefix.  Before tile 0 the prefix is 0.
__device__ uint64_t look_back(const EncArgs &a, const uint64_t *flags, uint32_t t) {
    const uint32_t lane = lane_id();
    uint64_t G = 0;
    int64_t end = (int64_t)t - 1;   // nearest predecessor not yet added
    uint32_t polls = 0;
    for (;;) {
        const int64_t j = end - (int64_t)lane;
        const uint64_t v = j >= 0 ? flag_load(flags + (uint64_t)j * kFlagStride) : kInclusive;
        const uint64_t inc = __ballot((v >> 62) == 2u), pub = __ballot((v >> 62) != 0u);
        const uint32_t k = inc ? (uint32_t)__builtin_ctzll(inc) : 64u;   // nearest inclusive lane
        const uint64_t need = k >= 63u ? ~0ull : ((2ull << k) - 1u);      // lanes 0 .. k
        if ((pub & need) != need) {   // a nearer predecessor has not published yet
            if (++polls > kSpinLimit) {
                if (lane == 0) report_internal(a);
                return G;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        G += wave_sum<uint64_t>(lane <= k ? (v & kValMask) : 0ull);
        if (k < 64u) return G;
        end -= 64;
    }
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
    const uint32_t lane = lane_id();
    v |= xor_lane32<32>(v, lane);
    v |= xor_lane32<16>(v, lane);
    v |= xor_lane32<8>(v, lane);
    v |= xor_lane32<4>(v, lane);
    v |= xor_lane32<2>(v, lane);
    v |= xor_lane32<1>(v, lane);
    return v;
}

// The first 32 bits of the stream after padded position p (MSB-first, zero
// past the end of the stream), one whole wave; c is the code at p + lane.
template <bool WIDE>
__device__ uint32_t stream_head(const EncArgs &a, const typename Codeword<WIDE>::T *s_book, uint64_t p, uint32_t c) {
    typedef Codeword<WIDE> CW;
    const uint32_t lane = lane_id();
    uint32_t word = 0, off = 0;
    for (;;) {
        const typename CW::T e = c != kNoSymbol ? s_book[c] : (typename CW::T)0;
        const uint32_t len = CW::len(e);
        const uint32_t incl = wave_incl_scan<uint32_t>(len);
        const uint32_t start = off + incl - len;
        uint32_t part = 0;
        if (len && start < 32u) part = (uint32_t)(((CW::code(e) << (64u - len)) >> start) >> 32);
        word |= wave_or(part);
        off += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        p += 64;
        if (off >= 32u || p >= a.g.padded) return word;
        c = p + lane < a.g.padded ? a.b.codes[p + lane] : kNoSymbol;
    }
}

// One packing run: PER consecutive positions per thread from padded position
// p0 + PER * tid, codes q[] (their codewords pre[] when PRE, else looked up
// again), the run's first bit at stream bit
// `base`, the thread's bits at base + excl.  Codewords are built MSB-first
// in a 64-bit register (current word in bits 63..32); words wholly inside
// the thread's bit range are stored plainly into the LDS word buffer, the
// first and last ones (shared with the neighbouring threads) are ORed.  The
// run's words then leave in one contiguous pass, except: a first word begun
// before the tile (its owner completes it), and a last word left partial,
// which is carried into the tile's next run or, after the last run,
// completed with `head` (the next 32 stream bits) when the tile owns it.
template <bool WIDE, uint32_t PER, bool PRE>
__device__ __forceinline__ void pack_run(const EncArgs &a, uint64_t p0, uint64_t base, uint32_t run_bits,
                                         uint32_t excl, const uint16_t (&q)[PER],
                                         const typename Codeword<WIDE>::T (&pre)[PER],
                                         const typename Codeword<WIDE>::T *s_book,
                                         uint32_t *s_words, uint64_t tile_start, bool last_run,
                                         const uint32_t *s_carry_in, uint32_t *s_carry_out, const uint32_t *s_head,
                                         const EncCtl &cc) {
    typedef Codeword<WIDE> CW;
    const uint32_t tid = threadIdx.x;
    const uint64_t my0 = p0 + (uint64_t)PER * tid;
    const uint32_t lead = (uint32_t)(base & 31u);
    const uint32_t nwords = (lead + run_bits + 31u) >> 5;
    for (uint32_t i = tid; i < nwords; i += 256) s_words[i] = 0u;
    if (tid == 0 && s_carry_out) *s_carry_out = 0u;
    // chunk offsets that start inside this run (chunk_subs is a power of two)
    if ((my0 & (a.L.sub_size - 1)) == 0 && my0 < a.g.padded) {
        const uint64_t sub = my0 >> a.L.sub_shift;
        if ((sub & (a.L.chunk_subs - 1)) == 0)
            *reinterpret_cast<uint64_t *>(a.archive + a.L.off_chunk + 8ull * (sub >> (__ffs(a.L.chunk_subs) - 1))) =
                base + excl;
    }
    // the thread's codewords, all lookups in flight together (a padding
    // position reads entry 0 and counts as an empty codeword)
    typename CW::T ent[PER];
#pragma unroll
    for (uint32_t i = 0; i < PER; i++) ent[i] = PRE ? pre[i] : s_book[q[i] != kNoSymbol ? q[i] : 0u];
    __syncthreads();
    {
        const uint32_t bit = lead + excl;
        uint32_t w = bit >> 5, fill = bit & 31u;
        bool head = fill != 0;
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t i = 0; i < PER; i++) {
            const bool real = q[i] != kNoSymbol;
            const uint32_t len = real ? CW::len(ent[i]) : 0u;
            const uint64_t code = real ? CW::code(ent[i]) : 0u;
#pragma unroll
            for (uint32_t part = 0; part < (WIDE ? 2u : 1u); part++) {
                // WIDE codes over 32 bits go in two parts, high part first
                uint32_t l = len;
                uint64_t c = code;
                if (WIDE) {
                    if (part == 0) { l = len > 32u ? len - 32u : 0u; c = code >> 32; }
                    else { l = len > 32u ? 32u : len; c = code & 0xFFFFFFFFull; }
                }
                if (WIDE && l == 0) continue;
                acc |= (c << ((64u - l) & 63u)) >> fill;   // an empty codeword adds nothing
                fill += l;
                if (fill >= 32u) {
                    const uint32_t v = (uint32_t)(acc >> 32);
                    if (head) atomicOr(&s_words[w], v);
                    else s_words[w] = v;
                    head = false;
                    acc <<= 32;
                    fill -= 32u;
                    w++;
                }
            }
        }
        if (fill) atomicOr(&s_words[w], (uint32_t)(acc >> 32));
    }
    __syncthreads();
    uint32_t *stream = reinterpret_cast<uint32_t *>(a.archive + cc.off_str);
    const uint64_t W0 = base >> 5;
    const uint32_t tail = (lead + run_bits) & 31u;   // bits used in the last word (0: it is full)
    for (uint32_t i = tid; i < nwords; i += 256) {
        uint32_t v = s_words[i];
        if (i == 0 && s_carry_in) v |= *s_carry_in;
        if (i == nwords - 1 && tail) {
            if (!last_run) {
                *s_carry_out = v;
                continue;
            }
            v |= *s_head >> tail;
        }
        if (32ull * (W0 + i) >= tile_start && W0 + i < cc.n_words) stream[W0 + i] = v;
    }
}

// A run spans at most PackWords<WIDE>::n words: a whole tile of codes up to
// 24 bits (32-bit codewords), or half a tile of codes up to 64 bits (the
// 64-bit codeword path packs a tile in two runs).  Each kernel's LDS holds
// its word buffer and its codebook.
constexpr uint32_t kRuns64 = 2;
template <bool WIDE> struct PackWords { static constexpr uint32_t n = kTile * 24 / 32 + 2; };
template <> struct PackWords<true> { static constexpr uint32_t n = kTile / kRuns64 * 64 / 32 + 2; };
__host__ __device__ constexpr uint32_t book_offset_u64(bool wide) {
    return ((wide ? PackWords<true>::n : PackWords<false>::n) + 1) / 2;
}
size_t enc_lds_bytes(bool wide, uint32_t nsym) {
    return 8 * (size_t)book_offset_u64(wide) + (wide ? 8 : 4) * (size_t)nsym;
}

struct EncLds {
    uint32_t sub[kTile / 32];
    uint64_t scan[10];
    uint64_t G;
    uint32_t head;
    uint32_t carry[2];
};

// Staged exception records of quantize tile t -> archive, by one wave (the
// records' offset: the segment totals before the tile's, plus its offset
// inside its segment).  Records past the tile's slot come from its run of
// the overflow pool (this kernel does not run when the pool was too small).
__device__ void copy_exceptions(const EncArgs &a, uint32_t t, uint32_t lane) {
    const uint32_t cnt = a.b.qscan.val[0][t];
    const uint32_t in_slot = cnt < a.b.cap ? cnt : a.b.cap;
    uint64_t part = 0;
    for (uint32_t i = lane; i < t / kSegTiles; i += 64) part += a.b.qscan.seg_total[0][i];
    const uint64_t off = wave_sum<uint64_t>(part) + a.b.qscan.excl[0][t];
    uint2 *dst = reinterpret_cast<uint2 *>(a.archive + a.L.off_exc) + off;
    const uint2 *src = a.b.stage + (uint64_t)t * a.b.cap;
    for (uint32_t i = lane; i < in_slot; i += 64) dst[i] = src[i];
    if (cnt > in_slot) {
        const uint2 *ovf = a.b.pool + a.b.ovf_base[t];
        for (uint32_t i = lane; i < cnt - in_slot; i += 64) dst[in_slot + i] = ovf[i];
    }
}

// q: the tile's codes (RUNS runs of PER per thread, loaded by the caller)
template <bool WIDE>
__device__ __forceinline__ void enc_tile(const EncArgs &a, uint32_t t, uint32_t *s_words, uint64_t *s_book_raw,
                                         EncLds &S, const EncCtl &cc,
                                         const uint16_t (&q)[WIDE ? kRuns64 : 1][kEncPer / (WIDE ? kRuns64 : 1)]) {
    typedef Codeword<WIDE> CW;
    typedef typename CW::T Entry;
    constexpr uint32_t RUNS = WIDE ? kRuns64 : 1;
    constexpr uint32_t PER = kEncPer / RUNS;
    Entry *s_book = reinterpret_cast<Entry *>(s_book_raw);
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / 64;
    const uint64_t p0 = (uint64_t)t * kTile;
    const bool coder = t < a.n_tiles_e;
    if (!coder) {   // a quantize tile past the last encode tile: its records only
        if (w == 0 && t < a.b.n_tiles_q) copy_exceptions(a, t, lane);
        return;
    }
    // the codebook and (wave 1) the codes just after the tile in flight
    // together (the tile's codes are already on their way)
    uint32_t after = kNoSymbol;
    {
        const uint64_t pn = p0 + kTile + lane;
        if (w == 1 && pn < a.g.padded) after = a.b.codes[pn];
    }
    {
        const Entry *gbook = WIDE ? reinterpret_cast<const Entry *>(a.b.book) : reinterpret_cast<const Entry *>(a.b.book32);
        Entry ev[kMaxSyms / 256];
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) ev[k] = gbook[i];
        }
        for (uint32_t i = tid; i < kTile / 32; i += 256) S.sub[i] = 0;
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) s_book[i] = ev[k];
        }
    }
    __syncthreads();
    // widths, subchunk sums (a thread's positions never straddle a
    // subchunk), the runs' scans and the tile's bit count
    uint32_t bits[RUNS], excl[RUNS];
    uint64_t tot[RUNS];
    Entry keep[RUNS][PER];   // the 32-bit path keeps its codewords for the packing
#pragma unroll
    for (uint32_t r = 0; r < RUNS; r++) {
        bits[r] = 0;
        Entry (&ent)[PER] = keep[r];
#pragma unroll
        for (uint32_t i = 0; i < PER; i++) ent[i] = s_book[q[r][i] != kNoSymbol ? q[r][i] : 0u];
#pragma unroll
        for (uint32_t i = 0; i < PER; i++) bits[r] += q[r][i] != kNoSymbol ? CW::len(ent[i]) : 0u;
        if (bits[r]) atomicAdd(&S.sub[(r * (kTile / RUNS) + PER * tid) >> a.L.sub_shift], bits[r]);
    }
#pragma unroll
    for (uint32_t r = 0; r < RUNS; r++) excl[r] = (uint32_t)block_excl_scan256(bits[r], S.scan, &tot[r]);
    uint64_t tile_bits = 0;
#pragma unroll
    for (uint32_t r = 0; r < RUNS; r++) tile_bits += tot[r];
    // wave 0: the tile's stream offset; wave 1: the stream bits after the
    // tile; wave 2: the quantize tile's exception records
    uint64_t *flags = a.b.eflag;
    if (w == 0) {
        uint64_t G = 0;
        if (t == 0) {
            if (tid == 0) flag_store(flags, kInclusive | tile_bits);
        } else {
            if (tid == 0) flag_store(flags + (uint64_t)t * kFlagStride, kAggregate | tile_bits);
            G = look_back(a, flags, t);
            if (tid == 0) flag_store(flags + (uint64_t)t * kFlagStride, kInclusive | ((G + tile_bits) & kValMask));
        }
        if (tid == 0) {
            S.G = G;
            // the stream ends where the codebook's total says
            if (t + 1 == a.n_tiles_e && G + tile_bits != cc.total_bits) report_internal(a);
        }
    } else if (w == 1) {
        const uint32_t hb = stream_head<WIDE>(a, s_book, p0 + kTile, after);
        if (lane == 0) S.head = hb;
    } else if (w == 2) {
        if (t < a.b.n_tiles_q) copy_exceptions(a, t, lane);
    }
    __syncthreads();
    // subchunk bit counts (u16, little-endian)
    {
        const uint32_t sub_per_tile = kTile >> a.L.sub_shift;
        const uint64_t sub0 = p0 >> a.L.sub_shift;
        for (uint32_t j = tid; j < sub_per_tile; j += 256) {
            const uint64_t s2 = sub0 + j;
            if (s2 < a.L.n_sub) {
                const uint32_t v = S.sub[j];
                uint8_t *dst = a.archive + a.L.off_sub + 2ull * s2;
                dst[0] = (uint8_t)v;
                dst[1] = (uint8_t)(v >> 8);
            }
        }
    }
    const uint64_t G = S.G;
    uint64_t base = G;
#pragma unroll
    for (uint32_t r = 0; r < RUNS; r++) {
        if (r) __syncthreads();   // the word buffer is reused
        pack_run<WIDE, PER, !WIDE>(a, p0 + r * (kTile / RUNS), base, (uint32_t)tot[r], excl[r], q[r], keep[r],
                                   s_book, s_words, G, r + 1 == RUNS, r ? &S.carry[(r - 1) & 1] : nullptr,
                                   r + 1 < RUNS ? &S.carry[r & 1] : nullptr, &S.head, cc);
        base += tot[r];
    }
}

// Both codeword widths in one kernel: the width is a device value (the
// longest code; over 24 bits is common at larger error bounds, where rare
// symbols get long codes), taken uniformly by every workgroup.  The
// launch reserves the larger of the two LDS layouts; the 32-bit path keeps
// its speed at the 64-bit path's register count (measured), and no second
// launch that returns at once is needed.
__global__ __launch_bounds__(256) void k_enc_stream(EncArgs a) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ EncLds S;
    const EncCtl cc = load_enc_ctl(a.ctl);
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    const uint64_t p0 = (uint64_t)t * kTile;
    const bool coder = t < a.n_tiles_e;
    // the tile's codes in the 32-bit path's order go out together with the
    // control fields (the common case; the 64-bit path loads its own order)
    uint16_t q32[1][kEncPer];
    if (coder) load_codes(a, p0 + (uint64_t)kEncPer * tid, q32[0]);
    if (cc.status & kBadStatus) return;
    uint32_t *s_words = reinterpret_cast<uint32_t *>(s_dyn);   // PackWords<WIDE>::n, then nsym codewords
    if (cc.max_len > 24) {
        constexpr uint32_t PER = kEncPer / kRuns64;
        uint16_t q64[kRuns64][PER];
        if (coder) {
#pragma unroll
            for (uint32_t r = 0; r < kRuns64; r++) load_codes(a, p0 + r * (kTile / kRuns64) + (uint64_t)PER * tid, q64[r]);
        }
        enc_tile<true>(a, t, s_words, s_dyn + book_offset_u64(true), S, cc, q64);
    } else {
        enc_tile<false>(a, t, s_words, s_dyn + book_offset_u64(false), S, cc, q32);
    }
}

// One workgroup per segment: exclusive prefix of the tile values inside
// the segment, and the segment total.
__global__ __launch_bounds__(256) void k_seg_scan(TileScan S, HistJob H) {
    __shared__ uint64_t sh[4];
    const uint32_t seg = blockIdx.x, t = seg * kSegTiles + threadIdx.x;
    for (uint32_t k = 0; k < S.nvals; k++) {
        const uint64_t v = (t < S.n_tiles) ? S.val[k][t] : 0u;
        uint64_t tot;
        const uint64_t ex = block_excl_scan256(v, sh, &tot);
        if (t < S.n_tiles) S.excl[k][t] = (uint32_t)ex;
        if (threadIdx.x == 0) S.seg_total[k][seg] = tot;
    }
    // side job: sum the histogram replicas (bins spread over the workgroups)
    if (H.hist_out) {
        for (uint32_t b = seg * 256 + threadIdx.x; b < H.nsym; b += gridDim.x * 256) {
            uint32_t v[kHistReplicas];
#pragma unroll
            for (uint32_t r = 0; r < kHistReplicas; r++) v[r] = H.replicas[r * H.nsym + b];
            uint32_t f = 0;
#pragma unroll
            for (uint32_t r = 0; r < kHistReplicas; r++) f += v[r];
            H.hist_out[b] = f;
        }
    }
}

void launch_seg_scan(hipStream_t s, const TileScan &S, const HistJob *hj) {
    if (S.n_segs == 0) return;
    HistJob H = {nullptr, nullptr, 0};
    if (hj) H = *hj;
    hipLaunchKernelGGL(k_seg_scan, dim3(S.n_segs), dim3(256), 0, s, S, H);
}

uint32_t encode_tiles(const Geom &g) { return (uint32_t)((g.padded + kTile - 1) / kTile); }

void launch_encode(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, Readback *rb, const EncodeBufs &b,
                   uint8_t *archive, int ncu) {
    EncArgs a;
    a.g = g;
    a.L = L;
    a.ctl = ctl;
    a.rb = rb;
    a.b = b;
    a.archive = archive;
    a.n_tiles_e = encode_tiles(g);
    const uint32_t grid = a.n_tiles_e > b.n_tiles_q ? a.n_tiles_e : b.n_tiles_q;
    if (grid == 0) return;
    (void)ncu;
    const size_t lds32 = enc_lds_bytes(false, L.nsym), lds64 = enc_lds_bytes(true, L.nsym);
    hipLaunchKernelGGL(k_enc_stream, dim3(grid), dim3(256), lds32 > lds64 ? lds32 : lds64, s, a);
}

}  // namespace dqz
