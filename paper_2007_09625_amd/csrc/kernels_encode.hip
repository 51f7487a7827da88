// kernels_encode.hip -- Huffman encode + deflate (Sec. 3.2.4).
//
// The paper encodes each symbol to a fixed-length (code, width) word in one
// fine-grained pass and then concatenates the words chunk by chunk with one
// thread per chunk.  Here the stream is produced by two tiled passes over
// the code array (tile = kTile padded positions, one workgroup per tile):
//
//   k_enc_count  code widths from the LDS length table -> subchunk bit
//                counts (written to the archive) and the tile's bit count
//                (scanned by k_seg_scan); the same launch copies the
//                quantize tiles' staged exception records to their final
//                place and clears the stream words.
//   k_enc_pack   the tile's global bit offset is now known: look codes up in
//                an LDS copy of the codebook (32-bit codewords when every
//                code fits in 24 bits, the paper's adaptive representation,
//                else 64-bit), scan widths across the workgroup, OR the
//                codewords into an LDS word buffer and write it out as one
//                contiguous run; the first and last words, shared with the
//                neighbouring tiles, are merged with atomic OR.  Chunk
//                offsets that fall inside the tile are written here.
#include "dqz_internal.h"

namespace dqz {

struct EncArgs {
    Geom g;
    Layout L;
    Ctl *ctl;
    EncodeBufs b;
    uint8_t *archive;
    uint32_t n_tiles_e;
};

constexpr uint32_t kEncPer = kTile / 256;              // positions per thread
constexpr uint32_t kBadStatus = ST_EINVAL | ST_ETOOSMALL | ST_EUNSUPPORTED | ST_EINTERNAL | ST_RETRY;

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
// kNoSymbol); N a multiple of 8
template <uint32_t N>
__device__ __forceinline__ void load_codes(const EncArgs &a, uint64_t my0, uint16_t (&q)[N]) {
    const uint32_t padded = a.g.padded;
    if (my0 + N <= padded) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.b.codes + my0);
#pragma unroll
        for (uint32_t v = 0; v < N / 8; v++) {
            const uint4 u4 = src[v];
            const uint32_t u[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
            for (uint32_t i = 0; i < 4; i++) {
                q[8 * v + 2 * i] = (uint16_t)(u[i] & 0xFFFF);
                q[8 * v + 2 * i + 1] = (uint16_t)(u[i] >> 16);
            }
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < N; i++) q[i] = (my0 + i < padded) ? a.b.codes[my0 + i] : kNoSymbol;
    }
}

// ---------------------------------------------------------------------------
// pass 1
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_enc_count(EncArgs a) {
    __shared__ uint8_t s_len[kMaxSyms];
    __shared__ uint32_t s_sub[kTile / 32];
    __shared__ uint64_t s_scan[10];
    Ctl *ctl = a.ctl;
    if (ctl->status & kBadStatus) return;
    const uint32_t tid = threadIdx.x, t = blockIdx.x;
    // the tile's codes are in flight during the copies below and while the
    // length table goes to LDS
    const uint64_t p0 = (uint64_t)t * kTile;
    const uint64_t my0 = p0 + (uint64_t)kEncPer * tid;
    uint16_t q[kEncPer];
    if (t < a.n_tiles_e) load_codes(a, my0, q);

    // staged exception records of quantize tile t -> archive
    if (t < a.b.n_tiles_q) {
        uint32_t cnt = a.b.qscan.val[0][t];
        if (cnt > a.b.cap) cnt = a.b.cap;   // overflowed: the host compresses again with full staging
        const uint64_t off = tile_offset(a.b.qscan, 0, t, s_scan);
        uint2 *dst = reinterpret_cast<uint2 *>(a.archive + a.L.off_exc) + off;
        const uint2 *src = a.b.stage + (uint64_t)t * a.b.cap;
        for (uint32_t i = tid; i < cnt; i += 256) dst[i] = src[i];
    }
    // clear the stream words (the packing pass ORs the tile edges)
    {
        uint32_t *stream = reinterpret_cast<uint32_t *>(a.archive + ctl->off_str);
        const uint64_t words = ctl->n_words;
        for (uint64_t i = (uint64_t)t * 256 + tid; i < words; i += (uint64_t)gridDim.x * 256) stream[i] = 0u;
    }
    if (t >= a.n_tiles_e) return;

    for (uint32_t i = tid; i < a.L.nsym; i += 256) s_len[i] = a.archive[a.L.off_len + i];
    for (uint32_t i = tid; i < kTile / 32; i += 256) s_sub[i] = 0;
    __syncthreads();
    uint32_t my_bits = 0;
#pragma unroll
    for (uint32_t i = 0; i < kEncPer; i++)
        if (q[i] != kNoSymbol) my_bits += s_len[q[i]];
    // subchunk sums (a thread's positions never straddle a subchunk)
    if (my_bits) atomicAdd(&s_sub[(kEncPer * tid) >> a.L.sub_shift], my_bits);
    uint64_t tile_bits;
    (void)block_excl_scan256(my_bits, s_scan, &tile_bits);
    const uint32_t sub_per_tile = kTile >> a.L.sub_shift;
    const uint64_t sub0 = p0 >> a.L.sub_shift;
    for (uint32_t j = tid; j < sub_per_tile; j += 256) {
        const uint64_t s = sub0 + j;
        if (s < a.L.n_sub) {
            const uint32_t v = s_sub[j];
            uint8_t *dst = a.archive + a.L.off_sub + 2ull * s;
            dst[0] = (uint8_t)v;
            dst[1] = (uint8_t)(v >> 8);
        }
    }
    tile_publish(a.b.escan, t, (uint32_t)tile_bits, 0u);
}

// ---------------------------------------------------------------------------
// pass 2
// ---------------------------------------------------------------------------
// One packing pass over PER consecutive positions per thread starting at
// padded position p0 + PER * tid, the pass's first bit at stream bit `base`.
// The thread's codewords are built MSB-first in a 64-bit register (current
// word in bits 63..32); words wholly inside the thread's bit range are stored
// plainly into the LDS word buffer, the first and last ones (shared with the
// neighbouring threads when the range starts or ends mid-word) are ORed.
// The buffer then leaves as one contiguous run; its first and last words are
// shared with the neighbouring passes and merged into the stream by atomic OR.
// Returns the pass's bit count.
template <bool WIDE, uint32_t PER>
__device__ __forceinline__ uint32_t pack_pass(const EncArgs &a, uint64_t p0, uint64_t base, const uint16_t (&q)[PER],
                                              const typename Codeword<WIDE>::T *s_book, uint32_t *s_words,
                                              uint64_t *s_scan) {
    typedef Codeword<WIDE> CW;
    typedef typename CW::T Entry;
    const uint32_t tid = threadIdx.x;
    const uint64_t my0 = p0 + (uint64_t)PER * tid;
    uint32_t my_bits = 0;
#pragma unroll
    for (uint32_t i = 0; i < PER; i++)
        if (q[i] != kNoSymbol) my_bits += CW::len(s_book[q[i]]);
    uint64_t pass_bits;
    const uint32_t excl = (uint32_t)block_excl_scan256(my_bits, s_scan, &pass_bits);
    const uint32_t lead = (uint32_t)(base & 31u);
    const uint32_t nwords = (lead + (uint32_t)pass_bits + 31u) >> 5;
    for (uint32_t i = tid; i < nwords; i += 256) s_words[i] = 0u;
    // chunk offsets that start inside this pass
    if ((my0 & (a.L.sub_size - 1)) == 0 && my0 < a.g.padded) {
        const uint64_t sub = my0 >> a.L.sub_shift;
        if ((sub & (a.L.chunk_subs - 1)) == 0)
            *reinterpret_cast<uint64_t *>(a.archive + a.L.off_chunk + 8ull * (sub / a.L.chunk_subs)) = base + excl;
    }
    __syncthreads();
    {
        const uint32_t bit = lead + excl;
        uint32_t w = bit >> 5, fill = bit & 31u;
        bool head = fill != 0;
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t i = 0; i < PER; i++) {
            if (q[i] == kNoSymbol) continue;
            const Entry e = s_book[q[i]];
            const uint32_t len = CW::len(e);
            const uint64_t code = CW::code(e);
#pragma unroll
            for (uint32_t part = 0; part < (WIDE ? 2u : 1u); part++) {
                // WIDE codes over 32 bits go in two parts, high part first
                uint32_t l = len;
                uint64_t c = code;
                if (WIDE) {
                    if (part == 0) { l = len > 32u ? len - 32u : 0u; c = code >> 32; }
                    else { l = len > 32u ? 32u : len; c = code & 0xFFFFFFFFull; }
                }
                if (l == 0) continue;
                acc |= (c << (64u - l)) >> fill;
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
    uint32_t *stream = reinterpret_cast<uint32_t *>(a.archive + a.ctl->off_str);
    const uint64_t W0 = base >> 5;
    const bool shared_first = lead != 0;
    const bool shared_last = ((lead + (uint32_t)pass_bits) & 31u) != 0;
    for (uint32_t i = tid; i < nwords; i += 256) {
        const uint32_t v = s_words[i];
        const bool edge = (i == 0 && shared_first) || (i == nwords - 1 && shared_last);
        if (edge) {
            if (v) atomicOr(stream + W0 + i, v);
        } else {
            stream[W0 + i] = v;
        }
    }
    return (uint32_t)pass_bits;
}

// A pass spans at most kPackWords words: a whole tile of codes up to 32 bits,
// or half a tile of codes up to 63 bits (the 64-bit codeword path packs a
// tile in two halves).
constexpr uint32_t kPackWords = kTile + 2;

template <bool WIDE>
__device__ __forceinline__ void pack_tile(const EncArgs &a, uint32_t *s_words, uint64_t *s_book_raw,
                                          uint64_t *s_scan, uint64_t *s_G) {
    typedef typename Codeword<WIDE>::T Entry;
    Entry *s_book = reinterpret_cast<Entry *>(s_book_raw);
    const uint32_t tid = threadIdx.x, t = blockIdx.x;
    const Entry *gbook = WIDE ? reinterpret_cast<const Entry *>(a.b.book) : reinterpret_cast<const Entry *>(a.b.book32);
    const uint64_t p0 = (uint64_t)t * kTile;
    // the tile's codes are in flight while the codebook goes to LDS (the
    // 64-bit path packs the tile in two halves)
    constexpr uint32_t PER = WIDE ? kEncPer / 2 : kEncPer;
    uint16_t q0[PER], q1[PER];
    load_codes(a, p0 + (uint64_t)PER * tid, q0);
    if (WIDE) load_codes(a, p0 + kTile / 2 + (uint64_t)PER * tid, q1);
    {
        // codebook into LDS: all loads of a thread in flight
        Entry e[kMaxSyms / 256];
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) e[k] = gbook[i];
        }
        // the tile's global bit offset: wave 0 sums the totals of the earlier segments
        if (tid < 64) {
            const uint32_t seg = t / kSegTiles;
            uint64_t part = 0;
            for (uint32_t i = tid; i < seg; i += 64) part += a.b.escan.seg_total[0][i];
            part = wave_sum<uint64_t>(part);
            if (tid == 0) *s_G = part + a.b.escan.excl[0][t];
        }
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) s_book[i] = e[k];
        }
    }
    __syncthreads();
    const uint64_t G = *s_G;
    if (!WIDE) {
        (void)pack_pass<false, PER>(a, p0, G, q0, reinterpret_cast<const uint32_t *>(s_book), s_words, s_scan);
    } else {
        const uint32_t b0 = pack_pass<true, PER>(a, p0, G, q0, reinterpret_cast<const uint64_t *>(s_book), s_words,
                                                 s_scan);
        __syncthreads();   // the word buffer is reused
        (void)pack_pass<true, PER>(a, p0 + kTile / 2, G + b0, q1, reinterpret_cast<const uint64_t *>(s_book),
                                   s_words, s_scan);
    }
}

__global__ __launch_bounds__(256) void k_enc_pack(EncArgs a) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ uint64_t s_scan[10];
    __shared__ uint64_t s_G;
    if (a.ctl->status & kBadStatus) return;
    uint32_t *s_words = reinterpret_cast<uint32_t *>(s_dyn);               // kPackWords
    uint64_t *s_book = s_dyn + (kPackWords + 1) / 2;                       // nsym entries
    if (a.ctl->max_len <= 24) pack_tile<false>(a, s_words, s_book, s_scan, &s_G);
    else pack_tile<true>(a, s_words, s_book, s_scan, &s_G);
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

static EncArgs enc_args(const Geom &g, const Layout &L, Ctl *ctl, const EncodeBufs &b, uint8_t *archive) {
    EncArgs a;
    a.g = g;
    a.L = L;
    a.ctl = ctl;
    a.b = b;
    a.archive = archive;
    a.n_tiles_e = encode_tiles(g);
    return a;
}

void launch_encode_count(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const EncodeBufs &b,
                         uint8_t *archive) {
    const EncArgs a = enc_args(g, L, ctl, b, archive);
    if (a.n_tiles_e == 0) return;
    const uint32_t grid1 = a.n_tiles_e > b.n_tiles_q ? a.n_tiles_e : b.n_tiles_q;
    hipLaunchKernelGGL(k_enc_count, dim3(grid1), dim3(256), 0, s, a);
    launch_seg_scan(s, b.escan);
}

void launch_encode_pack(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const EncodeBufs &b,
                        uint8_t *archive) {
    const EncArgs a = enc_args(g, L, ctl, b, archive);
    if (a.n_tiles_e == 0) return;
    const size_t lds = sizeof(uint64_t) * ((kPackWords + 1) / 2 + L.nsym);
    hipLaunchKernelGGL(k_enc_pack, dim3(a.n_tiles_e), dim3(256), lds, s, a);
}

}  // namespace dqz
