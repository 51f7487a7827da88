// kernels_encode.hip -- Huffman encode + deflate (Sec. 3.2.4).
//
// The paper encodes each symbol to a fixed-length (code, width) word in one
// fine-grained pass and then concatenates the words chunk by chunk with one
// thread per chunk.  Here both steps are one pass: each workgroup handles a
// tile of kTile padded positions (tile index = workgroup index), looks the
// codes up in an LDS copy of the codebook (32-bit codewords when every code
// fits in 24 bits, the paper's adaptive representation, else 64-bit), scans
// the code widths across the workgroup,
// obtains the tile's global bit offset by decoupled look-back, and packs the
// codewords into an LDS word buffer that is then written out as one
// contiguous run of stream words.  Words shared with the neighbouring tiles
// (first and last) are merged with atomic OR into the zeroed stream.  The
// tile also writes its subchunk bit counts and the chunk offsets that fall
// inside it, so the bitstream and tables come out in one read of the codes.
#include "dqz_internal.h"

namespace dqz {

__global__ __launch_bounds__(256) void k_zero_stream(Ctl *ctl, uint8_t *archive) {
    if (ctl->status & (ST_EINVAL | ST_ETOOSMALL | ST_EUNSUPPORTED)) return;
    const uint64_t words = ctl->n_words;
    uint32_t *w = reinterpret_cast<uint32_t *>(archive + ctl->off_str);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = tid; i < words; i += stride) w[i] = 0u;
}

struct EncArgs {
    Geom g;
    Layout L;
    Ctl *ctl;
    const uint16_t *codes;
    const uint64_t *book;
    const uint32_t *book32;
    uint64_t *lb;
    uint8_t *archive;
    uint32_t n_tiles;
};

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

constexpr uint32_t kEncPer = kTile / 256;              // positions per thread
constexpr uint32_t kEncWords = kTile * 64 / 32 + 2;    // worst case tile span in words

__device__ __forceinline__ void or_bits(uint32_t *buf, uint32_t bit, uint64_t code, uint32_t len) {
    // write `len` bits of `code` (MSB first) starting at buffer bit `bit`
    while (len) {
        const uint32_t w = bit >> 5, o = bit & 31u;
        const uint32_t take = (32u - o) < len ? (32u - o) : len;
        const uint32_t chunk = (uint32_t)((code >> (len - take)) & ((take == 32u) ? 0xFFFFFFFFull : ((1ull << take) - 1ull)));
        atomicOr(buf + w, chunk << (32u - o - take));
        bit += take;
        len -= take;
    }
}

struct EncLds {
    uint32_t sub[kTile / 32];
    uint32_t wave[4];
    unsigned long long G;
};

template <bool WIDE>
__device__ __forceinline__ void encode_tile(const EncArgs &a, uint64_t *s_dyn, EncLds &sh) {
    typedef Codeword<WIDE> CW;
    typedef typename CW::T Entry;
    uint32_t *s_words = reinterpret_cast<uint32_t *>(s_dyn);                // kEncWords
    Entry *s_book = reinterpret_cast<Entry *>(s_dyn + (kEncWords + 1) / 2);
    uint32_t *s_sub = sh.sub;
    uint32_t *s_wave = sh.wave;
    unsigned long long &s_G = sh.G;
    Ctl *ctl = a.ctl;
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / 64;
    const Entry *gbook = WIDE ? reinterpret_cast<const Entry *>(a.book) : reinterpret_cast<const Entry *>(a.book32);
    {
        // codebook into LDS: up to kMaxSyms / 256 loads per thread, all in flight
        Entry e[kMaxSyms / 256];
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) e[k] = gbook[i];
        }
#pragma unroll
        for (uint32_t k = 0; k < kMaxSyms / 256; k++) {
            const uint32_t i = tid + 256 * k;
            if (i < a.L.nsym) s_book[i] = e[k];
        }
    }
    for (uint32_t i = tid; i < kTile / 32; i += 256) s_sub[i] = 0;
    __syncthreads();
    const uint32_t tile = blockIdx.x;
    const uint64_t p0 = (uint64_t)tile * kTile;
    const uint64_t my0 = p0 + (uint64_t)kEncPer * tid;
    const uint32_t padded = a.g.padded;

    uint16_t q[kEncPer];
    if (my0 + kEncPer <= padded) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.codes + my0);
        const uint4 v0 = src[0], v1 = src[1];
        const uint32_t u[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
        for (uint32_t i = 0; i < 8; i++) {
            q[2 * i] = (uint16_t)(u[i] & 0xFFFF);
            q[2 * i + 1] = (uint16_t)(u[i] >> 16);
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kEncPer; i++) q[i] = (my0 + i < padded) ? a.codes[my0 + i] : kNoSymbol;
    }
    uint32_t my_bits = 0;
#pragma unroll
    for (uint32_t i = 0; i < kEncPer; i++)
        if (q[i] != kNoSymbol) my_bits += CW::len(s_book[q[i]]);

    // workgroup exclusive scan of bit counts
    const uint32_t incl = wave_incl_scan<uint32_t>(my_bits);
    if (lane == 63) s_wave[w] = incl;
    // subchunk sums (a thread's positions never straddle a subchunk)
    if (my_bits) atomicAdd(&s_sub[(kEncPer * tid) >> a.L.sub_shift], my_bits);
    __syncthreads();
    uint32_t wave_off = 0, tile_bits = 0;
    for (uint32_t i = 0; i < 4; i++) {
        if (i < w) wave_off += s_wave[i];
        tile_bits += s_wave[i];
    }
    const uint32_t excl = wave_off + incl - my_bits;
    if (w == 0) {
        uint64_t G = 0;
        if (tile == 0) {
            if (lane == 0) lb_publish(a.lb, 0, tile_bits, 2);
        } else {
            if (lane == 0) lb_publish(a.lb, tile, tile_bits, 1);
            G = lb_exclusive(a.lb, tile, &ctl->status);
            if (lane == 0) lb_publish(a.lb, tile, G + tile_bits, 2);
        }
        if (lane == 0) s_G = G;
    }
    __syncthreads();
    const uint64_t G = s_G;
    const uint32_t lead = (uint32_t)(G & 31u);
    const uint32_t nwords = (lead + tile_bits + 31u) >> 5;
    for (uint32_t i = tid; i < nwords; i += 256) s_words[i] = 0u;

    // tables: subchunk bit counts, chunk offsets at chunk starts
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
    if ((my0 & (a.L.sub_size - 1)) == 0 && my0 < padded) {
        const uint64_t s = my0 >> a.L.sub_shift;
        if ((s & (a.L.chunk_subs - 1)) == 0)
            *reinterpret_cast<uint64_t *>(a.archive + a.L.off_chunk + 8ull * (s / a.L.chunk_subs)) = G + excl;
    }
    __syncthreads();
    // pack
    uint32_t bit = lead + excl;
#pragma unroll
    for (uint32_t i = 0; i < kEncPer; i++) {
        if (q[i] == kNoSymbol) continue;
        const Entry e = s_book[q[i]];
        const uint32_t len = CW::len(e);
        or_bits(s_words, bit, CW::code(e), len);
        bit += len;
    }
    __syncthreads();
    // write out: words shared with neighbours via atomic OR
    uint32_t *stream = reinterpret_cast<uint32_t *>(a.archive + ctl->off_str);
    const uint64_t W0 = G >> 5;
    const bool shared_first = lead != 0;
    const bool shared_last = ((lead + tile_bits) & 31u) != 0;
    for (uint32_t i = tid; i < nwords; i += 256) {
        const uint32_t v = s_words[i];
        const bool edge = (i == 0 && shared_first) || (i == nwords - 1 && shared_last);
        if (edge) {
            if (v) atomicOr(stream + W0 + i, v);
        } else {
            stream[W0 + i] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_encode(EncArgs a) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ EncLds sh;
    if (a.ctl->status & (ST_EINVAL | ST_ETOOSMALL | ST_EUNSUPPORTED | ST_EINTERNAL)) return;
    if (a.ctl->max_len <= 24) encode_tile<false>(a, s_dyn, sh);
    else encode_tile<true>(a, s_dyn, sh);
}

void launch_zero_stream(hipStream_t s, const Geom &g, Ctl *ctl, uint8_t *archive) {
    if (g.nelem == 0) return;
    hipLaunchKernelGGL(k_zero_stream, dim3(512), dim3(256), 0, s, ctl, archive);
}

uint32_t encode_tiles(const Geom &g) { return (uint32_t)((g.padded + kTile - 1) / kTile); }

void launch_encode(hipStream_t s, const Geom &g, const Layout &L, Ctl *ctl, const uint16_t *codes,
                   const uint64_t *book, const uint32_t *book32, uint64_t *lb, uint8_t *archive) {
    EncArgs a;
    a.g = g;
    a.L = L;
    a.ctl = ctl;
    a.codes = codes;
    a.book = book;
    a.book32 = book32;
    a.lb = lb;
    a.archive = archive;
    a.n_tiles = encode_tiles(g);
    if (a.n_tiles == 0) return;
    const size_t lds = sizeof(uint64_t) * ((kEncWords + 1) / 2 + L.nsym);
    hipLaunchKernelGGL(k_encode, dim3(a.n_tiles), dim3(256), lds, s, a);
}

}  // namespace dqz
