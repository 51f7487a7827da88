// kernels_huff.hip -- Huffman codebook (compression) and decoding tables
// (decompression), each in one workgroup that keeps everything in LDS.
//
// Code lengths (Sec. 3.2.2).  Leaves with nonzero frequency are sorted by
// (frequency, symbol); the tree is the classic two-queue construction where
// each pick takes the lighter of the next leaf and the oldest unmerged
// internal node, the leaf on equal weights.  Instead of one merge per step,
// the kernel merges in rounds: with T = the sum of the two lightest
// available items, every available item of weight <= T is consumed before
// any node created from now on (those weigh >= T, and ties go to leaves and
// then to older nodes), so that whole prefix of the merged order is paired
// up in parallel.  An odd item left over stays first in line for the next
// round.  This yields exactly the sequential algorithm's tree in about
// log2(N) rounds instead of n - 1 dependent steps.
//
// Canonical codes (Sec. 3.2.3): symbols sorted by (length, symbol) receive
// consecutive codes, the first code of each length following the counting
// rule of RFC 1951 Sec. 3.2.2.  The codebook entry packs the code with its
// bit width: (length << 56) | code (the paper's fixed-length codeword
// representation, Sec. 3.2.2, widened so one form serves every length).
#include "dqz_internal.h"

namespace dqz {

constexpr uint32_t kBookThreads = 256;

template <typename K>
__device__ void bitonic_sort(K *key, uint32_t ns) {
    for (uint32_t k = 2; k <= ns; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const K a = key[i], b = key[ixj];
                    const bool asc = (i & k) == 0;
                    if ((a > b) == asc) {
                        key[i] = b;
                        key[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

struct HeaderArgs {
    uint64_t dims[3];
    double eb_param;
    uint32_t ndim, eb_mode;
};

__device__ void put_le(uint8_t *p, uint32_t off, uint64_t v, uint32_t bytes) {
    for (uint32_t i = 0; i < bytes; i++) p[off + i] = (uint8_t)(v >> (8 * i));
}

// Canonical numbering shared by the codebook and the decoding tables: sorts
// symbols by (length, symbol) into `order`, fills count / first_index /
// first_code, returns max length.  `len` has ns entries (0 = unused).
struct CanonScratch {
    uint64_t key[kMaxSyms];
    uint32_t count[66];
    uint32_t first_index[66];
    uint64_t first_code[66];
    uint32_t n_used;
    uint32_t max_len;
};

__device__ void canonical_order(const uint8_t *len, uint32_t ns, CanonScratch &c) {
    for (uint32_t s = threadIdx.x; s < ns; s += blockDim.x)
        c.key[s] = len[s] ? (((uint64_t)len[s] << 16) | s) : ~0ull;
    for (uint32_t l = threadIdx.x; l < 66; l += blockDim.x) {
        c.count[l] = 0;
        c.first_index[l] = 0;
        c.first_code[l] = 0;
    }
    if (threadIdx.x == 0) { c.n_used = 0; c.max_len = 0; }
    __syncthreads();
    bitonic_sort<uint64_t>(c.key, ns);
    for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x) {
        const uint64_t k = c.key[i];
        if (k == ~0ull) continue;
        const uint32_t l = (uint32_t)(k >> 16);
        const bool first = (i == 0) || ((uint32_t)(c.key[i - 1] >> 16) != l);
        if (first) c.first_index[l] = i;
        const bool last = (i + 1 == ns) || c.key[i + 1] == ~0ull || ((uint32_t)(c.key[i + 1] >> 16) != l);
        if (last) {
            c.count[l] = i + 1;   // fixed up to a count below
            if ((i + 1 == ns) || c.key[i + 1] == ~0ull) { c.n_used = i + 1; c.max_len = l; }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t l = 1; l <= 64; l++)
            if (c.count[l]) c.count[l] -= c.first_index[l];
        uint64_t code = 0;
        for (uint32_t bits = 1; bits <= 64; bits++) {
            code = (code + c.count[bits - 1]) << 1;
            c.first_code[bits] = code;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// K2: histogram -> lengths -> canonical codebook -> header + lengths section
// ---------------------------------------------------------------------------
struct BookLds {
    union {
        uint64_t key[kMaxSyms];
        CanonScratch canon;
    };
    uint32_t leaf_w[kMaxSyms];
    uint16_t leaf_sym[kMaxSyms];
    uint32_t int_w[kMaxSyms];
    uint32_t merged_w[kMaxSyms];
    uint16_t parent_leaf[kMaxSyms];
    uint16_t parent_int[kMaxSyms];
    uint16_t round_start[kMaxSyms + 1];
    uint8_t depth_int[kMaxSyms];
    uint8_t len[kMaxSyms];
    uint32_t n, la, ib, ic, nl, ni, T, rounds, done;
    unsigned long long total_bits;
    uint32_t max_len;
};

__global__ __launch_bounds__(kBookThreads) void k_codebook(const uint32_t *__restrict__ hist, Ctl *ctl,
                                                           uint64_t *__restrict__ book, uint8_t *archive,
                                                           Layout L, Geom g, HeaderArgs hdr) {
    __shared__ BookLds s;
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t ns = L.nsym;
    if (ctl->status & ST_EINVAL) return;

    for (uint32_t i = tid; i < ns; i += T) {
        const uint32_t f = hist[i];
        s.key[i] = f ? (((uint64_t)f << 16) | i) : ~0ull;
        s.len[i] = 0;
    }
    if (tid == 0) { s.n = 0; s.total_bits = 0; s.max_len = 0; }
    __syncthreads();
    bitonic_sort<uint64_t>(s.key, ns);
    for (uint32_t i = tid; i < ns; i += T) {
        const uint64_t k = s.key[i];
        if (k != ~0ull) {
            s.leaf_w[i] = (uint32_t)(k >> 16);
            s.leaf_sym[i] = (uint16_t)(k & 0xFFFF);
            if (i + 1 == ns || s.key[i + 1] == ~0ull) s.n = i + 1;
        }
    }
    __syncthreads();
    const uint32_t n = s.n;
    if (n == 1) {
        if (tid == 0) s.len[s.leaf_sym[0]] = 1;
    } else if (n > 1) {
        if (tid == 0) { s.la = 0; s.ib = 0; s.ic = 0; s.rounds = 0; s.done = 0; }
        __syncthreads();
        for (;;) {
            if (tid == 0) {
                const uint32_t la = s.la, ib = s.ib, ic = s.ic;
                if ((n - la) + (ic - ib) <= 1) {
                    s.done = 1;
                } else {
                    uint32_t a = la, b = ib, tsum = 0;
                    for (int k = 0; k < 2; k++) {
                        const bool leaf = a < n && (b >= ic || s.leaf_w[a] <= s.int_w[b]);
                        tsum += leaf ? s.leaf_w[a++] : s.int_w[b++];
                    }
                    s.T = tsum;
                    s.nl = 0;
                    s.ni = 0;
                }
            }
            __syncthreads();
            if (s.done) break;
            const uint32_t la = s.la, ib = s.ib, ic = s.ic, Tw = s.T;
            // the items of weight <= T form a prefix of each sorted queue
            for (uint32_t i = la + tid; i < n; i += T)
                if (s.leaf_w[i] <= Tw && (i + 1 == n || s.leaf_w[i + 1] > Tw)) s.nl = i + 1 - la;
            for (uint32_t i = ib + tid; i < ic; i += T)
                if (s.int_w[i] <= Tw && (i + 1 == ic || s.int_w[i + 1] > Tw)) s.ni = i + 1 - ib;
            __syncthreads();
            if (tid == 0) {
                uint32_t nl = s.nl, ni = s.ni;
                if ((nl + ni) & 1u) {   // odd: the last item of the merged order waits
                    const bool int_last = ni > 0 && (nl == 0 || s.int_w[ib + ni - 1] >= s.leaf_w[la + nl - 1]);
                    if (int_last) ni--; else nl--;
                }
                s.nl = nl;
                s.ni = ni;
            }
            __syncthreads();
            const uint32_t nl = s.nl, ni = s.ni;
            // merge ranks: a leaf goes after internals strictly lighter; an
            // internal goes after leaves of equal or lower weight
            for (uint32_t k = tid; k < nl; k += T) {
                const uint32_t w = s.leaf_w[la + k];
                uint32_t lo = 0, hi = ni;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s.int_w[ib + mid] < w) lo = mid + 1; else hi = mid;
                }
                const uint32_t rank = k + lo;
                s.merged_w[rank] = w;
                s.parent_leaf[la + k] = (uint16_t)(ic + rank / 2);
            }
            for (uint32_t k = tid; k < ni; k += T) {
                const uint32_t w = s.int_w[ib + k];
                uint32_t lo = 0, hi = nl;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s.leaf_w[la + mid] <= w) lo = mid + 1; else hi = mid;
                }
                const uint32_t rank = k + lo;
                s.merged_w[rank] = w;
                s.parent_int[ib + k] = (uint16_t)(ic + rank / 2);
            }
            __syncthreads();
            const uint32_t p = (nl + ni) / 2;
            for (uint32_t k = tid; k < p; k += T) s.int_w[ic + k] = s.merged_w[2 * k] + s.merged_w[2 * k + 1];
            __syncthreads();
            if (tid == 0) {
                s.round_start[s.rounds++] = (uint16_t)ic;
                s.la = la + nl;
                s.ib = ib + ni;
                s.ic = ic + p;
            }
            __syncthreads();
        }
        // depths: the root is the last internal node; every node's parent
        // was created in a later round, so walk the rounds backwards
        const uint32_t nint = s.ic, rounds = s.rounds;
        if (tid == 0) s.round_start[rounds] = (uint16_t)nint;
        __syncthreads();
        for (int32_t rd = (int32_t)rounds - 1; rd >= 0; rd--) {
            const uint32_t b0 = s.round_start[rd], b1 = s.round_start[rd + 1];
            for (uint32_t k = b0 + tid; k < b1; k += T)
                s.depth_int[k] = (k == nint - 1) ? 0 : (uint8_t)(s.depth_int[s.parent_int[k]] + 1);
            __syncthreads();
        }
        for (uint32_t i = tid; i < n; i += T) {
            const uint32_t d = (uint32_t)s.depth_int[s.parent_leaf[i]] + 1u;
            s.len[s.leaf_sym[i]] = (uint8_t)(d > 255 ? 255 : d);
        }
    }
    __syncthreads();

    // canonical codes
    canonical_order(s.len, ns, s.canon);
    for (uint32_t i = tid; i < ns; i += T) {
        const uint64_t k = s.canon.key[i];
        if (k == ~0ull) continue;
        const uint32_t l = (uint32_t)(k >> 16), sym = (uint32_t)(k & 0xFFFF);
        const uint64_t code = s.canon.first_code[l] + (i - s.canon.first_index[l]);
        book[sym] = ((uint64_t)l << 56) | code;
    }
    for (uint32_t sym = tid; sym < ns; sym += T) {
        if (s.len[sym] == 0) book[sym] = 0;
        const uint64_t c = (uint64_t)hist[sym] * s.len[sym];
        if (c) atomicAdd(&s.total_bits, (unsigned long long)c);
    }
    __syncthreads();

    if (tid == 0) {
        const uint32_t max_len = s.canon.max_len;
        if (max_len > 64) atomicOr(&ctl->status, ST_EUNSUPPORTED);
        const uint64_t total_bits = s.total_bits;
        const uint64_t n_words = (total_bits + 31) / 32;
        const uint32_t n_exc = ctl->n_exc;
        const uint64_t off_str = L.off_exc + 8ull * n_exc;
        const uint64_t end = off_str + 4ull * n_words;
        ctl->max_len = max_len;
        ctl->total_bits = total_bits;
        ctl->n_words = n_words;
        ctl->off_str = off_str;
        ctl->archive_bytes = end;
        if (end > L.cap) atomicOr(&ctl->status, ST_ETOOSMALL);
        // header
        uint8_t *hb = ctl->header;
        for (uint32_t i = 0; i < kHeaderBytes; i++) hb[i] = 0;
        put_le(hb, 0, kMagic, 4);
        put_le(hb, 4, kVersion, 2);
        put_le(hb, 6, hdr.ndim, 1);
        put_le(hb, 7, hdr.eb_mode, 1);
        for (int a = 0; a < 3; a++) put_le(hb, 8 + 8 * a, g.n[a], 8);
        for (int a = 0; a < 3; a++) put_le(hb, 32 + 4 * a, g.b[a], 4);
        put_le(hb, 44, L.radius, 4);
        put_le(hb, 48, (uint64_t)__double_as_longlong(hdr.eb_param), 8);
        put_le(hb, 56, (uint64_t)__double_as_longlong(ctl->eb_abs), 8);
        put_le(hb, 64, __float_as_uint(ctl->h), 4);
        put_le(hb, 68, __float_as_uint(ctl->r), 4);
        if (hdr.eb_mode == 1 && ctl->vmin_key != 0xFFFFFFFFu) {
            put_le(hb, 72, key2f(ctl->vmin_key), 4);
            put_le(hb, 76, key2f(ctl->vmax_key), 4);
        }
        put_le(hb, 80, g.nelem, 8);
        put_le(hb, 88, ctl->n_out, 4);
        put_le(hb, 92, ctl->n_patch, 4);
        put_le(hb, 96, total_bits, 8);
        put_le(hb, 104, L.sub_size, 4);
        put_le(hb, 108, L.chunk_subs, 4);
        put_le(hb, 112, L.n_chunks, 4);
        put_le(hb, 116, max_len, 1);
        put_le(hb, 120, end, 8);
    }
    __syncthreads();
    // header + lengths into the archive (the host checked that the fixed
    // sections fit the capacity)
    for (uint32_t i = tid; i < kHeaderBytes; i += T) archive[i] = ctl->header[i];
    for (uint32_t i = tid; i < ns; i += T) archive[L.off_len + i] = s.len[i];
    for (uint64_t i = L.off_len + ns + tid; i < L.off_chunk; i += T) archive[i] = 0;   // alignment pads
    for (uint64_t i = L.off_sub + 2ull * L.n_sub + tid; i < L.off_exc; i += T) archive[i] = 0;
}

void launch_codebook(hipStream_t st, const Geom &g, const Layout &L, Ctl *ctl, const uint32_t *hist, uint64_t *book,
                     uint8_t *archive, int eb_mode, double eb_param) {
    HeaderArgs h;
    h.dims[0] = g.n[0];
    h.dims[1] = g.n[1];
    h.dims[2] = g.n[2];
    h.eb_param = eb_param;
    h.ndim = g.ndim;
    h.eb_mode = (uint32_t)eb_mode;
    hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kBookThreads), 0, st, hist, ctl, book, archive, L, g, h);
}

// ---------------------------------------------------------------------------
// D0: archive code lengths -> canonical decoding tables.  Validates that the
// lengths describe a complete prefix code (or one symbol of length 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBookThreads) void k_decode_tables(const uint8_t *__restrict__ archive, Layout L,
                                                                uint32_t max_len_hdr, DecodeTables *tab) {
    __shared__ CanonScratch c;
    __shared__ uint8_t len[kMaxSyms];
    __shared__ uint64_t s_short[kMaxSyms];   // left-aligned (to kLutBits) codes of length <= kLutBits
    __shared__ uint32_t s_nshort, s_bad;
    const uint32_t tid = threadIdx.x, T = blockDim.x, ns = L.nsym;
    for (uint32_t i = tid; i < ns; i += T) len[i] = archive[L.off_len + i];
    if (tid == 0) { s_bad = 0; s_nshort = 0; }
    __syncthreads();
    for (uint32_t i = tid; i < ns; i += T)
        if (len[i] > 63) s_bad = 1;
    __syncthreads();
    if (s_bad) {
        if (tid == 0) tab->status = ST_ECORRUPT;
        return;
    }
    canonical_order(len, ns, c);
    if (tid == 0) {
        // Kraft: the code space must be exactly filled (or a lone symbol of length 1)
        int64_t left = 1;
        bool over = false;
        for (uint32_t l = 1; l <= 63; l++) {
            left = 2 * left - (int64_t)c.count[l];
            if (left < 0) { over = true; break; }
            if (left > (1ll << 40)) left = 1ll << 40;   // stays positive: incomplete
        }
        const bool lone = c.n_used == 1 && c.count[1] == 1;
        uint32_t st = 0;
        if (over || (!lone && c.n_used > 0 && left != 0) || c.max_len != max_len_hdr) st = ST_ECORRUPT;
        tab->status = st;
        tab->max_len = c.max_len;
        uint32_t nshort = 0;
        for (uint32_t l = 1; l <= kLutBits; l++) nshort += c.count[l];
        s_nshort = nshort;
    }
    for (uint32_t l = tid; l < 65; l += T) {
        tab->first_code[l] = c.first_code[l];
        tab->count[l] = c.count[l];
        tab->first_index[l] = c.first_index[l];
    }
    __syncthreads();
    const uint32_t nshort = s_nshort;
    for (uint32_t i = tid; i < ns; i += T) {
        const uint64_t k = c.key[i];
        tab->sorted[i] = (k == ~0ull) ? 0 : (uint16_t)(k & 0xFFFF);
        if (i < nshort) {
            const uint32_t l = (uint32_t)(k >> 16);
            const uint64_t code = c.first_code[l] + (i - c.first_index[l]);
            s_short[i] = code << (kLutBits - l);
        }
    }
    __syncthreads();
    // each table slot: the short code whose left-aligned range covers it
    for (uint32_t v = tid; v < (1u << kLutBits); v += T) {
        uint32_t lo = 0, hi = nshort;   // last entry with start <= v
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_short[mid] <= v) lo = mid + 1; else hi = mid;
        }
        uint32_t e = 0;
        if (lo > 0) {
            const uint32_t i = lo - 1;
            const uint64_t k = c.key[i];
            const uint32_t l = (uint32_t)(k >> 16);
            if (v < s_short[i] + (1ull << (kLutBits - l))) e = (l << 16) | (uint32_t)(k & 0xFFFF);
        }
        tab->lut[v] = e;
    }
}

void launch_decode_tables(hipStream_t st, const Layout &L, const uint8_t *archive, uint32_t max_len_hdr,
                          DecodeTables *tab) {
    hipLaunchKernelGGL(k_decode_tables, dim3(1), dim3(kBookThreads), 0, st, archive, L, max_len_hdr, tab);
}

}  // namespace dqz
