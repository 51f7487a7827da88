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
constexpr uint32_t kTableThreads = 512;    // decoding tables: threads per workgroup
constexpr uint32_t kTableGroups = 16;      // workgroups that share the lookup tables' slots

template <typename K>
__device__ __forceinline__ K xor_lane(K v, uint32_t lane, uint32_t d) {   // d a compile-time constant
    switch (d) {
    case 1: return xor_lane_t<1>(v, lane);
    case 2: return xor_lane_t<2>(v, lane);
    case 4: return xor_lane_t<4>(v, lane);
    case 8: return xor_lane_t<8>(v, lane);
    case 16: return xor_lane_t<16>(v, lane);
    default: return xor_lane_t<32>(v, lane);
    }
}

// Bitonic sort of 256 * E keys (32- or 64-bit) held E per thread (thread t holds
// elements t*E .. t*E + E - 1).  Partners within a thread are compared in
// registers, partners within a wave through cross-lane exchanges, and only
// the strides spanning waves go through LDS (`xch`, 256 * E entries).  Every
// loop has a compile-time trip count, so register indices stay static.
template <int E, typename K>
__device__ __forceinline__ void sort_keys(K (&k)[E], K *xch) {
    constexpr uint32_t NS = 256u * E;
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t kk = 2; kk <= NS; kk <<= 1) {
#pragma unroll
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            if (j < (uint32_t)E) {
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)E; r++) {
                    if (r & j) continue;
                    const uint32_t e = t * E + r;
                    const bool asc = (e & kk) == 0;
                    const K a = k[r], b = k[r | j];
                    if ((a > b) == asc) { k[r] = b; k[r | j] = a; }
                }
            } else if (j < 64u * E) {
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)E; r++) {
                    const uint32_t e = t * E + r;
                    const K o = xor_lane(k[r], t & 63u, j / E);
                    const bool lower = (e & j) == 0, asc = (e & kk) == 0;
                    const K mn = o < k[r] ? o : k[r], mx = o < k[r] ? k[r] : o;
                    k[r] = (lower == asc) ? mn : mx;
                }
            } else {
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)E; r++) xch[t * E + r] = k[r];
                __syncthreads();
#pragma unroll
                for (uint32_t r = 0; r < (uint32_t)E; r++) {
                    const uint32_t e = t * E + r;
                    const K o = xch[e ^ j];
                    const bool lower = (e & j) == 0, asc = (e & kk) == 0;
                    const K mn = o < k[r] ? o : k[r], mx = o < k[r] ? k[r] : o;
                    k[r] = (lower == asc) ? mn : mx;
                }
                __syncthreads();
            }
        }
    }
}

// Sort `ns` keys of type K produced by make(i) (i < ns; padding slots get
// ~0) and store out(i, key) for i < max(ns, 256).  ns is a power of two <=
// kMaxSyms.
template <typename K, typename F, typename G>
__device__ __forceinline__ void sort_into(uint32_t ns, K *xch, F make, G out) {
    const uint32_t t = threadIdx.x;
    if (ns <= 256) {
        K k[1] = {t < ns ? make(t) : (K)~(K)0};
        sort_keys<1>(k, xch);
        out(t, k[0]);
    } else if (ns == 512) {
        K k[2];
#pragma unroll
        for (int r = 0; r < 2; r++) k[r] = make(t * 2 + r);
        sort_keys<2>(k, xch);
#pragma unroll
        for (int r = 0; r < 2; r++) out(t * 2 + r, k[r]);
    } else if (ns == 1024) {
        K k[4];
#pragma unroll
        for (int r = 0; r < 4; r++) k[r] = make(t * 4 + r);
        sort_keys<4>(k, xch);
#pragma unroll
        for (int r = 0; r < 4; r++) out(t * 4 + r, k[r]);
    } else {
        K k[8];
#pragma unroll
        for (int r = 0; r < 8; r++) k[r] = make(t * 8 + r);
        sort_keys<8>(k, xch);
#pragma unroll
        for (int r = 0; r < 8; r++) out(t * 8 + r, k[r]);
    }
    __syncthreads();
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
// symbols by (length, symbol) into `key` (entries (len << 16) | sym, unused
// symbols last as ~0), fills count / first_index / first_code per length.
struct CanonScratch {
    uint64_t key[kMaxSyms];
    uint64_t xch[kMaxSyms];
    uint64_t first_code[66];
    uint32_t count[66];
    uint32_t first_index[66];
    uint32_t wave_max[16];
    uint32_t n_used;
    uint32_t max_len;
    uint32_t kraft;   // 0: the lengths fill the code space exactly, 1: they overfill it, 2: they leave room
};

constexpr uint32_t kCanonGroups = kMaxSyms / 64;   // (chunk, wave) groups of 64 symbols
constexpr uint32_t kCanonStride = kCanonGroups + 1;

__device__ void canonical_order(const uint8_t *len, uint32_t ns, CanonScratch &c) {
    // stable counting sort of the symbols by code length.  Symbol tid + B * r
    // belongs to group (r, wave); the group's lanes of equal length are found
    // from eight ballots (one per bit of the length), which give each symbol
    // its rank within its group and lane L - 1 the group's count of length L.
    // One wave then turns the counts into per-length offsets of the groups.
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / 64, B = blockDim.x, W = B / 64;
    const uint32_t nk = ns < B ? B : ns;
    const uint32_t chunks = nk / B, groups = chunks * W;   // groups <= kCanonGroups
    uint32_t *cnt = reinterpret_cast<uint32_t *>(c.xch);   // [length - 1][group], row stride kCanonStride
    if (tid == 0) {
        c.count[0] = c.count[65] = 0;
        c.first_index[0] = c.first_index[65] = 0;
        c.first_code[0] = c.first_code[65] = 0;
    }
    constexpr uint32_t kChunks = kMaxSyms / 256;
    const uint64_t below = lanes_below(lane);
    uint32_t myrank[kChunks], mylen[kChunks];
    uint32_t ml = 0;
#pragma unroll
    for (uint32_t r = 0; r < kChunks; r++) {
        myrank[r] = 0;
        mylen[r] = 0;
        if (r >= chunks) continue;
        const uint32_t sym = tid + B * r;
        const uint32_t l = sym < ns ? len[sym] : 0u;
        ml = l > ml ? l : ml;
        uint64_t same = ~0ull, mine = ~0ull;
        const uint32_t L = lane + 1;
#pragma unroll
        for (uint32_t b = 0; b < 8; b++) {
            const uint64_t m = __ballot((l >> b) & 1u);
            same &= ((l >> b) & 1u) ? m : ~m;
            mine &= ((L >> b) & 1u) ? m : ~m;
        }
        myrank[r] = (uint32_t)__popcll(same & below);
        mylen[r] = l;
        cnt[lane * kCanonStride + r * W + w] = (uint32_t)__popcll(mine);
    }
    ml = wave_max<uint32_t>(ml);
    if (lane == 0) c.wave_max[w] = ml;
    __syncthreads();
    if (tid < 64) {
        // lane l - 1 stands for length l: exclusive prefix of its row over the
        // groups (in symbol order), then first_index is the exclusive prefix
        // of the counts; first_code[b] = sum_{j<b} count[j] << (b - j) (the
        // RFC 1951 recurrence code_b = (code_{b-1} + count_{b-1}) << 1, unrolled)
        // comes from a shift-weighted scan S_l = count_l + (S_{l-1} << 1),
        // first_code[l + 1] = S_l << 1; no partial sum exceeds 2^63 for l <= 62
        uint32_t max_len = 0;
        for (uint32_t k = 0; k < W; k++) max_len = c.wave_max[k] > max_len ? c.wave_max[k] : max_len;
        uint32_t v[kCanonGroups];
#pragma unroll
        for (uint32_t g = 0; g < kCanonGroups; g++) v[g] = g < groups ? cnt[tid * kCanonStride + g] : 0u;
        uint32_t run = 0;
#pragma unroll
        for (uint32_t g = 0; g < kCanonGroups; g++) {
            if (g < groups) cnt[tid * kCanonStride + g] = run;
            run += v[g];
        }
        const uint32_t l = tid + 1;
        const uint32_t cl = run;
        c.count[l] = cl;
        const uint32_t incl = wave_incl_scan<uint32_t>(cl);
        c.first_index[l] = incl - cl;
        // (the same doubling steps as a prefix sum: row shifts by 1, 2, 4, 8
        // weighted 2^k, then the row broadcasts weighted by the distance
        // from the broadcast lane)
        uint64_t S = cl;
        S += dpp_zero<0x111>(S) << 1;
        S += dpp_zero<0x112>(S) << 2;
        S += dpp_zero<0x114>(S) << 4;
        S += dpp_zero<0x118>(S) << 8;
        S += dpp_zero<0x142, 0xA>(S) << ((tid & 15u) + 1u);
        S += dpp_zero<0x143, 0xC>(S) << ((tid - 31u) & 63u);
        if (l + 1 <= 64) c.first_code[l + 1] = S << 1;
        if (tid == 0) c.first_code[1] = 0;
        // Kraft: S_l = sum_{j<=l} count_j 2^(l-j) may not exceed 2^l at any l
        // <= 63 (the first l that does is computed without overflow) and must
        // equal 2^max_len at the end
        const bool over = __ballot(l <= 63u && S > (1ull << (l & 63u))) != 0;
        const uint64_t S_top = __shfl(S, (int)((max_len >= 1u && max_len <= 64u ? max_len : 1u) - 1u), 64);
        if (tid == 63) {
            c.n_used = incl;
            c.max_len = max_len;
            c.kraft = over ? 1u : ((max_len >= 1u && max_len <= 63u && S_top == (1ull << max_len)) ? 0u : 2u);
        }
    }
    __syncthreads();
    // lengths above 64 (only reachable from damaged input) are reported
    // through max_len and otherwise left out of the order
    const uint32_t n_used = c.n_used;
#pragma unroll
    for (uint32_t r = 0; r < kChunks; r++) {
        if (r >= chunks) continue;
        const uint32_t sym = tid + B * r, l = mylen[r];
        if (l && l <= 64) c.key[c.first_index[l] + cnt[(l - 1) * kCanonStride + r * W + w] + myrank[r]] = ((uint64_t)l << 16) | sym;
    }
    for (uint32_t i = n_used + tid; i < nk; i += B) c.key[i] = ~0ull;
    __syncthreads();
}

// ---------------------------------------------------------------------------
// K2: histogram replicas -> lengths -> canonical codebook -> header + lengths
// ---------------------------------------------------------------------------
struct BookLds {
    CanonScratch canon;                  // key / xch double as the leaf sort buffers
    uint32_t leaf_w[kMaxSyms];
    uint32_t wave_fmax[kBookThreads / 64];
    uint16_t leaf_sym[kMaxSyms];
    uint32_t int_w[kMaxSyms];
    uint32_t merged_w[kMaxSyms];
    uint16_t parent_leaf[kMaxSyms];
    uint16_t parent_int[kMaxSyms];
    uint8_t depth_int[kMaxSyms];
    uint8_t len[kMaxSyms];
    uint32_t hist[kMaxSyms];
    uint8_t hdr[kHeaderBytes];
    uint32_t n;
    uint32_t ic_end, rounds;   // nodes made, merge rounds (for the other waves)
    unsigned long long total_bits;
};

// Numbers of entries <= t in the ascending arrays A[0, ma) and B[0, mb),
// found by one wave with 64-way probes of both arrays at once: about
// log64(m) dependent LDS reads.  The probe positions are uniform arithmetic,
// so no lane exchange is needed.
// Also returns A[ca - 1] and B[cb - 1] when ca, cb > 0 (read from the last
// probe window when they lie in it).
__device__ __forceinline__ void wave_count_le2(const uint32_t *A, uint32_t ma, const uint32_t *B, uint32_t mb,
                                               uint32_t t, uint32_t lane, uint32_t &ca, uint32_t &cb,
                                               uint32_t &lasta, uint32_t &lastb) {
    uint32_t loa = 0, hia = ma, lob = 0, hib = mb;   // each count lies in [lo, hi]
    while (hia - loa > 64 || hib - lob > 64) {
        const uint32_t sa = hia - loa, sb = hib - lob;
        const uint32_t ia = loa + (sa * (lane + 1)) / 65, ib = lob + (sb * (lane + 1)) / 65;
        const uint32_t va = A[sa > 64 ? ia : 0], vb = B[sb > 64 ? ib : 0];
        const uint32_t na = (uint32_t)__popcll(__ballot(va <= t)), nb = (uint32_t)__popcll(__ballot(vb <= t));
        if (sa > 64) {
            const uint32_t lo = na ? loa + (sa * na) / 65 + 1 : loa;
            hia = na < 64 ? loa + (sa * (na + 1)) / 65 : hia;
            loa = lo;
        }
        if (sb > 64) {
            const uint32_t lo = nb ? lob + (sb * nb) / 65 + 1 : lob;
            hib = nb < 64 ? lob + (sb * (nb + 1)) / 65 : hib;
            lob = lo;
        }
    }
    const uint32_t ia = loa + lane, ib = lob + lane;
    const uint32_t va = A[ia < hia ? ia : 0], vb = B[ib < hib ? ib : 0];
    ca = loa + (uint32_t)__popcll(__ballot(ia < hia && va <= t));
    cb = lob + (uint32_t)__popcll(__ballot(ib < hib && vb <= t));
    lasta = ca > loa ? (uint32_t)__builtin_amdgcn_readlane((int)va, (int)(ca - loa - 1)) : (ca ? A[ca - 1] : 0u);
    lastb = cb > lob ? (uint32_t)__builtin_amdgcn_readlane((int)vb, (int)(cb - lob - 1)) : (cb ? B[cb - 1] : 0u);
}

// LDS read at a clamped index: loads that may fall past a queue's end are
// issued unconditionally (their values are discarded), so independent
// reads go out together
__device__ __forceinline__ uint32_t ldc(const uint32_t *A, uint32_t i) { return A[i < kMaxSyms ? i : kMaxSyms - 1]; }

// Merges the ascending key sequences a and b (one key per lane each, 64
// each) in registers: afterwards a holds merged positions 0..63 and b
// positions 64..127, in lane order.  Bitonic: a followed by b reversed is
// bitonic; one in-lane compare splits it into two bitonic halves, each
// sorted by six cross-lane half-cleaners.
template <typename K>
__device__ __forceinline__ void wave_merge128(K &a, K &b, uint32_t lane) {
    const K br = __shfl(b, (int)(63u - lane), 64);
    K lo = a < br ? a : br, hi = a < br ? br : a;
#define DQZ_HALF_CLEAN(D)                                                   \
    {                                                                        \
        const K pl = xor_lane_t<D>(lo, lane), ph = xor_lane_t<D>(hi, lane);  \
        const bool low = (lane & (D)) == 0;                                  \
        lo = (low == (pl < lo)) ? pl : lo;                                   \
        hi = (low == (ph < hi)) ? ph : hi;                                   \
    }
    DQZ_HALF_CLEAN(32)
    DQZ_HALF_CLEAN(16)
    DQZ_HALF_CLEAN(8)
    DQZ_HALF_CLEAN(4)
    DQZ_HALF_CLEAN(2)
    DQZ_HALF_CLEAN(1)
#undef DQZ_HALF_CLEAN
    a = lo;
    b = hi;
}

// The merge rounds of the two-queue construction, in one wave (no barrier):
// leaf_w[0, n) ascending; internal nodes are appended to int_w (nondecreasing
// by construction) and parents recorded in parent_leaf / parent_int.  A round
// takes every item no heavier than T, the sum of the two lightest available
// items: nodes made later weigh at least T (and lose ties to leaves and to
// older nodes), so those items are exactly the next ones the sequential
// algorithm would merge, in the stable merge of the two queues (leaf first
// on equal weight), paired in order.  The merged order is built 64 positions
// at a time: the next 64 items of each queue, keyed (weight, queue, index),
// merged in registers; the first 64 results are the next 64 positions.  K:
// 32-bit keys when every weight (at most the total count) is below 2^25,
// else 64-bit.
template <typename K>
__device__ void wave_rounds(BookLds &s, uint32_t n, Ctl *ctl, uint32_t lane) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;   // no item (weights stay below 2^31)
    uint32_t la = 0, ib = 0, ic = 0, rounds = 0;
    for (;;) {
        if ((n - la) + (ic - ib) <= 1) break;
        if (la == n) {
            // Leaves used up: the internal queue is nondecreasing and every
            // node made from now on weighs at least its last item, so the
            // sequential algorithm pairs the queue front to back (oldest first
            // on ties) with no weight comparison left: item x of
            // [ib, ic + k - 2) gets parent ic + (x - ib) / 2 for the k = ic - ib
            // items left, the last node made being the root.
            const uint32_t k = ic - ib;
            for (uint32_t x = ib + lane; x < ic + k - 2; x += 64) s.parent_int[x] = (uint16_t)(ic + (x - ib) / 2);
            ib = ic + k - 2;
            ic += k - 1;
            rounds += 32u - __clz(k - 1u);   // ceil(log2 k) levels: the bound on the depth
            break;
        }
        // both queue windows requested together (clamped reads, the lanes
        // past a queue's end then set to kNone)
        const uint32_t lw_raw = ldc(s.leaf_w, la + lane), iw_raw = ldc(s.int_w, ib + lane);
        const uint32_t lw = la + lane < n ? lw_raw : kNone;
        const uint32_t iw = ib + lane < ic ? iw_raw : kNone;
        // T, from the first two items of each queue
        const uint32_t l0 = (uint32_t)__builtin_amdgcn_readlane((int)lw, 0);
        const uint32_t l1 = (uint32_t)__builtin_amdgcn_readlane((int)lw, 1);
        const uint32_t i0 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 0);
        const uint32_t i1 = (uint32_t)__builtin_amdgcn_readlane((int)iw, 1);
        uint32_t Tw;
        {
            uint32_t a = 0, b = 0, t = 0;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const uint32_t lv = a == 0 ? l0 : l1, iv = b == 0 ? i0 : i1;
                const bool leaf = la + a < n && (ib + b >= ic || lv <= iv);
                t += leaf ? lv : iv;
                a += leaf ? 1u : 0u;
                b += leaf ? 0u : 1u;
            }
            Tw = t;
        }
        // items of weight <= T: prefixes of both sorted queues (beyond the
        // windows by 64-way probes)
        uint32_t nl = (uint32_t)__popcll(__ballot(la + lane < n && lw <= Tw));
        uint32_t ni = (uint32_t)__popcll(__ballot(ib + lane < ic && iw <= Tw));
        uint32_t lastl, lasti;
        if (nl == 64 || ni == 64) {
            wave_count_le2(s.leaf_w + la, n - la, s.int_w + ib, ic - ib, Tw, lane, nl, ni, lastl, lasti);
        } else {
            lastl = nl ? (uint32_t)__builtin_amdgcn_readlane((int)lw, (int)(nl - 1)) : 0u;
            lasti = ni ? (uint32_t)__builtin_amdgcn_readlane((int)iw, (int)(ni - 1)) : 0u;
        }
        if ((nl + ni) & 1u) {   // odd: the last item of the merged order waits
            const bool int_last = ni > 0 && (nl == 0 || lasti >= lastl);
            if (int_last) ni--; else nl--;
        }
        if (nl + ni < 2) {   // cannot happen for sorted queues: stop rather than spin
            if (lane == 0) atomicOr(&ctl->status, ST_EINTERNAL);
            break;
        }
        const uint32_t m = nl + ni;
        uint32_t i = 0, j = 0;   // leaves and internals placed so far this round
        for (uint32_t d = 0; d < m; d += 64) {
            const uint32_t wl_raw = d == 0 ? lw : ldc(s.leaf_w, la + i + lane);
            const uint32_t wi_raw = d == 0 ? iw : ldc(s.int_w, ib + j + lane);
            const uint32_t wl = d == 0 ? lw : (i + lane < nl ? wl_raw : kNone);
            const uint32_t wi = d == 0 ? iw : (j + lane < ni ? wi_raw : kNone);
            // key: weight, then queue (leaf first), then position in the queue
            K ka = i + lane < nl ? ((K)wl << 7) | lane : (K)~(K)0;
            K kb = j + lane < ni ? ((K)wi << 7) | 64u | lane : (K)~(K)0;
            wave_merge128<K>(ka, kb, lane);
            const uint32_t cnt = m - d < 64 ? m - d : 64u;   // even
            const bool mine = lane < cnt;
            const bool is_leaf = (ka & 64u) == 0;
            const uint32_t k = (uint32_t)(ka & 63u), w = (uint32_t)(ka >> 7);
            const uint32_t node = ic + ((d + lane) >> 1);
            if (mine) {
                if (is_leaf) s.parent_leaf[la + i + k] = (uint16_t)node;
                else s.parent_int[ib + j + k] = (uint16_t)node;
            }
            const uint32_t wp = xor_lane32<1>(w, lane);
            if (mine && !(lane & 1u)) s.int_w[node] = w + wp;
            const uint32_t leaves = (uint32_t)__popcll(__ballot(mine && is_leaf));
            i += leaves;
            j += cnt - leaves;
        }
        la += nl;
        ib += ni;
        ic += m / 2;
        rounds++;
    }
    if (lane == 0) {
        s.ic_end = ic;
        s.rounds = rounds;
    }
}

__global__ __launch_bounds__(kBookThreads) void k_codebook(const uint32_t *__restrict__ hist, Ctl *ctl,
                                                           uint64_t *__restrict__ book, uint32_t *__restrict__ book32,
                                                           uint8_t *archive, Layout L, Geom g, HeaderArgs hdr,
                                                           TileScan qscan,
                                                           Readback *rb) {
    __shared__ BookLds s;
    __shared__ uint64_t s_red[4];
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t ns = L.nsym;
    if (ctl->status & (ST_EINVAL | ST_EINTERNAL)) {
        if (tid == 0) publish_status(rb, ctl->status);   // the host reads this block after the stream ends
        return;
    }
    if (tid == 0) ctl->phase[0] = wall_clock64();

    // the histogram (replicas already summed by the segment scan)
    {
        constexpr uint32_t kPer = kMaxSyms / kBookThreads;
        uint32_t f[kPer];
#pragma unroll
        for (uint32_t k = 0; k < kPer; k++) {
            const uint32_t i = tid + kBookThreads * k;
            f[k] = (i < ns) ? hist[i] : 0u;
        }
        uint32_t fm = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPer; k++) {
            const uint32_t i = tid + kBookThreads * k;
            if (i < ns) { s.hist[i] = f[k]; s.len[i] = 0; }
            fm = f[k] > fm ? f[k] : fm;
        }
        fm = wave_max<uint32_t>(fm);
        if (lane_id() == 0) s.wave_fmax[tid / 64] = fm;
    }
    if (tid == 0) { s.n = 0; s.total_bits = 0; s.ic_end = 0; s.rounds = 0; }
    __syncthreads();
    // exception totals from the quantize tiles' segment totals
    {
        const uint64_t exc = scan_total(qscan, 0, s_red);
        const uint64_t out = scan_total(qscan, 1, s_red);
        if (tid == 0) { ctl->exc_total = exc; ctl->out_total = out; }
    }
    if (tid == 0) ctl->phase[1] = wall_clock64();
    // leaves with nonzero frequency sorted by (frequency, symbol), on 32-bit
    // keys (frequency << symbol bits | symbol) when they fit, else 64-bit;
    // sorted entries go to key[] as (frequency << 16) | symbol
    {
        uint32_t fmax = 0;
        for (uint32_t k = 0; k < kBookThreads / 64; k++) fmax = s.wave_fmax[k] > fmax ? s.wave_fmax[k] : fmax;
        const uint32_t sb = 32u - __clz(ns - 1u);   // symbol bits (ns is a power of two >= 2)
        uint64_t *key = s.canon.key;
        if (sb < 32u && (uint64_t)fmax + 1u < (1ull << (32u - sb))) {
            sort_into<uint32_t>(ns, reinterpret_cast<uint32_t *>(s.canon.xch), [&](uint32_t i) -> uint32_t {
                return (i < ns && s.hist[i]) ? ((s.hist[i] << sb) | i) : ~0u;
            }, [&](uint32_t i, uint32_t k) {
                key[i] = k == ~0u ? ~0ull : (((uint64_t)(k >> sb) << 16) | (k & ((1u << sb) - 1u)));
            });
        } else {
            sort_into<uint64_t>(ns, s.canon.xch, [&](uint32_t i) -> uint64_t {
                return (i < ns && s.hist[i]) ? (((uint64_t)s.hist[i] << 16) | i) : ~0ull;
            }, [&](uint32_t i, uint64_t k) { key[i] = k; });
        }
    }
    const uint32_t nk = ns < 256 ? 256 : ns;
    for (uint32_t i = tid; i < nk; i += T) {
        const uint64_t k = s.canon.key[i];
        if (k != ~0ull) {
            s.leaf_w[i] = (uint32_t)(k >> 16);
            s.leaf_sym[i] = (uint16_t)(k & 0xFFFF);
            if (i + 1 == nk || s.canon.key[i + 1] == ~0ull) s.n = i + 1;
        }
    }
    __syncthreads();
    const uint32_t n = s.n;
    if (tid == 0) ctl->phase[2] = wall_clock64();
    if (n == 1) {
        if (tid == 0) s.len[s.leaf_sym[0]] = 1;
    } else if (n > 1) {
        if (tid < 64) {
            if (g.nelem < (1ull << 25)) wave_rounds<uint32_t>(s, n, ctl, tid);   // weights sum to the count of values
            else wave_rounds<uint64_t>(s, n, ctl, tid);
        }
        __syncthreads();
        const uint32_t ic = s.ic_end, rounds = s.rounds;
        if (tid == 0) { ctl->phase[3] = wall_clock64(); ctl->phase[8] = rounds; }
        // depths of the internal nodes by pointer jumping: the root is the last
        // node made; a node's depth is the length of its parent chain, doubled
        // per step (ping-pong between two copies), about log2(rounds) steps
        {
            uint16_t *pa = s.parent_int, *pb = reinterpret_cast<uint16_t *>(s.merged_w);
            uint8_t *da = s.depth_int, *db = reinterpret_cast<uint8_t *>(s.merged_w) + 2 * kMaxSyms;
            const uint32_t root = ic - 1;
            for (uint32_t k = tid; k < ic; k += T) {
                da[k] = k == root ? 0 : 1;
                if (k == root) pa[k] = (uint16_t)root;
            }
            __syncthreads();
            for (uint32_t span = 1; span < rounds + 1; span <<= 1) {
                for (uint32_t k = tid; k < ic; k += T) {
                    const uint32_t q = pa[k];
                    db[k] = (uint8_t)(da[k] + da[q]);
                    pb[k] = pa[q];
                }
                __syncthreads();
                uint16_t *tp = pa; pa = pb; pb = tp;
                uint8_t *td = da; da = db; db = td;
            }
            if (da != s.depth_int)
                for (uint32_t k = tid; k < ic; k += T) s.depth_int[k] = da[k];
            __syncthreads();
        }
        for (uint32_t i = tid; i < n; i += T) {
            const uint32_t d = (uint32_t)s.depth_int[s.parent_leaf[i]] + 1u;
            s.len[s.leaf_sym[i]] = (uint8_t)(d > 255 ? 255 : d);
        }
    }
    __syncthreads();

    // canonical codes; the fixed-width codeword form (Sec. 3.2.2) is 32-bit
    // (len << 24 | code) when every code fits in 24 bits, else 64-bit
    if (tid == 0) ctl->phase[4] = wall_clock64();
    canonical_order(s.len, ns, s.canon);
    if (tid == 0) ctl->phase[5] = wall_clock64();
    const uint32_t max_len = s.canon.max_len;
    for (uint32_t i = tid; i < nk; i += T) {
        const uint64_t k = s.canon.key[i];
        if (k == ~0ull) continue;
        const uint32_t l = (uint32_t)(k >> 16), sym = (uint32_t)(k & 0xFFFF);
        const uint64_t code = s.canon.first_code[l] + (i - s.canon.first_index[l]);
        book[sym] = ((uint64_t)l << 56) | code;
        if (max_len <= 24) book32[sym] = (l << 24) | (uint32_t)code;
    }
    uint64_t my_bits = 0;
    for (uint32_t sym = tid; sym < ns; sym += T) {
        if (s.len[sym] == 0) {
            book[sym] = 0;
            book32[sym] = 0;
        }
        my_bits += (uint64_t)s.hist[sym] * s.len[sym];
    }
    {
        const uint64_t tb = block_sum256(my_bits, s_red);
        if (tid == 0) s.total_bits = tb;
    }
    __syncthreads();

    if (tid == 0) {
        ctl->phase[6] = wall_clock64();
        if (max_len > 64) atomicOr(&ctl->status, ST_EUNSUPPORTED);
        const uint64_t total_bits = s.total_bits;
        const uint64_t n_words = (total_bits + 31) / 32;
        const uint32_t n_exc = (uint32_t)ctl->exc_total;
        ctl->n_exc = n_exc;
        ctl->n_out = (uint32_t)ctl->out_total;
        ctl->n_patch = (uint32_t)(ctl->exc_total - ctl->out_total);
        const uint64_t off_str = L.off_exc + 8ull * n_exc;
        const uint64_t end = off_str + 4ull * n_words;
        ctl->max_len = max_len;
        ctl->total_bits = total_bits;
        ctl->n_words = n_words;
        ctl->off_str = off_str;
        ctl->archive_bytes = end;
        if (end > L.cap) atomicOr(&ctl->status, ST_ETOOSMALL);
        // header (assembled in LDS, then copied out by all threads)
        uint8_t *hb = s.hdr;
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
        put_le(hb, 117, L.layers - 1, 1);
        put_le(hb, 120, end, 8);
    }
    __syncthreads();
    // header + lengths into the archive (the host checked that the fixed
    // sections fit the capacity); zero the alignment pads
    for (uint32_t i = tid; i < kHeaderBytes; i += T) {
        archive[i] = s.hdr[i];
        ctl->header[i] = s.hdr[i];
        rb->header[i] = s.hdr[i];
    }
    if (tid == 0) {
        // the host's readback block (pinned host memory): final once this
        // kernel ends, since the encoding kernels add no status
        rb->archive_bytes = ctl->archive_bytes;
        rb->workspace_need = (ctl->status & ST_ENOMEM) ? L.ws_fixed + 8ull * ctl->pool_used : 0ull;
        publish_status(rb, ctl->status);
    }
    for (uint32_t i = tid; i < ns; i += T) archive[L.off_len + i] = s.len[i];
    for (uint64_t i = L.off_len + ns + tid; i < L.off_chunk; i += T) archive[i] = 0;
    for (uint64_t i = L.off_sub + 2ull * L.n_sub + tid; i < L.off_exc; i += T) archive[i] = 0;
    if (tid == 0) ctl->phase[7] = wall_clock64();
}

void launch_codebook(hipStream_t st, const Geom &g, const Layout &L, Ctl *ctl, const uint32_t *hist, uint64_t *book,
                     uint32_t *book32, uint8_t *archive, int eb_mode, double eb_param, const TileScan &qscan,
                     Readback *rb) {
    HeaderArgs h;
    h.dims[0] = g.n[0];
    h.dims[1] = g.n[1];
    h.dims[2] = g.n[2];
    h.eb_param = eb_param;
    h.ndim = g.ndim;
    h.eb_mode = (uint32_t)eb_mode;
    hipLaunchKernelGGL(k_codebook, dim3(1), dim3(kBookThreads), 0, st, hist, ctl, book, book32, archive, L, g, h, qscan, rb);
}

// ---------------------------------------------------------------------------
// D0: archive code lengths -> canonical decoding tables (the first
// kTableGroups workgroups, each ordering the codes and filling a share of
// the lookup tables).  Workgroup 0 validates that the lengths describe a
// complete prefix code (or one symbol of length 1).  The other workgroups
// index the exception list by
// reconstruction unit (512 padded positions): unit_exc[u] is the first
// record at or after the unit's first position, found by binary search, and
// every adjacent pair of keys is checked to increase.
// ---------------------------------------------------------------------------
__device__ void exception_index(const uint2 *exc, uint32_t n_exc, uint32_t *unit_exc, uint32_t n_units,
                                Readback *rb, uint32_t i) {
    if (i <= n_units) {
        const uint64_t key = 2ull * ((uint64_t)i << kUnitShift);
        uint32_t lo = 0, hi = n_exc;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((uint64_t)exc[mid].x < key) lo = mid + 1; else hi = mid;
        }
        unit_exc[i] = lo;
    }
    if (i > 0 && i < n_exc && exc[i - 1].x >= exc[i].x) publish_status(rb, ST_ECORRUPT);
    // with increasing keys, every record then lies in some unit
    if (i + 1 == n_exc && ((exc[i].x >> 1) >> kUnitShift) >= n_units) publish_status(rb, ST_ECORRUPT);
}

// Second-level table: the long-code prefixes are the top of the first
// level, [V0, 2^kLutBits) (canonical codes of <= kLutBits bits come first).
// With b the largest width in 1..7 for which all of them fit kLut2Max
// entries (or as many as fit at width 1), entry (v - V0) * 2^b + i holds the
// code whose first kLutBits + b bits are v, i, when it is that short (0
// otherwise: the decoder then takes the canonical limits).
// The length of the code that a left-aligned stream window w starts with,
// given that it is longer than kLutBits: the first l in (kLutBits, max_len)
// with w < lim[l], else max_len (lim is nondecreasing: the left-aligned end
// of the codes of length <= l), by binary search.
__device__ __forceinline__ uint32_t long_code_len(const uint64_t *lim, uint64_t w, uint32_t max_len) {
    uint32_t lo = kLutBits + 1, hi = max_len > lo ? max_len : lo;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (w >= lim[mid]) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// lim[l] for l = 0..64 (lim[0] = 0, lim[64] = ~0), one workgroup
__device__ void build_limits(const CanonScratch &c, uint64_t *lim) {
    for (uint32_t l = threadIdx.x; l < 65; l += blockDim.x)
        lim[l] = (l == 0) ? 0ull : (l == 64 ? ~0ull : ((c.first_code[l] + c.count[l]) << (64 - l)));
}

// Entries [part * ceil(n / parts), ...) of the second level (workgroup
// `part` of `parts`; part 0 also stores the table's parameters).
__device__ void build_lut2(const CanonScratch &c, DecodeTables *tab, const uint64_t *lim, uint32_t part,
                           uint32_t parts) {
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t max_len = c.max_len;
    // codes of <= kLutBits bits fill [0, V0) of the prefixes; no long codes: V0 = 2^kLutBits
    const uint32_t V0 = max_len > kLutBits ? (uint32_t)(lim[kLutBits] >> (64 - kLutBits)) : (1u << kLutBits);
    const uint32_t n_long = (1u << kLutBits) - V0;
    uint32_t b = 7;
    while (b > 1 && (n_long << b) > kLut2Max) b--;
    const uint32_t n2 = (n_long << b) < kLut2Max ? (n_long << b) : kLut2Max;
    if (part == 0 && tid == 0) {
        tab->lut2_v0 = V0;
        tab->lut2_bits = b;
        tab->lut2_n = n2;
    }
    const uint32_t per = (n2 + parts - 1) / parts, j1 = (part + 1) * per < n2 ? (part + 1) * per : n2;
    for (uint32_t j = part * per + tid; j < j1; j += T) {
        const uint64_t wv = (uint64_t)((V0 << b) + j) << (64 - kLutBits - b);
        const uint32_t l = long_code_len(lim, wv, max_len);
        uint32_t e = 0;
        if (l <= kLutBits + b) {
            const uint64_t code = wv >> (64 - l);
            const uint64_t d = code - c.first_code[l];
            if (code >= c.first_code[l] && d < c.count[l])
                e = (l << 11) | (uint32_t)(c.key[c.first_index[l] + (uint32_t)d] & 0x7FF);
        }
        // when not every long prefix fits, the last entry stands for the rest
        // (lookups past the table are clamped to it): it must send them on
        if (j + 1 == n2 && (n_long << b) > kLut2Max) e = 0;
        tab->lut2[j] = (uint16_t)e;
    }
}

__global__ __launch_bounds__(kTableThreads) void k_decode_tables(const uint8_t *__restrict__ archive, Layout L,
                                                                uint32_t max_len_hdr, DecodeTables *tab, Readback *rb,
                                                                uint32_t n_exc, uint32_t *unit_exc, uint32_t n_units) {
    if (blockIdx.x >= kTableGroups) {
        exception_index(reinterpret_cast<const uint2 *>(archive + L.off_exc), n_exc, unit_exc, n_units, rb,
                        (blockIdx.x - kTableGroups) * blockDim.x + threadIdx.x);
        return;
    }
    // each table workgroup orders the codes itself and fills its share of
    // both lookup levels; workgroup 0 also stores the validation result and
    // the canonical arrays
    const uint32_t part = blockIdx.x;
    __shared__ CanonScratch c;
    __shared__ uint8_t len[kMaxSyms];
    __shared__ uint32_t s_bad;
    const uint32_t tid = threadIdx.x, T = blockDim.x, ns = L.nsym;
    if (tid == 0) s_bad = 0;
    if (part == 0 && tid == 0) {
        s_bad = 0;
        tab->phase[0] = wall_clock64();
        tab->phase[3] = 0;
        tab->phase[8] = ~0ull;
        for (uint32_t k = 9; k < 16; k++) tab->phase[k] = 0;
    }
    __syncthreads();
    for (uint32_t i = tid; i < ns; i += T) {
        len[i] = archive[L.off_len + i];
        if (len[i] > 63) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (part == 0 && tid == 0) { tab->status = ST_ECORRUPT; tab->max_len = 0; publish_status(rb, ST_ECORRUPT); }
        return;
    }
    canonical_order(len, ns, c);
    if (part == 0 && tid == 0) {
        tab->phase[1] = wall_clock64();
        // Kraft: the code space must be exactly filled (or a lone symbol of length 1)
        const bool lone = c.n_used == 1 && c.count[1] == 1;
        uint32_t st = 0;
        if (c.kraft == 1u || (!lone && c.n_used > 0 && c.kraft != 0u) || c.max_len != max_len_hdr || c.max_len > 63)
            st = ST_ECORRUPT;
        tab->status = st;
        if (st) publish_status(rb, st);   // the host reads this block after the stream ends
        tab->max_len = c.max_len;
    }
    if (part == 0) {
        for (uint32_t l = tid; l < 65; l += T) {
            tab->first_code[l] = c.first_code[l];
            tab->count[l] = c.count[l];
            tab->first_index[l] = c.first_index[l];
            // codes of length <= l occupy [0, limit) of the left-aligned code space
            tab->limit[l] = (l == 0) ? 0ull : (l == 64 ? ~0ull : ((c.first_code[l] + c.count[l]) << (64 - l)));
        }
        for (uint32_t i = tid; i < ns; i += T) {
            const uint64_t k = c.key[i];
            tab->sorted[i] = (k == ~0ull) ? 0 : (uint16_t)(k & 0xFFFF);
        }
    }
    // the left-aligned limits (the long-code searches below read them)
    build_limits(c, c.xch);
    __syncthreads();
    // each table slot v (the next kLutBits stream bits): its code length is
    // 1 + the number of lengths l <= kLutBits whose codes all lie below v
    // (canonical codes of length <= l fill [0, limit_l)); longer codes get the
    // shortest length that can follow the prefix
    // (the slot's code of length l is its top l bits; the codes of length l
    // are those of [lim_{l-1}, lim_l), so it is the code of canonical index
    // first_index_l + code - first_code_l)
    uint32_t lim[kLutBits + 1];
    int32_t base[kLutBits + 1];
#pragma unroll
    for (uint32_t l = 1; l <= kLutBits; l++) {
        lim[l] = (uint32_t)((c.first_code[l] + c.count[l]) << (kLutBits - l));
        base[l] = (int32_t)c.first_index[l] - (int32_t)c.first_code[l];
    }
    // the shortest length after a long-code prefix (computed once per
    // workgroup for the prefixes, which are the top of the table)
    constexpr uint32_t kSlots = (1u << kLutBits) / kTableGroups;   // this workgroup's: [part * kSlots, ...)
    constexpr uint32_t kPer = kSlots / kTableThreads;
    static_assert(kPer * kTableThreads * kTableGroups == (1u << kLutBits), "table slots per thread");
    const uint32_t v0 = part * kSlots;
    uint32_t slot_len[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
        const uint32_t v = v0 + tid + kTableThreads * i;
        uint32_t l = 1;
#pragma unroll
        for (uint32_t k = 1; k <= kLutBits; k++) l += (lim[k] <= v) ? 1u : 0u;
        slot_len[i] = l;
    }
    uint64_t key[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
        const uint32_t v = v0 + tid + kTableThreads * i, l = slot_len[i];
        int32_t b = 0;
#pragma unroll
        for (uint32_t k = 1; k <= kLutBits; k++) b = (l == k) ? base[k] : b;
        const uint32_t idx = (uint32_t)(b + (int32_t)(v >> ((kLutBits - l) & 31u)));
        key[i] = l <= kLutBits ? c.key[idx < kMaxSyms ? idx : 0u] : 0ull;
    }
#pragma unroll
    for (uint32_t i = 0; i < kPer; i++) {
        const uint32_t v = v0 + tid + kTableThreads * i, l = slot_len[i];
        uint32_t e = 0;
        if (l <= kLutBits) {
            e = (l << 11) | (uint32_t)(key[i] & 0x7FF);
        } else if (c.max_len > kLutBits) {
            // a long-code prefix: the shortest length that can follow
            e = 0x8000u | long_code_len(c.xch, (uint64_t)v << (64 - kLutBits), c.max_len);
        }
        tab->lut[v] = (uint16_t)e;
    }
    __syncthreads();
    // the second-level table (its limits, in the sort exchange buffer, were
    // built before the first level)
    build_lut2(c, tab, c.xch, part, kTableGroups);
    __syncthreads();
    if (part == 0 && tid == 0) tab->phase[2] = wall_clock64();
}

void launch_decode_tables(hipStream_t st, const Layout &L, const uint8_t *archive, uint32_t max_len_hdr,
                          DecodeTables *tab, Readback *rb, uint32_t n_exc, uint32_t *unit_exc,
                          uint32_t n_units) {
    // the first kTableGroups workgroups build the tables; the others index
    // the exception list
    const uint32_t idx_items = unit_exc ? (n_units + 1 > n_exc ? n_units + 1 : n_exc) : 0u;
    const uint32_t blocks = kTableGroups + (idx_items + kTableThreads - 1) / kTableThreads;
    hipLaunchKernelGGL(k_decode_tables, dim3(blocks), dim3(kTableThreads), 0, st, archive, L, max_len_hdr, tab,
                       rb, n_exc, unit_exc, n_units);
}

}  // namespace dqz
