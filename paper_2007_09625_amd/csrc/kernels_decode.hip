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
    const uint2 *exc;
    uint32_t n_exc;
    const DecodeTables *tab;
    uint32_t *status;
    float *out;
    float h;
    uint32_t wave_tasks;
    uint32_t qstride;   // LDS code-buffer stride per subchunk (sub_size + 2: spreads lanes over banks)
};

// Per-lane bit reader: `cur` holds the next 64 stream bits MSB-first
// (`avail` of them valid).  Stream words arrive through a queue of three
// prefetched 8-byte word pairs (q0 is being consumed, `qpos` = next word of
// q0), so each load is issued about 24 symbols before its bits are needed.
struct BitReader {
    uint64_t cur;
    uint64_t bp;       // stream position of the top bit of `cur`
    uint64_t q0, q1, q2;
    uint64_t pidx;     // next pair to load
    uint32_t qpos;
    int32_t avail;
};

__device__ __forceinline__ uint32_t ld_word(const DecArgs &a, uint64_t i) {
    return i < a.n_words ? a.words[i] : 0u;
}

__device__ __forceinline__ uint64_t ld_pair(const DecArgs &a, uint64_t p) {
    const uint64_t w = 2 * p;
    if (w + 1 < a.n_words) return reinterpret_cast<const uint64_t *>(a.words)[p];
    return (uint64_t)ld_word(a, w) | ((uint64_t)ld_word(a, w + 1) << 32);
}

__device__ __forceinline__ void br_init(const DecArgs &a, BitReader &br, uint64_t start) {
    const uint64_t w = start >> 5;
    const uint32_t o = (uint32_t)(start & 31u);
    const uint64_t p = w >> 1;
    const uint64_t P0 = ld_pair(a, p), P1 = ld_pair(a, p + 1), P2 = ld_pair(a, p + 2), P3 = ld_pair(a, p + 3);
    uint32_t w0, w1;
    if (w & 1u) { w0 = (uint32_t)(P0 >> 32); w1 = (uint32_t)P1; br.qpos = 1; }
    else { w0 = (uint32_t)P0; w1 = (uint32_t)(P0 >> 32); br.qpos = 0; }
    br.cur = (((uint64_t)w0 << 32) | w1) << o;
    br.avail = 64 - (int32_t)o;
    br.q0 = P1;
    br.q1 = P2;
    br.q2 = P3;
    br.pidx = p + 4;
    br.bp = start;
}

__device__ __forceinline__ void br_refill(const DecArgs &a, BitReader &br) {
    if (br.avail <= 32) {
        const uint32_t w = br.qpos ? (uint32_t)(br.q0 >> 32) : (uint32_t)br.q0;
        br.cur |= (uint64_t)w << (32 - br.avail);
        br.avail += 32;
        if (br.qpos) {
            br.q0 = br.q1;
            br.q1 = br.q2;
            br.q2 = ld_pair(a, br.pidx++);
            br.qpos = 0;
        } else {
            br.qpos = 1;
        }
    }
}

// LDS copy of the decoding tables
struct DecLds {
    uint64_t limit[65];
    uint64_t first_code[65];
    uint32_t first_index[65];
};

__device__ __forceinline__ uint32_t decode_one(const DecArgs &a, BitReader &br, const uint16_t *lut,
                                               const DecLds &t, const uint16_t *sorted, uint32_t max_len,
                                               bool &bad) {
    br_refill(a, br);
    const uint32_t e = lut[(uint32_t)(br.cur >> (64 - kLutBits))];
    uint32_t len, sym;
    if (!(e & 0x8000u)) {
        len = e >> 11;
        sym = e & 0x7FFu;
        if (len == 0) { bad = true; len = 1; }
    } else {
        // a longer code: canonical limits from the shortest possible length
        // (codes over 32 bits need a full 64-bit window from memory)
        uint32_t l = e & 63u;
        uint64_t win = br.cur;
        if (max_len > 32) {
            const uint64_t w = br.bp >> 5;
            const uint32_t o = (uint32_t)(br.bp & 31u);
            const uint64_t hi = ((uint64_t)ld_word(a, w) << 32) | ld_word(a, w + 1);
            win = o ? ((hi << o) | (ld_word(a, w + 2) >> (32 - o))) : hi;
        }
        while (l < max_len && win >= t.limit[l]) l++;
        const uint64_t c = win >> (64 - l);
        const uint64_t idx = t.first_index[l] + (c - t.first_code[l]);
        if (idx >= a.L.nsym) { bad = true; sym = a.L.radius; }
        else sym = sorted[idx];
        if ((int32_t)l > br.avail) {   // only possible for codes over 32 bits
            br_init(a, br, br.bp + l);
            return sym;
        }
        len = l;
    }
    br.cur <<= len;
    br.avail -= (int32_t)len;
    br.bp += len;
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

// code buffer slot -> wrapping delta
__device__ __forceinline__ uint32_t slot_delta(const DecArgs &a, uint16_t q, uint32_t e0, bool &bad) {
    if (q & 0x8000u) return a.exc[e0 + (q & 0x7FFFu)].y;
    if (q == 0) bad = true;
    return (uint32_t)q - a.L.radius;
}

__device__ __forceinline__ uint32_t lower_bound_key(const uint2 *exc, uint32_t n, uint64_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)exc[mid].x < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(64 * kDecMaxWaves) void k_decode(DecArgs a) {
    extern __shared__ uint32_t s_dyn[];
    __shared__ DecLds s_t;
    uint16_t *s_lut = reinterpret_cast<uint16_t *>(s_dyn);                       // 1 << kLutBits
    uint16_t *s_sorted = s_lut + (1u << kLutBits);                               // nsym
    uint16_t *s_q = s_sorted + a.L.nsym;                                         // waves * 64 * qstride
    if (a.tab->status) return;   // the code lengths failed validation: tables are not usable
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.tab->lut);
        uint32_t *dst = reinterpret_cast<uint32_t *>(s_lut);
        for (uint32_t i = threadIdx.x; i < (1u << kLutBits) / 2; i += blockDim.x) dst[i] = src[i];
        for (uint32_t i = threadIdx.x; i < a.L.nsym; i += blockDim.x) s_sorted[i] = a.tab->sorted[i];
        for (uint32_t i = threadIdx.x; i < 65; i += blockDim.x) {
            s_t.limit[i] = a.tab->limit[i];
            s_t.first_code[i] = a.tab->first_code[i];
            s_t.first_index[i] = a.tab->first_index[i];
        }
    }
    __syncthreads();

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

    if (active) {
        // ---- start bit of this lane's subchunk
        const uint64_t s = sub0 + lane;
        const bool has = s < a.L.n_sub;
        const uint8_t *subp = a.archive + a.L.off_sub;
        const uint32_t bits_s = has ? ((uint32_t)subp[2 * s] | ((uint32_t)subp[2 * s + 1] << 8)) : 0u;
        const uint32_t incl = wave_incl_scan<uint32_t>(bits_s);
        const uint32_t excl = incl - bits_s;
        const uint32_t C = a.L.chunk_subs;
        const uint64_t *chunks = reinterpret_cast<const uint64_t *>(a.archive + a.L.off_chunk);
        uint64_t start;
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
        // ---- inflate the subchunk into the LDS code buffer
        if (has) {
            const uint64_t pa = s << sh;
            const uint64_t pb = (pa + S) < a.g.padded ? (pa + S) : a.g.padded;
            uint16_t *myq = wq + lane * a.qstride;
            bool full;
            if (a.g.ndim == 1) {
                full = pb <= a.g.nelem;
            } else {
                full = true;
                for (uint32_t blk = (uint32_t)(pa / a.g.bvol); blk <= (uint32_t)((pb - 1) / a.g.bvol); blk++)
                    full = full && block_full(a.g, blk);
            }
            BitReader br;
            br_init(a, br, start);
            const uint32_t max_len = a.tab->max_len < 63u ? a.tab->max_len : 63u;
            const uint32_t cnt = (uint32_t)(pb - pa);
            if (full) {
                for (uint32_t i = 0; i < cnt; i++)
                    myq[i] = (uint16_t)decode_one(a, br, s_lut, s_t, s_sorted, max_len, bad);
            } else {
                for (uint32_t i = 0; i < cnt; i++)
                    myq[i] = pos_real(a.g, pa + i) ? (uint16_t)decode_one(a, br, s_lut, s_t, s_sorted, max_len, bad)
                                                   : (uint16_t)a.L.radius;
            }
            if (br.bp - start != bits_s) bad = true;
        }
        // ---- exception range of this wave
        uint32_t r0 = 0, r1 = 0;
        if (lane == 0) r0 = lower_bound_key(a.exc, a.n_exc, 2ull * P0);
        if (lane == 1) r1 = lower_bound_key(a.exc, a.n_exc, 2ull * P1);
        e0 = __shfl(r0, 0, 64);
        e1 = __shfl(r1, 1, 64);
    }
    __syncthreads();
    if (active) {
        // ---- outliers: mark their slots with an index into the exception list
        for (uint32_t e = e0 + lane; e < e1; e += 64) {
            const uint32_t key = a.exc[e].x;
            if (key & 1u) continue;
            const uint64_t loc = (uint64_t)(key >> 1) - P0;
            uint16_t *slot = wq + (loc >> sh) * a.qstride + (loc & (S - 1));
            if (*slot != 0 || e - e0 > 0x7FFFu) bad = true;
            else *slot = (uint16_t)(0x8000u | (e - e0));
        }
    }
    __syncthreads();
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
                for (uint32_t z = 0; z < 8; z++) {
                    uint32_t t = v[z];
                    uint32_t o = __shfl_up(t, 8, 64);  if (ly >= 1) t += o;
                    o = __shfl_up(t, 16, 64);           if (ly >= 2) t += o;
                    o = __shfl_up(t, 32, 64);           if (ly >= 4) t += o;
                    o = __shfl_up(t, 1, 64);            if (lx >= 1) t += o;
                    o = __shfl_up(t, 2, 64);            if (lx >= 2) t += o;
                    o = __shfl_up(t, 4, 64);            if (lx >= 4) t += o;
                    v[z] = t;
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
                uint32_t col = 0;
                for (uint32_t y = 0; y < 16; y++) {
                    if (ok) col += slot_delta(a, qat(base + y * 16 + lx), e0, bad);
                    uint32_t t = col;
                    uint32_t o = __shfl_up(t, 1, 64);  if (lx >= 1) t += o;
                    o = __shfl_up(t, 2, 64);            if (lx >= 2) t += o;
                    o = __shfl_up(t, 4, 64);            if (lx >= 4) t += o;
                    o = __shfl_up(t, 8, 64);            if (lx >= 8) t += o;
                    const uint32_t yy = By * 16 + y;
                    if (ok && x < g.n[2] && yy < g.n[1]) a.out[(uint64_t)yy * g.n[2] + x] = dequant((int32_t)t, h);
                }
            }
        } else {
            const uint32_t hl = lane % 32;
            for (uint64_t off = 0; P0 + off < P1; off += 64) {
                const uint64_t loc = off + lane;
                const uint64_t p = P0 + loc;
                uint32_t t = (p < P1) ? slot_delta(a, qat(loc), e0, bad) : 0u;
                uint32_t o = __shfl_up(t, 1, 64);  if (hl >= 1) t += o;
                o = __shfl_up(t, 2, 64);            if (hl >= 2) t += o;
                o = __shfl_up(t, 4, 64);            if (hl >= 4) t += o;
                o = __shfl_up(t, 8, 64);            if (hl >= 8) t += o;
                o = __shfl_up(t, 16, 64);           if (hl >= 16) t += o;
                if (p < g.nelem) a.out[p] = dequant((int32_t)t, h);
            }
        }
    }
    __syncthreads();   // all regular values are stored before patches overwrite some
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
}

static uint32_t decode_waves(const Layout &L) { return L.sub_size <= 256 ? kDecMaxWaves : 1u; }

size_t decode_lds_bytes(const Layout &L) {
    return sizeof(uint16_t) * ((1u << kLutBits) + L.nsym + (size_t)decode_waves(L) * 64 * (L.sub_size + 2));
}

void launch_decode(hipStream_t s, const Geom &g, const Layout &L, const uint8_t *archive, uint64_t off_str,
                   uint64_t n_words, uint32_t n_exc, float h, DecodeTables *tab, float *out) {
    DecArgs a;
    a.g = g;
    a.L = L;
    a.archive = archive;
    a.words = reinterpret_cast<const uint32_t *>(archive + off_str);
    a.n_words = n_words;
    a.exc = reinterpret_cast<const uint2 *>(archive + L.off_exc);
    a.n_exc = n_exc;
    a.tab = tab;
    a.status = &tab->status;
    a.out = out;
    a.h = h;
    a.wave_tasks = (L.n_sub + 63) / 64;
    a.qstride = L.sub_size + 2;
    if (a.wave_tasks == 0) return;
    const uint32_t waves = decode_waves(L);
    const uint32_t blocks = (a.wave_tasks + waves - 1) / waves;
    const size_t lds = decode_lds_bytes(L);
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)k_decode, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(64 * waves), lds, s, a);
}

}  // namespace dqz
