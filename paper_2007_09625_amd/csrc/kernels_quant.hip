// kernels_quant.hip -- error bound, range reduction and dual-quantization.
//
//   k_init      clears the control block and device counters; absolute-eb
//               mode derives h = fl32(2 eb), r = fl32(1 / (2 eb)) here.
//   k_minmax    finite min / max in IEEE total order for the
//               value-range-relative bound (footnote in Sec. 3.2.2); the
//               last workgroup derives eb_abs, h and r on the device.
//   k_quant{1,2,3}d
//               prequantization d° = round(x / 2eb) (Sec. 3.1.2), the
//               1-layer Lorenzo delta inside zero-padded blocks (Sec. 3.1.1),
//               postquantization with the +-R cap and outliers (Algorithm 2),
//               the rehearsal check that turns a missed bound into a patch
//               (Algorithm 1's watchdog), an LDS-privatized histogram of the
//               codes (Sec. 3.2.1), and the per-tile exception records.
//
// Each quantize workgroup handles one tile of kTile padded positions.  Its
// exception records (in stream order) go to the tile's staging slots and
// its record count is scanned across tiles by k_seg_scan; the encoder later
// copies the records to their final place.  The tile is staged in LDS
// with fully coalesced row loads; the Lorenzo delta is the mixed backward
// difference, computed per axis with registers (slow axis) and cross-lane
// shuffles (fast axes).
#include "dqz_internal.h"

#include <float.h>

namespace dqz {

// ---------------------------------------------------------------------------
// init / error bound
// ---------------------------------------------------------------------------
__device__ void derive_eb(Ctl *ctl, double e) {
    bool ok = isfinite(e) && e >= (double)FLT_MIN;
    const double two_e = 2.0 * e;
    const float h = (float)two_e;
    const float r = (float)(1.0 / two_e);
    ok = ok && isfinite(h) && isfinite(r) && r >= FLT_MIN;
    if (!ok) atomicOr(&ctl->status, ST_EINVAL);
    ctl->eb_abs = e;
    ctl->h = h;
    ctl->r = r;
}

// Clears the control block and the zeroed scratch (histogram replicas and
// their sum, encoder look-back states); shared by k_init and, in the
// value-range-relative mode, the range kernel (which saves a launch).
__device__ __forceinline__ void clear_scratch(Ctl *ctl, uint32_t *zero_base, uint64_t zero_words) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = tid; i < zero_words; i += stride) zero_base[i] = 0u;
    if (tid == 0) {
        uint32_t *c = reinterpret_cast<uint32_t *>(ctl);
        for (uint32_t i = 0; i < sizeof(Ctl) / 4; i++) c[i] = 0u;
        ctl->vmin_key = 0xFFFFFFFFu;
        ctl->vmax_key = 0u;
    }
}

__global__ void k_init(Ctl *ctl, uint32_t *zero_base, uint64_t zero_words, int eb_mode, double eb) {
    clear_scratch(ctl, zero_base, zero_words);
    if (blockIdx.x == 0 && threadIdx.x == 0 && eb_mode == 0) derive_eb(ctl, eb);
}

void launch_init(hipStream_t s, Ctl *ctl, void *zero_base, uint64_t zero_bytes, int eb_mode, double eb) {
    const uint64_t words = zero_bytes / 4;
    uint32_t blocks = (uint32_t)((words + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, ctl, (uint32_t *)zero_base, words, eb_mode, eb);
}

// One thread: a readback block's status and archive size (the asynchronous
// decompression's result before its kernels run; they overwrite it on damage).
__global__ void k_publish(Readback *rb, uint32_t bits, uint64_t archive_bytes) {
    rb->archive_bytes = archive_bytes;
    rb->workspace_need = 0;
    publish_status(rb, bits);
}

void launch_publish(hipStream_t s, Readback *rb, uint32_t bits, uint64_t archive_bytes) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, s, rb, bits, archive_bytes);
}

__device__ __forceinline__ void key_acc(uint32_t u, uint32_t &lo, uint32_t &hi) {
    if ((u & 0x7F800000u) != 0x7F800000u) {   // finite
        const uint32_t k = f2key(u);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
}

// Pass 1: each workgroup reduces its grid-stride share and writes one
// (min key, max key) pair; no atomics (same-address device atomics
// serialize across the whole chip).
__global__ __launch_bounds__(256) void k_minmax(const float *__restrict__ x, uint64_t n, uint32_t *partials, Ctl *ctl,
                                                uint32_t *zero_base, uint64_t zero_words) {
    clear_scratch(ctl, zero_base, zero_words);
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t *u = reinterpret_cast<const uint32_t *>(x);
    if ((reinterpret_cast<uintptr_t>(x) & 15u) == 0) {
        const uint64_t n4 = n / 4;
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 *v = reinterpret_cast<const u32x4 *>(x);
        // four independent 16-byte loads in flight per thread per iteration
        uint64_t i = tid;
        for (; i + 3 * stride < n4; i += 4 * stride) {
            u32x4 w[4];
#pragma unroll
            for (int k = 0; k < 4; k++) w[k] = __builtin_nontemporal_load(v + i + k * stride);
#pragma unroll
            for (int k = 0; k < 4; k++) {
                key_acc(w[k].x, lo, hi);
                key_acc(w[k].y, lo, hi);
                key_acc(w[k].z, lo, hi);
                key_acc(w[k].w, lo, hi);
            }
        }
        for (; i < n4; i += stride) {
            const u32x4 w = __builtin_nontemporal_load(v + i);
            key_acc(w.x, lo, hi);
            key_acc(w.y, lo, hi);
            key_acc(w.z, lo, hi);
            key_acc(w.w, lo, hi);
        }
        for (uint64_t j = n4 * 4 + tid; j < n; j += stride) key_acc(u[j], lo, hi);
    } else {
        for (uint64_t j = tid; j < n; j += stride) key_acc(u[j], lo, hi);
    }
    lo = ~wave_max<uint32_t>(~lo);
    hi = wave_max<uint32_t>(hi);
    __shared__ uint32_t s_lo[4], s_hi[4];
    const uint32_t w = threadIdx.x / 64;
    if (lane_id() == 0) { s_lo[w] = lo; s_hi[w] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t k = 1; k < blockDim.x / 64; k++) {
            lo = s_lo[k] < lo ? s_lo[k] : lo;
            hi = s_hi[k] > hi ? s_hi[k] : hi;
        }
        partials[2 * blockIdx.x] = lo;
        partials[2 * blockIdx.x + 1] = hi;
    }
}

// Pass 2 (one workgroup): combine the partials, derive eb_abs, h, r.
__global__ __launch_bounds__(256) void k_minmax_final(const uint32_t *partials, uint32_t nparts, Ctl *ctl,
                                                      double valrel) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) {
        const uint32_t a = partials[2 * i], b = partials[2 * i + 1];
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    lo = ~wave_max<uint32_t>(~lo);
    hi = wave_max<uint32_t>(hi);
    __shared__ uint32_t s_lo[4], s_hi[4];
    const uint32_t w = threadIdx.x / 64;
    if (lane_id() == 0) { s_lo[w] = lo; s_hi[w] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t i = 1; i < blockDim.x / 64; i++) {
            lo = s_lo[i] < lo ? s_lo[i] : lo;
            hi = s_hi[i] > hi ? s_hi[i] : hi;
        }
        ctl->vmin_key = lo;
        ctl->vmax_key = hi;
        double range = 1.0;
        if (lo != 0xFFFFFFFFu) {   // at least one finite value
            const float fmin = __uint_as_float(key2f(lo));
            const float fmax = __uint_as_float(key2f(hi));
            const double d = (double)fmax - (double)fmin;
            if (d > 0.0) range = d;
        }
        derive_eb(ctl, valrel * range);
    }
}

void launch_minmax(hipStream_t s, const float *x, uint64_t n, Ctl *ctl, uint32_t *partials, double valrel, int ncu,
                   void *zero_base, uint64_t zero_bytes) {
    uint64_t want = (n / 4 + 255) / 256;
    uint64_t cap = (uint64_t)ncu * 8;
    if (cap > kMinmaxMaxBlocks) cap = kMinmaxMaxBlocks;
    uint32_t blocks = (uint32_t)(want < cap ? want : cap);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_minmax, dim3(blocks), dim3(256), 0, s, x, n, partials, ctl, (uint32_t *)zero_base,
                       zero_bytes / 4);
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(256), 0, s, partials, blocks, ctl, valrel);
}

// Range of a field compressed slab by slab: fold one slab's (min key, max
// key), as the range kernels left them in the control block, into acc[0..1]
// (the first slab initializes it).  One thread.
__global__ void k_range_fold(const Ctl *ctl, uint32_t *acc, uint32_t first) {
    const uint32_t lo = ctl->vmin_key, hi = ctl->vmax_key;
    acc[0] = (first || lo < acc[0]) ? lo : acc[0];
    acc[1] = (first || hi > acc[1]) ? hi : acc[1];
}

void launch_range_fold(hipStream_t s, const Ctl *ctl, uint32_t *acc, bool first) {
    hipLaunchKernelGGL(k_range_fold, dim3(1), dim3(1), 0, s, ctl, acc, first ? 1u : 0u);
}

// ---------------------------------------------------------------------------
// shared pieces of the quantize kernels
// ---------------------------------------------------------------------------
struct QuantArgs {
    const float *x;
    Geom g;
    Layout L;
    Ctl *ctl;
    QuantBufs b;
    uint32_t n_tiles;
    uint32_t tiles_per_row;
};

// LDS histogram privatization: one replica per workgroup, flushed once into
// one of kHistReplicas global copies (summed by the codebook kernel).
__device__ __forceinline__ void hist_flush(uint32_t *sh_hist, uint32_t nsym, uint32_t *ghist) {
    uint32_t *dst = ghist + (blockIdx.x % kHistReplicas) * nsym;
    for (uint32_t b = threadIdx.x; b < nsym; b += blockDim.x) {
        const uint32_t c = sh_hist[b];
        if (c) atomicAdd(dst + b, c);
    }
}

// Each wave reports its record count; returns the wave's first record index
// inside the tile and the tile totals.
__device__ __forceinline__ uint32_t wave_base_in_tile(uint32_t wave_count, uint32_t wave_out, uint32_t *sh,
                                                      uint32_t &tile_count, uint32_t &tile_out) {
    const uint32_t w = threadIdx.x / 64, nw = blockDim.x / 64;
    if (lane_id() == 0) { sh[w] = wave_count; sh[8 + w] = wave_out; }
    __syncthreads();
    uint32_t base = 0, tot = 0, tout = 0;
    for (uint32_t i = 0; i < nw; i++) {
        if (i < w) base += sh[i];
        tot += sh[i];
        tout += sh[8 + i];
    }
    tile_count = tot;
    tile_out = tout;
    return base;
}

// Record idx of the tile (in stream order): the first `cap` go to the tile's
// staging slot, the rest to its run of the overflow pool starting at `ovf`.
__device__ __forceinline__ void put_exc(const QuantArgs &a, uint32_t tile, uint32_t idx, uint32_t key, uint32_t payload,
                                        uint32_t ovf) {
    uint2 rec;
    rec.x = key;
    rec.y = payload;
    if (idx < a.b.cap) {
        a.b.stage[(uint64_t)tile * a.b.cap + idx] = rec;
    } else {
        const uint64_t j = (uint64_t)ovf + (idx - a.b.cap);
        if (j < a.b.pool_cap) a.b.pool[j] = rec;
    }
}

// A tile with more records than its slot takes a run of the overflow pool
// (one device atomic, on this rare path only); a pool too small for every
// run is reported as ST_ENOMEM, with the records it needed in pool_used.
// tile_count is the same for every thread, so the barrier is uniform.
__device__ __forceinline__ uint32_t reserve_overflow(const QuantArgs &a, uint32_t tile, uint32_t tile_count,
                                                     uint32_t *sh) {
    if (tile_count <= a.b.cap) return 0u;
    if (threadIdx.x == 0) {
        const uint64_t n = tile_count - a.b.cap;
        const uint64_t base = atomicAdd((unsigned long long *)&a.ctl->pool_used, (unsigned long long)n);
        if (base + n > a.b.pool_cap) atomicOr(&a.ctl->status, ST_ENOMEM);
        a.b.ovf_base[tile] = (uint32_t)base;
        sh[12] = (uint32_t)base;
    }
    __syncthreads();
    return sh[12];
}

// Tile epilogue shared by all dimensionalities: overflow flag, histogram
// flush, and the wait-free scan of the record counts.
__device__ __forceinline__ void tile_epilogue(const QuantArgs &a, uint32_t tile, uint32_t tile_count, uint32_t tile_out,
                                              uint32_t *sh_hist, uint64_t *sh64) {
    (void)tile_count;
    __syncthreads();
    hist_flush(sh_hist, a.L.nsym, a.b.hist);
    tile_publish(a.b.scan, tile, tile_count, tile_out);
    (void)sh64;
}

// ---------------------------------------------------------------------------
// 3D: tile = 8 consecutive 8x8x8 blocks along x in one block row.
// Wave w handles blocks 2w, 2w+1; lane (y, x) = (lane / 8, lane % 8) holds
// the 8 points of its z column in registers.
// ---------------------------------------------------------------------------
constexpr uint32_t kT3 = 8;           // blocks per 3D tile
constexpr uint32_t kRow3 = 8 * kT3 + 8;   // LDS row pitch (floats), padded against bank conflicts

template <uint32_t LAYERS>
__global__ __launch_bounds__(256) void k_quant3d(QuantArgs a) {
    extern __shared__ uint32_t sh_hist[];
    __shared__ float s_tile[8][8][kRow3];
    __shared__ uint32_t s_misc[16];
    __shared__ uint64_t s_scan[10];

    Ctl *ctl = a.ctl;
    if (ctl->status & ST_EINVAL) return;
    const float r = ctl->r, h = ctl->h;
    const double eb = ctl->eb_abs;
    const float thr = patch_threshold(eb);
    const int32_t R = (int32_t)a.L.radius;
    for (uint32_t b = threadIdx.x; b < a.L.nsym; b += blockDim.x) sh_hist[b] = 0;

    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t tx = tile % a.tiles_per_row;
    const uint32_t rowid = tile / a.tiles_per_row;
    const uint32_t By = rowid % a.g.nb[1], Bz = rowid / a.g.nb[1];
    const uint32_t z0 = Bz * 8, y0 = By * 8, x0 = tx * kT3 * 8;
    const uint32_t nz = a.g.n[0], ny = a.g.n[1], nx = a.g.n[2];

    // stage the tile: 64 rows (z, y) of 64 floats, one wave per row; all 16
    // loads of a thread are issued before any is used
    {
        // row rr = w0 + 4k is (z, y) = (k / 2, w0 + 4 (k & 1)): one base
        // address per thread plus uniform plane and 4-row strides
        float v[16];
        const uint32_t xx = lane_id(), w0 = threadIdx.x / 64;
        const float *base = a.x + ((uint64_t)z0 * ny + (y0 + w0)) * nx + (x0 + xx);
        const uint64_t plane = (uint64_t)ny * nx, four_rows = 4ull * nx;
        const bool x_ok = x0 + xx < nx;
#pragma unroll
        for (uint32_t k = 0; k < 16; k++) {
            const uint32_t z = k / 2, y = w0 + 4 * (k & 1);
            v[k] = 0.0f;
            if (z0 + z < nz && y0 + y < ny && x_ok)
                v[k] = __builtin_nontemporal_load(base + (uint64_t)z * plane + ((k & 1) ? four_rows : 0ull));
        }
#pragma unroll
        for (uint32_t k = 0; k < 16; k++) {
            const uint32_t rr = w0 + 4 * k;
            s_tile[rr / 8][rr % 8][xx] = v[k];
        }
    }
    __syncthreads();

    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t ly = lane / 8, lx = lane % 8;
    int32_t delta[2][8];
    uint32_t flags_o = 0, flags_p = 0;   // bit (j*8 + z)
    uint32_t n_zero = 0;   // codes of delta 0 (bin R), added once per wave
#pragma unroll
    for (uint32_t j = 0; j < 2; j++) {
        const uint32_t bxl = 2 * w + j;              // block within tile
        const uint32_t Bx = tx * kT3 + bxl;
        const bool blk_ok = Bx < a.g.nb[2];
        const uint32_t gx = x0 + bxl * 8 + lx, gy = y0 + ly;
        const uint64_t blk = ((uint64_t)Bz * a.g.nb[1] + By) * a.g.nb[2] + Bx;
        const bool col_ok = blk_ok && gx < nx && gy < ny;
        // the block column's eight values and prequantized codes (LDS reads
        // all in flight), then the mixed backward difference: z in registers,
        // y and x across lanes, each axis for all eight z at once
        float v[8];
        int32_t d[8];
#pragma unroll
        for (uint32_t z = 0; z < 8; z++) v[z] = s_tile[z][ly][bxl * 8 + lx];
#pragma unroll
        for (uint32_t z = 0; z < 8; z++) d[z] = prequant(v[z], r);
        // (LAYERS layers: each axis's difference taken LAYERS times, the
        // padding being 0 at every step, which is the binomial form)
        uint32_t t[8];
#pragma unroll
        for (uint32_t z = 0; z < 8; z++) t[z] = (uint32_t)d[z] - (z ? (uint32_t)d[z - 1] : 0u);   // padding layer is 0
#pragma unroll
        for (uint32_t l = 1; l < LAYERS; l++)
#pragma unroll
            for (uint32_t z = 7; z > 0; z--) t[z] -= t[z - 1];
        uint32_t up[8];
#pragma unroll
        for (uint32_t l = 0; l < LAYERS; l++) {
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) up[z] = __shfl_up(t[z], 8, 64);
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) t[z] -= ly > 0 ? up[z] : 0u;
        }
#pragma unroll
        for (uint32_t l = 1; l < LAYERS; l++) {
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) up[z] = __shfl_up(t[z], 1, 64);
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) t[z] -= lx > 0 ? up[z] : 0u;
        }
#pragma unroll
        for (uint32_t z = 0; z < 8; z++) up[z] = __shfl_up(t[z], 1, 64);
#pragma unroll
        for (uint32_t z = 0; z < 8; z++) {
            const int32_t del = (int32_t)(t[z] - (lx > 0 ? up[z] : 0u));
            delta[j][z] = del;
            const bool real = col_ok && (z0 + z) < nz;
            const bool incap = del > -R && del < R;
            // the patch test in single precision (the exact one, for the few
            // values it cannot settle, runs after the loop)
            const bool pre = real && !(fabsf(__fsub_rn(v[z], dequant(d[z], h))) <= thr);
            uint16_t q = kNoSymbol;
            if (real) {
                q = incap ? (uint16_t)(del + R) : (uint16_t)0;
                if (del == 0) n_zero++;   // the usually hottest bin: counted in a register
                else atomicAdd(&sh_hist[q], 1u);
            }
            if (blk_ok) a.b.codes[blk * 512 + z * 64 + lane] = q;
            flags_o |= (real && !incap ? 1u : 0u) << (j * 8 + z);
            flags_p |= (pre ? 1u : 0u) << (j * 8 + z);
        }
    }
    if (__builtin_expect(__any((int)(flags_p != 0u)), 0)) {
        // values the single-precision test could not settle: the exact test
#pragma unroll
        for (uint32_t j = 0; j < 2; j++) {
            const uint32_t bxl = 2 * w + j;
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) {
                if (!((flags_p >> (j * 8 + z)) & 1u)) continue;
                const float v = s_tile[z][ly][bxl * 8 + lx];
                if (!needs_patch(v, prequant(v, r), h, eb)) flags_p &= ~(1u << (j * 8 + z));
            }
        }
    }
    const uint32_t wave_out = wave_sum_xor((uint32_t)__popc(flags_o));
    const uint32_t wave_count = wave_out + wave_sum_xor((uint32_t)__popc(flags_p));

    uint32_t tile_count, tile_out;
    const uint32_t base0 = wave_base_in_tile(wave_count, wave_out, s_misc, tile_count, tile_out);
    const uint32_t ovf = reserve_overflow(a, tile, tile_count, s_misc);
    if (wave_count) {
        uint32_t base = base0;
        const uint64_t below = lanes_below(lane);
#pragma unroll
        for (uint32_t j = 0; j < 2; j++) {
            const uint32_t bxl = 2 * w + j;
            const uint64_t blk = ((uint64_t)Bz * a.g.nb[1] + By) * a.g.nb[2] + (tx * kT3 + bxl);
#pragma unroll
            for (uint32_t z = 0; z < 8; z++) {
                const bool o = (flags_o >> (j * 8 + z)) & 1u, p = (flags_p >> (j * 8 + z)) & 1u;
                const uint64_t mo = __ballot(o), mp = __ballot(p);
                if ((mo | mp) == 0) continue;
                const uint32_t idx = base + __popcll(mo & below) + __popcll(mp & below);
                const uint32_t pos = (uint32_t)(blk * 512 + z * 64 + lane);
                if (o) put_exc(a, tile, idx, 2u * pos, (uint32_t)delta[j][z], ovf);
                if (p) put_exc(a, tile, idx + (o ? 1 : 0), 2u * pos + 1u, __float_as_uint(s_tile[z][ly][bxl * 8 + lx]), ovf);
                base += __popcll(mo) + __popcll(mp);
            }
        }
    }
    n_zero = wave_sum_xor(n_zero);
    if (lane_id() == 0 && n_zero) atomicAdd(&sh_hist[R], n_zero);
    tile_epilogue(a, tile, tile_count, tile_out, sh_hist, s_scan);
}

// ---------------------------------------------------------------------------
// 2D: tile = 16 consecutive 16x16 blocks along x in one block row.  Wave w
// handles blocks 4w..4w+3; lane -> (block 4w + lane/16, column lane%16)
// walking the 16 rows, so the y difference stays in registers and the x
// difference is a shuffle inside each 16-lane row.
// ---------------------------------------------------------------------------
constexpr uint32_t kT2 = 16;

template <uint32_t LAYERS>
__global__ __launch_bounds__(256) void k_quant2d(QuantArgs a) {
    extern __shared__ uint32_t sh_hist[];
    __shared__ float s_tile[16][16 * kT2];
    __shared__ uint32_t s_misc[16];
    __shared__ uint64_t s_scan[10];

    Ctl *ctl = a.ctl;
    if (ctl->status & ST_EINVAL) return;
    const float r = ctl->r, h = ctl->h;
    const double eb = ctl->eb_abs;
    const float thr = patch_threshold(eb);
    const int32_t R = (int32_t)a.L.radius;
    for (uint32_t b = threadIdx.x; b < a.L.nsym; b += blockDim.x) sh_hist[b] = 0;

    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t tx = tile % a.tiles_per_row, By = tile / a.tiles_per_row;
    const uint32_t y0 = By * 16, x0 = tx * kT2 * 16;
    const uint32_t ny = a.g.n[1], nx = a.g.n[2];
    {
        float v[16];
        const uint32_t xx = threadIdx.x;
#pragma unroll
        for (uint32_t rr = 0; rr < 16; rr++) {
            v[rr] = 0.0f;
            if (y0 + rr < ny && x0 + xx < nx) v[rr] = __builtin_nontemporal_load(a.x + (uint64_t)(y0 + rr) * nx + x0 + xx);
        }
#pragma unroll
        for (uint32_t rr = 0; rr < 16; rr++) s_tile[rr][xx] = v[rr];
    }
    __syncthreads();

    const uint32_t lane = lane_id(), w = threadIdx.x / 64;
    const uint32_t grp = lane / 16, lx = lane % 16;
    const uint32_t bxl = 4 * w + grp;
    const uint32_t Bx = tx * kT2 + bxl;
    const bool blk_ok = Bx < a.g.nb[2];
    const uint32_t gx = x0 + bxl * 16 + lx;
    const uint64_t blk = (uint64_t)By * a.g.nb[2] + Bx;
    int32_t delta[16];
    uint32_t flags_o = 0, flags_p = 0;
    uint32_t n_zero = 0;   // codes of delta 0 (bin R), added once per wave
    const bool col_ok = blk_ok && gx < nx;
    int32_t prev = 0;   // d° of (y-1) in this column; padding row is 0
    uint32_t prev_e = 0;   // the first layer's y difference of (y-1) (2 layers)
#pragma unroll
    for (uint32_t y0h = 0; y0h < 16; y0h += 8) {
        // eight rows at a time: LDS reads, prequantization and the x
        // exchanges of the eight in flight together
        float v[8];
        int32_t d[8];
        uint32_t t[8], up[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) v[k] = s_tile[y0h + k][bxl * 16 + lx];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) d[k] = prequant(v[k], r);
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) t[k] = (uint32_t)d[k] - (uint32_t)(k ? d[k - 1] : prev);
        prev = d[7];
        if (LAYERS == 2) {
            // the y difference again (its padding row is 0 too), then x twice
            const uint32_t last = t[7];
#pragma unroll
            for (uint32_t k = 7; k > 0; k--) t[k] -= t[k - 1];
            t[0] -= prev_e;
            prev_e = last;
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) up[k] = __shfl_up(t[k], 1, 64);
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) t[k] -= lx > 0 ? up[k] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) up[k] = __shfl_up(t[k], 1, 64);
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t y = y0h + k;
            const int32_t del = (int32_t)(t[k] - (lx > 0 ? up[k] : 0u));
            delta[y] = del;
            const bool real = col_ok && (y0 + y) < ny;
            const bool incap = del > -R && del < R;
            // single-precision patch test; the exact one runs after the loop
            const bool pre = real && !(fabsf(__fsub_rn(v[k], dequant(d[k], h))) <= thr);
            uint16_t q = kNoSymbol;
            if (real) {
                q = incap ? (uint16_t)(del + R) : (uint16_t)0;
                if (del == 0) n_zero++;   // the usually hottest bin: counted in a register
                else atomicAdd(&sh_hist[q], 1u);
            }
            if (blk_ok) a.b.codes[blk * 256 + y * 16 + lx] = q;
            flags_o |= (real && !incap ? 1u : 0u) << y;
            flags_p |= (pre ? 1u : 0u) << y;
        }
    }
    if (__builtin_expect(__any((int)(flags_p != 0u)), 0)) {
#pragma unroll
        for (uint32_t y = 0; y < 16; y++) {
            if (!((flags_p >> y) & 1u)) continue;
            const float v = s_tile[y][bxl * 16 + lx];
            if (!needs_patch(v, prequant(v, r), h, eb)) flags_p &= ~(1u << y);
        }
    }
    const uint32_t my_count = (uint32_t)__popc(flags_o) + (uint32_t)__popc(flags_p);
    const uint32_t wave_out = wave_sum_xor((uint32_t)__popc(flags_o));
    // records are ordered block by block: group totals, then exclusive over groups
    uint32_t grp_total = my_count;
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) grp_total += __shfl_xor(grp_total, off, 16);
    const uint32_t g0 = __shfl(grp_total, 0, 64), g1 = __shfl(grp_total, 16, 64), g2 = __shfl(grp_total, 32, 64),
                   g3 = __shfl(grp_total, 48, 64);
    const uint32_t wave_count = g0 + g1 + g2 + g3;
    const uint32_t grp_off = (grp > 0 ? g0 : 0u) + (grp > 1 ? g1 : 0u) + (grp > 2 ? g2 : 0u);
    uint32_t tile_count, tile_out;
    const uint32_t base0 = wave_base_in_tile(wave_count, wave_out, s_misc, tile_count, tile_out);
    const uint32_t ovf = reserve_overflow(a, tile, tile_count, s_misc);
    if (wave_count) {
        uint32_t base = base0 + grp_off;
        const uint64_t gmask = 0xFFFFull << (16 * grp);
        const uint64_t below = lanes_below(lane) & gmask;
#pragma unroll
        for (uint32_t y = 0; y < 16; y++) {
            const bool o = (flags_o >> y) & 1u, p = (flags_p >> y) & 1u;
            const uint64_t mo = __ballot(o), mp = __ballot(p);
            if ((mo | mp) == 0) continue;
            const uint32_t idx = base + __popcll(mo & below) + __popcll(mp & below);
            const uint32_t pos = (uint32_t)(blk * 256 + y * 16 + lx);
            if (o) put_exc(a, tile, idx, 2u * pos, (uint32_t)delta[y], ovf);
            if (p) put_exc(a, tile, idx + (o ? 1 : 0), 2u * pos + 1u, __float_as_uint(s_tile[y][bxl * 16 + lx]), ovf);
            base += __popcll(mo & gmask) + __popcll(mp & gmask);
        }
    }
    n_zero = wave_sum_xor(n_zero);
    if (lane_id() == 0 && n_zero) atomicAdd(&sh_hist[R], n_zero);
    tile_epilogue(a, tile, tile_count, tile_out, sh_hist, s_scan);
}

// ---------------------------------------------------------------------------
// 1D: tile = 4096 consecutive points (128 blocks of 32).  Thread t owns the
// 16 consecutive points [16t, 16t + 16), half a block; the first point of an
// odd thread takes its neighbour from the previous lane.
// ---------------------------------------------------------------------------
// (five waves per SIMD, a few registers spilled: 503 us against 525 at four
// waves on a 281-million-value field)
template <uint32_t LAYERS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_quant1d(QuantArgs a) {
    extern __shared__ uint32_t sh_hist[];
    __shared__ float s_tile[kTile];
    __shared__ uint32_t s_misc[16];
    __shared__ uint64_t s_scan[10];

    Ctl *ctl = a.ctl;
    if (ctl->status & ST_EINVAL) return;
    const float r = ctl->r, h = ctl->h;
    const double eb = ctl->eb_abs;
    const float thr = patch_threshold(eb);
    const int32_t R = (int32_t)a.L.radius;
    for (uint32_t b = threadIdx.x; b < a.L.nsym; b += blockDim.x) sh_hist[b] = 0;

    __syncthreads();
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint64_t p0 = (uint64_t)tile * kTile;
    const uint64_t n = a.g.nelem;
    {
        float v[kTile / 256];
#pragma unroll
        for (uint32_t k = 0; k < kTile / 256; k++) {
            const uint64_t e = p0 + threadIdx.x + 256 * k;
            v[k] = (e < n) ? __builtin_nontemporal_load(a.x + e) : 0.0f;
        }
#pragma unroll
        for (uint32_t k = 0; k < kTile / 256; k++) s_tile[threadIdx.x + 256 * k] = v[k];
    }
    __syncthreads();

    const uint32_t t = threadIdx.x;
    int32_t d[16];
#pragma unroll
    for (uint32_t i = 0; i < 16; i++) d[i] = prequant(s_tile[16 * t + i], r);
    // backward differences inside the 32-blocks (a thread holds half a block;
    // an odd thread continues the previous one's half), LAYERS times
    uint32_t e[16];
    {
        const uint32_t nb_prev = __shfl_up((uint32_t)d[15], 1, 64);
#pragma unroll
        for (uint32_t i = 0; i < 16; i++) e[i] = (uint32_t)d[i] - (i > 0 ? (uint32_t)d[i - 1] : ((t & 1u) ? nb_prev : 0u));
#pragma unroll
        for (uint32_t l = 1; l < LAYERS; l++) {
            const uint32_t e_prev = __shfl_up(e[15], 1, 64);
#pragma unroll
            for (uint32_t i = 15; i > 0; i--) e[i] -= e[i - 1];
            e[0] -= (t & 1u) ? e_prev : 0u;
        }
    }
    int32_t delta[16];
    uint32_t flags_o = 0, flags_p = 0, my_count = 0;
    uint32_t n_zero = 0;   // codes of delta 0 (bin R), added once per wave
    uint16_t q[16];
#pragma unroll
    for (uint32_t i = 0; i < 16; i++) {
        const int32_t del = (int32_t)e[i];   // lane t-1 is in the same wave (t odd)
        delta[i] = del;
        const uint64_t pos = p0 + 16 * t + i;
        const bool real = pos < n;
        const bool incap = del > -R && del < R;
        const bool o = real && !incap;
        // single-precision patch test; the exact one runs after the loop
        const bool pre = real && !(fabsf(__fsub_rn(s_tile[16 * t + i], dequant(d[i], h))) <= thr);
        uint16_t qq = kNoSymbol;
        if (real) {
            qq = incap ? (uint16_t)(del + R) : (uint16_t)0;
            if (del == 0) n_zero++;   // the usually hottest bin: counted in a register
            else atomicAdd(&sh_hist[qq], 1u);
        }
        q[i] = qq;
        flags_o |= (o ? 1u : 0u) << i;
        flags_p |= (pre ? 1u : 0u) << i;
    }
    if (__builtin_expect(__any((int)(flags_p != 0u)), 0)) {
#pragma unroll
        for (uint32_t i = 0; i < 16; i++)
            if (((flags_p >> i) & 1u) && !needs_patch(s_tile[16 * t + i], prequant(s_tile[16 * t + i], r), h, eb))
                flags_p &= ~(1u << i);
    }
    my_count = (uint32_t)__popc(flags_o) + (uint32_t)__popc(flags_p);
    // codes: 16 consecutive u16 per thread (two 16-byte stores)
    {
        const uint64_t pos0 = p0 + 16 * t;
        if (pos0 + 16 <= a.g.padded) {
            uint4 v0, v1;
            v0.x = q[0] | ((uint32_t)q[1] << 16); v0.y = q[2] | ((uint32_t)q[3] << 16);
            v0.z = q[4] | ((uint32_t)q[5] << 16); v0.w = q[6] | ((uint32_t)q[7] << 16);
            v1.x = q[8] | ((uint32_t)q[9] << 16); v1.y = q[10] | ((uint32_t)q[11] << 16);
            v1.z = q[12] | ((uint32_t)q[13] << 16); v1.w = q[14] | ((uint32_t)q[15] << 16);
            uint4 *dst = reinterpret_cast<uint4 *>(a.b.codes + pos0);
            dst[0] = v0;
            dst[1] = v1;
        } else {
#pragma unroll
            for (uint32_t i = 0; i < 16; i++)
                if (pos0 + i < a.g.padded) a.b.codes[pos0 + i] = q[i];
        }
    }
    const uint32_t incl = wave_incl_scan<uint32_t>(my_count);
    const uint32_t wave_count = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t wave_out = wave_sum_xor(__popc(flags_o));
    const uint32_t wave_patch = wave_sum_xor(__popc(flags_p));
    uint32_t tile_count, tile_out;
    const uint32_t base0 = wave_base_in_tile(wave_count, wave_out, s_misc, tile_count, tile_out);
    const uint32_t ovf = reserve_overflow(a, tile, tile_count, s_misc);
    (void)wave_patch;
    if (my_count) {
        uint32_t idx = base0 + incl - my_count;
#pragma unroll
        for (uint32_t i = 0; i < 16; i++) {
            const uint32_t pos = (uint32_t)(p0 + 16 * t + i);
            if ((flags_o >> i) & 1u) put_exc(a, tile, idx++, 2u * pos, (uint32_t)delta[i], ovf);
            if ((flags_p >> i) & 1u) put_exc(a, tile, idx++, 2u * pos + 1u, __float_as_uint(s_tile[16 * t + i]), ovf);
        }
    }
    n_zero = wave_sum_xor(n_zero);
    if (lane_id() == 0 && n_zero) atomicAdd(&sh_hist[R], n_zero);
    tile_epilogue(a, tile, tile_count, tile_out, sh_hist, s_scan);
}

uint32_t quantize_tiles(const Geom &g) {
    if (g.nelem == 0) return 0;
    if (g.ndim == 3) return g.nb[0] * g.nb[1] * ((g.nb[2] + kT3 - 1) / kT3);
    if (g.ndim == 2) return g.nb[1] * ((g.nb[2] + kT2 - 1) / kT2);
    return (uint32_t)((g.padded + kTile - 1) / kTile);
}

void launch_quantize(hipStream_t s, const float *x, const Geom &g, const Layout &L, Ctl *ctl, const QuantBufs &b) {
    QuantArgs a;
    a.x = x;
    a.g = g;
    a.L = L;
    a.ctl = ctl;
    a.b = b;
    a.n_tiles = quantize_tiles(g);
    if (a.n_tiles == 0) return;
    const size_t lds = sizeof(uint32_t) * L.nsym;
    if (g.ndim == 3) {
        a.tiles_per_row = (g.nb[2] + kT3 - 1) / kT3;
        if (L.layers == 2) hipLaunchKernelGGL(k_quant3d<2>, dim3(a.n_tiles), dim3(256), lds, s, a);
        else hipLaunchKernelGGL(k_quant3d<1>, dim3(a.n_tiles), dim3(256), lds, s, a);
    } else if (g.ndim == 2) {
        a.tiles_per_row = (g.nb[2] + kT2 - 1) / kT2;
        if (L.layers == 2) hipLaunchKernelGGL(k_quant2d<2>, dim3(a.n_tiles), dim3(256), lds, s, a);
        else hipLaunchKernelGGL(k_quant2d<1>, dim3(a.n_tiles), dim3(256), lds, s, a);
    } else {
        a.tiles_per_row = 1;
        if (L.layers == 2) hipLaunchKernelGGL(k_quant1d<2>, dim3(a.n_tiles), dim3(256), lds, s, a);
        else hipLaunchKernelGGL(k_quant1d<1>, dim3(a.n_tiles), dim3(256), lds, s, a);
    }
}

void launch_quantize_scan(hipStream_t s, const Geom &g, const Layout &L, const QuantBufs &b) {
    if (quantize_tiles(g) == 0) return;
    HistJob hj;
    hj.replicas = b.hist;
    hj.hist_out = b.hist_sum;
    hj.nsym = L.nsym;
    launch_seg_scan(s, b.scan, &hj);
}

}  // namespace dqz
