/*
 * dqz_oracle.c -- plain, slow, single-threaded CPU oracle of the cuSZ
 * compression method (Tian et al., "cuSZ: An Efficient GPU-Based
 * Error-Bounded Lossy Compression Framework for Scientific Data", PACT'20).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP implementation; the archive layout is restated here from its
 * definition, not included.
 *
 * Every step follows the paper's order and notation and is written for a
 * reader to check by eye, not for speed:
 *   - value-range-relative error bound        (footnote in Sec. 3.2.2)
 *   - prequantization d° = round(d / 2eb)      (Sec. 3.1.2, Algorithm 2)
 *   - chunking with a zero padding layer       (Sec. 3.1.1)
 *   - 1-layer Lorenzo predictor                (Sec. 3.1.2, "Lorenzo predictor
 *                                               with binomial coefficients"),
 *     and its 2-layer form as an archive option (the same paragraph's
 *     generalized n-layer predictor)
 *   - postquantization delta = d° - p°, cap    (Sec. 3.1.2, Algorithm 2)
 *   - outliers recorded verbatim               (Algorithm 2)
 *   - rehearsal + verbatim fallback (patches)  (Algorithm 1's watchdog)
 *   - histogram of quantization codes          (Sec. 3.2.1)
 *   - Huffman tree -> code lengths             (Sec. 3.2.2)
 *   - canonical codebook                       (Sec. 3.2.3)
 *   - encode + deflate into a bitstream        (Sec. 3.2.4)
 *   - inflate + reversed dual-quantization     (Sec. 3.3, Algorithm 2)
 *
 * Readings of passages the paper leaves open (tie rules, payloads, bit
 * order, archive layout) are the ones listed in the design notes; each is
 * repeated at the point of use below.
 *
 * Build: gcc -O2 -std=gnu99 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (no FMA contraction: every float operation is the single IEEE operation
 * written in the source, rounded to nearest-even).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ETOOSMALL (-2)
#define ORC_ENOMEM (-3)
#define ORC_ECORRUPT (-4)
#define ORC_EUNSUPPORTED (-5)

#define ORC_MAGIC 0x315A5144u /* bytes 'D' 'Q' 'Z' '1' */
#define ORC_VERSION 1u
#define ORC_HEADER_BYTES 128u

/* ------------------------------------------------------------------ */
/* little-endian byte helpers (the archive is little-endian)           */
/* ------------------------------------------------------------------ */
static void put_u8(uint8_t *p, uint64_t off, uint8_t v) { p[off] = v; }
static void put_u16(uint8_t *p, uint64_t off, uint16_t v)
{
    p[off] = (uint8_t)(v & 0xff);
    p[off + 1] = (uint8_t)(v >> 8);
}
static void put_u32(uint8_t *p, uint64_t off, uint32_t v)
{
    for (int i = 0; i < 4; i++) p[off + i] = (uint8_t)((v >> (8 * i)) & 0xff);
}
static void put_u64(uint8_t *p, uint64_t off, uint64_t v)
{
    for (int i = 0; i < 8; i++) p[off + i] = (uint8_t)((v >> (8 * i)) & 0xff);
}
static uint8_t get_u8(const uint8_t *p, uint64_t off) { return p[off]; }
static uint16_t get_u16(const uint8_t *p, uint64_t off)
{
    return (uint16_t)(p[off] | ((uint16_t)p[off + 1] << 8));
}
static uint32_t get_u32(const uint8_t *p, uint64_t off)
{
    uint32_t v = 0;
    for (int i = 0; i < 4; i++) v |= (uint32_t)p[off + i] << (8 * i);
    return v;
}
static uint64_t get_u64(const uint8_t *p, uint64_t off)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v |= (uint64_t)p[off + i] << (8 * i);
    return v;
}
static uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}
static float bits_f32(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}
static uint64_t f64_bits(double d)
{
    uint64_t u;
    memcpy(&u, &d, 8);
    return u;
}
static double bits_f64(uint64_t u)
{
    double d;
    memcpy(&d, &u, 8);
    return d;
}
static uint64_t align8(uint64_t v) { return (v + 7u) & ~(uint64_t)7u; }
static int is_pow2(uint64_t v) { return v != 0 && (v & (v - 1)) == 0; }

/* ------------------------------------------------------------------ */
/* Geometry: every field is viewed as (nz, ny, nx), slowest -> fastest. */
/* Prediction blocks (Sec. 3.1.1): 32 for 1D, 16x16 for 2D, 8x8x8 for 3D; */
/* a 1D/2D field gets block extent 1 on its missing leading axes.        */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t n[3];  /* field extents (nz, ny, nx) */
    uint64_t b[3];  /* block extents (bz, by, bx) */
    uint64_t nb[3]; /* number of blocks per axis */
    uint64_t bvol;  /* bz*by*bx */
    uint64_t nblocks;
    uint64_t padded; /* nblocks * bvol : size of the padded position space */
    uint64_t nelem;
} geom_t;

static int make_geom(int ndim, const uint64_t *dims, geom_t *g)
{
    if (ndim < 1 || ndim > 3) return ORC_EINVAL;
    g->n[0] = g->n[1] = 1;
    for (int i = 0; i < ndim; i++) g->n[3 - ndim + i] = dims[i];
    if (ndim == 1) { g->b[0] = 1; g->b[1] = 1; g->b[2] = 32; }
    else if (ndim == 2) { g->b[0] = 1; g->b[1] = 16; g->b[2] = 16; }
    else { g->b[0] = 8; g->b[1] = 8; g->b[2] = 8; }
    g->nelem = 1;
    g->nblocks = 1;
    for (int a = 0; a < 3; a++) {
        g->nb[a] = (g->n[a] + g->b[a] - 1) / g->b[a];
        g->nelem *= g->n[a];
        g->nblocks *= g->nb[a];
    }
    g->bvol = g->b[0] * g->b[1] * g->b[2];
    g->padded = g->nblocks * g->bvol;
    return ORC_OK;
}

/* Padded block-major position of element (z, y, x): blocks in row-major
 * order of block coordinates, then row-major inside the (full-size) block. */
static uint64_t padded_pos(const geom_t *g, uint64_t z, uint64_t y, uint64_t x)
{
    uint64_t Bz = z / g->b[0], By = y / g->b[1], Bx = x / g->b[2];
    uint64_t iz = z % g->b[0], iy = y % g->b[1], ix = x % g->b[2];
    uint64_t blk = (Bz * g->nb[1] + By) * g->nb[2] + Bx;
    return blk * g->bvol + (iz * g->b[1] + iy) * g->b[2] + ix;
}

/* ------------------------------------------------------------------ */
/* Step 1: error bound (footnote in Sec. 3.2.2: valrel = eb relative to   */
/* the value range).  Range over finite values only; IEEE total order   */
/* (-0 < +0) so the chosen min/max bit patterns do not depend on order.  */
/* ------------------------------------------------------------------ */
static int total_less(float a, float b)
{
    /* a < b in IEEE-754 totalOrder, both finite */
    if (a < b) return 1;
    if (a > b) return 0;
    return signbit(a) && !signbit(b);
}

int orc_value_range(const float *x, uint64_t n, float *vmin, float *vmax, uint64_t *nfinite)
{
    uint64_t cnt = 0;
    float lo = 0.0f, hi = 0.0f;
    for (uint64_t i = 0; i < n; i++) {
        float v = x[i];
        if (!isfinite(v)) continue;
        if (cnt == 0) { lo = v; hi = v; }
        else {
            if (total_less(v, lo)) lo = v;
            if (total_less(hi, v)) hi = v;
        }
        cnt++;
    }
    *vmin = lo;
    *vmax = hi;
    *nfinite = cnt;
    return ORC_OK;
}

/* eb_abs, h = fl32(2 eb_abs), r = fl32(1 / (2 eb_abs)).
 * mode 0: eb is absolute.  mode 1: eb is relative to max - min (finite
 * values); a field with no finite values or max == min uses range 1. */
int orc_eb_params(int mode, double eb, float vmin, float vmax, uint64_t nfinite,
                  double *eb_abs, float *h, float *r)
{
    if (!(eb > 0.0) || !isfinite(eb)) return ORC_EINVAL;
    double e;
    if (mode == 0) e = eb;
    else if (mode == 1) {
        double range = (double)vmax - (double)vmin;
        if (nfinite == 0 || !(range > 0.0)) range = 1.0;
        e = eb * range;
    } else return ORC_EINVAL;
    if (!isfinite(e) || e < (double)FLT_MIN) return ORC_EINVAL;
    float hh = (float)(2.0 * e);
    float rr = (float)(1.0 / (2.0 * e));
    if (!isfinite(hh) || !(rr >= FLT_MIN) || !isfinite(rr)) return ORC_EINVAL;
    *eb_abs = e;
    *h = hh;
    *r = rr;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 2: prequantization, d° = round(d / (2 eb)) (Sec. 3.1.2).        */
/* Reading: multiply by r = fl32(1/(2eb)) in fp32, round half to even,  */
/* store as int32; values whose |t| is not below 2^30 (and NaN/Inf) map  */
/* to 0 and are then caught by the rehearsal below.                     */
/* ------------------------------------------------------------------ */
void orc_prequant(const float *x, uint64_t n, float r, int32_t *dq)
{
    for (uint64_t i = 0; i < n; i++) {
        float t = x[i] * r;
        if (fabsf(t) < 1073741824.0f) dq[i] = (int32_t)rintf(t);
        else dq[i] = 0;
    }
}

/* Reconstructed value of a prequantized integer: (float)d° * fl32(2eb). */
static float dequant(int32_t d, float h) { return (float)d * h; }

/* Rehearsal (Algorithm 1's watchdog, applied to the final fp32 value):
 * an element whose reconstruction misses the bound is stored verbatim. */
static int needs_patch(float x, float xr, double eb_abs)
{
    return !(fabs((double)x - (double)xr) <= eb_abs);
}

/* ------------------------------------------------------------------ */
/* Step 3: 1-layer Lorenzo predictor with a zero padding layer per block */
/* (Sec. 3.1.1 and the Lorenzo paragraph of Sec. 3.1.2).  For a point at */
/* offset 0/1 steps back along each axis, the coefficient of the        */
/* neighbour k in {0,1}^3 \ {0} is (-1)^(|k|+1); neighbours outside the */
/* point's own block read the padding value 0.                          */
/* ------------------------------------------------------------------ */
static int64_t lorenzo_predict(const int32_t *dq, const geom_t *g, uint64_t z, uint64_t y, uint64_t x)
{
    int64_t p = 0;
    for (int kz = 0; kz <= 1; kz++)
        for (int ky = 0; ky <= 1; ky++)
            for (int kx = 0; kx <= 1; kx++) {
                if (kz == 0 && ky == 0 && kx == 0) continue;
                /* the neighbour must lie in the same block */
                if (kz && (z % g->b[0]) == 0) continue;
                if (ky && (y % g->b[1]) == 0) continue;
                if (kx && (x % g->b[2]) == 0) continue;
                uint64_t zz = z - (uint64_t)kz, yy = y - (uint64_t)ky, xx = x - (uint64_t)kx;
                int64_t v = dq[(zz * g->n[1] + yy) * g->n[2] + xx];
                int s = kz + ky + kx;
                p += (s % 2 == 1) ? v : -v; /* (-1)^(|k|+1) */
            }
    return p;
}

/* 32-bit two's-complement wrap of an exact integer. */
static int32_t wrap32(int64_t v) { return (int32_t)(uint32_t)(uint64_t)v; }

/* delta = d° - p° for every element, row-major output (pins use this). */
int orc_lorenzo_delta(const int32_t *dq, int ndim, const uint64_t *dims, int32_t *delta)
{
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_EINVAL;
    for (uint64_t z = 0; z < g.n[0]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[2]; x++) {
                uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
                delta[i] = wrap32((int64_t)dq[i] - lorenzo_predict(dq, &g, z, y, x));
            }
    return ORC_OK;
}

/* Reversed Lorenzo (decompression loop of Algorithm 2): reconstruct
 * cascadingly, d° = delta + p°(already reconstructed neighbours), visiting
 * points in an order where every lower-index neighbour comes first. */
int orc_lorenzo_reconstruct(const int32_t *delta, int ndim, const uint64_t *dims, int32_t *dq)
{
    geom_t g;
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_EINVAL;
    for (uint64_t z = 0; z < g.n[0]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[2]; x++) {
                uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
                dq[i] = wrap32((int64_t)delta[i] + lorenzo_predict(dq, &g, z, y, x));
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 3, n layers: the generalized Lorenzo predictor with binomial      */
/* coefficients (Sec. 3.1.2), in the same sign reading as the 1-layer     */
/* predictor above: the neighbour k in {0..n}^3 \ {0} steps back has      */
/* coefficient (-1)^(|k|+1) C(n,kz) C(n,ky) C(n,kx), which sums to 1 (unit */
/* weight, as the paper requires).  A neighbour outside the point's own    */
/* block (more steps back than the point lies into its block along some   */
/* axis) reads the padding value 0.  Only n = 2 is used with this form;   */
/* n = 1 keeps the explicit predictor above.                              */
/* ------------------------------------------------------------------ */
#define ORC_MAX_LAYERS 2

static int64_t binomial(int n, int k)
{
    int64_t c = 1;
    for (int i = 1; i <= k; i++) c = c * (n - k + i) / i;
    return c;
}

static int64_t lorenzo_predict_n(const int32_t *dq, const geom_t *g, uint64_t z, uint64_t y, uint64_t x, int n)
{
    int64_t p = 0;
    for (int kz = 0; kz <= n; kz++)
        for (int ky = 0; ky <= n; ky++)
            for (int kx = 0; kx <= n; kx++) {
                if (kz == 0 && ky == 0 && kx == 0) continue;
                /* the neighbour must lie in the same block */
                if ((uint64_t)kz > z % g->b[0] || (uint64_t)ky > y % g->b[1] || (uint64_t)kx > x % g->b[2])
                    continue;
                int64_t v = dq[((z - (uint64_t)kz) * g->n[1] + (y - (uint64_t)ky)) * g->n[2] + (x - (uint64_t)kx)];
                int64_t c = binomial(n, kz) * binomial(n, ky) * binomial(n, kx);
                p += ((kz + ky + kx) % 2 == 1) ? c * v : -c * v; /* (-1)^(|k|+1) */
            }
    return p;
}

int orc_lorenzo_delta_n(const int32_t *dq, int ndim, const uint64_t *dims, int layers, int32_t *delta)
{
    geom_t g;
    if (layers < 1 || layers > ORC_MAX_LAYERS) return ORC_EINVAL;
    if (layers == 1) return orc_lorenzo_delta(dq, ndim, dims, delta);
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_EINVAL;
    for (uint64_t z = 0; z < g.n[0]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[2]; x++) {
                uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
                delta[i] = wrap32((int64_t)dq[i] - lorenzo_predict_n(dq, &g, z, y, x, layers));
            }
    return ORC_OK;
}

/* The cascading reconstruction of Algorithm 2 with the n-layer predictor. */
int orc_lorenzo_reconstruct_n(const int32_t *delta, int ndim, const uint64_t *dims, int layers, int32_t *dq)
{
    geom_t g;
    if (layers < 1 || layers > ORC_MAX_LAYERS) return ORC_EINVAL;
    if (layers == 1) return orc_lorenzo_reconstruct(delta, ndim, dims, dq);
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_EINVAL;
    for (uint64_t z = 0; z < g.n[0]; z++)
        for (uint64_t y = 0; y < g.n[1]; y++)
            for (uint64_t x = 0; x < g.n[2]; x++) {
                uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
                dq[i] = wrap32((int64_t)delta[i] + lorenzo_predict_n(dq, &g, z, y, x, layers));
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 5: Huffman code lengths (Sec. 3.2.2).  Reading of the tie rules: */
/* leaves with nonzero frequency sorted by (frequency, symbol); the      */
/* classic two-queue construction (sorted leaves, FIFO of merged nodes); */
/* each pick takes the lighter front, the leaf on equal weights.  One    */
/* used symbol gets length 1.  Returns the maximum length, or -1.        */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t f;
    uint32_t s;
} leaf_t;

static int leaf_cmp(const void *a, const void *b)
{
    const leaf_t *x = (const leaf_t *)a, *y = (const leaf_t *)b;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    return x->s < y->s ? -1 : (x->s > y->s ? 1 : 0);
}

int orc_huffman_lengths(const uint64_t *freq, uint32_t nsym, uint8_t *len)
{
    memset(len, 0, nsym);
    uint32_t n = 0;
    for (uint32_t s = 0; s < nsym; s++)
        if (freq[s]) n++;
    if (n == 0) return 0;
    leaf_t *lv = (leaf_t *)malloc(sizeof(leaf_t) * n);
    if (!lv) return -1;
    n = 0;
    for (uint32_t s = 0; s < nsym; s++)
        if (freq[s]) { lv[n].f = freq[s]; lv[n].s = s; n++; }
    qsort(lv, n, sizeof(leaf_t), leaf_cmp);
    if (n == 1) {
        len[lv[0].s] = 1;
        free(lv);
        return 1;
    }
    uint32_t tot = 2 * n - 1;
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * tot);
    uint32_t *parent = (uint32_t *)malloc(sizeof(uint32_t) * tot);
    uint32_t *depth = (uint32_t *)malloc(sizeof(uint32_t) * tot);
    if (!w || !parent || !depth) { free(lv); free(w); free(parent); free(depth); return -1; }
    for (uint32_t i = 0; i < n; i++) w[i] = lv[i].f;
    uint32_t next_leaf = 0, next_int = n, created = n;
    for (uint32_t k = 0; k + 1 < n; k++) {
        uint32_t pick[2];
        for (int j = 0; j < 2; j++) {
            int take_leaf;
            if (next_leaf >= n) take_leaf = 0;
            else if (next_int >= created) take_leaf = 1;
            else take_leaf = (w[next_leaf] <= w[next_int]);
            pick[j] = take_leaf ? next_leaf++ : next_int++;
        }
        w[created] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = created;
        parent[pick[1]] = created;
        created++;
    }
    depth[tot - 1] = 0;
    for (int64_t i = (int64_t)tot - 2; i >= 0; i--) depth[i] = depth[parent[i]] + 1;
    int maxlen = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (depth[i] > 255) { maxlen = -1; break; }
        len[lv[i].s] = (uint8_t)depth[i];
        if ((int)depth[i] > maxlen) maxlen = (int)depth[i];
    }
    free(lv); free(w); free(parent); free(depth);
    return maxlen;
}

/* ------------------------------------------------------------------ */
/* Step 6: canonical codebook (Sec. 3.2.3).  Reading: the canonical rule */
/* of RFC 1951 Sec. 3.2.2 -- count codes per length, first code of each  */
/* length from the counts, consecutive codes in increasing symbol order  */
/* inside a length; codes are emitted most significant bit first.        */
/* ------------------------------------------------------------------ */
int orc_canonical_codes(const uint8_t *len, uint32_t nsym, uint64_t *code)
{
    uint64_t bl_count[65] = {0}, next_code[65] = {0};
    for (uint32_t s = 0; s < nsym; s++) {
        if (len[s] > 64) return ORC_EINVAL;
        bl_count[len[s]]++;
    }
    bl_count[0] = 0;
    uint64_t c = 0;
    for (int bits = 1; bits <= 64; bits++) {
        c = (c + bl_count[bits - 1]) << 1;
        next_code[bits] = c;
    }
    for (uint32_t s = 0; s < nsym; s++) {
        code[s] = 0;
        if (len[s]) code[s] = next_code[len[s]]++;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Bit writer / reader.  One bit-dense stream of little-endian u32 words; */
/* stream bit i is bit (31 - i mod 32) of word i / 32.                    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint8_t *base; /* start of the stream section in the archive */
    uint64_t nbits;
} bitw_t;

static void bw_put_bit(bitw_t *w, int bit)
{
    if (bit) {
        uint64_t word = w->nbits >> 5;
        uint32_t v = get_u32(w->base, word * 4);
        v |= 1u << (31 - (w->nbits & 31));
        put_u32(w->base, word * 4, v);
    }
    w->nbits++;
}

static void bw_put_code(bitw_t *w, uint64_t code, int len)
{
    for (int i = len - 1; i >= 0; i--) bw_put_bit(w, (int)((code >> i) & 1u));
}

typedef struct {
    const uint8_t *base;
    uint64_t limit; /* total bits */
    uint64_t pos;
} bitr_t;

static int br_get_bit(bitr_t *r, int *bit)
{
    if (r->pos >= r->limit) return 0;
    uint32_t v = get_u32(r->base, (r->pos >> 5) * 4);
    *bit = (int)((v >> (31 - (r->pos & 31))) & 1u);
    r->pos++;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Archive layout (little-endian).  A fixed 128-byte header, then:        */
/*   lengths   u8[2R]                         at 128                       */
/*   chunks    u64[n_chunks]                  at align8(128 + 2R)          */
/*   subchunks u16[n_sub]                     right after                  */
/*   exceptions {u32 key, u32 payload}[..]    at align8(after subchunks)   */
/*   stream    u32[ceil(total_bits / 32)]     right after                  */
/* A subchunk is S consecutive padded positions; its entry is the number */
/* of stream bits of its symbols.  A chunk is C consecutive subchunks;   */
/* its entry is the stream bit offset of its first symbol.  Exception    */
/* key = 2*position + kind, kind 0 = outlier (payload = delta, int32),   */
/* kind 1 = patch (payload = the input's raw fp32 bits); ascending keys. */
/* ------------------------------------------------------------------ */
enum {
    H_MAGIC = 0, H_VERSION = 4, H_NDIM = 6, H_EBMODE = 7, H_DIMS = 8, H_BLOCK = 32,
    H_RADIUS = 44, H_EBPARAM = 48, H_EBABS = 56, H_H = 64, H_R = 68, H_VMIN = 72,
    H_VMAX = 76, H_NELEM = 80, H_NOUT = 88, H_NPATCH = 92, H_TOTBITS = 96,
    H_SUBSIZE = 104, H_CHUNKSUBS = 108, H_NCHUNKS = 112, H_MAXLEN = 116,
    H_LAYERS = 117, /* Lorenzo layers - 1 (0: the 1-layer predictor) */
    H_ARCBYTES = 120
};

typedef struct {
    uint64_t off_len, off_chunk, off_sub, off_exc, off_str, end;
    uint64_t n_sub, n_chunks, n_exc, n_words;
} layout_t;

static void make_layout(uint32_t radius, uint64_t padded, uint32_t sub, uint32_t csubs,
                        uint64_t n_exc, uint64_t total_bits, layout_t *L)
{
    L->n_sub = (padded + sub - 1) / sub;
    L->n_chunks = (L->n_sub + csubs - 1) / csubs;
    L->n_exc = n_exc;
    L->n_words = (total_bits + 31) / 32;
    L->off_len = ORC_HEADER_BYTES;
    L->off_chunk = align8(L->off_len + 2ull * radius);
    L->off_sub = L->off_chunk + 8ull * L->n_chunks;
    L->off_exc = align8(L->off_sub + 2ull * L->n_sub);
    L->off_str = L->off_exc + 8ull * n_exc;
    L->end = L->off_str + 4ull * L->n_words;
}

typedef struct {
    uint32_t key;
    uint32_t payload;
} exc_t;

static int check_params(uint32_t radius, uint32_t sub, uint32_t csubs)
{
    if (!is_pow2(radius) || radius > 4096) return ORC_EINVAL;
    if (!is_pow2(sub) || sub < 32 || sub > 1024) return ORC_EINVAL;
    if (!is_pow2(csubs) || csubs > 65536) return ORC_EINVAL;
    return ORC_OK;
}

/* Walk the real elements in stream order: blocks in block-major order,
 * row-major inside a block, skipping padded positions outside the field. */
#define FOR_EACH_STREAM_ELEMENT(g, z, y, x, pos)                                         \
    for (uint64_t Bz_ = 0; Bz_ < (g)->nb[0]; Bz_++)                                      \
        for (uint64_t By_ = 0; By_ < (g)->nb[1]; By_++)                                  \
            for (uint64_t Bx_ = 0; Bx_ < (g)->nb[2]; Bx_++)                              \
                for (uint64_t iz_ = 0; iz_ < (g)->b[0]; iz_++)                           \
                    for (uint64_t iy_ = 0; iy_ < (g)->b[1]; iy_++)                       \
                        for (uint64_t ix_ = 0; ix_ < (g)->b[2]; ix_++)                   \
                            for (uint64_t z = Bz_ * (g)->b[0] + iz_,                     \
                                          y = By_ * (g)->b[1] + iy_,                     \
                                          x = Bx_ * (g)->b[2] + ix_,                     \
                                          pos = padded_pos((g), z, y, x), once_ = 1;     \
                                 once_ && z < (g)->n[0] && y < (g)->n[1] && x < (g)->n[2]; \
                                 once_ = 0)

/* ------------------------------------------------------------------ */
/* Compression: the whole pipeline, in the paper's order.              */
/* ------------------------------------------------------------------ */
int orc_compress_layers(const float *xin, int ndim, const uint64_t *dims, double eb, int eb_mode,
                        uint32_t radius, uint32_t sub, uint32_t csubs, int layers,
                        uint8_t *out, uint64_t cap, uint64_t *out_bytes)
{
    geom_t g;
    int st;
    if (layers < 1 || layers > ORC_MAX_LAYERS) return ORC_EINVAL;
    if ((st = make_geom(ndim, dims, &g)) != ORC_OK) return st;
    if ((st = check_params(radius, sub, csubs)) != ORC_OK) return st;
    if (g.padded >= (1ull << 31)) return ORC_EUNSUPPORTED;
    const uint64_t N = g.nelem;
    const uint32_t nsym = 2 * radius;

    /* error bound */
    float vmin = 0.0f, vmax = 0.0f;
    uint64_t nfinite = 0;
    if (eb_mode == 1) orc_value_range(xin, N, &vmin, &vmax, &nfinite);
    double eb_abs;
    float h, r;
    if ((st = orc_eb_params(eb_mode, eb, vmin, vmax, nfinite, &eb_abs, &h, &r)) != ORC_OK) return st;
    if (eb_mode == 0) { vmin = 0.0f; vmax = 0.0f; }

    int32_t *dq = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
    int32_t *delta = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
    uint16_t *q = (uint16_t *)malloc(sizeof(uint16_t) * (N ? N : 1));
    uint64_t *posv = (uint64_t *)malloc(sizeof(uint64_t) * (N ? N : 1));
    exc_t *exc = (exc_t *)malloc(sizeof(exc_t) * (2 * N + 1));
    uint64_t *freq = (uint64_t *)calloc(nsym, sizeof(uint64_t));
    uint8_t *len = (uint8_t *)calloc(nsym, 1);
    uint64_t *code = (uint64_t *)calloc(nsym, sizeof(uint64_t));
    if (!dq || !delta || !q || !posv || !exc || !freq || !len || !code) { st = ORC_ENOMEM; goto done; }

    /* prequantization (whole field first: Algorithm 2's barrier) */
    orc_prequant(xin, N, r, dq);
    /* prediction + postquantization delta */
    orc_lorenzo_delta_n(dq, ndim, dims, layers, delta);

    /* postquantization into codes, outliers and patches, in stream order */
    uint64_t n_exc = 0, n_out = 0, n_patch = 0, ns = 0;
    FOR_EACH_STREAM_ELEMENT(&g, z, y, x, pos) {
        uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
        int32_t d = delta[i];
        uint16_t qq;
        if (d > -(int32_t)radius && d < (int32_t)radius) qq = (uint16_t)(d + (int32_t)radius);
        else {
            qq = 0; /* code slot 0 marks an outlier; delta kept verbatim */
            exc[n_exc].key = (uint32_t)(2 * pos + 0);
            exc[n_exc].payload = (uint32_t)d;
            n_exc++;
            n_out++;
        }
        float xr = dequant(dq[i], h);
        if (needs_patch(xin[i], xr, eb_abs)) {
            exc[n_exc].key = (uint32_t)(2 * pos + 1);
            exc[n_exc].payload = f32_bits(xin[i]);
            n_exc++;
            n_patch++;
        }
        q[ns] = qq;
        posv[ns] = pos;
        ns++;
    }

    /* histogram (Sec. 3.2.1) */
    for (uint64_t k = 0; k < ns; k++) freq[q[k]]++;
    /* code lengths and canonical codes (Sec. 3.2.2, 3.2.3) */
    int maxlen = orc_huffman_lengths(freq, nsym, len);
    if (maxlen < 0 || maxlen > 64) { st = ORC_EUNSUPPORTED; goto done; }
    orc_canonical_codes(len, nsym, code);
    uint64_t total_bits = 0;
    for (uint64_t k = 0; k < ns; k++) total_bits += len[q[k]];

    layout_t L;
    make_layout(radius, g.padded, sub, csubs, n_exc, total_bits, &L);
    if (L.end > cap) { st = ORC_ETOOSMALL; *out_bytes = L.end; goto done; }
    memset(out, 0, L.end);

    /* header */
    put_u32(out, H_MAGIC, ORC_MAGIC);
    put_u16(out, H_VERSION, ORC_VERSION);
    put_u8(out, H_NDIM, (uint8_t)ndim);
    put_u8(out, H_EBMODE, (uint8_t)eb_mode);
    for (int a = 0; a < 3; a++) put_u64(out, H_DIMS + 8 * a, g.n[a]);
    for (int a = 0; a < 3; a++) put_u32(out, H_BLOCK + 4 * a, (uint32_t)g.b[a]);
    put_u32(out, H_RADIUS, radius);
    put_u64(out, H_EBPARAM, f64_bits(eb));
    put_u64(out, H_EBABS, f64_bits(eb_abs));
    put_u32(out, H_H, f32_bits(h));
    put_u32(out, H_R, f32_bits(r));
    put_u32(out, H_VMIN, f32_bits(vmin));
    put_u32(out, H_VMAX, f32_bits(vmax));
    put_u64(out, H_NELEM, N);
    put_u32(out, H_NOUT, (uint32_t)n_out);
    put_u32(out, H_NPATCH, (uint32_t)n_patch);
    put_u64(out, H_TOTBITS, total_bits);
    put_u32(out, H_SUBSIZE, sub);
    put_u32(out, H_CHUNKSUBS, csubs);
    put_u32(out, H_NCHUNKS, (uint32_t)L.n_chunks);
    put_u8(out, H_MAXLEN, (uint8_t)maxlen);
    put_u8(out, H_LAYERS, (uint8_t)(layers - 1));
    put_u64(out, H_ARCBYTES, L.end);

    /* lengths */
    for (uint32_t s = 0; s < nsym; s++) put_u8(out, L.off_len + s, len[s]);
    /* exceptions, already in ascending key order */
    for (uint64_t k = 0; k < n_exc; k++) {
        put_u32(out, L.off_exc + 8 * k, exc[k].key);
        put_u32(out, L.off_exc + 8 * k + 4, exc[k].payload);
    }
    /* encode + deflate: every codeword in stream order into one stream; the
     * subchunk entry collects the bits of its symbols, the chunk entry the
     * offset of its first subchunk */
    {
        bitw_t w = {out + L.off_str, 0};
        uint64_t *subbits = (uint64_t *)calloc(L.n_sub ? L.n_sub : 1, sizeof(uint64_t));
        if (!subbits) { st = ORC_ENOMEM; goto done; }
        for (uint64_t k = 0; k < ns; k++) {
            bw_put_code(&w, code[q[k]], len[q[k]]);
            subbits[posv[k] / sub] += len[q[k]];
        }
        uint64_t acc = 0;
        for (uint64_t j = 0; j < L.n_sub; j++) {
            if (j % csubs == 0) put_u64(out, L.off_chunk + 8 * (j / csubs), acc);
            put_u16(out, L.off_sub + 2 * j, (uint16_t)subbits[j]);
            acc += subbits[j];
        }
        free(subbits);
    }
    *out_bytes = L.end;
    st = ORC_OK;
done:
    free(dq); free(delta); free(q); free(posv); free(exc); free(freq); free(len); free(code);
    return st;
}

int orc_compress(const float *xin, int ndim, const uint64_t *dims, double eb, int eb_mode,
                 uint32_t radius, uint32_t sub, uint32_t csubs,
                 uint8_t *out, uint64_t cap, uint64_t *out_bytes)
{
    return orc_compress_layers(xin, ndim, dims, eb, eb_mode, radius, sub, csubs, 1, out, cap, out_bytes);
}

/* Size of the archive orc_compress would write (runs the whole method). */
int orc_compressed_size(const float *xin, int ndim, const uint64_t *dims, double eb, int eb_mode,
                        uint32_t radius, uint32_t sub, uint32_t csubs, uint64_t *bytes)
{
    uint8_t dummy[1];
    int st = orc_compress(xin, ndim, dims, eb, eb_mode, radius, sub, csubs, dummy, 0, bytes);
    if (st == ORC_ETOOSMALL) return ORC_OK;
    return st;
}

/* ------------------------------------------------------------------ */
/* Decompression (Sec. 3.3): inflate, then reversed dual-quantization.  */
/* The archive is validated as it is read; any inconsistency is          */
/* ORC_ECORRUPT.                                                          */
/* ------------------------------------------------------------------ */
int orc_decompress(const uint8_t *arc, uint64_t nbytes, float *out, uint64_t cap_elems)
{
    if (nbytes < ORC_HEADER_BYTES) return ORC_ECORRUPT;
    if (get_u32(arc, H_MAGIC) != ORC_MAGIC || get_u16(arc, H_VERSION) != ORC_VERSION) return ORC_ECORRUPT;
    int ndim = get_u8(arc, H_NDIM);
    if (ndim < 1 || ndim > 3) return ORC_ECORRUPT;
    uint64_t dims[3];
    geom_t g;
    uint64_t n3[3];
    for (int a = 0; a < 3; a++) n3[a] = get_u64(arc, H_DIMS + 8 * a);
    for (int a = 0; a < 3 - ndim; a++)
        if (n3[a] != 1) return ORC_ECORRUPT;
    for (int i = 0; i < ndim; i++) dims[i] = n3[3 - ndim + i];
    if (make_geom(ndim, dims, &g) != ORC_OK) return ORC_ECORRUPT;
    for (int a = 0; a < 3; a++)
        if (get_u32(arc, H_BLOCK + 4 * a) != g.b[a]) return ORC_ECORRUPT;
    if (get_u64(arc, H_NELEM) != g.nelem) return ORC_ECORRUPT;
    if (g.padded >= (1ull << 31)) return ORC_ECORRUPT;
    uint32_t radius = get_u32(arc, H_RADIUS);
    uint32_t sub = get_u32(arc, H_SUBSIZE), csubs = get_u32(arc, H_CHUNKSUBS);
    if (check_params(radius, sub, csubs) != ORC_OK) return ORC_ECORRUPT;
    uint32_t nsym = 2 * radius;
    double eb_abs = bits_f64(get_u64(arc, H_EBABS));
    float h = bits_f32(get_u32(arc, H_H));
    (void)eb_abs;
    uint64_t n_out = get_u32(arc, H_NOUT), n_patch = get_u32(arc, H_NPATCH);
    uint64_t total_bits = get_u64(arc, H_TOTBITS);
    int maxlen_hdr = get_u8(arc, H_MAXLEN);
    int layers = get_u8(arc, H_LAYERS) + 1;
    if (layers > ORC_MAX_LAYERS) return ORC_ECORRUPT;
    if (n_out > g.nelem || n_patch > g.nelem) return ORC_ECORRUPT;
    if (total_bits > 64ull * g.nelem) return ORC_ECORRUPT;
    layout_t L;
    make_layout(radius, g.padded, sub, csubs, n_out + n_patch, total_bits, &L);
    if (get_u32(arc, H_NCHUNKS) != L.n_chunks) return ORC_ECORRUPT;
    if (get_u64(arc, H_ARCBYTES) != L.end || nbytes < L.end) return ORC_ECORRUPT;
    if (cap_elems < g.nelem) return ORC_ETOOSMALL;
    const uint64_t N = g.nelem;

    /* lengths -> canonical decoding tables */
    uint8_t *len = (uint8_t *)malloc(nsym);
    uint32_t *sorted = (uint32_t *)malloc(sizeof(uint32_t) * nsym);
    int32_t *delta = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
    int32_t *dq = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
    uint64_t *subbits = (uint64_t *)calloc(L.n_sub ? L.n_sub : 1, sizeof(uint64_t));
    int st = ORC_OK;
    if (!len || !sorted || !delta || !dq || !subbits) { st = ORC_ENOMEM; goto done; }
    uint64_t bl_count[65] = {0};
    int maxlen = 0;
    for (uint32_t s = 0; s < nsym; s++) {
        len[s] = get_u8(arc, L.off_len + s);
        if (len[s] > 64) { st = ORC_ECORRUPT; goto done; }
        bl_count[len[s]]++;
        if (len[s] > maxlen) maxlen = len[s];
    }
    if (maxlen != maxlen_hdr) { st = ORC_ECORRUPT; goto done; }
    {
        /* the lengths must describe a complete prefix code (Kraft sum 1),
         * or a single symbol of length 1 */
        uint64_t used = 0;
        for (int l = 1; l <= 64; l++) used += bl_count[l];
        if (used == 1) {
            if (bl_count[1] != 1) { st = ORC_ECORRUPT; goto done; }
        } else if (used > 1) {
            /* Kraft sum in units of 2^-maxlen, exact in 128-bit integers */
            unsigned __int128 kr = 0;
            for (int l = 1; l <= maxlen; l++) kr += (unsigned __int128)bl_count[l] << (maxlen - l);
            if (kr != ((unsigned __int128)1 << maxlen)) { st = ORC_ECORRUPT; goto done; }
        }
        uint32_t k = 0;
        for (int l = 1; l <= 64; l++)
            for (uint32_t s = 0; s < nsym; s++)
                if (len[s] == l) sorted[k++] = s;
    }

    /* inflate every symbol in stream order; map codes back to deltas */
    {
        bitr_t br = {arc + L.off_str, total_bits, 0};
        uint64_t e = 0; /* next exception */
        FOR_EACH_STREAM_ELEMENT(&g, z, y, x, pos) {
            uint64_t i = (z * g.n[1] + y) * g.n[2] + x;
            uint64_t start = br.pos;
            /* canonical decode, one bit at a time */
            int64_t codev = 0, first = 0, index = 0;
            int found = 0;
            uint32_t sym = 0;
            for (int l = 1; l <= maxlen; l++) {
                int bit;
                if (!br_get_bit(&br, &bit)) break;
                codev |= bit;
                int64_t count = (int64_t)bl_count[l];
                if (codev - first < count) {
                    sym = sorted[index + (codev - first)];
                    found = 1;
                    break;
                }
                index += count;
                first += count;
                first <<= 1;
                codev <<= 1;
            }
            if (!found) { st = ORC_ECORRUPT; goto done; }
            subbits[pos / sub] += br.pos - start;
            if (sym == 0) {
                /* outlier: the next exception must be this position's delta */
                if (e >= L.n_exc || get_u32(arc, L.off_exc + 8 * e) != (uint32_t)(2 * pos)) {
                    st = ORC_ECORRUPT;
                    goto done;
                }
                delta[i] = (int32_t)get_u32(arc, L.off_exc + 8 * e + 4);
                e++;
            } else {
                delta[i] = (int32_t)sym - (int32_t)radius;
            }
            /* skip this position's patch record, if any, applied later */
            if (e < L.n_exc && get_u32(arc, L.off_exc + 8 * e) == (uint32_t)(2 * pos + 1)) e++;
        }
        if (e != L.n_exc || br.pos != total_bits) { st = ORC_ECORRUPT; goto done; }
    }
    /* the subchunk and chunk tables must agree with the decoded stream */
    {
        uint64_t acc = 0;
        for (uint64_t j = 0; j < L.n_sub; j++) {
            if (j % csubs == 0 && get_u64(arc, L.off_chunk + 8 * (j / csubs)) != acc) { st = ORC_ECORRUPT; goto done; }
            if (get_u16(arc, L.off_sub + 2 * j) != subbits[j]) { st = ORC_ECORRUPT; goto done; }
            acc += subbits[j];
        }
    }
    /* reversed dual-quantization: cascading Lorenzo reconstruction, then
     * d = d° * 2eb */
    orc_lorenzo_reconstruct_n(delta, ndim, dims, layers, dq);
    for (uint64_t i = 0; i < N; i++) out[i] = dequant(dq[i], h);
    /* patches: verbatim values */
    {
        uint64_t prev_key = 0;
        for (uint64_t e = 0; e < L.n_exc; e++) {
            uint32_t key = get_u32(arc, L.off_exc + 8 * e);
            if (e > 0 && key <= prev_key) { st = ORC_ECORRUPT; goto done; }
            prev_key = key;
            if (key & 1u) {
                uint64_t pos = key >> 1;
                uint64_t blk = pos / g.bvol, in = pos % g.bvol;
                uint64_t Bx = blk % g.nb[2], By = (blk / g.nb[2]) % g.nb[1], Bz = blk / (g.nb[2] * g.nb[1]);
                uint64_t ix = in % g.b[2], iy = (in / g.b[2]) % g.b[1], iz = in / (g.b[2] * g.b[1]);
                uint64_t z = Bz * g.b[0] + iz, y = By * g.b[1] + iy, x = Bx * g.b[2] + ix;
                if (z >= g.n[0] || y >= g.n[1] || x >= g.n[2]) { st = ORC_ECORRUPT; goto done; }
                out[(z * g.n[1] + y) * g.n[2] + x] = bits_f32(get_u32(arc, L.off_exc + 8 * e + 4));
            }
        }
    }
done:
    free(len); free(sorted); free(delta); free(dq); free(subbits);
    return st;
}

/* Intermediate results of compression, for the pins and for stage-by-stage
 * comparison: prequantized values (row-major), codes in stream order and the
 * histogram.  Arrays are caller-allocated: dq[N], codes[N], freq[2R]. */
int orc_stages(const float *xin, int ndim, const uint64_t *dims, double eb, int eb_mode,
               uint32_t radius, int32_t *dq_out, uint16_t *codes_out, uint64_t *freq_out,
               double *eb_abs_out)
{
    geom_t g;
    int st;
    if ((st = make_geom(ndim, dims, &g)) != ORC_OK) return st;
    if (!is_pow2(radius) || radius > 4096) return ORC_EINVAL;
    uint64_t N = g.nelem;
    float vmin = 0.0f, vmax = 0.0f;
    uint64_t nfinite = 0;
    if (eb_mode == 1) orc_value_range(xin, N, &vmin, &vmax, &nfinite);
    double eb_abs;
    float h, r;
    if ((st = orc_eb_params(eb_mode, eb, vmin, vmax, nfinite, &eb_abs, &h, &r)) != ORC_OK) return st;
    int32_t *delta = (int32_t *)malloc(sizeof(int32_t) * (N ? N : 1));
    if (!delta) return ORC_ENOMEM;
    orc_prequant(xin, N, r, dq_out);
    orc_lorenzo_delta(dq_out, ndim, dims, delta);
    memset(freq_out, 0, sizeof(uint64_t) * 2 * radius);
    uint64_t ns = 0;
    FOR_EACH_STREAM_ELEMENT(&g, z, y, x, pos) {
        (void)pos;
        int32_t d = delta[(z * g.n[1] + y) * g.n[2] + x];
        uint16_t qq = (d > -(int32_t)radius && d < (int32_t)radius) ? (uint16_t)(d + (int32_t)radius) : 0;
        codes_out[ns++] = qq;
        freq_out[qq]++;
    }
    *eb_abs_out = eb_abs;
    free(delta);
    return ORC_OK;
}
