/*
 * golomb_ref.c -- TEST INFRASTRUCTURE ONLY: plain scalar CPU oracle for
 * PivCo-Golomb (App. G of the paper).  Nothing in the product path may call
 * this file.
 *
 * App. G applies the pivoted layout to a unary code: instead of a tree
 * there is a list of bitmaps, one per code-bit position.  Reading of the
 * appendix used here: a value v (0..255) is coded as v 0-bits followed by a
 * 1-bit; bitmap k holds, in stream order, the k-th code bit of every value
 * that has one (the values >= k), so its bit is 1 exactly for the values
 * equal to k.  Decoding bottom-up walks the list from the last bitmap to the
 * first: at bitmap k a 1 bit gives 0 and a 0 bit gives 1 + the value the
 * next bitmap holds for that position (the appendix's merge_vec_cst_plus1
 * with constant 0xFF).
 *
 * Stream format (ours, little-endian):
 *   header, 32 bytes: magic u32 "PVG1" | version u16 = 1 | flags u16 = 0
 *                     | n_total u64 | block_size u32 | n_blocks u32 | reserved u64 = 0
 *   block_off u64[n_blocks + 1]: byte offset of each block; the last entry is
 *                     the stream size
 *   blocks, each at a multiple of 4 bytes:
 *     comp_size u32 | n u32 | K u16 (bitmaps = largest value + 1) | pad u16 = 0
 *     | n_k u32 for k = 1 .. K-1 (values >= k; n_0 = n)
 *     | bitmaps k = 0 .. K-1: ceil(n_k / 8) bytes, LSB first, padding bits 0
 *   comp_size counts the block's bytes up to the end of its last bitmap; the
 *   block is padded with zero bytes to a multiple of 4.
 */
#include "pivco_ref.h"

#include <stdlib.h>
#include <string.h>

#define GHDR 32
#define GMAGIC 0x31475650u   /* "PVG1" */

static void gput32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void gput64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t gget32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t gget64(const uint8_t *p) { return (uint64_t)gget32(p) | ((uint64_t)gget32(p + 4) << 32); }

uint64_t pivco_ref_golomb_bound(uint64_t n, uint32_t block_size) {
    if (block_size == 0) return 0;
    uint64_t nb = (n + block_size - 1) / block_size;
    /* a value takes at most 256 code bits; a block at most 256 bitmaps */
    return GHDR + 8 * (nb + 1) + nb * (12 + 4 * 255 + 256 + 4) + 32 * n;
}

int pivco_ref_golomb_encode(const uint8_t *in, uint64_t n, uint32_t block_size, uint8_t *out,
                            uint64_t cap, uint64_t *out_len) {
    if (!out || !out_len || block_size == 0 || (n && !in)) return PVO_E_ARG;
    uint64_t nb = (n + block_size - 1) / block_size;
    if (nb > 0xFFFFFFFFull) return PVO_E_ARG;
    uint64_t o = GHDR + 8 * (nb + 1);
    if (o > cap) return PVO_E_CAPACITY;
    memset(out, 0, (size_t)o);
    gput32(out, GMAGIC);
    out[4] = 1;                                   /* version 1, flags 0 */
    gput64(out + 8, n);
    gput32(out + 16, block_size);
    gput32(out + 20, (uint32_t)nb);
    for (uint64_t b = 0; b < nb; b++) {
        const uint8_t *x = in + b * block_size;
        uint64_t bn = n - b * block_size < block_size ? n - b * block_size : block_size;
        gput64(out + GHDR + 8 * b, o);
        uint32_t K = 0;
        uint64_t nk[257];
        memset(nk, 0, sizeof(nk));
        for (uint64_t i = 0; i < bn; i++) {
            if ((uint32_t)x[i] + 1 > K) K = (uint32_t)x[i] + 1;
            for (uint32_t k = 0; k <= x[i]; k++) nk[k]++;   /* value v has code bits 0..v */
        }
        uint64_t hlen = 12 + 4 * (uint64_t)(K ? K - 1 : 0);
        uint64_t boff[257], body = 0;
        for (uint32_t k = 0; k < K; k++) { boff[k] = hlen + body; body += (nk[k] + 7) / 8; }
        uint64_t comp = hlen + body, padded = (comp + 3) & ~3ull;
        if (o + padded > cap) return PVO_E_CAPACITY;
        uint8_t *p = out + o;
        memset(p, 0, (size_t)padded);
        gput32(p, (uint32_t)comp);
        gput32(p + 4, (uint32_t)bn);
        p[8] = (uint8_t)K; p[9] = (uint8_t)(K >> 8);
        for (uint32_t k = 1; k < K; k++) gput32(p + 12 + 4 * (k - 1), (uint32_t)nk[k]);
        /* value i appends, for k = 0 .. v, the bit (k == v) to bitmap k */
        uint64_t cur[256];
        memset(cur, 0, sizeof(cur));
        for (uint64_t i = 0; i < bn; i++) {
            for (uint32_t k = 0; k <= x[i]; k++) {
                if (k == x[i]) p[boff[k] + (cur[k] >> 3)] |= (uint8_t)(1u << (cur[k] & 7));
                cur[k]++;
            }
        }
        o += padded;
    }
    gput64(out + GHDR + 8 * nb, o);
    *out_len = o;
    return PVO_OK;
}

typedef struct {
    uint64_t n;
    uint32_t K;
    uint64_t nk[256];
    const uint8_t *bm[256];
} gblock_t;

static int gbit(const uint8_t *bm, uint64_t j) { return (bm[j >> 3] >> (j & 7)) & 1; }

/* Parses and validates block b: sizes, every bitmap's count of 0 bits equals
 * the next bitmap's size, the last bitmap has no 0 bit, padding bits zero. */
static int gparse(const uint8_t *in, uint64_t in_len, uint64_t nb, uint32_t bs, uint64_t n_total,
                  uint64_t b, gblock_t *g) {
    uint64_t off = gget64(in + GHDR + 8 * b), end = gget64(in + GHDR + 8 * (b + 1));
    if (off < GHDR + 8 * (nb + 1) || end < off || end > in_len || (off & 3) || end - off < 12)
        return PVO_E_CORRUPT;
    const uint8_t *p = in + off;
    uint64_t comp = gget32(p);
    g->n = gget32(p + 4);
    g->K = (uint32_t)p[8] | ((uint32_t)p[9] << 8);
    uint64_t want = n_total - b * bs < bs ? n_total - b * bs : bs;
    if (g->n != want || p[10] || p[11] || g->K > 256 || (g->n == 0) != (g->K == 0)) return PVO_E_CORRUPT;
    uint64_t hlen = 12 + 4 * (uint64_t)(g->K ? g->K - 1 : 0);
    if (comp < hlen || comp > end - off || ((comp + 3) & ~3ull) != end - off) return PVO_E_CORRUPT;
    uint64_t o = hlen;
    for (uint32_t k = 0; k < g->K; k++) {
        g->nk[k] = k ? gget32(p + 12 + 4 * (k - 1)) : g->n;
        if (k && g->nk[k] > g->nk[k - 1]) return PVO_E_CORRUPT;
        uint64_t nbytes = (g->nk[k] + 7) / 8;
        if (o + nbytes > comp) return PVO_E_CORRUPT;
        g->bm[k] = p + o;
        if ((g->nk[k] & 7) && (p[o + nbytes - 1] >> (g->nk[k] & 7))) return PVO_E_CORRUPT;
        o += nbytes;
    }
    if (o != comp) return PVO_E_CORRUPT;
    for (uint64_t i = comp; i < end - off; i++) if (p[i]) return PVO_E_CORRUPT;
    for (uint32_t k = 0; k < g->K; k++) {
        uint64_t zeros = 0;
        for (uint64_t j = 0; j < g->nk[k]; j++) zeros += (uint64_t)(1 - gbit(g->bm[k], j));
        uint64_t next = k + 1 < g->K ? g->nk[k + 1] : 0;
        if (zeros != next) return PVO_E_CORRUPT;
    }
    return PVO_OK;
}

static int gdecode(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap, uint64_t *n_out,
                   int merge) {
    if (!in || in_len < GHDR || gget32(in) != GMAGIC || in[4] != 1 || in[5] || in[6] || in[7])
        return PVO_E_CORRUPT;
    uint64_t n_total = gget64(in + 8);
    uint32_t bs = gget32(in + 16), nb = gget32(in + 20);
    if (bs == 0 || (n_total + bs - 1) / bs != nb || GHDR + 8 * ((uint64_t)nb + 1) > in_len) return PVO_E_CORRUPT;
    if (gget64(in + GHDR + 8 * (uint64_t)nb) != in_len) return PVO_E_CORRUPT;
    if (n_total > cap) return PVO_E_CAPACITY;
    uint64_t o = 0;
    for (uint64_t b = 0; b < nb; b++) {
        gblock_t g;
        int rc = gparse(in, in_len, nb, bs, n_total, b, &g);
        if (rc) return rc;
        if (!merge) {
            /* each value: count the 0 bits read, one bitmap after the other,
             * up to the first 1 bit (one read cursor per bitmap) */
            uint64_t cur[256];
            memset(cur, 0, sizeof(cur));
            for (uint64_t i = 0; i < g.n; i++) {
                uint32_t k = 0;
                while (!gbit(g.bm[k], cur[k]++)) k++;
                out[o + i] = (uint8_t)k;
            }
        } else {
            /* bottom-up from the last bitmap: position j of bitmap k is 0
             * for a 1 bit, else 1 + entry (j - ones before j) of bitmap k+1 */
            uint8_t *next = NULL;
            for (int k = (int)g.K - 1; k >= 0; k--) {
                uint8_t *cur = k ? (uint8_t *)malloc((size_t)g.nk[k] + 1) : out + o;
                uint64_t ones = 0;
                for (uint64_t j = 0; j < g.nk[k]; j++) {
                    int bit = gbit(g.bm[k], j);
                    cur[j] = bit ? 0 : (uint8_t)(next[j - ones] + 1);
                    ones += (uint64_t)bit;
                }
                free(next);
                next = k ? cur : NULL;
            }
        }
        o += g.n;
    }
    if (n_out) *n_out = o;
    return PVO_OK;
}

int pivco_ref_golomb_decode(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap, uint64_t *n_out) {
    return gdecode(in, in_len, out, cap, n_out, 0);
}

int pivco_ref_golomb_decode_merge(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                                  uint64_t *n_out) {
    return gdecode(in, in_len, out, cap, n_out, 1);
}
