/*
 * fse_ref.c -- TEST INFRASTRUCTURE ONLY: the oracle's selective tANS ("FSE")
 * coding of node bitmaps as bytes (Sec. 5.2 of the paper; App. D's FSE
 * marker; the x-cursor layout of App. F).  Nothing in the product path may
 * call this file.
 *
 * Readings (the paper fixes the ideas, not the numbers below):
 *   - A table serves bitmaps whose 1-bit fraction is s = t + 49 percent,
 *     t = 1..50 (the "50 static tables for skew 50..99%").  It is built for
 *     bytes whose 8 bits are independent with P(1) = s: P(b) = s^k (1-s)^(8-k)
 *     with k = popcount(b).
 *   - Table size 2^11.  Normalized counts by largest remainders, exact in
 *     integers (s as a percentage): n_b = floor(P(b) 2^11), at least 1; if
 *     they sum to less than 2^11, one more to each of the bytes with the
 *     largest remainders P(b) 2^11 - floor (lower byte first on equal
 *     remainders) until the sum is 2^11; if the forced 1s make it more, the
 *     excess comes off the largest count (lowest byte among equal ones).
 *   - Spread: symbols 0..255 in order, each n_b times, to positions p, p +
 *     step, ... (mod 2^11), step = 2^10 + 2^8 + 3 (odd: every position once).
 *   - Decoding state X in [0, 2^11): b = spread[X]; the k-th state of b in
 *     increasing X has k = n_b, n_b + 1, ...; it reads nb = 11 - floor(log2 k)
 *     bits v and goes to (k << nb) - 2^11 + v.  Encoding is its inverse: from
 *     x in [2^11, 2^12), emit the low nb bits of x with x >> nb in [n_b,
 *     2 n_b), then x = 2^11 + (the state of b numbered x >> nb).
 *   - Layout: a node's bitmap is ceil(n_v / 8) bytes; chunks of 2^chunk_log2
 *     bits (as the rANS chunks); in a chunk byte j goes to cursor j mod 32 at
 *     step j / 32 (32 cursors, the paper's x-cursor idea at the GPU's width),
 *     each cursor with its own bit stream: the bits read at steps 0, 1, ...
 *     follow each other LSB first.  Chunk: X0 u16[32] (each cursor's first
 *     state) | nbytes u16[32] (each cursor's stream bytes) | the 32 streams |
 *     zero padding to 4 bytes.  After its last step every cursor is back at
 *     state 0 (the encoder's first state), which the decoder checks.
 *   - XOR marker: a bitmap with more 0 than 1 bits is coded complemented
 *     (every byte XOR 0xFF) with the table of its 0-bit fraction.
 *   - Selection (Sec. 5.2): at least 256 bits (32 bytes); skew max(f, 1-f)
 *     above 0.625 (8 max(n_right, n_v - n_right) > 5 n_v); table t = round
 *     (100 skew) - 49, halves rounding up; benefit (depth + H_t) / (depth +
 *     1) < 0.95 with H_t the table's expected bits per bitmap bit at its own
 *     skew, sum over b of P(b) (11 - log2 n_b) / 8, in double.
 */
#include "pivco_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FSE_LOG 11
#define FSE_SIZE (1u << FSE_LOG)
#define FSE_LANES 32

static int popcount8(uint32_t b) {
    int k = 0;
    for (int i = 0; i < 8; i++) k += (int)((b >> i) & 1);
    return k;
}

static uint64_t ipow(uint64_t a, int e) {
    uint64_t r = 1;
    for (int i = 0; i < e; i++) r *= a;
    return r;
}

int pivco_ref_fse_norm(uint32_t t, uint16_t norm[256]) {
    if (t < 1 || t > 50 || !norm) return PVO_E_ARG;
    const uint64_t s = t + 49, q = 100 - s;
    const unsigned __int128 den = (unsigned __int128)ipow(100, 8);
    unsigned __int128 rem[256];
    int32_t sum = 0;
    for (int b = 0; b < 256; b++) {
        const int k = popcount8((uint32_t)b);
        const unsigned __int128 num = (unsigned __int128)(ipow(s, k) * ipow(q, 8 - k)) * FSE_SIZE;
        uint32_t n = (uint32_t)(num / den);
        rem[b] = num % den;
        if (n < 1) { n = 1; rem[b] = 0; }        /* forced: takes no extra unit */
        norm[b] = (uint16_t)n;
        sum += (int32_t)n;
    }
    while (sum < (int32_t)FSE_SIZE) {           /* largest remainder, lowest byte on ties */
        int best = -1;
        for (int b = 0; b < 256; b++)
            if (rem[b] && (best < 0 || rem[b] > rem[best])) best = b;
        if (best < 0) return PVO_E_ARG;
        norm[best]++;
        rem[best] = 0;
        sum++;
    }
    if (sum > (int32_t)FSE_SIZE) {
        int big = 0;
        for (int b = 1; b < 256; b++) if (norm[b] > norm[big]) big = b;
        const int32_t fixed = (int32_t)norm[big] - (sum - (int32_t)FSE_SIZE);
        if (fixed < 1) return PVO_E_ARG;
        norm[big] = (uint16_t)fixed;
    }
    return PVO_OK;
}

typedef struct {
    uint16_t norm[256];
    uint8_t sym[FSE_SIZE];      /* decoding: symbol of state X */
    uint8_t nb[FSE_SIZE];       /* bits read in state X */
    uint16_t base[FSE_SIZE];    /* next state before adding the bits read */
    uint16_t first[256];        /* encoding: symbol b's states start here ... */
    uint16_t state[FSE_SIZE];   /* ... in increasing X */
} fse_t;

static int floor_log2(uint32_t v) {
    int r = -1;
    while (v) { v >>= 1; r++; }
    return r;
}

static int fse_build(uint32_t t, fse_t *T) {
    if (pivco_ref_fse_norm(t, T->norm)) return PVO_E_ARG;
    const uint32_t step = (FSE_SIZE >> 1) + (FSE_SIZE >> 3) + 3;
    uint32_t pos = 0;
    for (int b = 0; b < 256; b++)
        for (uint32_t i = 0; i < T->norm[b]; i++) {
            T->sym[pos] = (uint8_t)b;
            pos = (pos + step) & (FSE_SIZE - 1);
        }
    uint32_t next[256], at = 0;
    for (int b = 0; b < 256; b++) { next[b] = T->norm[b]; T->first[b] = (uint16_t)at; at += T->norm[b]; }
    for (uint32_t X = 0; X < FSE_SIZE; X++) {
        const int b = T->sym[X];
        const uint32_t k = next[b]++;
        const int nb = FSE_LOG - floor_log2(k);
        T->nb[X] = (uint8_t)nb;
        T->base[X] = (uint16_t)((k << nb) - FSE_SIZE);
        T->state[T->first[b] + (k - T->norm[b])] = (uint16_t)X;
    }
    return PVO_OK;
}

double pivco_ref_fse_cost(uint32_t t) {
    uint16_t norm[256];
    if (pivco_ref_fse_norm(t, norm)) return -1.0;
    const double s = (double)(t + 49) / 100.0;
    double h = 0.0;
    for (int b = 0; b < 256; b++) {
        const int k = popcount8((uint32_t)b);
        const double p = pow(s, k) * pow(1.0 - s, 8 - k);
        h += p * ((double)FSE_LOG - log2((double)norm[b])) / 8.0;
    }
    return h;
}

int pivco_ref_fse_select(uint64_t n_v, uint64_t n_right, uint32_t depth, uint32_t *marker) {
    if (n_v < 256 || n_right > n_v) return 0;
    const uint64_t ones = n_right, zeros = n_v - n_right;
    const uint64_t maj = ones >= zeros ? ones : zeros;
    if (8 * maj <= 5 * n_v) return 0;                          /* skew <= 0.625 */
    uint64_t pct = (200 * maj + n_v) / (2 * n_v);              /* round(100 skew), halves up */
    if (pct > 99) pct = 99;
    const uint32_t t = (uint32_t)pct - 49;
    const double h = pivco_ref_fse_cost(t);
    if (!((double)depth + h < 0.95 * ((double)depth + 1.0))) return 0;
    if (marker) *marker = t | (ones < zeros ? 0x80u : 0u);
    return 1;
}

static void put16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static uint32_t get16(const uint8_t *p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }

int pivco_ref_fse_encode(const uint8_t *bits, uint64_t nbits, uint32_t marker, uint32_t chunk_log2,
                         uint8_t *out, uint64_t cap, uint64_t *out_len) {
    const uint32_t t = marker & 0x7F;
    const uint8_t flip = (marker & 0x80) ? 0xFF : 0x00;
    if (chunk_log2 < 8 || chunk_log2 > 24 || !out_len) return PVO_E_ARG;
    fse_t *T = (fse_t *)malloc(sizeof(fse_t));
    if (fse_build(t, T)) { free(T); return PVO_E_ARG; }
    const uint64_t nbytes = (nbits + 7) / 8, cbytes = ((uint64_t)1 << chunk_log2) / 8;
    uint64_t o = 0;
    int rc = PVO_OK;
    /* per cursor: the bits emitted for each of its steps (at most 11 each) */
    const uint64_t smax = (cbytes + FSE_LANES - 1) / FSE_LANES;
    uint16_t *val = (uint16_t *)malloc(sizeof(uint16_t) * smax);
    uint8_t *cnt = (uint8_t *)malloc(smax);
    for (uint64_t c0 = 0; c0 < nbytes; c0 += cbytes) {
        const uint64_t cb = nbytes - c0 < cbytes ? nbytes - c0 : cbytes;
        if (o + 4 * FSE_LANES > cap) { rc = PVO_E_CAPACITY; break; }
        uint8_t *hdr = out + o;
        uint64_t so = o + 4 * FSE_LANES;
        for (uint32_t lane = 0; lane < FSE_LANES; lane++) {
            const uint64_t steps = cb > lane ? (cb - lane + FSE_LANES - 1) / FSE_LANES : 0;
            uint32_t x = FSE_SIZE;                              /* encoder state in [2^11, 2^12) */
            for (uint64_t i = steps; i-- > 0;) {                /* the last byte first */
                const uint8_t b = (uint8_t)(bits[c0 + lane + FSE_LANES * i] ^ flip);
                const uint32_t n = T->norm[b];
                uint32_t nb = 0;
                while ((x >> nb) >= 2 * n) nb++;
                val[i] = (uint16_t)(x & ((1u << nb) - 1));
                cnt[i] = (uint8_t)nb;
                x = FSE_SIZE + T->state[T->first[b] + ((x >> nb) - n)];
            }
            uint64_t tb = 0;
            for (uint64_t i = 0; i < steps; i++) tb += cnt[i];
            const uint64_t lb = (tb + 7) / 8;
            if (so + lb > cap || lb > 0xFFFF) { rc = PVO_E_CAPACITY; goto end; }
            memset(out + so, 0, (size_t)lb);
            uint64_t p = 0;
            for (uint64_t i = 0; i < steps; i++)
                for (uint32_t k = 0; k < cnt[i]; k++, p++)
                    if ((val[i] >> k) & 1) out[so + (p >> 3)] |= (uint8_t)(1u << (p & 7));
            put16(hdr + 2 * lane, x - FSE_SIZE);
            put16(hdr + 2 * FSE_LANES + 2 * lane, (uint32_t)lb);
            so += lb;
        }
        while (so & 3) { if (so >= cap) { rc = PVO_E_CAPACITY; goto end; } out[so++] = 0; }
        o = so;
    }
end:
    free(val); free(cnt); free(T);
    if (rc == PVO_OK) *out_len = o;
    return rc;
}

int pivco_ref_fse_decode(const uint8_t *body, uint64_t body_len, uint64_t nbits, uint32_t marker,
                         uint32_t chunk_log2, uint8_t *bits) {
    const uint32_t t = marker & 0x7F;
    const uint8_t flip = (marker & 0x80) ? 0xFF : 0x00;
    if (chunk_log2 < 8 || chunk_log2 > 24 || (marker & 0x7F) < 1 || (marker & 0x7F) > 50) return PVO_E_CORRUPT;
    fse_t *T = (fse_t *)malloc(sizeof(fse_t));
    if (fse_build(t, T)) { free(T); return PVO_E_CORRUPT; }
    const uint64_t nbytes = (nbits + 7) / 8, cbytes = ((uint64_t)1 << chunk_log2) / 8;
    uint64_t o = 0;
    int rc = PVO_OK;
    for (uint64_t c0 = 0; c0 < nbytes && rc == PVO_OK; c0 += cbytes) {
        const uint64_t cb = nbytes - c0 < cbytes ? nbytes - c0 : cbytes;
        if (o + 4 * FSE_LANES > body_len) { rc = PVO_E_CORRUPT; break; }
        const uint8_t *hdr = body + o;
        uint64_t so = o + 4 * FSE_LANES;
        for (uint32_t lane = 0; lane < FSE_LANES && rc == PVO_OK; lane++) {
            const uint64_t steps = cb > lane ? (cb - lane + FSE_LANES - 1) / FSE_LANES : 0;
            const uint64_t lb = get16(hdr + 2 * FSE_LANES + 2 * lane);
            uint32_t X = get16(hdr + 2 * lane);
            if (so + lb > body_len || X >= FSE_SIZE) { rc = PVO_E_CORRUPT; break; }
            uint64_t p = 0;
            for (uint64_t i = 0; i < steps; i++) {
                const uint8_t b = T->sym[X];
                const uint32_t nb = T->nb[X];
                if (p + nb > 8 * lb) { rc = PVO_E_CORRUPT; break; }
                uint32_t v = 0;
                for (uint32_t k = 0; k < nb; k++, p++) v |= (uint32_t)((body[so + (p >> 3)] >> (p & 7)) & 1) << k;
                X = T->base[X] + v;
                bits[c0 + lane + FSE_LANES * i] = (uint8_t)(b ^ flip);
            }
            /* every bit used, padding bits zero, back at the first state */
            if (rc == PVO_OK && (X != 0 || (p + 7) / 8 != lb ||
                                 ((p & 7) && (body[so + lb - 1] >> (p & 7)))))
                rc = PVO_E_CORRUPT;
            so += lb;
        }
        while (rc == PVO_OK && (so & 3)) { if (so >= body_len || body[so]) rc = PVO_E_CORRUPT; so++; }
        o = so;
    }
    if (rc == PVO_OK && o != body_len) rc = PVO_E_CORRUPT;
    /* the bitmap's padding bits (past n_v) must be zero */
    if (rc == PVO_OK && (nbits & 7) && (bits[nbytes - 1] >> (nbits & 7))) rc = PVO_E_CORRUPT;
    free(T);
    return rc;
}
