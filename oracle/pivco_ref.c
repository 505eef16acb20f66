/*
 * pivco_ref.c -- TEST INFRASTRUCTURE ONLY: plain scalar CPU oracle for the
 * PivCo-Huffman codec.  Nothing in the product path may call this file; it
 * exists so that tests can check the GPU library against an implementation
 * that can be read against the paper line by line.  See pivco_ref.h for the
 * passage each function follows.
 *
 * Wire format v1 (all integers little-endian):
 *
 *   stream header, 48 bytes:
 *     magic u32 = "PVC1" | version u16 = 1 | flags u16 = 0 | n_total u64
 *     | block_size u32 | n_blocks u32 | max_len u8 | chunk_log2 u8
 *     | reserved u16 = 0 | reserved u32 = 0 | ans_words u64 | reserved u64 = 0
 *   block_off u64[n_blocks + 1]   byte offset of each block from the stream
 *                                 start; the last entry is the stream size
 *   ans_off   u64[n_blocks + 1]   running count of scratch words (u32) that
 *                                 the rANS-coded nodes of earlier blocks
 *                                 decode into: sum of ceil(n_v / 32)
 *   blocks, each starting at a multiple of 4 bytes:
 *     comp_size u32 | n u32 | mode u8 (0 coded, 1 constant) | const_sym u8
 *     | cnt_width u8 (2 if n <= 65535 else 4) | pad u8 = 0
 *     mode 0 only:
 *       code_len u8[128]: symbol 2j in the low nibble of byte j, 2j+1 in the
 *                         high nibble; 0 = absent (App. D)
 *       kind u8[ceil(I/8)]: bit i (LSB first) = internal node i is rANS-coded
 *       n_right u16|u32 [I]: number of 1 bits (symbols going right) of every
 *                         internal node
 *       raw bodies of nodes with kind 0, node order: ceil(n_v/8) bytes, bit j
 *                         of the node in byte j>>3 at bit j&7, pad bits zero
 *       rANS bodies of nodes with kind 1, node order, each at a multiple of 4
 *                         bytes: p1q u16 | pad u16 | body_len u32 | chunks
 *     comp_size counts the block's bytes from its first header byte to the
 *     end of its last body.
 *   Internal nodes are numbered breadth-first: by depth, then left to right.
 *   Bit 0 = left child, bit 1 = right child (Listing 1).
 *
 * Stream flags bit 0 (encoder ans_mode 3): entropy-coded nodes use the
 * selective tANS of bitmap bytes (fse_ref.c) instead of binary rANS; such a
 * body is marker u8 (table id 1..50 | 0x80 complemented) | 0 u8 | 0 u16 |
 * body_len u32 | chunks.
 *
 * Wire format v2 (version u16 = 2) is v1 with the flat-subtree tree of
 * Sec. 2.2.3-2.2.4 in place of the canonical one, derived from the same
 * length table (build_flat_tree).  Its nodes are numbered the same way; a
 * flat node of depth D keeps n_right = 0 and kind 0, and its raw body is
 * ceil(n_v D / 8) bytes holding one D-bit field per passing symbol, field j
 * at bits [jD, jD + D) (LSB first; bit k of the field is bit k of the
 * value), whose value is the index of the symbol in the node's group.
 */
#include "pivco_ref.h"

#include <stdlib.h>
#include <string.h>

#define MAXSYM 256
#define MAXNODE 511   /* 255 internal + 256 leaves */

/* ------------------------------------------------------------------ */
/* little-endian helpers                                               */
/* ------------------------------------------------------------------ */
static void put16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t get16(const uint8_t *p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t get32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t get64(const uint8_t *p) { return (uint64_t)get32(p) | ((uint64_t)get32(p + 4) << 32); }

static int getbit(const uint8_t *bm, uint64_t j) { return (bm[j >> 3] >> (j & 7)) & 1; }
static void setbit(uint8_t *bm, uint64_t j) { bm[j >> 3] |= (uint8_t)(1u << (j & 7)); }

/* ------------------------------------------------------------------ */
/* Code lengths: package-merge (coin collector)                        */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t w;     /* weight */
    int kind;       /* 0 = leaf, 1 = package */
    int sym;        /* leaf symbol */
    int a, b;       /* package: indices of its two items in the deeper list */
} pm_item;

int pivco_ref_lengths(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]) {
    if (!counts || !len || max_len < 1 || max_len > 15) return PVO_E_ARG;
    int syms[MAXSYM], m = 0;
    memset(len, 0, 256);
    for (int s = 0; s < 256; s++)
        if (counts[s]) syms[m++] = s;
    if (m < 2 || ((uint32_t)1 << max_len) < (uint32_t)m) return PVO_E_ARG;
    /* leaves sorted by (weight asc, symbol asc): insertion sort, stable */
    for (int i = 1; i < m; i++) {
        int s = syms[i], j = i - 1;
        while (j >= 0 && counts[syms[j]] > counts[s]) { syms[j + 1] = syms[j]; j--; }
        syms[j + 1] = s;
    }
    int L = (int)max_len;
    pm_item *lists[16];
    int nlist[16];
    /* list[L] = leaves; list[l-1] = merge(leaves, packages of list[l]) */
    for (int l = 0; l < 16; l++) lists[l] = NULL;
    lists[L] = (pm_item *)malloc(sizeof(pm_item) * (size_t)m);
    for (int i = 0; i < m; i++) {
        lists[L][i].w = counts[syms[i]]; lists[L][i].kind = 0; lists[L][i].sym = syms[i];
        lists[L][i].a = lists[L][i].b = -1;
    }
    nlist[L] = m;
    for (int l = L; l >= 2; l--) {
        int np = nlist[l] / 2;
        pm_item *out = (pm_item *)malloc(sizeof(pm_item) * (size_t)(m + np));
        int i = 0, p = 0, o = 0;
        while (i < m || p < np) {
            int take_leaf;
            if (p >= np) take_leaf = 1;
            else if (i >= m) take_leaf = 0;
            else {
                uint64_t pw = lists[l][2 * p].w + lists[l][2 * p + 1].w;
                take_leaf = counts[syms[i]] <= pw; /* leaf first on equal weight */
            }
            if (take_leaf) {
                out[o].w = counts[syms[i]]; out[o].kind = 0; out[o].sym = syms[i];
                out[o].a = out[o].b = -1; i++;
            } else {
                out[o].w = lists[l][2 * p].w + lists[l][2 * p + 1].w; out[o].kind = 1;
                out[o].sym = -1; out[o].a = 2 * p; out[o].b = 2 * p + 1; p++;
            }
            o++;
        }
        lists[l - 1] = out;
        nlist[l - 1] = o;
    }
    /* select the first 2m-2 items of list[1]; expand packages downwards */
    int cnt[256];
    memset(cnt, 0, sizeof(cnt));
    char *sel = (char *)calloc((size_t)(2 * m + 2), 1);
    char *nsel = (char *)calloc((size_t)(2 * m + 2), 1);
    for (int i = 0; i < 2 * m - 2 && i < nlist[1]; i++) sel[i] = 1;
    for (int l = 1; l <= L; l++) {
        memset(nsel, 0, (size_t)(2 * m + 2));
        for (int i = 0; i < nlist[l]; i++) {
            if (!sel[i]) continue;
            if (lists[l][i].kind == 0) cnt[lists[l][i].sym]++;
            else { nsel[lists[l][i].a] = 1; nsel[lists[l][i].b] = 1; }
        }
        char *t = sel; sel = nsel; nsel = t;
    }
    free(sel); free(nsel);
    for (int l = 1; l <= L; l++) free(lists[l]);
    /* deterministic assignment: ascending lengths to (count desc, sym asc) */
    int hist[16];
    memset(hist, 0, sizeof(hist));
    for (int s = 0; s < 256; s++)
        if (counts[s]) hist[cnt[s]]++;
    int order[MAXSYM];
    for (int i = 0; i < m; i++) order[i] = syms[i];
    /* syms sorted by (w asc, sym asc); want (w desc, sym asc) */
    for (int i = 1; i < m; i++) {
        int s = order[i], j = i - 1;
        while (j >= 0 && (counts[order[j]] < counts[s] ||
                          (counts[order[j]] == counts[s] && order[j] > s))) {
            order[j + 1] = order[j]; j--;
        }
        order[j + 1] = s;
    }
    int k = 0;
    for (int l = 1; l <= L; l++)
        for (int c = 0; c < hist[l]; c++) len[order[k++]] = (uint8_t)l;
    return k == m ? PVO_OK : PVO_E_ARG;
}

int pivco_ref_codes(const uint8_t len[256], uint16_t code[256]) {
    if (!len || !code) return PVO_E_ARG;
    memset(code, 0, 256 * sizeof(uint16_t));
    uint32_t c = 0;
    int prevlen = 0, first = 1;
    for (int l = 1; l <= 15; l++) {
        for (int s = 0; s < 256; s++) {
            if (len[s] != l) continue;
            if (first) { c = 0; first = 0; }
            else c = (c + 1) << (l - prevlen);
            prevlen = l;
            if (c >> l) return PVO_E_ARG; /* over-subscribed */
            code[s] = (uint16_t)c;
        }
    }
    return PVO_OK;
}

/* ------------------------------------------------------------------ */
/* Explicit code tree (trie) built from the canonical codes            */
/* ------------------------------------------------------------------ */
typedef struct {
    int leaf, sym, child[2], depth;
    int flat, g0;        /* flat node: its depth D >= 2 and its group's first
                            index in tree_t.order; 0 for other nodes */
    int id;              /* breadth-first index among internal nodes */
    uint64_t n, n_right; /* symbols passing / symbols going right */
} tnode;

typedef struct {
    tnode nd[MAXNODE];
    int nn;
    int bfs[255];        /* node index of internal node i (BFS order) */
    int ni;              /* number of internal nodes */
    uint16_t code[256];  /* every symbol's code: the branch bits of its path
                            from the root, then (below a flat node) its
                            index in the node's group, D bits */
    uint8_t order[256];  /* symbols ordered by (length, symbol) */
} tree_t;

/* Breadth-first numbering of the internal nodes (binary and flat; a flat
 * node's leaves are not nodes of the tree).  Every binary node must have two
 * children. */
static int number_nodes(tree_t *t) {
    int queue[MAXNODE], qh = 0, qt = 0;
    queue[qt++] = 0;
    t->ni = 0;
    while (qh < qt) {
        int v = queue[qh++];
        if (t->nd[v].leaf) continue;
        t->nd[v].id = t->ni;
        t->bfs[t->ni++] = v;
        if (t->nd[v].flat) continue;
        if (t->nd[v].child[0] < 0 || t->nd[v].child[1] < 0) return PVO_E_CORRUPT;
        queue[qt++] = t->nd[v].child[0];
        queue[qt++] = t->nd[v].child[1];
    }
    return PVO_OK;
}

static int new_node(tree_t *t, int depth) {
    int c = t->nn++;
    memset(&t->nd[c], 0, sizeof(tnode));
    t->nd[c].child[0] = t->nd[c].child[1] = -1;
    t->nd[c].depth = depth;
    return c;
}

/* Kraft sum of the lengths == 1 with at least two symbols. */
static int complete_code(const uint8_t len[256]) {
    uint64_t kraft = 0;
    int m = 0;
    for (int s = 0; s < 256; s++) {
        if (len[s] > 15) return 0;
        if (len[s]) { kraft += (uint64_t)1 << (15 - len[s]); m++; }
    }
    return m >= 2 && kraft == ((uint64_t)1 << 15);
}

/* Returns 0 if the lengths form a complete prefix code (Kraft sum == 1) with
 * at least two symbols, and builds the canonical code tree. */
static int build_tree(const uint8_t len[256], tree_t *t) {
    if (!complete_code(len)) return PVO_E_CORRUPT;
    memset(t, 0, sizeof(*t));
    if (pivco_ref_codes(len, t->code)) return PVO_E_CORRUPT;
    int no = 0;
    for (int l = 1; l <= 15; l++)
        for (int s = 0; s < 256; s++) if (len[s] == l) t->order[no++] = (uint8_t)s;
    new_node(t, 0);
    for (int s = 0; s < 256; s++) {
        if (!len[s]) continue;
        int cur = 0;
        for (int d = 0; d < len[s]; d++) {
            int b = (t->code[s] >> (len[s] - 1 - d)) & 1;
            if (t->nd[cur].leaf) return PVO_E_CORRUPT;
            int c = t->nd[cur].child[b];
            if (d == len[s] - 1) {
                if (c != -1) return PVO_E_CORRUPT;
                c = new_node(t, d + 1);
                t->nd[c].leaf = 1; t->nd[c].sym = s;
                t->nd[cur].child[b] = c;
            } else {
                if (c == -1) { c = new_node(t, d + 1); t->nd[cur].child[b] = c; }
                cur = c;
            }
        }
    }
    if (number_nodes(t)) return PVO_E_CORRUPT;
    return (t->ni == no - 1) ? PVO_OK : PVO_E_CORRUPT;
}

/* ------------------------------------------------------------------ */
/* Flat-subtree tree (Sec. 2.2.3 and 2.2.4)                            */
/* ------------------------------------------------------------------ */
/* The regrouping of Sec. 2.2.4, applied once the code lengths are fixed:
 * the symbols of each length, in ascending order, are cut into groups, each
 * the largest power of two of the symbols still left.  A group of 2^D
 * symbols of length l stands for one subtree of depth D whose leaves all
 * have length l, hanging at depth l - D.  These groups ("items") take
 * canonical codes of their own depths, ordered by (depth, D descending), so
 * the tree has the same code lengths as the canonical one and, usually, a
 * different shape.  An item with D >= 2 is a flat node (Sec. 2.2.3): it
 * keeps one D-bit value per passing symbol, the symbol's index in the group.
 * An item with D = 1 is an ordinary internal node with two leaf children; an
 * item with D = 0 is a leaf.  Grouping keeps the Kraft sum, so the items
 * form a complete code. */
typedef struct { int depth, d, first; } item_t;   /* first: index into order[] */

static int flat_items(const uint8_t len[256], uint8_t order[256], item_t *it) {
    int no = 0, n = 0;
    for (int l = 1; l <= 15; l++) {
        int pos = no;
        for (int s = 0; s < 256; s++) if (len[s] == l) order[no++] = (uint8_t)s;
        int left = no - pos;
        while (left > 0) {
            int d = 0;
            while ((2 << d) <= left) d++;          /* 2^d: largest power of two <= left */
            it[n].depth = l - d; it[n].d = d; it[n].first = pos; n++;
            pos += 1 << d;
            left -= 1 << d;
        }
    }
    /* (depth ascending, D descending); stable insertion sort */
    for (int i = 1; i < n; i++) {
        item_t x = it[i];
        int j = i - 1;
        while (j >= 0 && (it[j].depth > x.depth || (it[j].depth == x.depth && it[j].d < x.d))) {
            it[j + 1] = it[j];
            j--;
        }
        it[j + 1] = x;
    }
    return n;
}

/* Canonical codes of the items: the first is 0; the next is (previous + 1)
 * shifted left by the growth in depth. */
static void item_codes(const item_t *it, int n, uint32_t *code) {
    uint32_t c = 0;
    for (int i = 0; i < n; i++) {
        if (i) c = (c + 1) << (it[i].depth - it[i - 1].depth);
        code[i] = c;
    }
}

static int build_flat_tree(const uint8_t len[256], tree_t *t) {
    if (!complete_code(len)) return PVO_E_CORRUPT;
    memset(t, 0, sizeof(*t));
    item_t it[256];
    uint32_t icode[256];
    int n = flat_items(len, t->order, it);
    item_codes(it, n, icode);
    new_node(t, 0);
    for (int i = 0; i < n; i++) {
        const item_t *x = &it[i];
        if (icode[i] >> x->depth) return PVO_E_CORRUPT;     /* over-subscribed */
        int cur = 0;
        for (int k = 0; k < x->depth; k++) {
            int b = (icode[i] >> (x->depth - 1 - k)) & 1;
            if (t->nd[cur].leaf || t->nd[cur].flat) return PVO_E_CORRUPT;
            int c = t->nd[cur].child[b];
            if (c == -1) { c = new_node(t, k + 1); t->nd[cur].child[b] = c; }
            cur = c;
        }
        tnode *v = &t->nd[cur];
        if (v->leaf || v->flat || v->child[0] != -1 || v->child[1] != -1) return PVO_E_CORRUPT;
        if (x->d == 0) {
            v->leaf = 1;
            v->sym = t->order[x->first];
        } else if (x->d == 1) {
            for (int b = 0; b < 2; b++) {
                int c = new_node(t, x->depth + 1);
                t->nd[c].leaf = 1;
                t->nd[c].sym = t->order[x->first + b];
                t->nd[cur].child[b] = c;
            }
        } else {
            v->flat = x->d;
            v->g0 = x->first;
        }
        /* a symbol's code: the item's code, then its index in the group */
        for (int q = 0; q < (1 << x->d); q++)
            t->code[t->order[x->first + q]] = (uint16_t)((icode[i] << x->d) | (uint32_t)q);
    }
    return number_nodes(t);
}

/* ------------------------------------------------------------------ */
/* rANS (binary alphabet, 12-bit probabilities, 32 interleaved lanes)   */
/* ------------------------------------------------------------------ */
#define RANS_M 4096u
#define RANS_L 65536u

uint32_t pivco_ref_p1q(uint64_t n_v, uint64_t n_right) {
    if (n_v == 0) return 2048;
    uint64_t q = (n_right * 4096u + n_v / 2) / n_v;
    if (q < 1) q = 1;
    if (q > 4095) q = 4095;
    return (uint32_t)q;
}

int pivco_ref_select_ans(uint32_t mode, uint64_t n_v, uint64_t n_right) {
    if (n_v == 0) return 0;
    if (mode == 1) return (10 * n_right < n_v) || (10 * n_right > 9 * n_v);
    if (mode == 2) return 1;
    return 0;
}

int pivco_ref_rans_encode(const uint8_t *bits, uint64_t nbits, uint32_t p1q,
                          uint32_t chunk_log2, uint8_t *out, uint64_t cap,
                          uint64_t *out_len) {
    if (p1q < 1 || p1q > 4095 || chunk_log2 < 5 || chunk_log2 > 24) return PVO_E_ARG;
    uint64_t C = (uint64_t)1 << chunk_log2;
    uint32_t f[2] = {RANS_M - p1q, p1q};
    uint32_t c[2] = {0, RANS_M - p1q};
    uint16_t *stack = (uint16_t *)malloc(sizeof(uint16_t) * (C + 1));
    uint64_t o = 0;
    for (uint64_t start = 0; start < nbits; start += C) {
        uint64_t cl = nbits - start < C ? nbits - start : C;
        uint64_t K = (cl + 31) / 32;
        uint32_t x[32];
        for (int l = 0; l < 32; l++) x[l] = RANS_L;
        uint64_t nw = 0;
        for (uint64_t k = K; k-- > 0;) {
            for (int lane = 31; lane >= 0; lane--) {
                uint64_t j = 32 * k + (uint64_t)lane;
                if (j >= cl) continue;
                int b = getbit(bits, start + j);
                if (x[lane] >= (f[b] << 20)) { stack[nw++] = (uint16_t)(x[lane] & 0xFFFF); x[lane] >>= 16; }
                x[lane] = (x[lane] / f[b]) * RANS_M + (x[lane] % f[b]) + c[b];
            }
        }
        uint64_t need = 4 + 128 + 2 * nw;
        need = (need + 3) & ~(uint64_t)3;
        if (o + need > cap) { free(stack); return PVO_E_CAPACITY; }
        put32(out + o, (uint32_t)nw);
        for (int l = 0; l < 32; l++) put32(out + o + 4 + 4 * l, x[l]);
        for (uint64_t i = 0; i < nw; i++) put16(out + o + 132 + 2 * i, stack[nw - 1 - i]);
        for (uint64_t i = 132 + 2 * nw; i < need; i++) out[o + i] = 0;
        o += need;
    }
    free(stack);
    *out_len = o;
    return PVO_OK;
}

int pivco_ref_rans_decode(const uint8_t *body, uint64_t body_len, uint64_t nbits,
                          uint32_t p1q, uint32_t chunk_log2, uint8_t *bits_out) {
    if (p1q < 1 || p1q > 4095 || chunk_log2 < 5 || chunk_log2 > 24) return PVO_E_ARG;
    uint64_t C = (uint64_t)1 << chunk_log2;
    uint32_t f0 = RANS_M - p1q, f[2] = {RANS_M - p1q, p1q}, c[2] = {0, RANS_M - p1q};
    memset(bits_out, 0, (size_t)((nbits + 7) / 8));
    uint64_t o = 0;
    for (uint64_t start = 0; start < nbits; start += C) {
        uint64_t cl = nbits - start < C ? nbits - start : C;
        uint64_t K = (cl + 31) / 32;
        if (o + 132 > body_len) return PVO_E_CORRUPT;
        uint64_t nw = get32(body + o);
        uint64_t size = (132 + 2 * nw + 3) & ~(uint64_t)3;
        if (nw > C || o + size > body_len) return PVO_E_CORRUPT;
        uint32_t x[32];
        for (int l = 0; l < 32; l++) {
            x[l] = get32(body + o + 4 + 4 * l);
            if (x[l] < RANS_L) return PVO_E_CORRUPT;
        }
        const uint8_t *w = body + o + 132;
        uint64_t pos = 0;
        for (uint64_t k = 0; k < K; k++) {
            for (int lane = 0; lane < 32; lane++) {
                uint64_t j = 32 * k + (uint64_t)lane;
                if (j >= cl) continue;
                uint32_t slot = x[lane] & (RANS_M - 1);
                int b = slot >= f0;
                x[lane] = f[b] * (x[lane] >> 12) + slot - c[b];
                if (x[lane] < RANS_L) {
                    if (pos >= nw) return PVO_E_CORRUPT;
                    x[lane] = (x[lane] << 16) | get16(w + 2 * pos);
                    pos++;
                }
                if (b) setbit(bits_out, start + j);
            }
        }
        if (pos != nw) return PVO_E_CORRUPT;
        for (int l = 0; l < 32; l++)
            if (x[l] != RANS_L) return PVO_E_CORRUPT;
        for (uint64_t i = 132 + 2 * nw; i < size; i++)
            if (body[o + i]) return PVO_E_CORRUPT;
        o += size;
    }
    return o == body_len ? PVO_OK : PVO_E_CORRUPT;
}

/* ------------------------------------------------------------------ */
/* Encoder                                                              */
/* ------------------------------------------------------------------ */
#define HDR 48

uint64_t pivco_ref_encode_bound(uint64_t n, uint32_t block_size, uint32_t ans_mode) {
    if (block_size == 0) return 0;
    uint64_t nb = (n + block_size - 1) / block_size;
    uint64_t b = HDR + 16 * (nb + 1);
    /* per block: fixed header, length table, kind bits, counts, padding */
    b += nb * (12 + 128 + 32 + 4 * 255 + 8);
    /* bodies: every symbol contributes at most 15 bits; one byte of padding
     * per node; rANS adds per-chunk headers and up to 2 bytes per bit */
    if (ans_mode == 0) b += (15 * n) / 8 + nb * 255;
    else b += 2 * 15 * n + nb * 255 * (12 + 136) + 136 * ((15 * n) >> 16);
    return b;
}

/* Bits a node's raw body holds: one per passing symbol, D for a flat node. */
static uint64_t body_bits(const tnode *v) { return v->flat ? v->n * (uint64_t)v->flat : v->n; }

static int encode_block(const uint8_t *in, uint64_t n, uint32_t max_len, uint32_t ans_mode,
                        uint32_t chunk_log2, const uint8_t *tree_len, int flat, uint8_t *out,
                        uint64_t cap, uint64_t *out_len, uint64_t *ans_words) {
    uint64_t counts[256];
    memset(counts, 0, sizeof(counts));
    for (uint64_t i = 0; i < n; i++) counts[in[i]]++;
    int m = 0, last = 0;
    for (int s = 0; s < 256; s++) if (counts[s]) { m++; last = s; }
    *ans_words = 0;
    if (cap < 12) return PVO_E_CAPACITY;
    uint32_t cw = n <= 65535 ? 2 : 4;
    put32(out + 4, (uint32_t)n);
    out[10] = (uint8_t)cw; out[11] = 0;
    if (!tree_len && m == 1) {           /* constant block */
        put32(out, 12); out[8] = 1; out[9] = (uint8_t)last;
        *out_len = 12;
        return PVO_OK;
    }
    uint8_t len[256];
    if (tree_len) {
        memcpy(len, tree_len, 256);
        for (int s = 0; s < 256; s++)
            if (counts[s] && !len[s]) return PVO_E_ARG;
        for (int s = 0; s < 256; s++) if (len[s] > max_len) return PVO_E_ARG;
    } else {
        int r = pivco_ref_lengths(counts, max_len, len);
        if (r) return r;
    }
    tree_t *t = (tree_t *)malloc(sizeof(tree_t));
    if (flat ? build_flat_tree(len, t) : build_tree(len, t)) { free(t); return PVO_E_ARG; }
    const uint16_t *code = t->code;
    /* n_v and n_right from the symbol counts: a symbol passes every node on
     * its path; below a flat node there are no more nodes */
    for (int s = 0; s < 256; s++) {
        if (!len[s] || !counts[s]) continue;
        int cur = 0;
        for (int d = 0; !t->nd[cur].leaf; d++) {
            t->nd[cur].n += counts[s];
            if (t->nd[cur].flat) break;
            int b = (code[s] >> (len[s] - 1 - d)) & 1;
            if (b) t->nd[cur].n_right += counts[s];
            cur = t->nd[cur].child[b];
        }
    }
    int I = t->ni;
    uint8_t *bm[255];
    uint64_t cur_pos[255];
    for (int i = 0; i < I; i++) {
        bm[i] = (uint8_t *)calloc((size_t)((body_bits(&t->nd[t->bfs[i]]) + 7) / 8 + 1), 1);
        cur_pos[i] = 0;
    }
    /* bitmaps: each symbol appends one bit to every binary node on its path
     * (the branch it takes) and, at a flat node of depth D, the D bits of its
     * index in the node's group (the packN step of Table 11) */
    for (uint64_t i = 0; i < n; i++) {
        int s = in[i], cur = 0;
        for (int d = 0; !t->nd[cur].leaf; d++) {
            const tnode *v = &t->nd[cur];
            int id = v->id;
            if (v->flat) {
                uint32_t q = code[s] & ((1u << v->flat) - 1);
                for (int k = 0; k < v->flat; k++)
                    if ((q >> k) & 1) setbit(bm[id], cur_pos[id] * (uint64_t)v->flat + (uint64_t)k);
                cur_pos[id]++;
                break;
            }
            int b = (code[s] >> (len[s] - 1 - d)) & 1;
            if (b) setbit(bm[id], cur_pos[id]);
            cur_pos[id]++;
            cur = v->child[b];
        }
    }
    int rc = PVO_OK;
    uint64_t o = 12;
    out[8] = 0; out[9] = 0;
    if (o + 128 > cap) { rc = PVO_E_CAPACITY; goto done; }
    for (int j = 0; j < 128; j++) out[o + j] = (uint8_t)(len[2 * j] | (len[2 * j + 1] << 4));
    o += 128;
    uint8_t kind[255];
    uint32_t marker[255];
    for (int i = 0; i < I; i++) {
        tnode *v = &t->nd[t->bfs[i]];
        marker[i] = 0;
        if (v->flat) kind[i] = 0;
        else if (ans_mode == 3) kind[i] = (uint8_t)pivco_ref_fse_select(v->n, v->n_right, (uint32_t)v->depth, &marker[i]);
        else kind[i] = (uint8_t)pivco_ref_select_ans(ans_mode, v->n, v->n_right);
    }
    uint64_t kb = ((uint64_t)I + 7) / 8;
    if (o + kb + (uint64_t)cw * I > cap) { rc = PVO_E_CAPACITY; goto done; }
    memset(out + o, 0, (size_t)kb);
    for (int i = 0; i < I; i++) if (kind[i]) out[o + i / 8] |= (uint8_t)(1u << (i % 8));
    o += kb;
    for (int i = 0; i < I; i++) {
        uint64_t r = t->nd[t->bfs[i]].n_right;
        if (cw == 2) put16(out + o, (uint32_t)r); else put32(out + o, (uint32_t)r);
        o += cw;
    }
    for (int i = 0; i < I; i++) {
        if (kind[i]) continue;
        uint64_t nb = (body_bits(&t->nd[t->bfs[i]]) + 7) / 8;
        if (o + nb > cap) { rc = PVO_E_CAPACITY; goto done; }
        memcpy(out + o, bm[i], (size_t)nb);
        o += nb;
    }
    for (int i = 0; i < I; i++) {
        if (!kind[i]) continue;
        tnode *v = &t->nd[t->bfs[i]];
        while (o & 3) { if (o >= cap) { rc = PVO_E_CAPACITY; goto done; } out[o++] = 0; }
        if (o + 8 > cap) { rc = PVO_E_CAPACITY; goto done; }
        uint64_t blen;
        if (ans_mode == 3) {
            rc = pivco_ref_fse_encode(bm[i], v->n, marker[i], chunk_log2, out + o + 8, cap - o - 8, &blen);
            if (rc) goto done;
            out[o] = (uint8_t)marker[i]; out[o + 1] = 0; put16(out + o + 2, 0);
        } else {
            uint32_t p1q = pivco_ref_p1q(v->n, v->n_right);
            rc = pivco_ref_rans_encode(bm[i], v->n, p1q, chunk_log2, out + o + 8, cap - o - 8, &blen);
            if (rc) goto done;
            put16(out + o, p1q); put16(out + o + 2, 0);
        }
        put32(out + o + 4, (uint32_t)blen);
        o += 8 + blen;
        *ans_words += (v->n + 31) / 32;
    }
    put32(out, (uint32_t)o);
    *out_len = o;
done:
    for (int i = 0; i < I; i++) free(bm[i]);
    free(t);
    return rc;
}

static int encode_stream(const uint8_t *in, uint64_t n, uint32_t block_size,
                         uint32_t max_len, uint32_t ans_mode, uint32_t chunk_log2,
                         const uint8_t *tree_len, int flat, uint8_t *out, uint64_t cap,
                         uint64_t *out_len) {
    if ((!in && n) || !out || !out_len || block_size == 0 || max_len < 1 || max_len > 15 ||
        ans_mode > 3 || chunk_log2 < 5 || chunk_log2 > 24 || (ans_mode == 3 && chunk_log2 < 8))
        return PVO_E_ARG;
    uint64_t nb64 = (n + block_size - 1) / block_size;
    if (nb64 > 0xFFFFFFFFull) return PVO_E_ARG;
    uint32_t nb = (uint32_t)nb64;
    uint64_t o = HDR + 16 * ((uint64_t)nb + 1);
    if (o > cap) return PVO_E_CAPACITY;
    memset(out, 0, (size_t)o);
    put32(out, 0x31435650u);  /* "PVC1" */
    put16(out + 4, flat ? 2 : 1); put16(out + 6, ans_mode == 3 ? 1 : 0);
    put64(out + 8, n);
    put32(out + 16, block_size); put32(out + 20, nb);
    out[24] = (uint8_t)max_len; out[25] = (uint8_t)chunk_log2;
    uint64_t ans_total = 0;
    for (uint32_t b = 0; b < nb; b++) {
        uint64_t start = (uint64_t)b * block_size;
        uint64_t bn = n - start < block_size ? n - start : block_size;
        put64(out + HDR + 8 * (uint64_t)b, o);
        put64(out + HDR + 8 * ((uint64_t)nb + 1) + 8 * (uint64_t)b, ans_total);
        uint64_t bl, aw;
        int rc = encode_block(in + start, bn, max_len, ans_mode, chunk_log2, tree_len, flat,
                              out + o, cap - o, &bl, &aw);
        if (rc) return rc;
        o += bl;
        while (o & 3) { if (o >= cap) return PVO_E_CAPACITY; out[o++] = 0; }
        ans_total += aw;
    }
    put64(out + HDR + 8 * (uint64_t)nb, o);
    put64(out + HDR + 8 * ((uint64_t)nb + 1) + 8 * (uint64_t)nb, ans_total);
    put64(out + 32, ans_total);
    *out_len = o;
    return PVO_OK;
}

int pivco_ref_encode(const uint8_t *in, uint64_t n, uint32_t block_size,
                     uint32_t max_len, uint32_t ans_mode, uint32_t chunk_log2,
                     const uint8_t *tree_len, uint8_t *out, uint64_t cap,
                     uint64_t *out_len) {
    return encode_stream(in, n, block_size, max_len, ans_mode, chunk_log2, tree_len, 0, out,
                         cap, out_len);
}

int pivco_ref_encode_flat(const uint8_t *in, uint64_t n, uint32_t block_size,
                          uint32_t max_len, uint32_t ans_mode, uint32_t chunk_log2,
                          const uint8_t *tree_len, uint8_t *out, uint64_t cap,
                          uint64_t *out_len) {
    return encode_stream(in, n, block_size, max_len, ans_mode, chunk_log2, tree_len, 1, out,
                         cap, out_len);
}

/* ------------------------------------------------------------------ */
/* Stream parsing and validation (shared by both decoders)             */
/* ------------------------------------------------------------------ */
int pivco_ref_stream_info(const uint8_t *in, uint64_t in_len, uint64_t *n_total,
                          uint32_t *n_blocks, uint32_t *block_size, uint64_t *ans_words) {
    if (!in || in_len < HDR) return PVO_E_CORRUPT;
    if (get32(in) != 0x31435650u) return PVO_E_CORRUPT;
    if (n_total) *n_total = get64(in + 8);
    if (block_size) *block_size = get32(in + 16);
    if (n_blocks) *n_blocks = get32(in + 20);
    if (ans_words) *ans_words = get64(in + 32);
    return PVO_OK;
}

typedef struct {
    uint32_t mode, cw, I;
    uint32_t version;    /* 1: canonical tree, 2: flat-subtree tree */
    uint8_t const_sym;
    uint8_t len[256];
    tree_t *t;
    uint8_t kind[255];
    uint8_t *bm[255];    /* raw bitmap of every internal node (decoded) */
    uint64_t n;
} block_t;

static void free_block(block_t *bk) {
    if (bk->t) {
        for (uint32_t i = 0; i < bk->I; i++) free(bk->bm[i]);
        free(bk->t);
        bk->t = NULL;
    }
}

/* Parse and fully validate block b; all node bitmaps decoded into bk->bm. */
static int parse_block(const uint8_t *in, uint64_t in_len, uint32_t b, block_t *bk) {
    memset(bk, 0, sizeof(*bk));
    uint32_t version = in_len >= HDR ? get16(in + 4) : 0;
    uint32_t flags = in_len >= HDR ? get16(in + 6) : 0;
    if (in_len < HDR || get32(in) != 0x31435650u || (version != 1 && version != 2) || flags > 1)
        return PVO_E_CORRUPT;
    bk->version = version;
    uint64_t n_total = get64(in + 8);
    uint32_t bs = get32(in + 16), nb = get32(in + 20), max_len = in[24], cl2 = in[25];
    if (bs == 0 || max_len < 1 || max_len > 15 || cl2 < 5 || cl2 > 24 || (flags && cl2 < 8)) return PVO_E_CORRUPT;
    if ((n_total + bs - 1) / bs != nb || b >= nb) return PVO_E_CORRUPT;
    uint64_t tab = HDR + 16 * ((uint64_t)nb + 1);
    if (tab > in_len) return PVO_E_CORRUPT;
    uint64_t off = get64(in + HDR + 8 * (uint64_t)b), end = get64(in + HDR + 8 * ((uint64_t)b + 1));
    uint64_t a0 = get64(in + HDR + 8 * ((uint64_t)nb + 1) + 8 * (uint64_t)b);
    uint64_t a1 = get64(in + HDR + 8 * ((uint64_t)nb + 1) + 8 * ((uint64_t)b + 1));
    if (off < tab || end < off || end > in_len || (off & 3) || end - off < 12 || a1 < a0)
        return PVO_E_CORRUPT;
    const uint8_t *p = in + off;
    uint64_t comp = get32(p);
    if (comp > end - off || comp < 12) return PVO_E_CORRUPT;
    uint64_t n = get32(p + 4);
    uint64_t want = n_total - (uint64_t)b * bs < bs ? n_total - (uint64_t)b * bs : bs;
    if (n != want) return PVO_E_CORRUPT;
    bk->n = n;
    bk->mode = p[8]; bk->const_sym = p[9]; bk->cw = p[10];
    if (p[11] != 0 || bk->cw != (n <= 65535 ? 2u : 4u)) return PVO_E_CORRUPT;
    if (bk->mode == 1) return (comp == 12 && a1 == a0 && n > 0) ? PVO_OK : PVO_E_CORRUPT;
    if (bk->mode != 0 || bk->const_sym != 0) return PVO_E_CORRUPT;
    if (comp < 12 + 128) return PVO_E_CORRUPT;
    for (int j = 0; j < 128; j++) { bk->len[2 * j] = p[12 + j] & 15; bk->len[2 * j + 1] = p[12 + j] >> 4; }
    for (int s = 0; s < 256; s++) if (bk->len[s] > max_len) return PVO_E_CORRUPT;
    bk->t = (tree_t *)malloc(sizeof(tree_t));
    if (version == 2 ? build_flat_tree(bk->len, bk->t) : build_tree(bk->len, bk->t)) {
        free(bk->t); bk->t = NULL; return PVO_E_CORRUPT;
    }
    tree_t *t = bk->t;
    uint32_t I = (uint32_t)t->ni;
    uint64_t o = 140, kb = (I + 7) / 8;
    if (o + kb + (uint64_t)bk->cw * I > comp) { free(t); bk->t = NULL; return PVO_E_CORRUPT; }
    for (uint32_t i = 0; i < I; i++) {
        bk->kind[i] = (p[o + i / 8] >> (i % 8)) & 1;
        if (bk->kind[i] && t->nd[t->bfs[i]].flat) { free(t); bk->t = NULL; return PVO_E_CORRUPT; }
    }
    for (uint32_t i = I; i < kb * 8; i++)
        if ((p[o + i / 8] >> (i % 8)) & 1) { free(t); bk->t = NULL; return PVO_E_CORRUPT; }
    o += kb;
    /* node sizes top-down: root sees n symbols; left child n_v - n_right */
    t->nd[0].n = n;
    for (uint32_t i = 0; i < I; i++) {
        tnode *v = &t->nd[t->bfs[i]];
        v->n_right = bk->cw == 2 ? get16(p + o) : get32(p + o);
        o += bk->cw;
        if (v->n_right > v->n || (v->flat && v->n_right)) { free(t); bk->t = NULL; return PVO_E_CORRUPT; }
        if (v->flat) continue;                 /* its leaves need no sizes */
        t->nd[v->child[0]].n = v->n - v->n_right;
        t->nd[v->child[1]].n = v->n_right;
    }
    bk->I = I;
    for (uint32_t i = 0; i < I; i++) bk->bm[i] = NULL;
    int rc = PVO_OK;
    uint64_t aw = 0;
    for (uint32_t i = 0; i < I; i++) {
        tnode *v = &t->nd[t->bfs[i]];
        uint64_t nbits = body_bits(v);
        bk->bm[i] = (uint8_t *)calloc((size_t)((nbits + 7) / 8 + 1), 1);
        if (bk->kind[i]) continue;
        uint64_t nbytes = (nbits + 7) / 8;
        if (o + nbytes > comp) { rc = PVO_E_CORRUPT; goto fail; }
        memcpy(bk->bm[i], p + o, (size_t)nbytes);
        if ((nbits & 7) && (p[o + nbytes - 1] >> (nbits & 7))) { rc = PVO_E_CORRUPT; goto fail; }
        o += nbytes;
    }
    for (uint32_t i = 0; i < I; i++) {
        if (!bk->kind[i]) continue;
        tnode *v = &t->nd[t->bfs[i]];
        while (o & 3) { if (o >= comp || p[o]) { rc = PVO_E_CORRUPT; goto fail; } o++; }
        if (o + 8 > comp || v->n == 0) { rc = PVO_E_CORRUPT; goto fail; }
        uint32_t blen = get32(p + o + 4);
        if (get16(p + o + 2) != 0 || o + 8 + blen > comp) { rc = PVO_E_CORRUPT; goto fail; }
        if (flags) {
            if (p[o + 1] != 0 || pivco_ref_fse_decode(p + o + 8, blen, v->n, p[o], cl2, bk->bm[i])) {
                rc = PVO_E_CORRUPT; goto fail;
            }
        } else {
            uint32_t p1q = get16(p + o);
            if (pivco_ref_rans_decode(p + o + 8, blen, v->n, p1q, cl2, bk->bm[i])) { rc = PVO_E_CORRUPT; goto fail; }
        }
        o += 8 + blen;
        aw += (v->n + 31) / 32;
    }
    if (o != comp || aw != a1 - a0) { rc = PVO_E_CORRUPT; goto fail; }
    /* every binary node's bitmap must hold exactly n_right ones (any D-bit
     * value of a flat node names a symbol of its group) */
    for (uint32_t i = 0; i < I; i++) {
        tnode *v = &t->nd[t->bfs[i]];
        if (v->flat) continue;
        uint64_t ones = 0;
        for (uint64_t j = 0; j < v->n; j++) ones += (uint64_t)getbit(bk->bm[i], j);
        if (ones != v->n_right) { rc = PVO_E_CORRUPT; goto fail; }
    }
    return PVO_OK;
fail:
    free_block(bk);
    return rc;
}

static int check_stream(const uint8_t *in, uint64_t in_len, uint64_t *n_total, uint32_t *nb,
                        uint32_t *bs) {
    if (!in || in_len < HDR || get32(in) != 0x31435650u || (get16(in + 4) != 1 && get16(in + 4) != 2) ||
        get16(in + 6) > 1)
        return PVO_E_CORRUPT;
    *n_total = get64(in + 8); *bs = get32(in + 16); *nb = get32(in + 20);
    if (*bs == 0 || (*n_total + *bs - 1) / *bs != *nb) return PVO_E_CORRUPT;
    uint64_t tab = HDR + 16 * ((uint64_t)*nb + 1);
    if (tab > in_len) return PVO_E_CORRUPT;
    if (get64(in + HDR + 8 * (uint64_t)*nb) > in_len) return PVO_E_CORRUPT;
    if (get64(in + HDR + 8 * ((uint64_t)*nb + 1)) != 0) return PVO_E_CORRUPT;
    if (get64(in + HDR + 8 * ((uint64_t)*nb + 1) + 8 * (uint64_t)*nb) != get64(in + 32)) return PVO_E_CORRUPT;
    return PVO_OK;
}

/* Decoder A, from the definition of the pivoted layout (Sec. 2): the symbol at
 * position i of a block is the one whose code is the sequence of bits that
 * position left in the internal nodes on its path, and every internal node
 * keeps its bits in stream order.  So the code of position i is read one bit
 * at a time -- the next unread bit (a read count per node) of the internal
 * node named by the code prefix read so far -- until the prefix equals a
 * codeword of its length (the canonical codes of Sec. 1.1).  Internal nodes
 * are numbered breadth-first: by depth, then by prefix value. */
typedef struct {
    uint16_t pfx[16][256];     /* internal-node prefixes at depth d, ascending */
    int npfx[16], first[16];   /* their number; number of internal nodes above d */
    uint16_t cw[16][256];      /* codewords of length d, ascending */
    uint8_t cwsym[16][256];    /* their symbols */
    int ncw[16];
} codebook_t;

/* index of v in the ascending array a[0..n), or -1 */
static int find16(const uint16_t *a, int n, uint32_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo] == v) ? lo : -1;
}

/* insert v into the ascending array a[0..*n) unless present; returns its index */
static int insert16(uint16_t *a, int *n, uint32_t v) {
    int k = find16(a, *n, v);
    if (k >= 0) return k;
    int j = *n;
    while (j > 0 && a[j - 1] > v) { a[j] = a[j - 1]; j--; }
    a[j] = (uint16_t)v;
    (*n)++;
    return j;
}

static void build_codebook(const uint8_t len[256], codebook_t *cb) {
    uint16_t code[256];
    pivco_ref_codes(len, code);
    memset(cb, 0, sizeof(*cb));
    for (int s = 0; s < 256; s++) {
        int l = len[s];
        if (!l) continue;
        for (int d = 0; d < l; d++) insert16(cb->pfx[d], &cb->npfx[d], (uint32_t)code[s] >> (l - d));
        int k = insert16(cb->cw[l], &cb->ncw[l], code[s]);
        for (int j = cb->ncw[l] - 1; j > k; j--) cb->cwsym[l][j] = cb->cwsym[l][j - 1];
        cb->cwsym[l][k] = (uint8_t)s;
    }
    for (int d = 1; d < 16; d++) cb->first[d] = cb->first[d - 1] + cb->npfx[d - 1];
}

static void walk_block(const block_t *bk, uint8_t *out) {
    if (bk->mode == 1) { memset(out, bk->const_sym, (size_t)bk->n); return; }
    codebook_t *cb = (codebook_t *)malloc(sizeof(codebook_t));
    build_codebook(bk->len, cb);
    uint64_t cur[255];
    memset(cur, 0, sizeof(cur));
    for (uint64_t i = 0; i < bk->n; i++) {
        uint32_t v = 0;                 /* code prefix read so far */
        int d = 0;                      /* its length */
        int sym = -1;
        while (sym < 0 && d < 15) {
            int id = cb->first[d] + find16(cb->pfx[d], cb->npfx[d], v);
            v = 2 * v + (uint32_t)getbit(bk->bm[id], cur[id]++);
            d++;
            int k = find16(cb->cw[d], cb->ncw[d], v);
            if (k >= 0) sym = cb->cwsym[d][k];
        }
        out[i] = (uint8_t)sym;         /* the block was validated: a codeword is always reached */
    }
    free(cb);
}

/* Decoder A for a v2 block: the same reading with the items of Sec. 2.2.4
 * (build_flat_tree) in place of the symbols.  The code of position i is read
 * bit by bit from the binary nodes named by the prefix read so far until the
 * prefix is an item's code; an item with D >= 1 is itself a node, whose next
 * D-bit value is the index of the symbol in its group (D = 1: one bit). */
typedef struct {
    uint16_t pfx[16][256];     /* node prefixes at depth d (binary and group nodes), ascending */
    int npfx[16], first[16];   /* their number; number of nodes above d */
    uint16_t ic[16][256];      /* item codes of depth d, ascending */
    item_t item[16][256];      /* their items */
    int nic[16];
} itembook_t;

static void build_itembook(const uint8_t len[256], uint8_t order[256], itembook_t *ib) {
    item_t it[256];
    uint32_t code[256];
    int n = flat_items(len, order, it);
    item_codes(it, n, code);
    memset(ib, 0, sizeof(*ib));
    for (int i = 0; i < n; i++) {
        int m = it[i].depth;
        for (int d = 0; d < m; d++) insert16(ib->pfx[d], &ib->npfx[d], code[i] >> (m - d));
        if (it[i].d >= 1) insert16(ib->pfx[m], &ib->npfx[m], code[i]);
        int k = insert16(ib->ic[m], &ib->nic[m], code[i]);
        for (int j = ib->nic[m] - 1; j > k; j--) ib->item[m][j] = ib->item[m][j - 1];
        ib->item[m][k] = it[i];
    }
    for (int d = 1; d < 16; d++) ib->first[d] = ib->first[d - 1] + ib->npfx[d - 1];
}

static void walk_flat_block(const block_t *bk, uint8_t *out) {
    itembook_t *ib = (itembook_t *)malloc(sizeof(itembook_t));
    uint8_t order[256];
    build_itembook(bk->len, order, ib);
    uint64_t cur[255];
    memset(cur, 0, sizeof(cur));
    for (uint64_t i = 0; i < bk->n; i++) {
        uint32_t v = 0;                 /* item-code prefix read so far */
        int d = 0;                      /* its length */
        for (;;) {
            int k = find16(ib->ic[d], ib->nic[d], v);
            if (k >= 0) {
                const item_t *x = &ib->item[d][k];
                uint32_t q = 0;
                if (x->d) {
                    int id = ib->first[d] + find16(ib->pfx[d], ib->npfx[d], v);
                    for (int b = 0; b < x->d; b++)
                        q |= (uint32_t)getbit(bk->bm[id], cur[id] * (uint64_t)x->d + (uint64_t)b) << b;
                    cur[id]++;
                }
                out[i] = order[x->first + (int)q];
                break;
            }
            int id = ib->first[d] + find16(ib->pfx[d], ib->npfx[d], v);
            v = 2 * v + (uint32_t)getbit(bk->bm[id], cur[id]++);
            d++;                        /* the block was validated: an item is always reached */
        }
    }
    free(ib);
}

/* Decoder B, the bottom-up merge of Sec. 3: every internal node v, deepest
 * first, forms the symbol sequence of its subtree; output j of v comes from
 * the child its bitmap bit selects (0 left, 1 right), at the position given
 * by the count of equal bits before j (a leaf child's sequence is its symbol
 * repeated). */
static void merge_block(const block_t *bk, uint8_t *out) {
    if (bk->mode == 1) { memset(out, bk->const_sym, (size_t)bk->n); return; }
    const tree_t *t = bk->t;
    uint8_t *seq[255];
    for (int i = (int)bk->I - 1; i >= 0; i--) {
        const tnode *v = &t->nd[t->bfs[i]];
        uint8_t *o = (i == 0) ? out : (uint8_t *)malloc((size_t)v->n + 1);
        if (v->flat) {
            /* merge_flat_D (Sec. 3.2): output j is the group's symbol named by
             * the node's j-th D-bit value */
            for (uint64_t j = 0; j < v->n; j++) {
                uint32_t q = 0;
                for (int b = 0; b < v->flat; b++)
                    q |= (uint32_t)getbit(bk->bm[i], j * (uint64_t)v->flat + (uint64_t)b) << b;
                o[j] = t->order[v->g0 + (int)q];
            }
            seq[i] = o;
            continue;
        }
        const tnode *kid[2] = {&t->nd[v->child[0]], &t->nd[v->child[1]]};
        /* ones[j] = 1 bits of the node's bitmap before position j */
        uint64_t *ones = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)v->n + 1));
        ones[0] = 0;
        for (uint64_t j = 0; j < v->n; j++) ones[j + 1] = ones[j] + (uint64_t)getbit(bk->bm[i], j);
        for (uint64_t j = 0; j < v->n; j++) {
            int b = getbit(bk->bm[i], j);
            uint64_t rank = b ? ones[j] : j - ones[j];
            const tnode *c = kid[b];
            o[j] = c->leaf ? (uint8_t)c->sym : seq[c->id][rank];
        }
        free(ones);
        seq[i] = o;
        for (int b = 0; b < 2; b++)
            if (!kid[b]->leaf) free(seq[kid[b]->id]);
    }
}

static int decode_range(const uint8_t *in, uint64_t in_len, uint32_t b0, uint32_t b1,
                        uint8_t *out, uint64_t cap, uint64_t *n_out, int merge) {
    uint64_t n_total; uint32_t nb, bs;
    int rc = check_stream(in, in_len, &n_total, &nb, &bs);
    if (rc) return rc;
    if (b1 > nb) b1 = nb;
    if (b0 > b1) return PVO_E_ARG;
    uint64_t o = 0;
    for (uint32_t b = b0; b < b1; b++) {
        block_t bk;
        rc = parse_block(in, in_len, b, &bk);
        if (rc) return rc;
        if (o + bk.n > cap) { free_block(&bk); return PVO_E_CAPACITY; }
        if (merge) merge_block(&bk, out + o);
        else if (bk.version == 2 && bk.mode == 0) walk_flat_block(&bk, out + o);
        else walk_block(&bk, out + o);
        o += bk.n;
        free_block(&bk);
    }
    if (n_out) *n_out = o;
    return PVO_OK;
}

int pivco_ref_decode(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                     uint64_t *n_out) {
    return decode_range(in, in_len, 0, 0xFFFFFFFFu, out, cap, n_out, 0);
}

int pivco_ref_decode_merge(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                           uint64_t *n_out) {
    return decode_range(in, in_len, 0, 0xFFFFFFFFu, out, cap, n_out, 1);
}

int pivco_ref_decode_blocks(const uint8_t *in, uint64_t in_len, uint32_t b0, uint32_t b1,
                            uint8_t *out, uint64_t cap, uint64_t *n_out) {
    return decode_range(in, in_len, b0, b1, out, cap, n_out, 0);
}

int pivco_ref_block_info(const uint8_t *in, uint64_t in_len, uint32_t block, uint8_t len[256],
                         uint32_t *mode, uint32_t *n_internal, uint8_t depth[255],
                         uint64_t n_v[255], uint64_t n_right[255], uint8_t kind[255],
                         uint8_t flat[255]) {
    uint64_t n_total; uint32_t nb, bs;
    int rc = check_stream(in, in_len, &n_total, &nb, &bs);
    if (rc) return rc;
    block_t bk;
    rc = parse_block(in, in_len, block, &bk);
    if (rc) return rc;
    *mode = bk.mode;
    *n_internal = bk.mode == 0 ? bk.I : 0;
    memcpy(len, bk.len, 256);
    for (uint32_t i = 0; i < *n_internal; i++) {
        const tnode *v = &bk.t->nd[bk.t->bfs[i]];
        depth[i] = (uint8_t)v->depth; n_v[i] = v->n; n_right[i] = v->n_right; kind[i] = bk.kind[i];
        if (flat) flat[i] = (uint8_t)v->flat;
    }
    free_block(&bk);
    return PVO_OK;
}

/* ------------------------------------------------------------------ */
/* Classical (code-after-code) streams, for the cross-checks            */
/* ------------------------------------------------------------------ */
int pivco_ref_classical_encode(const uint8_t *in, uint64_t n, const uint8_t len[256],
                               uint8_t *out, uint64_t cap, uint64_t *nbits) {
    uint16_t code[256];
    if (pivco_ref_codes(len, code)) return PVO_E_ARG;
    uint64_t nb = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (!len[in[i]]) return PVO_E_ARG;
        nb += len[in[i]];
    }
    if ((nb + 7) / 8 > cap) return PVO_E_CAPACITY;
    memset(out, 0, (size_t)((nb + 7) / 8));
    uint64_t p = 0;
    for (uint64_t i = 0; i < n; i++) {
        int s = in[i];
        for (int d = 0; d < len[s]; d++, p++)
            if ((code[s] >> (len[s] - 1 - d)) & 1) out[p >> 3] |= (uint8_t)(0x80u >> (p & 7));
    }
    *nbits = nb;
    return PVO_OK;
}

int pivco_ref_classical_decode(const uint8_t *bits, uint64_t nbits, const uint8_t len[256],
                               uint8_t *out, uint64_t n) {
    tree_t *t = (tree_t *)malloc(sizeof(tree_t));
    if (build_tree(len, t)) { free(t); return PVO_E_ARG; }
    uint64_t p = 0;
    for (uint64_t i = 0; i < n; i++) {
        int node = 0;
        while (!t->nd[node].leaf) {                 /* one tree edge per bit */
            if (p >= nbits) { free(t); return PVO_E_CORRUPT; }
            int bit = (bits[p >> 3] >> (7 - (p & 7))) & 1;
            p++;
            node = bit ? t->nd[node].child[1] : t->nd[node].child[0];
        }
        out[i] = (uint8_t)t->nd[node].sym;
    }
    free(t);
    return p == nbits ? PVO_OK : PVO_E_CORRUPT;
}

int pivco_ref_pivoted_to_classical(const uint8_t *in, uint64_t in_len, uint8_t *out,
                                   uint64_t cap, uint64_t *nbits) {
    uint64_t n_total; uint32_t nb, bs;
    int rc = check_stream(in, in_len, &n_total, &nb, &bs);
    if (rc) return rc;
    if (nb < 1) return PVO_E_ARG;
    block_t bk;
    rc = parse_block(in, in_len, 0, &bk);
    if (rc) return rc;
    if (bk.mode != 0 || bk.version != 1) { free_block(&bk); return PVO_E_UNSUPPORTED; }
    const tree_t *t = bk.t;
    uint64_t cur[255], p = 0;
    memset(cur, 0, sizeof(cur));
    memset(out, 0, (size_t)cap);
    for (uint64_t i = 0; i < bk.n; i++) {
        int node = 0;
        while (!t->nd[node].leaf) {
            int id = t->nd[node].id;
            int bit = getbit(bk.bm[id], cur[id]++);
            if ((p >> 3) >= cap) { free_block(&bk); return PVO_E_CAPACITY; }
            if (bit) out[p >> 3] |= (uint8_t)(0x80u >> (p & 7));
            p++;
            node = t->nd[node].child[bit];
        }
    }
    *nbits = p;
    free_block(&bk);
    return PVO_OK;
}
