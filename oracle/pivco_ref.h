/*
 * pivco_ref.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, scalar CPU reference ("oracle") for the PivCo-Huffman codec.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the GPU library and the GPU library
 * never calls it.
 *
 * Every function follows a passage of the paper (Zukowski, "PivCo-Huffman",
 * v1.0, 2026):
 *   - Sec. 1.1 (canonical codes)   codes read bit by bit; a bit-by-bit tree
 *                                  walk (the decoding Listing 1 shows) is the
 *                                  classical-stream cross-check
 *   - Sec. 2 / Fig. 2-3            one bitmap per internal node ("pivoting")
 *   - Sec. 3 / naive merge loop    bottom-up merge decoder
 *   - Sec. 2.2.3-2.2.4, 3.2        flat subtrees and the non-canonical
 *                                  regrouping (v2 streams, merge_flat_D)
 *   - Sec. 4 / Table 11            encoder = build node bitmaps top-down
 *   - App. D                       128-byte 4-bit code-length table, blocks,
 *                                  per-node records in traversal order
 *   - Sec. 5 + ref. [4] (Duda)     selective entropy coding of skewed nodes;
 *                                  here binary rANS with 32 interleaved lanes
 * The wire format is the repository's v1 format (magic "PVC1"); its layout
 * is documented at pivco_ref_encode below.
 *
 * All arithmetic is integer.  All pointers are host pointers.  Functions
 * return 0 on success or a negative PVO_E_* code.
 */
#ifndef PIVCO_REF_H
#define PIVCO_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PVO_OK            0
#define PVO_E_ARG        -1
#define PVO_E_CAPACITY   -2
#define PVO_E_CORRUPT    -3
#define PVO_E_UNSUPPORTED -4

/* Length-limited optimal code lengths (package-merge, Larmore-Hirschberg),
 * then a deterministic assignment: the ascending multiset of lengths goes to
 * symbols ordered by (count desc, symbol asc).  0 = symbol absent.
 * Needs at least 2 symbols with nonzero count and 2^max_len >= that number;
 * max_len in [1, 15]. */
int pivco_ref_lengths(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]);

/* Canonical codes (Schwartz-Kallick, ref. [5] of the paper): symbols ordered
 * by (len asc, symbol asc); first code 0; next = (prev + 1) << (len - prevlen). */
int pivco_ref_codes(const uint8_t len[256], uint16_t code[256]);

/* rANS probability of a 1 bit, 12-bit fixed point, from exact node counts. */
uint32_t pivco_ref_p1q(uint64_t n_v, uint64_t n_right);

/* Selection rule for entropy-coding a node: one-bit fraction < 0.1 or > 0.9,
 * in integer form.  mode 0 = never, 1 = that rule, 2 = every internal node. */
int pivco_ref_select_ans(uint32_t mode, uint64_t n_v, uint64_t n_right);

/* Binary rANS over a bit sequence (bits LSB-first in bytes).  Chunks of
 * 2^chunk_log2 bits; 32 interleaved lanes (bit j of a chunk -> lane j%32,
 * step j/32); state in [2^16, 2^32); 16-bit renormalisation words.
 * Body layout per chunk: n_words u32 | state u32[32] | u16 words[n_words] |
 * zero pad to 4 bytes.  Returns body length in *out_len. */
int pivco_ref_rans_encode(const uint8_t *bits, uint64_t nbits, uint32_t p1q,
                          uint32_t chunk_log2, uint8_t *out, uint64_t cap,
                          uint64_t *out_len);
int pivco_ref_rans_decode(const uint8_t *body, uint64_t body_len, uint64_t nbits,
                          uint32_t p1q, uint32_t chunk_log2, uint8_t *bits_out);

/* Upper bound on the encoded stream size. */
uint64_t pivco_ref_encode_bound(uint64_t n, uint32_t block_size, uint32_t ans_mode);

/* Encode n bytes into a v1 stream.  tree_len: optional 256 code lengths to
 * use for every block (NULL = one optimal tree per block). */
int pivco_ref_encode(const uint8_t *in, uint64_t n, uint32_t block_size,
                     uint32_t max_len, uint32_t ans_mode, uint32_t chunk_log2,
                     const uint8_t *tree_len, uint8_t *out, uint64_t cap,
                     uint64_t *out_len);

/* The same, writing a v2 stream: every coded block uses the flat-subtree
 * tree that Sec. 2.2.3-2.2.4 derive from its code lengths (the symbols of
 * each length cut into power-of-two groups, largest first; a group of 2^D
 * >= 4 symbols is one flat node holding a D-bit index per passing symbol).
 * Both decoders read v1 and v2 streams; on v2, decoder B merges flat nodes
 * with merge_flat_D (Sec. 3.2). */
int pivco_ref_encode_flat(const uint8_t *in, uint64_t n, uint32_t block_size,
                          uint32_t max_len, uint32_t ans_mode, uint32_t chunk_log2,
                          const uint8_t *tree_len, uint8_t *out, uint64_t cap,
                          uint64_t *out_len);

/* Stream header fields (no validation beyond the magic). */
int pivco_ref_stream_info(const uint8_t *in, uint64_t in_len, uint64_t *n_total,
                          uint32_t *n_blocks, uint32_t *block_size,
                          uint64_t *ans_words);

/* Decoder A: validates the stream, then reads the code of every output
 * position bit by bit -- the next unread bit of the internal node named by
 * the prefix read so far -- until the prefix is a canonical codeword
 * (Sec. 1.1 and Sec. 2: a position's bits along its path are its code). */
int pivco_ref_decode(const uint8_t *in, uint64_t in_len, uint8_t *out,
                     uint64_t cap, uint64_t *n_out);

/* Decoder B: same validation, then the bottom-up merge of Sec. 3: every
 * internal node, deepest first, builds the dense symbol sequence of its
 * subtree from its bitmap and its two children (a leaf child is a constant). */
int pivco_ref_decode_merge(const uint8_t *in, uint64_t in_len, uint8_t *out,
                           uint64_t cap, uint64_t *n_out);

/* Decode only blocks [b0, b1) of a stream (decoder A); output written at
 * out[0 .. n of those blocks). */
int pivco_ref_decode_blocks(const uint8_t *in, uint64_t in_len, uint32_t b0,
                            uint32_t b1, uint8_t *out, uint64_t cap,
                            uint64_t *n_out);

/* Classical (non-pivoted) Huffman stream: codes of in[0..n) concatenated,
 * MSB of each code first, bits packed MSB-first into bytes. */
int pivco_ref_classical_encode(const uint8_t *in, uint64_t n, const uint8_t len[256],
                               uint8_t *out, uint64_t cap, uint64_t *nbits);
/* Bit-by-bit tree walk (the decoding of Listing 1) over a classical stream. */
int pivco_ref_classical_decode(const uint8_t *bits, uint64_t nbits,
                               const uint8_t len[256], uint8_t *out, uint64_t n);
/* Convert the first block of a pivoted stream into the classical stream. */
int pivco_ref_pivoted_to_classical(const uint8_t *in, uint64_t in_len,
                                   uint8_t *out, uint64_t cap, uint64_t *nbits);

/* Selective tANS of node bitmaps as bytes (Sec. 5.2, App. D, App. F;
 * fse_ref.c documents the readings): ans_mode 3 of the encoder, stream flags
 * bit 0.  fse_norm: table t's (1..50) normalized counts (sum 2^11).
 * fse_cost: its expected bits per bitmap bit at its own skew.  fse_select:
 * the selection rule; sets *marker = t | 0x80 if coded complemented.
 * fse_encode/fse_decode: a node body's chunks (without the 8-byte node
 * header) for a bitmap of nbits bits (ceil(nbits/8) bytes). */
int pivco_ref_fse_norm(uint32_t t, uint16_t norm[256]);
double pivco_ref_fse_cost(uint32_t t);
int pivco_ref_fse_select(uint64_t n_v, uint64_t n_right, uint32_t depth, uint32_t *marker);
int pivco_ref_fse_encode(const uint8_t *bits, uint64_t nbits, uint32_t marker, uint32_t chunk_log2,
                         uint8_t *out, uint64_t cap, uint64_t *out_len);
int pivco_ref_fse_decode(const uint8_t *body, uint64_t body_len, uint64_t nbits, uint32_t marker,
                         uint32_t chunk_log2, uint8_t *bits);

/* Per-block introspection of a stream: code lengths, internal-node count,
 * per-node (BFS order) depth, n_v, n_right, coding kind and flat depth D (0
 * for binary nodes; may be NULL). Arrays of 255. */
int pivco_ref_block_info(const uint8_t *in, uint64_t in_len, uint32_t block,
                         uint8_t len[256], uint32_t *mode, uint32_t *n_internal,
                         uint8_t depth[255], uint64_t n_v[255],
                         uint64_t n_right[255], uint8_t kind[255], uint8_t flat[255]);

/* PivCo-Golomb (App. G, golomb_ref.c): the pivoted layout applied to a
 * unary code -- value v is v 0-bits and a 1-bit, bitmap k holds the k-th code
 * bit of every value >= k.  Stream format "PVG1" documented in golomb_ref.c.
 * Decoder A reads each value's code bit by bit with a cursor per bitmap;
 * decoder B merges bottom-up from the last bitmap (merge_vec_cst_plus1). */
uint64_t pivco_ref_golomb_bound(uint64_t n, uint32_t block_size);
int pivco_ref_golomb_encode(const uint8_t *in, uint64_t n, uint32_t block_size, uint8_t *out,
                            uint64_t cap, uint64_t *out_len);
int pivco_ref_golomb_decode(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                            uint64_t *n_out);
int pivco_ref_golomb_decode_merge(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                                  uint64_t *n_out);

#ifdef __cplusplus
}
#endif
#endif
