// encode.hip -- gfx950 kernels and host driver for PivCo-Huffman encoding.
//
// Encoding (Sec. 4 of the paper) uses the same tree as decoding and walks it
// top-down: each internal node receives the codes of the symbols passing
// through it, emits one bit per symbol (its bitmap) and partitions the
// symbols between its children (the enc_partition primitives of Table 11).
// The driver:
//   1. k_hist        symbol histogram of every block and of every 4Ki-symbol
//                    slice of it (end-to-end encode time is dominated by this
//                    count, Sec. 4); k_slice_prefix turns the slice counts
//                    into per-slice prefixes;
//   2. k_tree        optimal length-limited lengths per block (package-merge,
//                    one wave per block, the host's tie rules), or the
//                    supplied tree;
//   3. k_layout      per block, from its lengths and histogram: canonical
//                    codes, breadth-first node table, n_v and n_right, the
//                    rANS selection rule, body sizes and offsets, and the
//                    block header bytes;
//   4. k_scan        offsets of every block's areas (exclusive scans);
//   5. k_split       per slice of a block: per level, one wave per node turns
//                    64 symbols at a time into a 64-bit ballot of code bits
//                    (LSB first = stream order), ORs it into the node's
//                    bitmap -- raw nodes straight into the block's byte-packed
//                    raw image, rANS nodes into word-aligned scratch -- and
//                    scatters the symbols to the children's segments in LDS
//                    with ballot + mbcnt ranks (stable);
//   6. k_chunks      the entropy-coded chunk jobs; k_rans_enc codes them
//                    (32-lane interleaved binary rANS, one wave per chunk,
//                    steps in reverse order), or k_fse_enc (byte tANS);
//   7. k_sizes       block sizes from the rANS body sizes; k_scan2 the block
//                    offsets and the stream size;
//   8. k_assemble    stream header, offset tables, block headers and raw
//                    images (aligned 4-byte words); k_assemble_rans the rANS
//                    bodies.
//   9. k_finish      the stream length and the call's status into device
//                    memory.
// Nothing waits on the host: pivco_encode_async leaves the length and status
// in device memory; pivco_encode reads them back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "pivco_int.h"

namespace pivco {

bool tree_is_complete(const uint8_t len[256], uint32_t max_len);

namespace {

constexpr int kWaveE = 64;
constexpr uint32_t kHistSlice = 1u << 12;   // one split tile: a 4 MiB block is 1024 workgroups
constexpr int kSplitNT = 256;
constexpr uint32_t kSplitT = 4096;      // input symbols per tile
constexpr uint32_t kHdrStride = 1216;   // block header bytes: 12 + 128 + 32 + 4 * 255 <= this
constexpr uint32_t kLayoutWaves = 4;
constexpr uint32_t kAsmSeg = 16384;     // output words per assembling workgroup
constexpr uint32_t kScanNT = 1024;
// Error word of one encode (in its status area); the first error wins.
constexpr uint32_t kErrArg = 1;          // a block's tree: PIVCO_E_ARG
constexpr uint32_t kErrUnsupported = 2;  // a tANS cursor stream past its 16-bit length: PIVCO_E_UNSUPPORTED

// Per-block description for the split kernel, written by k_layout.
struct EncBlock {
  uint64_t in_off;        // first input symbol
  uint32_t n;             // symbols
  uint32_t I;             // internal nodes (0: constant block, nothing to split)
  uint32_t maxlen;        // node levels
  uint32_t pad;
  uint32_t lvl[16];       // first node id of each depth
  uint32_t off[17];       // internal node at depth d with code prefix p: lvl[d] + p - off[d]
  uint32_t code[256];     // code | len << 16 | D << 20 | group node << 24: a symbol
                          // whose group of 2^D >= 2 symbols is a node ends its
                          // path there (D = 0: no such node)
  uint16_t child[256][2]; // internal id or 0x8000 | symbol (0x8000 for a flat node's)
  uint32_t bit[256];      // node's first bit: in the block's raw image (raw
                          // node) or in its rANS bitmap words (rANS node)
  uint32_t kind[8];       // bit i: node i is rANS-coded
  uint8_t fd[256];        // flat node: its depth D (>= 2), 0 for binary nodes
  uint32_t pad2;
};
static_assert(sizeof(EncBlock) % 16 == 0, "EncBlock copies in 16-byte units");

// Node on a symbol's path at depth d (cl = EncBlock::code of the symbol; lvl
// and off as in EncBlock):
// above the symbol's group the internal node of its code prefix, at the
// group's depth the group node.  The path has len - D + (D ? 1 : 0) nodes.
__device__ __forceinline__ uint32_t path_node(const uint32_t *lvl, const uint32_t *off, uint32_t cl, uint32_t d) {
  const uint32_t len = (cl >> 16) & 15, D = (cl >> 20) & 15;
  if (D && d == len - D) return cl >> 24;
  return lvl[d] + ((cl & 0xFFFF) >> (len - d)) - off[d];
}

__device__ __forceinline__ uint32_t path_len(uint32_t cl) {
  const uint32_t len = (cl >> 16) & 15, D = (cl >> 20) & 15;
  return len - D + (D ? 1u : 0u);
}

// Per-block layout (k_layout), offsets (k_scan) and size (k_sizes, k_scan2).
struct BlockLay {
  uint32_t n;             // symbols
  uint32_t hlen;          // header bytes
  uint32_t raw_bytes;     // raw bodies
  uint32_t ans_words;     // words its rANS nodes decode into: sum of ceil(n_v / 32)
  uint32_t n_rnodes;      // rANS-coded nodes
  uint32_t n_chunks;      // their chunks
  uint64_t slot_bytes;    // output slot bytes of its chunks
  uint64_t img_off;       // its raw image in the image area (bytes, 16-aligned)
  uint64_t rbm_off;       // its rANS bitmaps in the rANS bitmap area (words)
  uint64_t chunk0;        // its first chunk job
  uint64_t slot0;         // its first slot byte
  uint64_t ans0;          // scratch words of the blocks before it (stream table)
  uint64_t out_off;       // the block in the stream (bytes)
  uint32_t comp;          // block bytes (comp_size)
  uint32_t pad;
};

// A rANS-coded node of a block, in node order (k_layout; blen and boff by
// k_sizes).
struct RansNode {
  uint32_t rword;         // first word of its bitmap among the block's rANS words
  uint32_t nv;            // bits
  uint32_t p1q;           // 12-bit probability of a 1 bit (ans_mode 3: the tANS marker)
  uint32_t ch0;           // its first chunk among the block's chunks
  uint64_t sl0;           // its first slot byte among the block's slots
  uint32_t blen;          // body bytes (all its chunks)
  uint32_t boff;          // offset of its 8-byte body header in the block
};

struct RansJob {
  uint64_t bmp_word;      // word of the chunk's first bit in the rANS bitmap area
  uint64_t slot;          // byte offset of the chunk's output slot
  uint32_t nbits;
  uint32_t p1q;
  uint32_t block;
  uint32_t rnode;         // its node among the block's rANS nodes
  uint32_t first;         // 1: first chunk of its node
  uint32_t dst;           // byte offset of the chunk in its block (k_sizes)
};

// Batch totals (k_scan, k_scan2).
struct Totals {
  uint64_t img_bytes, rbm_words, chunks, slot_bytes, ans_words, out_bytes;
  uint64_t pad[2];
};

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Probability of a 1 bit in 12-bit fixed point, rounded to nearest and
// clamped to [1, 4095] (the format's reading of the 12-bit binary coder).
__device__ __forceinline__ uint32_t p1q_of(uint32_t nv, uint32_t nr) {
  const uint64_t q = (static_cast<uint64_t>(nr) * 4096 + nv / 2) / nv;
  return static_cast<uint32_t>(q < 1 ? 1 : q > 4095 ? 4095 : q);
}

// The rANS selection rule: ans_mode 1 codes nodes whose one-bit fraction is
// below 0.1 or above 0.9; 2 codes every node; nodes no symbol passes never.
__device__ __forceinline__ bool select_ans(uint32_t mode, uint32_t nv, uint32_t nr) {
  if (nv == 0) return false;
  if (mode == 1) return 10ull * nr < nv || 10ull * nr > 9ull * nv;
  return mode == 2;
}

// The selection rule of the byte tANS coder (ans_mode 3, Sec. 5.2): a
// binary node of at least 256 bits whose majority bit has a fraction above
// 0.625 (8 maj > 5 n_v) takes table t = round(100 x that fraction) - 49
// (halves up, at most 50) when the table's expected bits per bitmap bit h_t
// make (depth + h_t) / (depth + 1) < 0.95; dmax[t] is the number of depths
// that pass (the test holds exactly for depth < 19 - 20 h_t).  Returns the
// marker (t, | 0x80 when 1 bits are the minority and the bitmap is coded
// complemented), or 0.
__device__ __forceinline__ uint32_t fse_marker(uint32_t nv, uint32_t nr, uint32_t depth,
                                               const uint8_t *dmax) {
  if (nv < 256 || nr > nv) return 0;
  const uint32_t zeros = nv - nr, maj = nr >= zeros ? nr : zeros;
  if (8ull * maj <= 5ull * nv) return 0;
  uint64_t pct = (200ull * maj + nv) / (2ull * nv);
  if (pct > 99) pct = 99;
  const uint32_t t = static_cast<uint32_t>(pct) - 49;
  if (depth >= dmax[t]) return 0;
  return t | (nr < zeros ? 0x80u : 0u);
}

// Output slot of a chunk of nbits bits: lane states, at most one 16-bit word
// per bit, padding.  A tANS chunk of the same bits fits too: 128 header
// bytes, per cursor at most 11 bits a byte rounded up to bytes, and padding
// come to at most 161 + 11 nbits / 64 bytes, within this size from 14 bits
// on; below that, two cursors of one step each take at most 132 bytes.
__host__ __device__ __forceinline__ uint32_t slot_size(uint32_t nbits) {
  return (kChunkHdr + 2 * nbits + 4 + 15) & ~15u;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint32_t *p, uint64_t nwords) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nwords;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// Zeroes the image and rANS bitmap areas up to the sizes k_scan found (the
// split kernel ORs bits into them).
__global__ void k_zero_areas(uint32_t *img, uint32_t *rbm, const Totals *tot) {
  const uint64_t ni = tot->img_bytes / 4, nr = tot->rbm_words;
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < ni + nr; i += step) {
    if (i < ni) img[i] = 0;
    else rbm[i - ni] = 0;
  }
}

// Histogram of every block, one workgroup per slice of kHistSlice symbols:
// the slice's counts go to its own row of slh (the split kernel's slices
// start at the same boundaries); a block of one slice also writes them to
// its row of hist (k_slice_prefix writes the totals of larger blocks).
__global__ __launch_bounds__(256) void k_hist(const uint8_t *in, uint64_t n, uint32_t bs,
                                              uint32_t spb, uint32_t *hist, uint32_t *slh) {
  __shared__ uint32_t h[4][256];
  const int tid = threadIdx.x, w = tid >> 6;
  for (int i = tid; i < 1024; i += 256) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t b = blockIdx.x / spb, sl = blockIdx.x % spb;
  const uint64_t bstart = b * bs;
  const uint64_t bend = bstart + bs < n ? bstart + bs : n;
  const uint64_t s0 = bstart + sl * kHistSlice;
  const uint64_t s1 = s0 + kHistSlice < bend ? s0 + kHistSlice : bend;
  if (s0 < s1) {
    // aligned middle with dword loads, byte loads at the edges
    const uint64_t a0 = (s0 + 3) & ~3ull, a1 = s1 & ~3ull;
    for (uint64_t i = s0 + tid; i < s1 && i < a0; i += 256) atomicAdd(&h[w][in[i]], 1u);
    if (a0 < a1) {
      const uint32_t *in4 = reinterpret_cast<const uint32_t *>(in + a0);
      const uint64_t nd = (a1 - a0) >> 2;
      for (uint64_t i = tid; i < nd; i += 256) {
        const uint32_t v = in4[i];
        atomicAdd(&h[w][v & 255], 1u);
        atomicAdd(&h[w][(v >> 8) & 255], 1u);
        atomicAdd(&h[w][(v >> 16) & 255], 1u);
        atomicAdd(&h[w][v >> 24], 1u);
      }
    }
    for (uint64_t i = (a1 > a0 ? a1 : a0) + tid; i < s1; i += 256) atomicAdd(&h[w][in[i]], 1u);
  }
  __syncthreads();
  const uint32_t v = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
  slh[static_cast<uint64_t>(blockIdx.x) * 256 + tid] = v;
  if (spb == 1) hist[b * 256 + tid] = v;
}

// Per block, the slice histograms become exclusive prefixes: row k holds the
// count of each symbol in the block's slices before slice k, and the block's
// row of hist the totals (one thread per symbol, one workgroup per block;
// 16 rows read before any is rewritten).
__global__ __launch_bounds__(256) void k_slice_prefix(uint32_t *slh, uint32_t spb, uint32_t *hist) {
  uint32_t *row = slh + static_cast<uint64_t>(blockIdx.x) * spb * 256 + threadIdx.x;
  uint32_t run = 0, k = 0;
  for (; k + 16 <= spb; k += 16) {
    uint32_t c[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) c[j] = row[256ull * (k + j)];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      row[256ull * (k + j)] = run;
      run += c[j];
    }
  }
  for (; k < spb; ++k) {
    const uint32_t c = row[256ull * k];
    row[256ull * k] = run;
    run += c;
  }
  hist[static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x] = run;
}

// Code lengths of every block on the device (one wave per block), the same
// package-merge and determinism rules as the host's lengths_from_counts
// (items by weight; on equal weight a single before a package, symbols by
// id, packages in creation order; the multiset of lengths handed out again
// ascending to the symbols by (count desc, id asc)), in parallel form:
//   * the present symbols are ranked by (count, id) by counting over all 256
//     keys (a broadcast LDS read each), which also gives each symbol's run of
//     equal counts;
//   * row L holds the first min(m, 2m - 2) singles; row r - 1 merges the m
//     singles with the packages (sums of consecutive pairs) of row r: single
//     i lands at i + #(packages lighter than it), package j at j + #(singles
//     no heavier), both by binary search, and positions past 2m - 2 are
//     dropped.  Each row keeps the positions of its singles;
//   * buying the first k = 2m - 2 items of row 1 buys the singles placed
//     below k and 2 (k - singles) items of the next row, and so on; a
//     symbol's length is the number of rows in which it was bought.
// A block with one symbol becomes a constant block; a supplied tree is
// copied (a present symbol without a code is an argument error).  A block
// in error gets the constant mode (nothing to split) and sets *err.
constexpr uint32_t kTreeRows = kMaxLenGpu + 1;
struct TreeSmem {
  uint64_t key[256];          // (count << 8 | symbol); ~0 for an absent symbol
  uint64_t w[256];            // counts in (count, id) order
  uint64_t row[2][512];       // item weights of two rows
  uint64_t pk[256];           // packages of the row below
  uint16_t spos[kTreeRows][256];   // row r: position of single i (0xFFFF: not in the row)
  uint32_t rlen[kTreeRows];
};

__global__ __launch_bounds__(kWaveE) void k_tree(const uint32_t *hist, uint32_t nb, uint32_t L,
                                                 pivco_tree tree, uint32_t use_tree, uint8_t *lenm,
                                                 uint32_t *modes, uint32_t *err) {
  __shared__ TreeSmem sm;
  const uint32_t b = blockIdx.x, lane = __lane_id();
  if (b >= nb) return;
  uint32_t c[4];
  bool pres[4];
  uint32_t nsym = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    c[e] = hist[256ull * b + 4 * lane + e];
    pres[e] = c[e] != 0;
  }
  uint64_t bal[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    bal[e] = __ballot(pres[e]);
    nsym += static_cast<uint32_t>(__popcll(bal[e]));
  }
  const uint32_t m = nsym;
  uint8_t *lb = lenm + 256ull * b;
  if (use_tree) {
    bool bad = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint8_t l = tree.code_len[4 * lane + e];
      bad |= pres[e] && l == 0;
      lb[4 * lane + e] = l;
    }
    const bool any = __ballot(bad) != 0;
    if (lane == 0) {
      modes[b] = any ? 1u : 0u;
      if (any) atomicCAS(err, 0u, kErrArg);
    }
    return;
  }
  if (m == 1 || m == 0 || (m > (1u << L))) {   // constant block, or no code of this length exists
    uint32_t sym = 256;                   // the smallest present symbol (the same in every lane)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (bal[e]) {
        const uint32_t cand = 4 * static_cast<uint32_t>(__ffsll(static_cast<long long>(bal[e])) - 1) + e;
        sym = cand < sym ? cand : sym;
      }
    sym &= 255;
#pragma unroll
    for (int e = 0; e < 4; ++e) lb[4 * lane + e] = 0;
    if (lane == 0) {
      modes[b] = 1u | (sym << 8);
      if (m != 1) atomicCAS(err, 0u, kErrArg);
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t sy = 4 * lane + e;
    sm.key[sy] = pres[e] ? (static_cast<uint64_t>(c[e]) << 8) | sy : ~0ull;
  }
  wave_sync();
  // rank by (count, id), and the run of equal counts: [lt, le)
  uint32_t rank[4] = {0, 0, 0, 0}, lt[4] = {0, 0, 0, 0}, le[4] = {0, 0, 0, 0};
  for (uint32_t t = 0; t < 256; ++t) {
    const uint64_t kt = sm.key[t];
    const bool pt = kt != ~0ull;
    const uint64_t ct = kt >> 8;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint64_t ke = (static_cast<uint64_t>(c[e]) << 8) | (4 * lane + e);
      rank[e] += pt && kt < ke ? 1u : 0u;
      lt[e] += pt && ct < c[e] ? 1u : 0u;
      le[e] += pt && ct <= c[e] ? 1u : 0u;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (pres[e]) sm.w[rank[e]] = c[e];
  const uint32_t cap = 2 * m - 2, top = m < cap ? m : cap;
  for (uint32_t i = lane; i < 256; i += kWaveE) sm.spos[L][i] = i < top ? static_cast<uint16_t>(i) : 0xFFFFu;
  if (lane == 0) sm.rlen[L] = top;
  wave_sync();
  for (uint32_t i = lane; i < top; i += kWaveE) sm.row[L & 1][i] = sm.w[i];
  wave_sync();
  uint32_t rl = top;
  for (uint32_t r = L; r > 1; --r) {
    const uint64_t *cur = sm.row[r & 1];
    uint64_t *nxt = sm.row[(r - 1) & 1];
    const uint32_t np = rl / 2;
    for (uint32_t j = lane; j < np; j += kWaveE) sm.pk[j] = cur[2 * j] + cur[2 * j + 1];
    wave_sync();
    const uint32_t total = m + np < cap ? m + np : cap;
    for (uint32_t i = lane; i < m; i += kWaveE) {      // singles: packages strictly lighter come first
      const uint64_t x = sm.w[i];
      uint32_t lo = 0, hi = np;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sm.pk[mid] < x) lo = mid + 1; else hi = mid;
      }
      const uint32_t pos = i + lo;
      if (pos < total) nxt[pos] = x;
      sm.spos[r - 1][i] = pos < total ? static_cast<uint16_t>(pos) : 0xFFFFu;
    }
    for (uint32_t j = lane; j < np; j += kWaveE) {     // packages: singles no heavier come first
      const uint64_t y = sm.pk[j];
      uint32_t lo = 0, hi = m;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sm.w[mid] <= y) lo = mid + 1; else hi = mid;
      }
      const uint32_t pos = j + lo;
      if (pos < total) nxt[pos] = y;
    }
    if (lane == 0) sm.rlen[r - 1] = total;
    rl = total;
    wave_sync();
  }
  // bought items, row by row
  uint32_t depth[4] = {0, 0, 0, 0};
  bool bad = false;
  uint32_t k = cap;
  for (uint32_t r = 1; r <= L && k; ++r) {
    if (k > sm.rlen[r]) { bad = true; break; }
    uint32_t sg = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t i = 4 * lane + e;
      sg += static_cast<uint32_t>(__popcll(__ballot(i < m && sm.spos[r][i] < k)));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) depth[e] += 4 * lane + e < sg ? 1u : 0u;
    k = 2 * (k - sg);
  }
  // lengths: the ascending multiset to the symbols by (count desc, id asc)
  uint32_t cum[kTreeRows + 1];
  cum[0] = 0;
  for (uint32_t l = 1; l <= L; ++l) {
    uint32_t nl = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) nl += static_cast<uint32_t>(__popcll(__ballot(4 * lane + e < m && depth[e] == l)));
    cum[l] = cum[l - 1] + nl;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (4 * lane + e < m && (depth[e] < 1 || depth[e] > L)) bad = true;
  bad = __ballot(bad) != 0 || cum[L] != m;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t len = 0;
    if (pres[e]) {
      const uint32_t pd = (m - le[e]) + (rank[e] - lt[e]);
      for (uint32_t l = 1; l <= L; ++l)
        if (len == 0 && cum[l] > pd) len = l;
    }
    lb[4 * lane + e] = bad ? 0 : static_cast<uint8_t>(len);
  }
  if (lane == 0) {
    modes[b] = bad ? 1u : 0u;
    if (bad) atomicCAS(err, 0u, kErrArg);
  }
}

// Layout of one block per wave.  lenm holds, per block, its 256 code
// lengths; modes its mode (0 coded, 1 | symbol << 8 constant).  The code is
// canonical: with cnt(L) codes of length L and fc(L) the first of them,
// fc(L+1) = 2 (fc(L) + cnt(L)); a symbol's code is fc(len) plus its rank
// among the symbols of its length; the internal nodes at depth d are the
// prefixes [fc(d) + cnt(d), 2^d) numbered breadth-first, and child q of such
// a node is a leaf iff q < fc(d+1) + cnt(d+1).  With flat-subtree trees
// (shape 1, Sec. 2.2.3-2.2.4) the same closed form runs over the tree's
// items: the symbols of length L are cut by the binary digits of cnt(L),
// largest group first, a group of 2^D hanging at depth L - D; the items of a
// depth are ordered by D descending; a group of two or more symbols is a
// node (flat when D >= 2), numbered before the depth's internal nodes.
struct LayoutSmem {
  uint32_t nv[256], nr[256];
  uint32_t cnt[17], fc[18], lvl[18], lbase[17], ci[18], gn[18], off[18];
  uint32_t maxlen, I;
  uint8_t leafsym[256];
};

__global__ __launch_bounds__(kWaveE * kLayoutWaves) void k_layout(
    const uint8_t *lenm, const uint32_t *modes, const uint32_t *hist, uint32_t nb, uint64_t n,
    uint32_t bs, uint32_t ans_mode, uint32_t chunk_log2, uint32_t shape, const uint8_t *fse_dmax,
    EncBlock *eb, BlockLay *lay, RansNode *rnodes, uint8_t *hdr) {
  __shared__ LayoutSmem smem[kLayoutWaves];
  const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
  const uint32_t b = blockIdx.x * kLayoutWaves + wave;
  if (b >= nb) return;
  LayoutSmem &sm = smem[wave];
  EncBlock &E = eb[b];
  BlockLay &Lb = lay[b];
  uint8_t *H = hdr + static_cast<uint64_t>(b) * kHdrStride;
  const uint64_t start = static_cast<uint64_t>(b) * bs;
  const uint32_t nblk = static_cast<uint32_t>(n - start < bs ? n - start : bs);
  const uint32_t cw = nblk <= 65535 ? 2u : 4u;
  const uint32_t mode = modes[b];
  if (lane == 0) {
    E.in_off = start;
    E.n = nblk;
    Lb.n = nblk;
    *reinterpret_cast<uint32_t *>(H + 4) = nblk;
    H[8] = static_cast<uint8_t>(mode & 1);
    H[9] = static_cast<uint8_t>(mode >> 8);
    H[10] = static_cast<uint8_t>(cw);
    H[11] = 0;
  }
  if (mode & 1) {                        // constant block: its 12-byte header only
    if (lane == 0) {
      E.I = 0;
      E.maxlen = 0;
      Lb.hlen = kBlockFixed;
      Lb.raw_bytes = Lb.ans_words = Lb.n_rnodes = Lb.n_chunks = 0;
      Lb.slot_bytes = 0;
    }
    return;
  }
  // lane owns symbols 4 lane .. 4 lane + 3
  const uint32_t lw = *reinterpret_cast<const uint32_t *>(lenm + 256ull * b + 4 * lane);
  uint32_t l[4], c[4], rank[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    l[k] = (lw >> (8 * k)) & 255;
    c[k] = hist[256ull * b + 4 * lane + k];
  }
  const uint64_t below = (1ull << lane) - 1;
  for (uint32_t L = 1; L <= 15; ++L) {
    uint64_t mk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mk[k] = __ballot(l[k] == L);
    const uint32_t before = __popcll(mk[0] & below) + __popcll(mk[1] & below) +
                            __popcll(mk[2] & below) + __popcll(mk[3] & below);
    uint32_t own = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l[k] == L) { rank[k] = before + own; ++own; }
    if (lane == 0) sm.cnt[L] = __popcll(mk[0]) + __popcll(mk[1]) + __popcll(mk[2]) + __popcll(mk[3]);
  }
  if (lane == 0) {
    sm.cnt[0] = 0;
    sm.cnt[16] = 0;
    // items per depth: every symbol (shape 0), or one per set binary digit D
    // of cnt(d + D) (shape 1)
    uint32_t maxitem = 0, lb = 0;
    for (uint32_t d = 0; d <= 17; ++d) {
      uint32_t ci = 0, gn = 0;
      if (shape == 0) {
        ci = d <= 16 ? sm.cnt[d] : 0u;
      } else {
        for (uint32_t D = 0; D <= 8; ++D)
          if (d + D <= 15 && ((sm.cnt[d + D] >> D) & 1)) { ++ci; gn += D >= 1 ? 1u : 0u; }
      }
      sm.ci[d] = ci;
      sm.gn[d] = gn;
      if (ci) maxitem = d;
      if (d <= 16) { sm.lbase[d] = lb; lb += sm.cnt[d]; }
    }
    uint32_t fcd = 0, lv = 0;
    for (uint32_t d = 0; d <= 17; ++d) {
      sm.fc[d] = fcd;
      sm.lvl[d] = lv;
      sm.off[d] = fcd + sm.ci[d] - sm.gn[d];
      lv += sm.gn[d] + (d < maxitem ? (1u << d) - fcd - sm.ci[d] : 0u);
      fcd = 2 * (fcd + sm.ci[d]);
    }
    const uint32_t levels = maxitem + (sm.gn[maxitem] ? 1u : 0u);
    sm.maxlen = levels;
    sm.I = sm.lvl[levels];
    E.maxlen = levels;
    E.I = sm.lvl[levels];
  }
  wave_sync();
  const uint32_t I = sm.I;
  // codes and the symbols in (length, symbol) order
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t s = 4 * lane + k;
    uint32_t cl = 0;
    if (l[k]) {
      const uint32_t L = l[k], r = rank[k];
      if (shape == 0) {
        cl = (sm.fc[L] + r) | (L << 16);
      } else {
        // the symbol's group: binary digits of cnt(L), largest first
        const uint32_t cn = sm.cnt[L];
        uint32_t D = 0, hi = 0;
        for (uint32_t e = 9; e-- > 0;) {
          if (!((cn >> e) & 1)) continue;
          if (r < hi + (1u << e)) { D = e; break; }
          hi += 1u << e;
        }
        const uint32_t m = L - D;
        uint32_t idx = 0;                  // items of depth m with a larger D
        for (uint32_t e = D + 1; e <= 8; ++e)
          if (m + e <= 15 && ((sm.cnt[m + e] >> e) & 1)) ++idx;
        const uint32_t code = ((sm.fc[m] + idx) << D) | (r - hi);
        cl = code | (L << 16) | (D << 20) | (D ? (sm.lvl[m] + idx) << 24 : 0u);
      }
      sm.leafsym[sm.lbase[L] + r] = static_cast<uint8_t>(s);
    }
    E.code[s] = cl;
    sm.nv[s] = 0;
    sm.nr[s] = 0;
    rank[k] = cl;                        // kept for the path walk below
  }
  if (lane < 16) E.lvl[lane] = sm.lvl[lane];
  if (lane < 17) E.off[lane] = sm.off[lane];
  wave_sync();
  // symbols passing each node and going right: walk each present symbol's path
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!c[k] || !l[k]) continue;
    const uint32_t cl = rank[k], len = l[k], D = (cl >> 20) & 15;
    for (uint32_t d = 0; d < path_len(cl); ++d) {
      const uint32_t id = path_node(sm.lvl, sm.off, cl, d);
      atomicAdd(&sm.nv[id], c[k]);
      if (D >= 2 && d == len - D) break;  // a flat node has no right branch
      if (((cl & 0xFFFF) >> (len - 1 - d)) & 1) atomicAdd(&sm.nr[id], c[k]);
    }
  }
  wave_sync();
  // node table: lane owns nodes 4 lane .. 4 lane + 3
  uint32_t fdk[4] = {0, 0, 0, 0}, dk[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    if (i >= I) continue;
    uint32_t d = 0;
    while (sm.lvl[d + 1] <= i) ++d;
    dk[k] = d;
    const uint32_t r = i - sm.lvl[d];
    uint32_t cc = 0;
    if (r < sm.gn[d]) {                  // group r of depth d (shape 1)
      uint32_t D = 0, left = r;
      for (uint32_t e = 8; e >= 1; --e)
        if (d + e <= 15 && ((sm.cnt[d + e] >> e) & 1)) {
          if (left == 0) { D = e; break; }
          --left;
        }
      const uint32_t L = d + D;
      const uint32_t first = sm.lbase[L] + (sm.cnt[L] & ~((2u << D) - 1));
      if (D == 1) cc = (0x8000u | sm.leafsym[first]) | ((0x8000u | sm.leafsym[first + 1]) << 16);
      else { cc = 0x80008000u; fdk[k] = D; }
    } else {
      const uint32_t p = sm.fc[d] + sm.ci[d] + (r - sm.gn[d]);
      const uint32_t d1 = d + 1;
      const uint32_t leaf0 = sm.lbase[d1] + (shape ? (sm.cnt[d1] & ~1u) : 0u);
      for (int bb = 0; bb < 2; ++bb) {
        const uint32_t q = 2 * p + bb;
        const uint32_t rq = q - sm.fc[d1];
        const uint32_t ch = rq < sm.gn[d1] ? sm.lvl[d1] + rq
                            : rq < sm.ci[d1] ? 0x8000u | sm.leafsym[leaf0 + rq - sm.gn[d1]]
                                             : sm.lvl[d1] + sm.gn[d1] + (q - sm.fc[d1] - sm.ci[d1]);
        cc |= ch << (16 * bb);
      }
    }
    *reinterpret_cast<uint32_t *>(E.child[i]) = cc;
    E.fd[i] = static_cast<uint8_t>(fdk[k]);
  }
  // lane owns nodes 4 lane .. 4 lane + 3: kind, sizes and their prefixes
  const uint32_t C = 1u << chunk_log2;
  uint32_t kd[4], rb[4], aw[4], ch[4], sl[4], nvk[4], nrk[4], mk[4];
  uint32_t lraw = 0, lans = 0, lrn = 0, lch = 0, lsl = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    nvk[k] = i < I ? sm.nv[i] : 0u;
    nrk[k] = i < I ? sm.nr[i] : 0u;
    mk[k] = i < I && !fdk[k] && ans_mode == 3 ? fse_marker(nvk[k], nrk[k], dk[k], fse_dmax) : 0u;
    kd[k] = i < I && !fdk[k] && (ans_mode == 3 ? mk[k] != 0 : select_ans(ans_mode, nvk[k], nrk[k])) ? 1u : 0u;
    const uint32_t nch = kd[k] ? (nvk[k] + C - 1) / C : 0u;
    const uint32_t rem = nvk[k] - (nch ? (nch - 1) * C : 0u);
    const uint64_t bits = static_cast<uint64_t>(nvk[k]) * (fdk[k] ? fdk[k] : 1u);
    rb[k] = lraw; aw[k] = lans; ch[k] = lch; sl[k] = lsl;
    lraw += kd[k] || i >= I ? 0u : static_cast<uint32_t>((bits + 7) / 8);
    lans += kd[k] ? (nvk[k] + 31) / 32 : 0u;
    lch += nch;
    lsl += nch ? ((nch - 1) * slot_size(C) + slot_size(rem)) / 16 : 0u;   // 16-byte units
    lrn += kd[k];
  }
  const uint32_t iraw = wave_incl_scan(lraw), ians = wave_incl_scan(lans), irn = wave_incl_scan(lrn);
  const uint32_t ich = wave_incl_scan(lch), isl = wave_incl_scan(lsl);
  uint32_t rn = irn - lrn;
  uint32_t nib = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    nib |= kd[k] << k;
    if (i >= I) continue;
    const uint32_t raw_off = iraw - lraw + rb[k], rword = ians - lans + aw[k];
    E.bit[i] = kd[k] ? rword : raw_off;
    if (kd[k]) {
      RansNode r;
      r.rword = rword;
      r.nv = nvk[k];
      r.p1q = ans_mode == 3 ? mk[k] : p1q_of(nvk[k], nrk[k]);
      r.ch0 = ich - lch + ch[k];
      r.sl0 = 16ull * (isl - lsl + sl[k]);
      r.blen = 0;
      r.boff = 0;
      rnodes[255ull * b + rn] = r;
      ++rn;
    }
  }
  // header: code lengths (two nibbles a byte, symbol 2j low), kind bits, counts of 1 bits
  const uint32_t kb = (I + 7) / 8;
  H[12 + 2 * lane] = static_cast<uint8_t>(l[0] | (l[1] << 4));
  H[12 + 2 * lane + 1] = static_cast<uint8_t>(l[2] | (l[3] << 4));
  const uint32_t nib_hi = __shfl_down(nib, 1, kWaveE);
  if ((lane & 1) == 0 && lane / 2 < kb) H[140 + lane / 2] = static_cast<uint8_t>(nib | (nib_hi << 4));
  const uint64_t bm[4] = {__ballot(kd[0]), __ballot(kd[1]), __ballot(kd[2]), __ballot(kd[3])};
  if (lane < 8) {                        // kind mask word: nodes 32 lane .. 32 lane + 31
    uint32_t w = 0;
    for (uint32_t j = 0; j < 32; ++j) w |= static_cast<uint32_t>((bm[j & 3] >> (8 * lane + j / 4)) & 1) << j;
    E.kind[lane] = w;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    if (i >= I) continue;
    uint8_t *q = H + 140 + kb + cw * i;
    q[0] = static_cast<uint8_t>(nrk[k]);
    q[1] = static_cast<uint8_t>(nrk[k] >> 8);
    if (cw == 4) { q[2] = static_cast<uint8_t>(nrk[k] >> 16); q[3] = static_cast<uint8_t>(nrk[k] >> 24); }
  }
  if (lane == kWaveE - 1) {
    Lb.hlen = 140 + kb + cw * I;
    Lb.raw_bytes = iraw;
    Lb.ans_words = ians;
    Lb.n_rnodes = irn;
    Lb.n_chunks = ich;
    Lb.slot_bytes = 16ull * isl;
  }
}

// Exclusive scans over the blocks (one workgroup): image bytes (16-aligned,
// with 16 bytes of slack), rANS bitmap words (multiples of 4), chunk jobs,
// slot bytes and scratch words; their totals.
__global__ __launch_bounds__(kScanNT) void k_scan(BlockLay *lay, uint32_t nb, Totals *tot) {
  __shared__ uint64_t part[5][kScanNT];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (nb + kScanNT - 1) / kScanNT;
  const uint32_t b0 = tid * per, b1 = b0 + per < nb ? b0 + per : nb;
  uint64_t v[5] = {0, 0, 0, 0, 0};
  for (uint32_t b = b0; b < b1; ++b) {
    const BlockLay &L = lay[b];
    v[0] += (static_cast<uint64_t>(L.raw_bytes) + 16 + 15) & ~15ull;
    v[1] += (static_cast<uint64_t>(L.ans_words) + 3) & ~3ull;
    v[2] += L.n_chunks;
    v[3] += L.slot_bytes;
    v[4] += L.ans_words;
  }
  for (int q = 0; q < 5; ++q) part[q][tid] = v[q];
  __syncthreads();
  for (uint32_t off = 1; off < kScanNT; off <<= 1) {   // inclusive scan (Hillis-Steele)
    uint64_t a[5];
    for (int q = 0; q < 5; ++q) a[q] = tid >= off ? part[q][tid - off] : 0ull;
    __syncthreads();
    for (int q = 0; q < 5; ++q) part[q][tid] += a[q];
    __syncthreads();
  }
  uint64_t run[5];
  for (int q = 0; q < 5; ++q) run[q] = part[q][tid] - v[q];
  for (uint32_t b = b0; b < b1; ++b) {
    BlockLay &L = lay[b];
    L.img_off = run[0];
    L.rbm_off = run[1];
    L.chunk0 = run[2];
    L.slot0 = run[3];
    L.ans0 = run[4];
    run[0] += (static_cast<uint64_t>(L.raw_bytes) + 16 + 15) & ~15ull;
    run[1] += (static_cast<uint64_t>(L.ans_words) + 3) & ~3ull;
    run[2] += L.n_chunks;
    run[3] += L.slot_bytes;
    run[4] += L.ans_words;
  }
  if (tid == kScanNT - 1) {
    tot->img_bytes = part[0][tid];
    tot->rbm_words = part[1][tid];
    tot->chunks = part[2][tid];
    tot->slot_bytes = part[3][tid];
    tot->ans_words = part[4][tid];
  }
}

static_assert(kSplitNT == 256, "the split kernel's prefix walk has one thread per symbol");
static_assert(kHistSlice % kSplitT == 0, "split tiles never cross a slice");

struct SplitSmem {
  EncBlock B;
  uint32_t cur[256];      // symbols of the node in earlier tiles
  uint32_t tv[256];       // node's symbols in this tile
  uint32_t seg[256];      // node's segment in its level buffer
  uint32_t top[16];
  uint32_t hist[256];
  uint32_t fw[kSplitNT / kWaveE][20];   // per wave: a flat node's packed values (64 x D bits + 31)
  uint8_t buf[2][kSplitT];
};

// One workgroup per slice of kHistSlice symbols of a block (slice k of block
// b is workgroup b * spb + k), so that large blocks are split by many
// workgroups.  A node's bits from this slice start at the number of the
// block's symbols before the slice that pass the node: the sum, over the
// symbols on whose path the node lies, of their counts before the slice
// (the slice's row of the prefix histograms).  A raw node's bitmap is
// written at its byte offset in the block's raw image (the stream layout),
// a rANS node's at its word in the block's rANS bitmap words.  Slices and
// neighbouring nodes share words at their edges: every word is written with
// atomicOr into zeroed memory.
__global__ __launch_bounds__(kSplitNT) void k_split(const uint8_t *in, const EncBlock *blocks,
                                                    const BlockLay *lay, uint32_t nblocks, uint32_t spb,
                                                    const uint32_t *pre, uint32_t *img, uint32_t *rbm) {
  __shared__ SplitSmem sm;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const uint32_t lane = __lane_id();
  const uint32_t b = blockIdx.x / spb, slice = blockIdx.x % spb;
  if (b >= nblocks) return;
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(&blocks[b]);
    uint4 *dst = reinterpret_cast<uint4 *>(&sm.B);
    for (uint32_t i = tid; i < sizeof(EncBlock) / 16; i += kSplitNT) dst[i] = src[i];
  }
  __syncthreads();
  const EncBlock &B = sm.B;
  const uint32_t s_lo = slice * kHistSlice;
  if (B.I == 0 || s_lo >= B.n) return;
  const uint32_t s_hi = B.n - s_lo < kHistSlice ? B.n : s_lo + kHistSlice;
  const uint64_t img_bit = 8ull * lay[b].img_off, rbm_bit = 32ull * lay[b].rbm_off;
  for (uint32_t i = tid; i < 256; i += kSplitNT) sm.cur[i] = 0;
  __syncthreads();
  if (slice) {   // symbols of each node before this slice
    const uint32_t s = tid;
    const uint32_t c = pre[static_cast<uint64_t>(blockIdx.x) * 256 + s];
    const uint32_t cl = B.code[s];
    if (c && cl)
      for (uint32_t d = 0; d < path_len(cl); ++d) atomicAdd(&sm.cur[path_node(B.lvl, B.off, cl, d)], c);
    __syncthreads();
  }
  const uint8_t *bin = in + B.in_off;
  for (uint32_t t0 = s_lo; t0 < s_hi; t0 += kSplitT) {
    const uint32_t tn = s_hi - t0 < kSplitT ? s_hi - t0 : kSplitT;
    for (uint32_t i = tid; i < 256; i += kSplitNT) { sm.tv[i] = 0; sm.hist[i] = 0; }
    if (tid < 16) sm.top[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < tn; i += kSplitNT) {
      const uint8_t s = bin[t0 + i];
      sm.buf[0][i] = s;
      atomicAdd(&sm.hist[s], 1u);
    }
    __syncthreads();
    // symbols of the tile passing each node: walk each present symbol's path
    {
      const uint32_t s = tid;
      const uint32_t c = sm.hist[s];
      const uint32_t cl = B.code[s];
      if (c && cl)
        for (uint32_t d = 0; d < path_len(cl); ++d) atomicAdd(&sm.tv[path_node(B.lvl, B.off, cl, d)], c);
    }
    __syncthreads();
    for (uint32_t i = tid; i < B.I; i += kSplitNT) {
      uint32_t d = 0;
      while (B.lvl[d + 1] <= i) ++d;
      sm.seg[i] = sm.tv[i] ? atomicAdd(&sm.top[d], sm.tv[i]) : 0u;
    }
    __syncthreads();
    for (uint32_t d = 0; d < B.maxlen; ++d) {
      const uint8_t *lb = sm.buf[d & 1];
      uint8_t *cb = sm.buf[(d + 1) & 1];
      for (uint32_t v = B.lvl[d] + wave; v < B.lvl[d + 1]; v += kSplitNT / kWaveE) {
        const uint32_t tvv = sm.tv[v];
        const uint32_t seg = sm.seg[v];
        const uint16_t c0 = B.child[v][0], c1 = B.child[v][1];
        uint32_t r0 = (c0 & 0x8000) ? 0u : sm.seg[c0];
        uint32_t r1 = (c1 & 0x8000) ? 0u : sm.seg[c1];
        const bool rans = (B.kind[v >> 5] >> (v & 31)) & 1;
        uint32_t *area = rans ? rbm : img;
        const uint32_t D = B.fd[v];
        if (D) {
          // a flat node: each symbol's index in the node's group (its code's
          // last D bits), as D-bit fields in stream order, gathered per 64
          // symbols in LDS and ORed into the image word by word
          const uint64_t base = img_bit + 8ull * B.bit[v] + static_cast<uint64_t>(D) * sm.cur[v];
          uint32_t *fw = sm.fw[wave];
          for (uint32_t c = 0; c < tvv; c += kWaveE) {
            const bool act = c + lane < tvv;
            const uint32_t s = act ? lb[seg + c + lane] : 0u;
            const uint32_t q = B.code[s] & ((1u << D) - 1);
            const uint64_t P = base + static_cast<uint64_t>(D) * c;
            const uint32_t a = static_cast<uint32_t>(P & 31);
            const uint32_t nw = (a + D * kWaveE + 31) >> 5;
            if (lane < 20) fw[lane] = 0;
            wave_sync();
            if (act && q) {
              const uint32_t bp = a + D * lane;
              atomicOr(&fw[bp >> 5], q << (bp & 31));
              if ((bp & 31) + D > 32) atomicOr(&fw[(bp >> 5) + 1], q >> (32 - (bp & 31)));
            }
            wave_sync();
            if (lane < nw && fw[lane]) atomicOr(&area[(P >> 5) + lane], fw[lane]);
            wave_sync();
          }
          continue;
        }
        const uint64_t base_bit = (rans ? rbm_bit + 32ull * B.bit[v] : img_bit + 8ull * B.bit[v]) + sm.cur[v];
        for (uint32_t c = 0; c < tvv; c += kWaveE) {
          const bool act = c + lane < tvv;
          const uint32_t s = act ? lb[seg + c + lane] : 0u;
          const uint32_t cl = B.code[s], len = (cl >> 16) & 15, code = cl & 0xFFFF;
          const bool bit = act && ((code >> (len - 1 - d)) & 1);
          const uint64_t m1 = __ballot(bit);
          const uint64_t m0 = __ballot(act && !bit);
          const uint64_t lt = (1ull << lane) - 1;
          // bitmap: 64 bits at bit position base_bit + c
          const uint64_t P = base_bit + c;
          const uint64_t q = P >> 5;
          const uint32_t sh = static_cast<uint32_t>(P & 31);
          const uint32_t lo = static_cast<uint32_t>(m1), hi = static_cast<uint32_t>(m1 >> 32);
          uint32_t wv = 0;
          if (lane == 0) wv = lo << sh;
          if (lane == 1) wv = sh ? (lo >> (32 - sh)) | (hi << sh) : hi;
          if (lane == 2) wv = sh ? hi >> (32 - sh) : 0u;
          if (lane < 3 && wv) atomicOr(&area[q + lane], wv);
          // stable partition of the symbols into the children's segments
          if (act) {
            if (bit && !(c1 & 0x8000)) cb[r1 + __popcll(m1 & lt)] = static_cast<uint8_t>(s);
            if (!bit && !(c0 & 0x8000)) cb[r0 + __popcll(m0 & lt)] = static_cast<uint8_t>(s);
          }
          r1 += __popcll(m1);
          r0 += __popcll(m0);
        }
      }
      __syncthreads();
    }
    for (uint32_t i = tid; i < B.I; i += kSplitNT) sm.cur[i] += sm.tv[i];
    __syncthreads();
  }
}

// The chunk jobs of every rANS node (one wave per block, a lane per node).
__global__ __launch_bounds__(kWaveE * kLayoutWaves) void k_chunks(const BlockLay *lay, const RansNode *rnodes,
                                                                uint32_t nb, uint32_t chunk_log2,
                                                                RansJob *jobs) {
  const uint32_t wave = threadIdx.x >> 6, lane = __lane_id();
  const uint32_t b = blockIdx.x * kLayoutWaves + wave;
  if (b >= nb) return;
  const BlockLay &L = lay[b];
  const uint32_t C = 1u << chunk_log2;
  for (uint32_t r = lane; r < L.n_rnodes; r += kWaveE) {
    const RansNode rn = rnodes[255ull * b + r];
    uint32_t k = 0;
    for (uint32_t st = 0; st < rn.nv; st += C, ++k) {
      RansJob j;
      j.bmp_word = L.rbm_off + rn.rword + st / 32;
      j.slot = L.slot0 + rn.sl0 + static_cast<uint64_t>(k) * slot_size(C);
      j.nbits = rn.nv - st < C ? rn.nv - st : C;
      j.p1q = rn.p1q;
      j.block = b;
      j.rnode = r;
      j.first = st == 0;
      j.dst = 0;
      jobs[L.chunk0 + rn.ch0 + k] = j;
    }
  }
}

// One wave per chunk (persistent over the job list): encode steps k = K-1 ..
// 0; within a step the lanes push their renormalisation words in the order
// lane 31 .. 0, the reverse of the decoder's read order, so the decoder reads
// the pushed words backwards.
__global__ __launch_bounds__(256) void k_rans_enc(const RansJob *jobs, const Totals *tot,
                                                  const uint32_t *bmp, uint8_t *slots,
                                                  uint32_t *sizes) {
  const uint32_t lane = __lane_id();
  const uint64_t njobs = tot->chunks;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (256 / kWaveE);
  for (uint64_t j = blockIdx.x * (256 / kWaveE) + (threadIdx.x >> 6); j < njobs; j += nwaves) {
    const RansJob J = jobs[j];
    const uint32_t f0 = kRansM - J.p1q, f1 = J.p1q;
    const uint32_t K = (J.nbits + 31) / 32;
    uint8_t *slot = slots + J.slot;
    uint16_t *words = reinterpret_cast<uint16_t *>(slot + kChunkHdr);
    const uint32_t *bits = bmp + J.bmp_word;
    uint32_t x = kRansL;
    uint32_t pos = 0;
    const uint64_t gt = lane < 63 ? ~((2ull << lane) - 1) : 0ull;   // lanes above this one
    for (uint32_t k = K; k-- > 0;) {
      const uint32_t w = bits[k];
      const bool act = lane < kRansLanes && 32 * k + lane < J.nbits;
      const bool bit = act && ((w >> (lane & 31)) & 1);
      const uint32_t f = bit ? f1 : f0;
      const bool need = act && x >= (f << 20);
      const uint64_t m = __ballot(need);
      if (need) {
        words[pos + __popcll(m & gt)] = static_cast<uint16_t>(x & 0xFFFF);
        x >>= 16;
      }
      pos += __popcll(m);
      if (act) x = (x / f) * kRansM + (x % f) + (bit ? f0 : 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    __builtin_amdgcn_wave_barrier();
    // reverse the pushed words in place: decoder order
    for (uint32_t i = lane; i < pos / 2; i += kWaveE) {
      const uint16_t a = words[i], c = words[pos - 1 - i];
      words[i] = c;
      words[pos - 1 - i] = a;
    }
    if (lane == 0) *reinterpret_cast<uint32_t *>(slot) = pos;
    if (lane < kRansLanes) reinterpret_cast<uint32_t *>(slot)[1 + lane] = x;
    const uint32_t used = kChunkHdr + 2 * pos, size = (used + 3) & ~3u;
    if (lane < size - used) slot[used + lane] = 0;
    if (lane == 0) sizes[j] = size;
    __builtin_amdgcn_wave_barrier();
  }
}

// Byte tANS coding of the chunk jobs (ans_mode 3, Sec. 5.2), a half-wave
// per chunk (persistent over pairs of jobs).  Cursor l of a chunk codes its
// bytes l, l + 32, ... (XOR 0xFF when the marker says complemented) last
// first, from state 2^11: with n = norm(b), the step emits the low nb bits
// of the state, nb the smallest count with (state >> nb) < 2n (11 - k or
// 10 - k for 2^k <= n < 2^(k+1)), and moves to 2^11 + the (state >> nb) -
// n'th state of b.  A first pass finds the cursor's bit count; its stream
// starts after the 128-byte header and the streams of the cursors before it,
// and a second pass writes the bits backwards from the stream's end (the
// decoder reads step 0's bits first).  The table (norm, first, state) sits
// in LDS, reloaded when a half's table changes.
constexpr uint32_t kFseEncNT = 256;
__global__ __launch_bounds__(kFseEncNT) void k_fse_enc(const RansJob *jobs, const Totals *tot,
                                                       const uint32_t *bmp, const uint16_t *enc,
                                                       uint8_t *slots, uint32_t *sizes, uint32_t *err) {
  __shared__ uint16_t tabs[kFseEncNT / kWaveE][2][kFseEncWords];
  const uint32_t lane = __lane_id(), half = lane >> 5, hl = lane & 31;
  const uint32_t wave = threadIdx.x >> 6;
  const uint64_t njobs = tot->chunks;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (kFseEncNT / kWaveE);
  uint16_t *E = tabs[wave][half];
  uint32_t loaded = 0;
  for (uint64_t pr = blockIdx.x * (kFseEncNT / kWaveE) + wave; 2 * pr < njobs; pr += nwaves) {
    const uint64_t j = 2 * pr + half;
    const bool has = j < njobs;
    RansJob J{};
    if (has) J = jobs[j];
    const uint32_t t = has ? J.p1q & 0x7F : 0u;
    const uint32_t flip = (J.p1q & 0x80) ? 0xFFu : 0u;
    const uint32_t ta = __builtin_amdgcn_readlane(t, 0), tb = __builtin_amdgcn_readlane(t, 32);
    const uint32_t la = __builtin_amdgcn_readlane(loaded, 0), lb = __builtin_amdgcn_readlane(loaded, 32);
    const bool ra = ta && ta != la, rb = tb && tb != lb;
    if (ra || rb) {
      if (half ? rb : ra) {
        const uint4 *src = reinterpret_cast<const uint4 *>(enc + static_cast<uint64_t>(t - 1) * kFseEncWords);
        uint4 *dst = reinterpret_cast<uint4 *>(E);
        constexpr uint32_t n16 = kFseEncWords * 2 / 16;
        for (uint32_t i = hl; i < n16; i += 32) dst[i] = src[i];
        loaded = t;
      }
      wave_sync();
    }
    const uint16_t *norm = E, *first = E + 256, *state = E + 512;
    const uint8_t *bm = reinterpret_cast<const uint8_t *>(bmp + J.bmp_word);
    const uint32_t cb = (J.nbits + 7) >> 3;
    const uint32_t steps = has && cb > hl ? (cb - hl + 31) >> 5 : 0u;
    // pass 1: the cursor's bit count and final state
    uint32_t x = kFseSize, tbits = 0;
    for (uint32_t i = steps; i-- > 0;) {
      const uint32_t b = bm[hl + 32 * i] ^ flip;
      const uint32_t n = norm[b];
      const uint32_t k = 31 - __builtin_clz(n);
      const uint32_t nb = kFseLog - k - (x < (n << (kFseLog - k)) ? 1u : 0u);
      x = kFseSize + state[first[b] + (x >> nb) - n];
      tbits += nb;
    }
    const uint32_t len = (tbits + 7) >> 3;
    if (len > 0xFFFF) atomicCAS(err, 0u, kErrUnsupported);
    uint32_t incl = wave_incl_scan(len);
    const uint32_t lo = __builtin_amdgcn_readlane(incl, 31), all = __builtin_amdgcn_readlane(incl, 63);
    if (half) incl -= lo;
    const uint32_t total = half ? all - lo : lo;     // stream bytes of this half's chunk
    uint8_t *slot = slots + J.slot;
    uint8_t *sp = slot + kFseChunkHdr + (incl - len);
    // pass 2: the same steps, bits written from the stream's end backwards
    uint32_t acc = 0, accn = 8 * len - tbits, top = len, x2 = kFseSize;
    for (uint32_t i = steps; i-- > 0;) {
      const uint32_t b = bm[hl + 32 * i] ^ flip;
      const uint32_t n = norm[b];
      const uint32_t k = 31 - __builtin_clz(n);
      const uint32_t nb = kFseLog - k - (x2 < (n << (kFseLog - k)) ? 1u : 0u);
      acc = (acc << nb) | (x2 & ((1u << nb) - 1));
      accn += nb;
      x2 = kFseSize + state[first[b] + (x2 >> nb) - n];
      while (accn >= 8) {
        --top;
        sp[top] = static_cast<uint8_t>(acc >> (accn - 8));
        accn -= 8;
      }
    }
    if (has) {
      reinterpret_cast<uint16_t *>(slot)[hl] = static_cast<uint16_t>(x - kFseSize);
      reinterpret_cast<uint16_t *>(slot)[kFseLanes + hl] = static_cast<uint16_t>(len);
      const uint32_t used = kFseChunkHdr + total, size = (used + 3) & ~3u;
      if (hl < size - used) slot[used + hl] = 0;
      if (hl == 0) sizes[j] = size;
    }
  }
}

// Block sizes (one thread per block): header, raw bodies, then every rANS
// node at a multiple of 4 bytes with its 8-byte header and its chunks; the
// chunks' places in the block go to their jobs, comp_size to the header.
__global__ __launch_bounds__(256) void k_sizes(BlockLay *lay, RansNode *rnodes, RansJob *jobs,
                                               const uint32_t *sizes, uint32_t nb, uint32_t chunk_log2,
                                               uint8_t *hdr) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  BlockLay &L = lay[b];
  const uint32_t C = 1u << chunk_log2;
  uint64_t off = static_cast<uint64_t>(L.hlen) + L.raw_bytes;
  for (uint32_t r = 0; r < L.n_rnodes; ++r) {
    RansNode &rn = rnodes[255ull * b + r];
    off = (off + 3) & ~3ull;
    rn.boff = static_cast<uint32_t>(off);
    off += 8;
    const uint32_t nch = (rn.nv + C - 1) / C;
    uint32_t blen = 0;
    for (uint32_t k = 0; k < nch; ++k) {
      const uint64_t j = L.chunk0 + rn.ch0 + k;
      jobs[j].dst = static_cast<uint32_t>(off + blen);
      blen += sizes[j];
    }
    rn.blen = blen;
    off += blen;
  }
  L.comp = static_cast<uint32_t>(off);
  *reinterpret_cast<uint32_t *>(hdr + static_cast<uint64_t>(b) * kHdrStride) = static_cast<uint32_t>(off);
}

// Stream offsets of the blocks (one workgroup): each block starts at a
// multiple of 4 bytes after the header and the two offset tables.
__global__ __launch_bounds__(kScanNT) void k_scan2(BlockLay *lay, uint32_t nb, Totals *tot) {
  __shared__ uint64_t part[kScanNT];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (nb + kScanNT - 1) / kScanNT;
  const uint32_t b0 = tid * per, b1 = b0 + per < nb ? b0 + per : nb;
  uint64_t v = 0;
  for (uint32_t b = b0; b < b1; ++b) v += (static_cast<uint64_t>(lay[b].comp) + 3) & ~3ull;
  part[tid] = v;
  __syncthreads();
  for (uint32_t off = 1; off < kScanNT; off <<= 1) {
    const uint64_t a = tid >= off ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += a;
    __syncthreads();
  }
  const uint64_t tab = kHeaderBytes + 16ull * (nb + 1);
  uint64_t run = tab + part[tid] - v;
  for (uint32_t b = b0; b < b1; ++b) {
    lay[b].out_off = run;
    run += (static_cast<uint64_t>(lay[b].comp) + 3) & ~3ull;
  }
  if (tid == kScanNT - 1) tot->out_bytes = tab + part[tid];
}

// Stream header and the two offset tables (block offsets, scratch-word
// offsets), nothing written past out_cap.
__global__ __launch_bounds__(256) void k_stream_head(const BlockLay *lay, const Totals *tot, uint32_t nb,
                                                     uint64_t n, uint32_t bs, uint32_t max_len,
                                                     uint32_t chunk_log2, uint32_t version, uint8_t *out,
                                                     uint64_t out_cap) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (tot->out_bytes > out_cap) return;
  uint64_t *boff = reinterpret_cast<uint64_t *>(out + kHeaderBytes);
  uint64_t *aoff = boff + nb + 1;
  if (t <= nb) {
    boff[t] = t < nb ? lay[t].out_off : tot->out_bytes;
    aoff[t] = t < nb ? lay[t].ans0 : tot->ans_words;
  }
  if (t == 0) {
    uint32_t *h = reinterpret_cast<uint32_t *>(out);
    h[0] = kMagic;
    h[1] = version;                                   // version (1 or 2) | flags << 16
    h[2] = static_cast<uint32_t>(n);
    h[3] = static_cast<uint32_t>(n >> 32);
    h[4] = bs;
    h[5] = nb;
    h[6] = (max_len & 255) | ((chunk_log2 & 255) << 8);
    h[7] = 0;
    h[8] = static_cast<uint32_t>(tot->ans_words);
    h[9] = static_cast<uint32_t>(tot->ans_words >> 32);
    h[10] = 0;
    h[11] = 0;
  }
}

// Block header and raw image, as aligned 4-byte words (workgroup s of block b
// writes words [s kAsmSeg, (s + 1) kAsmSeg) of them): a word inside the raw
// bodies is a byte funnel of two image words, words at the edges are built
// byte by byte (bytes past the raw bodies are zero: the padding before the
// first rANS body or the next block).
__global__ __launch_bounds__(256) void k_assemble(const BlockLay *lay, const Totals *tot, uint32_t nb,
                                                  uint32_t segs, const uint8_t *hdr, const uint8_t *imgb,
                                                  uint8_t *out, uint64_t out_cap) {
  const uint32_t b = blockIdx.x / segs, s = blockIdx.x % segs;
  if (b >= nb || tot->out_bytes > out_cap) return;
  const BlockLay &L = lay[b];
  const uint32_t hlen = L.hlen;
  const uint64_t used = static_cast<uint64_t>(hlen) + L.raw_bytes;
  const uint64_t W = (used + 3) / 4;
  const uint64_t w0 = static_cast<uint64_t>(s) * kAsmSeg;
  if (w0 >= W) return;
  const uint64_t w1 = w0 + kAsmSeg < W ? w0 + kAsmSeg : W;
  const uint8_t *H = hdr + static_cast<uint64_t>(b) * kHdrStride;
  const uint8_t *img = imgb + L.img_off;
  const uint32_t *img32 = reinterpret_cast<const uint32_t *>(imgb);
  uint32_t *o32 = reinterpret_cast<uint32_t *>(out + L.out_off);
  for (uint64_t q = w0 + threadIdx.x; q < w1; q += 256) {
    const uint64_t x0 = 4 * q;
    uint32_t w;
    if (x0 + 4 <= hlen) {
      w = *reinterpret_cast<const uint32_t *>(H + x0);
    } else if (x0 >= hlen && x0 + 4 <= used) {
      const uint64_t so = L.img_off + (x0 - hlen);
      w = __builtin_amdgcn_alignbyte(img32[(so >> 2) + 1], img32[so >> 2], static_cast<uint32_t>(so & 3));
    } else {
      w = 0;
      for (uint32_t e = 0; e < 4; ++e) {
        const uint64_t x = x0 + e;
        const uint32_t v = x < hlen ? H[x] : x < used ? img[x - hlen] : 0u;
        w |= v << (8 * e);
      }
    }
    o32[q] = w;
  }
}

// rANS bodies: one wave per chunk copies its slot into the block; the first
// chunk of a node also writes the node's 8-byte body header.
__global__ __launch_bounds__(256) void k_assemble_rans(const BlockLay *lay, const RansNode *rnodes,
                                                       const RansJob *jobs, const uint32_t *sizes,
                                                       const Totals *tot, const uint8_t *slots,
                                                       uint8_t *out, uint64_t out_cap) {
  const uint32_t lane = __lane_id();
  if (tot->out_bytes > out_cap) return;
  const uint64_t njobs = tot->chunks;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (256 / kWaveE);
  for (uint64_t j = blockIdx.x * (256 / kWaveE) + (threadIdx.x >> 6); j < njobs; j += nwaves) {
    const RansJob J = jobs[j];
    const BlockLay &L = lay[J.block];
    uint8_t *dst = out + L.out_off + J.dst;
    if (J.first && lane == 0) {
      const RansNode &rn = rnodes[255ull * J.block + J.rnode];
      uint32_t *h = reinterpret_cast<uint32_t *>(dst - 8);
      h[0] = J.p1q;                                    // p1q u16, pad u16
      h[1] = rn.blen;
    }
    const uint32_t *src = reinterpret_cast<const uint32_t *>(slots + J.slot);
    uint32_t *d32 = reinterpret_cast<uint32_t *>(dst);
    const uint32_t nw = sizes[j] / 4;
    for (uint32_t i = lane; i < nw; i += kWaveE) d32[i] = src[i];
  }
}

// The call's result on the device: the stream length (also when it exceeds
// out_cap, in which case nothing was written) and a status.
__global__ void k_finish(const Totals *tot, const uint32_t *err, uint64_t out_cap, uint64_t *d_len,
                         int32_t *d_status) {
  if (threadIdx.x != 0) return;
  const uint64_t n = tot->out_bytes;
  const uint32_t e = *err;
  *d_len = n;
  *d_status = e == kErrArg ? PIVCO_E_ARG : e ? PIVCO_E_UNSUPPORTED : n > out_cap ? PIVCO_E_CAPACITY : PIVCO_OK;
}

// The stream of an empty input: header and the two one-entry tables.
struct EmptyStream {
  uint32_t w[16];
};
__global__ void k_empty(EmptyStream h, uint8_t *out, uint64_t out_cap, uint64_t *d_len, int32_t *d_status) {
  const uint32_t t = threadIdx.x;
  const bool fits = out_cap >= sizeof(h.w);
  if (t < 16 && fits) reinterpret_cast<uint32_t *>(out)[t] = h.w[t];
  if (t == 0) {
    *d_len = sizeof(h.w);
    *d_status = fits ? PIVCO_OK : PIVCO_E_CAPACITY;
  }
}

__global__ void k_zero_words(uint32_t *p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

bool opts_ok(const pivco_encode_opts *o) {
  return o && o->block_size >= 1 && o->block_size <= (1u << 30) && o->max_len >= 1 &&
         o->max_len <= kMaxLenGpu && o->ans_mode <= 3 && o->rans_chunk_log2 >= 5 &&
         o->rans_chunk_log2 <= 24 && (o->ans_mode != 3 || o->rans_chunk_log2 >= 8) &&
         o->tree_shape <= 1 && o->reserved == 0;
}

struct WsLayout {
  uint64_t hist, slh, lenm, modes, eb, lay, rnodes, hdr, img, rbm, jobs, sizes, slots, tot, stat, total;
};

// Sizes from n and the options alone (the data is not known yet): every
// area is bounded by the code-length limit and the block count.
WsLayout ws_layout(uint64_t n, const pivco_encode_opts *o) {
  WsLayout L{};
  const uint64_t nb = div_up(n, o->block_size);
  const uint64_t spb = div_up(o->block_size, kHistSlice);
  const uint64_t C = 1ull << o->rans_chunk_log2;
  const uint64_t bits = n * o->max_len;
  const uint64_t chunks = o->ans_mode ? bits / C + nb * 255 + 1 : 0;
  uint64_t x = 0;
  L.hist = x; x = align_up(x + nb * 1024 + 16, 256);
  L.slh = x; x = align_up(x + nb * spb * 1024 + 16, 256);
  L.lenm = x; x = align_up(x + nb * 256 + 16, 256);
  L.modes = x; x = align_up(x + nb * 4 + 16, 256);
  L.eb = x; x = align_up(x + nb * sizeof(EncBlock), 256);
  L.lay = x; x = align_up(x + nb * sizeof(BlockLay), 256);
  L.rnodes = x; x = align_up(x + (o->ans_mode ? nb * 255 * sizeof(RansNode) : 0), 256);
  L.hdr = x; x = align_up(x + nb * kHdrStride, 256);
  L.img = x; x = align_up(x + bits / 8 + nb * (255 + 32) + 64, 256);
  L.rbm = x; x = align_up(x + (o->ans_mode ? 4 * (bits / 32 + nb * (255 + 4)) : 0) + 64, 256);
  L.jobs = x; x = align_up(x + chunks * sizeof(RansJob), 256);
  L.sizes = x; x = align_up(x + chunks * 4, 256);
  L.slots = x; x = align_up(x + (o->ans_mode ? 2 * bits + chunks * 160 : 0) + 64, 256);
  L.tot = x; x = align_up(x + sizeof(Totals), 256);
  L.stat = x; x = align_up(x + 64, 256);     // error word, then the synchronous call's length and status
  L.total = x;
  return L;
}

#define HIPCHK(x) do { if ((x) != hipSuccess) return PIVCO_E_DEVICE; } while (0)

}  // namespace

uint64_t encode_bound(uint64_t n, const pivco_encode_opts *o) {
  if (!opts_ok(o)) return 0;
  const uint64_t nb = div_up(n, o->block_size);
  const uint64_t C = 1ull << o->rans_chunk_log2;
  const uint64_t bits = n * o->max_len;
  uint64_t b = kHeaderBytes + 16 * (nb + 1) + nb * (12 + 128 + 32 + 4 * 255 + 8);
  if (o->ans_mode == 0) b += bits / 8 + nb * 255;
  else b += 2 * bits + nb * 255 * (12 + 136) + 136 * (bits / C + 1);
  return b;
}

uint64_t encode_workspace(uint64_t n, const pivco_encode_opts *o) {
  if (!opts_ok(o)) return 0;
  return ws_layout(n, o).total;
}

namespace {

// Enqueues a whole encode on s: no host wait.  The stream length and the
// call's status go to d_len and d_status on the device.
pivco_status encode_enqueue(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap, uint64_t *d_len,
                            int32_t *d_status, const pivco_encode_opts *o, void *d_ws, uint64_t ws_bytes,
                            hipStream_t s) {
  if (!opts_ok(o) || (n && !d_in) || !d_out || !d_len || !d_status) return PIVCO_E_ARG;
  if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 15))
    return PIVCO_E_ARG;
  if (o->tree && !tree_is_complete(o->tree->code_len, o->max_len)) return PIVCO_E_ARG;
  const uint64_t bs = o->block_size;
  const uint64_t nb64 = div_up(n, bs);
  const uint64_t spb64 = div_up(bs, kHistSlice);
  if (nb64 > 0xFFFFFFFFull || nb64 * spb64 > 0x7FFFFFFFull) return PIVCO_E_ARG;
  const uint32_t nb = static_cast<uint32_t>(nb64), spb = static_cast<uint32_t>(spb64);
  const uint32_t flags = o->ans_mode == 3 ? 1u : 0u;
  const uint32_t version = o->tree_shape ? 2u : 1u;
  uint8_t *out = static_cast<uint8_t *>(d_out);
  if (nb == 0) {                         // header and the two one-entry tables
    EmptyStream h{};
    h.w[0] = kMagic;
    h.w[1] = version | (flags << 16);
    h.w[4] = static_cast<uint32_t>(bs);
    h.w[6] = (o->max_len & 255) | ((o->rans_chunk_log2 & 255) << 8);
    h.w[12] = static_cast<uint32_t>(sizeof(h.w));     // block_off[0] = the stream size
    hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, h, out, out_cap, d_len, d_status);
    HIPCHK(hipGetLastError());
    return PIVCO_OK;
  }
  const WsLayout L = ws_layout(n, o);
  if (ws_bytes < L.total || !d_ws) return PIVCO_E_CAPACITY;
  const FseTables *ft = nullptr;
  if (o->ans_mode == 3 && !(ft = fse_tables())) return PIVCO_E_DEVICE;   // copied once per device
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  const uint8_t *in = static_cast<const uint8_t *>(d_in);
  Totals *dtot = reinterpret_cast<Totals *>(ws + L.tot);
  BlockLay *dlay = reinterpret_cast<BlockLay *>(ws + L.lay);
  EncBlock *deb = reinterpret_cast<EncBlock *>(ws + L.eb);
  RansNode *drn = reinterpret_cast<RansNode *>(ws + L.rnodes);
  RansJob *djobs = reinterpret_cast<RansJob *>(ws + L.jobs);
  uint32_t *dsizes = reinterpret_cast<uint32_t *>(ws + L.sizes);
  uint32_t *derr = reinterpret_cast<uint32_t *>(ws + L.stat);
  uint8_t *dlenm = ws + L.lenm;
  uint32_t *dmodes = reinterpret_cast<uint32_t *>(ws + L.modes);

  // 1. histograms of the blocks and of their slices
  uint32_t *dh = reinterpret_cast<uint32_t *>(ws + L.hist);
  uint32_t *dslh = reinterpret_cast<uint32_t *>(ws + L.slh);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, derr, 1u);
  hipLaunchKernelGGL(k_fill_zero, dim3(std::min<uint64_t>(4096, div_up(nb64 * 256, 256))), dim3(256), 0, s,
                     dh, nb64 * 256);
  hipLaunchKernelGGL(k_hist, dim3(nb * spb), dim3(256), 0, s, in, n, static_cast<uint32_t>(bs), spb, dh, dslh);
  HIPCHK(hipGetLastError());
  if (spb > 1) hipLaunchKernelGGL(k_slice_prefix, dim3(nb), dim3(256), 0, s, dslh, spb, dh);

  // 2. code lengths (package-merge per block, or the supplied tree)
  pivco_tree tree{};
  if (o->tree) tree = *o->tree;
  hipLaunchKernelGGL(k_tree, dim3(nb), dim3(kWaveE), 0, s, dh, nb, o->max_len, tree, o->tree ? 1u : 0u,
                     dlenm, dmodes, derr);
  HIPCHK(hipGetLastError());

  // 3.-4. layout and offsets
  const uint32_t gl = (nb + kLayoutWaves - 1) / kLayoutWaves;
  hipLaunchKernelGGL(k_layout, dim3(gl), dim3(kWaveE * kLayoutWaves), 0, s, dlenm, dmodes, dh, nb, n,
                     static_cast<uint32_t>(bs), o->ans_mode, o->rans_chunk_log2, o->tree_shape,
                     ft ? ft->dmax : nullptr, deb, dlay, drn, ws + L.hdr);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanNT), 0, s, dlay, nb, dtot);
  uint32_t *dimg = reinterpret_cast<uint32_t *>(ws + L.img);
  uint32_t *drbm = reinterpret_cast<uint32_t *>(ws + L.rbm);
  hipLaunchKernelGGL(k_zero_areas, dim3(4096), dim3(256), 0, s, dimg, drbm, dtot);
  HIPCHK(hipGetLastError());

  // 5. bitmaps
  hipLaunchKernelGGL(k_split, dim3(nb * spb), dim3(kSplitNT), 0, s, in, deb, dlay, nb, spb, dslh, dimg, drbm);
  HIPCHK(hipGetLastError());

  // 6. entropy-coded chunks
  const bool ans = o->ans_mode != 0;
  if (ans) {
    hipLaunchKernelGGL(k_chunks, dim3(gl), dim3(kWaveE * kLayoutWaves), 0, s, dlay, drn, nb,
                       o->rans_chunk_log2, djobs);
    if (ft)
      hipLaunchKernelGGL(k_fse_enc, dim3(2048), dim3(kFseEncNT), 0, s, djobs, dtot, drbm, ft->enc,
                         ws + L.slots, dsizes, derr);
    else
      hipLaunchKernelGGL(k_rans_enc, dim3(2048), dim3(256), 0, s, djobs, dtot, drbm, ws + L.slots, dsizes);
    HIPCHK(hipGetLastError());
  }

  // 7. sizes and offsets
  hipLaunchKernelGGL(k_sizes, dim3((nb + 255) / 256), dim3(256), 0, s, dlay, drn, djobs, dsizes, nb,
                     o->rans_chunk_log2, ws + L.hdr);
  hipLaunchKernelGGL(k_scan2, dim3(1), dim3(kScanNT), 0, s, dlay, nb, dtot);

  // 8. the stream (nothing is written when it would not fit)
  hipLaunchKernelGGL(k_stream_head, dim3((nb + 1 + 255) / 256), dim3(256), 0, s, dlay, dtot, nb, n,
                     static_cast<uint32_t>(bs), o->max_len, o->rans_chunk_log2, version | (flags << 16), out,
                     out_cap);
  const uint64_t max_words = (kHdrStride + bs * o->max_len / 8 + 255 + 4) / 4 + 1;
  const uint32_t segs = static_cast<uint32_t>(div_up(max_words, kAsmSeg));
  if (static_cast<uint64_t>(nb) * segs > 0x7FFFFFFFull) return PIVCO_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_assemble, dim3(nb * segs), dim3(256), 0, s, dlay, dtot, nb, segs, ws + L.hdr,
                     ws + L.img, out, out_cap);
  if (ans)
    hipLaunchKernelGGL(k_assemble_rans, dim3(2048), dim3(256), 0, s, dlay, drn, djobs, dsizes, dtot,
                       ws + L.slots, out, out_cap);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, dtot, derr, out_cap, d_len, d_status);
  HIPCHK(hipGetLastError());
  return PIVCO_OK;
}

}  // namespace

pivco_status encode_stream_async(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                                 uint64_t *d_out_len, int32_t *d_status, const pivco_encode_opts *o,
                                 void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  return encode_enqueue(d_in, n, d_out, out_cap, d_out_len, d_status, o, d_ws, ws_bytes, s);
}

pivco_status encode_stream(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                           uint64_t *h_out_len, const pivco_encode_opts *o, void *d_ws,
                           uint64_t ws_bytes, hipStream_t s) {
  if (!opts_ok(o) || !h_out_len || !d_ws) return PIVCO_E_ARG;
  const WsLayout L = ws_layout(n, o);
  if (ws_bytes < L.total) return PIVCO_E_CAPACITY;
  // the result words sit in the workspace's status area
  uint8_t *res = static_cast<uint8_t *>(d_ws) + L.stat + 16;
  uint64_t *d_len = reinterpret_cast<uint64_t *>(res);
  int32_t *d_st = reinterpret_cast<int32_t *>(res + 8);
  const pivco_status st = encode_enqueue(d_in, n, d_out, out_cap, d_len, d_st, o, d_ws, ws_bytes, s);
  if (st) return st;
  struct {
    uint64_t len;
    int32_t status, pad;
  } r{};
  HIPCHK(hipMemcpyAsync(&r, res, 16, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (r.status) return static_cast<pivco_status>(r.status);
  *h_out_len = r.len;
  return PIVCO_OK;
}

}  // namespace pivco
