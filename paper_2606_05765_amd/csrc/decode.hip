// decode.hip -- gfx950 kernels for PivCo-Huffman decoding.
//
// Decoding follows the bottom-up scheme of the paper (Sec. 3): every internal
// node of the code tree produces the dense symbol sequence of its subtree by
// merging its two children's sequences under control of its bitmap
// (out[j] = bit_j ? right[#ones before j] : left[#zeros before j]); a leaf
// child contributes a constant.  The root's sequence is the block's output.
//
// GPU mapping (one workgroup per block, persistent over a work queue):
//   1. parse the block header: code lengths -> canonical code tree (the
//      internal nodes of a canonical tree at depth d are exactly the prefixes
//      [fc(d) + cnt(d), 2^d)), per-node symbol counts from the stored counts
//      of 1 bits, body offsets;
//   2. copy every node bitmap of the block into LDS with 16-byte loads
//      (entropy-coded nodes come from the scratch the rANS kernel wrote);
//   3. for each tile of T output symbols:
//      count phase, top-down by level: each node's share of the tile is
//        popcounted from its bitmap; the tile's bits are staged dword-aligned
//        together with a running popcount per 32-bit word (a rank directory);
//      merge phase, bottom-up by level: a lane makes 4 output bytes from 4
//        bitmap bits, their rank (directory + popcount), two unaligned 4-byte
//        LDS windows of the children's sequences and one v_perm_b32 whose
//        selector comes from a 16-entry table indexed by the 4 bits; the
//        root level stores straight to global memory.
// A second kernel decodes the rANS-coded node bitmaps: 32 interleaved lanes
// per chunk, renormalisation words addressed with ballot + mbcnt.
#include <hip/hip_runtime.h>

#include <utility>

#include "pivco_int.h"

namespace pivco {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void set_err(int32_t *status, int32_t e) {
  atomicCAS(reinterpret_cast<int *>(status), 0, e);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// 32 bits starting at bit position `bit` of a dword array (bits LSB-first).
__device__ __forceinline__ uint32_t bits32_lds(const uint32_t *w, uint32_t bit) {
  const uint32_t q = bit >> 5;
  return __builtin_amdgcn_alignbit(w[q + 1], w[q], bit & 31);
}

// Same from global memory with the dword index bounded by `lim`.
__device__ __forceinline__ uint32_t bits32_glb(const uint32_t *w, uint64_t bit, uint64_t lim) {
  const uint64_t q = bit >> 5;
  const uint32_t lo = q < lim ? w[q] : 0u;
  const uint32_t hi = q + 1 < lim ? w[q + 1] : 0u;
  return __builtin_amdgcn_alignbit(hi, lo, static_cast<uint32_t>(bit & 31));
}

// Unaligned 4-byte window at byte address a of an LDS dword array.
__device__ __forceinline__ uint32_t win4(const uint32_t *buf, uint32_t a) {
  const uint32_t q = a >> 2;
  return __builtin_amdgcn_alignbyte(buf[q + 1], buf[q], a);
}

__device__ __forceinline__ uint32_t load_u8(const uint8_t *p, uint64_t off, uint64_t len) {
  return off < len ? p[off] : 0u;
}

// Wave-wide inclusive scans with DPP (wave64): Hillis-Steele inside each
// 16-lane row (row_shr 1, 2, 4, 8), then row_bcast:15 and row_bcast:31
// carry the row totals to the following rows.  Lanes without a source get
// the identity (0).
template <class Op>
__device__ __forceinline__ uint32_t wave_incl_scan_op(uint32_t v, Op op) {
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false)));
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false)));
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false)));
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false)));
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false)));
  v = op(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false)));
  return v;
}

struct AddOp {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct MaxOp {
  __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) { return wave_incl_scan_op(v, AddOp()); }

// 64-bit sums as two 32-bit scans with the carries of the low half.
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
  const uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
  // low halves are small in every use here (< 2^31 in total): no carry
  return (static_cast<uint64_t>(wave_incl_scan(hi)) << 32) | wave_incl_scan(lo);
}

// tot[0] + ... + tot[n-1] for a wave-uniform n <= 64 (all lanes active):
// lane i reads tot[i], then one wave-wide sum, instead of n dependent reads.
__device__ __forceinline__ uint32_t sum_first(const uint32_t *tot, uint32_t n) {
  const uint32_t x = __lane_id() < n ? tot[__lane_id()] : 0u;
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wave_incl_scan(x)), kWave - 1));
}

// ---------------------------------------------------------------------------
// Block header state shared by the rANS and merge kernels
// ---------------------------------------------------------------------------
// The block's extent and owner: the first 48 bytes of its header state, all
// the merge kernel needs before it loads the rest.
struct BlockExt {
  uint64_t blk;        // byte offset of the block in the stream
  uint64_t end;        // byte offset of the next block
  uint64_t ans_word0;  // absolute scratch word of the block's first rANS node
  uint32_t ans_words;  // scratch words of its rANS nodes
  int32_t err;
  const uint8_t *in;   // the job's stream
  uint32_t job;        // the job's index in the batch
  uint32_t pad;
};

struct BlockHdr {
  uint64_t blk;        // (these seven as in BlockExt)
  uint64_t end;
  uint64_t ans_word0;
  uint32_t ans_words;
  int32_t err;
  const uint8_t *in;
  uint32_t job;
  uint32_t pad;
  uint64_t out_off;    // first output byte of the block
  uint32_t comp, n, mode, csym, cw, I, maxlen, kb;
  uint32_t raw_base, raw_end, n_ans;
  uint32_t kraft;
  uint32_t chunk0, nchunk; // the block's rANS chunks in the batch's chunk list
  uint32_t cnt[17], fc[18], lbase[17], lvl[18];
  uint16_t ci[18];         // per depth: items (leaves and groups; up to 256 in a canonical tree)
  uint8_t gn[18];          // per depth: group nodes (groups of two or more symbols)
  uint8_t nfl[18];         // per level: flat nodes (the level's first nodes)
  uint64_t lvl_total[17];  // bits staged per level (sum of n_v D); set by the merge kernel for streamed blocks
  uint32_t nflat;          // flat nodes of the block (0: binary nodes only)
  uint32_t pad2;           // the node tables start at a multiple of 16 bytes
};
static_assert(offsetof(BlockHdr, job) == offsetof(BlockExt, job) && sizeof(BlockExt) == 48, "BlockExt prefix");

// Per-node tables (breadth-first node ids).
// Field order: what a tile of a split block needs first (bodies, children,
// kinds, depths, flat nodes and their symbols), then the sizes a whole block
// needs, then what only the plan kernel uses; the merge kernel copies only
// the prefix it needs.
struct NodeTab {
  uint32_t boff[256];      // raw: byte offset of the body in the block;
                           // rANS: word offset in the block's scratch
  uint16_t child[256][2];  // internal id, or 0x8000 | symbol for a leaf; a
                           // flat node: 0x8000 | its group's first index in
                           // leafsym, 0x8000 | D (no children)
  uint8_t kind[256];       // 1 = rANS-coded
  uint8_t depth[256];
  uint8_t fd[256];         // flat node: its depth D (>= 2); 0: binary node
  uint8_t leafsym[256];    // symbols ordered by (length, symbol)
  uint32_t nv[256];        // symbols passing the node
  uint32_t nr[256];        // of which go right (1 bits; 0 for a flat node)
  uint8_t len[256];
};

// A block's parsed and validated header, written by the plan kernel and
// copied as is into the merge kernel's LDS.
struct alignas(16) ParsedBlock {
  BlockHdr h;
  NodeTab t;
};
static_assert(sizeof(ParsedBlock) == kParsedBlockBytes, "ParsedBlock layout");
// Bytes of the record a whole block needs (all but the plan kernel's own
// tables) and a tile of a split block needs (its shares come from the
// boundary table, not from the node sizes).
constexpr uint32_t kRecWhole16 = (offsetof(ParsedBlock, t) + offsetof(NodeTab, len) + 15) / 16;
constexpr uint32_t kRecTile16 = (offsetof(ParsedBlock, t) + offsetof(NodeTab, nv) + 15) / 16;
static_assert(offsetof(ParsedBlock, t) % 16 == 0 && offsetof(NodeTab, nv) % 16 == 0 &&
              offsetof(NodeTab, len) % 16 == 0, "record prefixes in 16-byte units");

// Byte readers for block-relative offsets: the block in global memory, or
// a copy of it in LDS.
struct GlbBytes {
  const uint8_t *p;
  __device__ uint32_t u8(uint32_t o) const { return p[o]; }
  __device__ uint32_t u32(uint32_t o) const { return *reinterpret_cast<const uint32_t *>(p + o); }
};
// The block's first hn bytes copied into LDS, the rest read from global memory.
struct SplitBytes {
  const uint8_t *l;
  uint32_t hn;
  const uint8_t *g;
  __device__ uint32_t u8(uint32_t o) const { return o < hn ? l[o] : g[o]; }
  __device__ uint32_t u32(uint32_t o) const {
    return o + 4 <= hn ? *reinterpret_cast<const uint32_t *>(l + o)
                       : u8(o) | (u8(o + 1) << 8) | (u8(o + 2) << 16) | (u8(o + 3) << 24);
  }
};

// Offsets of block b from the stream's tables (thread 0 only).
__device__ void parse_offsets(const JobDev &J, uint32_t b, BlockHdr &h) {
  const uint64_t nb = J.n_blocks;
  const uint64_t *tab = reinterpret_cast<const uint64_t *>(J.in + kHeaderBytes);
  const uint64_t tab_end = kHeaderBytes + 16 * (nb + 1);
  const uint64_t off = tab[b], end = tab[b + 1];
  const uint64_t a0 = tab[nb + 1 + b], a1 = tab[nb + 2 + b];
  int32_t err = 0;
  if (off < tab_end || end < off || end > J.in_len || (off & 3) || end - off < kBlockFixed ||
      end - off > 0xFFFFFFF0ull || a1 < a0 || a1 > J.ans_words || a1 - a0 > 0xFFFFFFFFull)
    err = PIVCO_E_CORRUPT;
  h.blk = off;
  h.end = err ? off : end;
  h.out_off = static_cast<uint64_t>(b) * J.block_size;
  h.ans_word0 = J.scratch_base + a0;
  h.ans_words = err ? 0u : static_cast<uint32_t>(a1 - a0);
  h.err = err;
  h.kraft = 0;
}

// The thread's index, opaque to loop-invariant code motion: the persistent
// merge loop would otherwise keep every LDS address derived from it live
// across items, and spill them.
__device__ __forceinline__ uint32_t item_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// A wave-uniform 64-bit value in scalar registers: the load that produced it
// is waited for here, once, not at its first use inside a loop.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// The wave's index in the workgroup, as a scalar (wave-uniform) value.
__device__ __forceinline__ uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the wave's global loads and stores in flight (the merge
// kernel's waves exchange data through LDS alone).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Parse and validate the rest of the header of block b (offsets already in
// h), run by ONE wave (wave-synchronous, no workgroup barrier); the caller
// synchronises the workgroup afterwards.  On return h.err != 0 or
// h.mode == 1 means the node tables are not filled.
//
// The canonical code is never materialised: with cnt(L) codes of length L
// and fc(L) the first of them, fc(L+1) = 2 (fc(L) + cnt(L)), the internal
// nodes at depth d are the prefixes [fc(d) + cnt(d), 2^d), numbered
// breadth-first; child q of such a node is a leaf iff q < fc(d+1) + cnt(d+1),
// and then it is the (q - fc(d+1))-th symbol of length d+1 by id.  A v2
// stream's flat-subtree tree (Sec. 2.2.3-2.2.4) follows the same closed form
// with its items (single symbols and power-of-two groups of one length) in
// place of the symbols; a group of two is a binary node over two leaves, a
// larger group a flat node.
template <class Rd>
__device__ void parse_block_wave(const JobDev &J, uint32_t b, BlockHdr &h, NodeTab &t, const Rd &rd) {
  const uint32_t lane = lane_id();
  int32_t err = h.err;
  uint32_t mode = 0, csym = 0, cw = 0, comp = 0, n = 0;
  if (!err) {
    comp = rd.u32(0);
    n = rd.u32(4);
    const uint32_t w2 = rd.u32(8);
    mode = w2 & 255; csym = (w2 >> 8) & 255; cw = (w2 >> 16) & 255;
    const uint64_t start = static_cast<uint64_t>(b) * J.block_size;
    const uint64_t want = J.n_total - start < J.block_size ? J.n_total - start : J.block_size;
    if (comp > h.end - h.blk || comp < kBlockFixed || n != want || (w2 >> 24) != 0 ||
        cw != (n <= 65535 ? 2u : 4u))
      err = PIVCO_E_CORRUPT;
    else if (mode == 1) {
      if (comp != kBlockFixed || h.ans_words != 0 || n == 0) err = PIVCO_E_CORRUPT;
    } else if (mode != 0 || csym != 0 || comp < kBlockFixed + kLenTable) {
      err = PIVCO_E_CORRUPT;
    }
  }
  if (lane == 0) { h.comp = comp; h.n = n; h.mode = mode; h.csym = csym; h.cw = cw; h.err = err; }
  if (err || mode == 1) { wave_sync_lds(); return; }
  // code lengths: lane owns symbols 4*lane .. 4*lane+3 (two table bytes)
  const uint32_t lb = rd.u8(kBlockFixed + 2 * lane) | (rd.u8(kBlockFixed + 2 * lane + 1) << 8);
  uint32_t l[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) l[k] = (lb >> (4 * k)) & 15;
  const uint64_t below = (1ull << lane) - 1;
  uint32_t rank[4] = {0, 0, 0, 0};
  // Per-length values are held lane-distributed (lane L holds the value for
  // length or depth L) and copied to h; dynamic lookups read h from LDS.
  uint32_t cnt_l = 0;
  uint32_t kraft = 0, m = 0, maxlen = 0;
#pragma unroll
  for (uint32_t L = 1; L <= 15; ++L) {
    uint64_t mk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mk[k] = __ballot(l[k] == L);
    const uint32_t c = __popcll(mk[0]) + __popcll(mk[1]) + __popcll(mk[2]) + __popcll(mk[3]);
    const uint32_t before = __popcll(mk[0] & below) + __popcll(mk[1] & below) +
                            __popcll(mk[2] & below) + __popcll(mk[3] & below);
    uint32_t own = 0;   // same-length symbols of this lane with a smaller id
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l[k] == L) { rank[k] = before + own; ++own; }
    if (lane == L) cnt_l = c;
    m += c;
    kraft += c << (15 - L);
    if (c) maxlen = L;
  }
  if (maxlen > J.max_len) err = PIVCO_E_CORRUPT;
  else if (m < 2 || kraft != (1u << 15)) err = PIVCO_E_CORRUPT;
  else if (maxlen > kMaxLenGpu) err = PIVCO_E_UNSUPPORTED;
  const bool flat = J.version == 2;
  const uint32_t lbase_l = wave_incl_scan(lane <= 16 ? cnt_l : 0u) - cnt_l;
  // The tree's leaves and groups ("items") per depth: lane d holds the
  // number of items at depth d (ci), of groups of two or more symbols (gn,
  // which are nodes) and of flat ones (nf).  Canonical tree: every symbol is
  // an item.  Flat-subtree tree (Sec. 2.2.4): the symbols of length l are cut
  // by the binary digits of their number cnt(l), largest group first; a
  // group of 2^D hangs at depth l - D, so depth d has one item for each D
  // with bit D of cnt(d + D) set, ordered by D descending.
  uint32_t ci_l = cnt_l, gn_l = 0, nf_l = 0;
  if (flat) {
    ci_l = 0;
#pragma unroll
    for (uint32_t D = 0; D <= 8; ++D) {
      const uint32_t src = lane + D;
      const uint32_t c = static_cast<uint32_t>(__shfl(static_cast<int>(cnt_l), static_cast<int>(src & 63), kWave));
      if (src <= 15 && ((c >> D) & 1)) {
        ++ci_l;
        gn_l += D >= 1 ? 1u : 0u;
        nf_l += D >= 2 ? 1u : 0u;
      }
    }
  }
  const uint64_t has_items = __ballot(lane <= 15 && ci_l != 0);
  const uint32_t maxitem = has_items ? 63u - static_cast<uint32_t>(__clzll(static_cast<long long>(has_items))) : 0u;
  // canonical codes of the items: fc(d+1) = 2 (fc(d) + ci(d)); below the
  // deepest items every other code of a depth is an internal (binary) node;
  // lvl(d) = nodes above depth d (groups of two or more, and internal nodes)
  uint32_t fc_l = 0, lvl_l = 0, fcd = 0, lvd = 0;
#pragma unroll
  for (uint32_t d = 0; d <= 16; ++d) {
    const uint32_t cd = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ci_l), d));
    const uint32_t gd = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(gn_l), d));
    const uint32_t Id = d < maxitem ? (1u << d) - fcd - cd : 0u;
    fcd = 2 * (fcd + cd);
    lvd += gd + Id;
    if (lane == d + 1) { fc_l = fcd; lvl_l = lvd; }
  }
  // node levels: the internal nodes above the deepest items, and the groups
  // at that depth
  const uint32_t gmax = static_cast<uint32_t>(__shfl(static_cast<int>(gn_l), static_cast<int>(maxitem), kWave));
  const uint32_t levels = maxitem + (gmax ? 1u : 0u);
  const uint32_t I = static_cast<uint32_t>(__shfl(static_cast<int>(lvl_l), static_cast<int>(levels), kWave));
  if (!err && (I == 0 || I > kMaxInternal || (!flat && I != m - 1))) err = PIVCO_E_CORRUPT;
  const uint32_t kb = (I + 7) / 8;
  const uint32_t raw_base = kBlockFixed + kLenTable + kb + cw * I;
  if (!err && raw_base > comp) err = PIVCO_E_CORRUPT;
  if (lane < 17) { h.cnt[lane] = cnt_l; h.lbase[lane] = lbase_l; }
  if (lane < 18) {
    h.fc[lane] = fc_l;
    h.lvl[lane] = lvl_l;
    h.ci[lane] = static_cast<uint16_t>(lane <= 15 ? ci_l : 0u);
    h.gn[lane] = static_cast<uint8_t>(gn_l);
    h.nfl[lane] = static_cast<uint8_t>(nf_l);
  }
  const uint32_t nflat = static_cast<uint32_t>(__shfl(static_cast<int>(wave_incl_scan(lane <= 17 ? nf_l : 0u)), kWave - 1, kWave));
  if (lane == 0) {
    h.I = I; h.maxlen = levels; h.kb = kb; h.raw_base = raw_base; h.err = err; h.kraft = kraft;
    h.nflat = nflat;
  }
  if (err) { wave_sync_lds(); return; }
  // symbols in canonical order
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t lb_k = __shfl(lbase_l, l[k], kWave);     // every lane takes part
    if (l[k]) t.leafsym[lb_k + rank[k]] = static_cast<uint8_t>(4 * lane + k);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) t.len[4 * lane + k] = static_cast<uint8_t>(l[k]);
  // node table: lane owns nodes 4*lane .. 4*lane+3.  A node's depth is the
  // number of levels that start at or before it.  At depth d the first
  // gn(d) nodes are the groups, in item order (flat ones first), then the
  // internal nodes, whose codes follow the items'.
  uint32_t dd[4] = {0, 0, 0, 0};
#pragma unroll
  for (uint32_t j = 1; j <= kMaxLenGpu; ++j) {
    const uint32_t lj = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lvl_l), j));
#pragma unroll
    for (int k = 0; k < 4; ++k) dd[k] += (4 * lane + k >= lj) ? 1u : 0u;
  }
  wave_sync_lds();                       // leaf symbols and per-depth values written
  const uint32_t kbase = kBlockFixed + kLenTable;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    if (i >= I) continue;
    const uint32_t d = dd[k];
    const uint32_t r = i - h.lvl[d];
    uint32_t cc = 0, fdv = 0;
    if (r < h.gn[d]) {
      // group r of depth d: the r-th D >= 1 with bit D of cnt(d + D) set, D descending
      uint32_t D = 0, left = r;
      for (uint32_t e = 8; e >= 1; --e) {
        const uint32_t le = d + e;
        if (le <= 15 && ((h.cnt[le] >> e) & 1)) {
          if (left == 0) { D = e; break; }
          --left;
        }
      }
      const uint32_t l0 = d + D;
      const uint32_t first = D ? h.lbase[l0] + (h.cnt[l0] & ~((2u << D) - 1)) : 0u;
      if (D == 0) err = PIVCO_E_CORRUPT;
      else if (D == 1) cc = (0x8000u | t.leafsym[first]) | ((0x8000u | t.leafsym[first + 1]) << 16);
      else { cc = (0x8000u | first) | ((0x8000u | D) << 16); fdv = D; }
    } else {
      const uint32_t p = h.fc[d] + h.ci[d] + (r - h.gn[d]);
      const uint32_t d1 = d + 1;
      // the D = 0 items of depth d+1: canonical tree, every symbol of length
      // d+1; flat-subtree tree, the one symbol left after the groups
      const uint32_t leaf0 = h.lbase[d1] + (flat ? (h.cnt[d1] & ~1u) : 0u);
      for (int bb = 0; bb < 2; ++bb) {
        const uint32_t q = 2 * p + bb;
        const uint32_t rq = q - h.fc[d1];
        const uint32_t c = rq < h.gn[d1] ? h.lvl[d1] + rq
                           : rq < h.ci[d1] ? 0x8000u | t.leafsym[leaf0 + rq - h.gn[d1]]
                                           : h.lvl[d1] + h.gn[d1] + (q - h.fc[d1] - h.ci[d1]);
        cc |= c << (16 * bb);
      }
    }
    *reinterpret_cast<uint32_t *>(t.child[i]) = cc;
    t.depth[i] = static_cast<uint8_t>(d);
    t.fd[i] = static_cast<uint8_t>(fdv);
    t.kind[i] = (rd.u8(kbase + (i >> 3)) >> (i & 7)) & 1;
    const uint32_t co = kbase + kb + cw * i;
    uint32_t nr = rd.u8(co) | (rd.u8(co + 1) << 8);
    if (cw == 4) nr |= (rd.u8(co + 2) << 16) | (rd.u8(co + 3) << 24);
    if (fdv && (nr || t.kind[i])) err = PIVCO_E_CORRUPT;   // a flat node has no 1-bit count and is raw
    t.nr[i] = nr;
  }
  if ((I & 7) && (rd.u8(kbase + (I >> 3)) >> (I & 7))) err = PIVCO_E_CORRUPT;  // unused kind bits
  if (lane == 0) t.nv[0] = n;
  wave_sync_lds();
  // symbol counts top-down, one level at a time (the wave stays in step)
  for (uint32_t d = 0; d < maxlen; ++d) {
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lvl_l), d));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(lvl_l), d + 1));
    for (uint32_t i = lo + lane; i < hi; i += kWave) {
      const uint32_t v = t.nv[i], r = t.nr[i];
      const uint32_t cc = *reinterpret_cast<const uint32_t *>(t.child[i]);
      if (r > v) err = PIVCO_E_CORRUPT;
      const uint32_t rr = r > v ? v : r;
      const uint32_t c0 = cc & 0xFFFF, c1 = cc >> 16;
      if (!(c0 & 0x8000)) t.nv[c0] = v - rr;
      if (!(c1 & 0x8000)) t.nv[c1] = rr;
    }
    wave_sync_lds();
  }
  // body offsets: lane owns nodes 4*lane .. 4*lane+3 (contiguous for the scan)
  uint32_t rawb[4], answ[4], lraw = 0, lans = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    uint32_t rb = 0, aw = 0;
    if (i < I) {
      const uint32_t v = t.nv[i];
      const uint64_t bits = static_cast<uint64_t>(v) * (t.fd[i] ? t.fd[i] : 1u);
      if (t.kind[i]) aw = (v + 31) / 32; else rb = static_cast<uint32_t>((bits + 7) / 8);
    }
    rawb[k] = lraw; answ[k] = lans;
    lraw += rb; lans += aw;
  }
  const uint32_t iraw = wave_incl_scan(lraw), ians = wave_incl_scan(lans);
  const uint32_t xraw = iraw - lraw, xans = ians - lans;
  uint32_t na = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    if (i >= I) continue;
    t.boff[i] = t.kind[i] ? xans + answ[k] : raw_base + xraw + rawb[k];
    na += t.kind[i];
  }
  const uint32_t raw_total = __shfl(iraw, kWave - 1, kWave);
  const uint32_t ans_total = __shfl(ians, kWave - 1, kWave);
  const uint32_t n_ans = __shfl(wave_incl_scan(na), kWave - 1, kWave);
  const uint64_t raw_end = static_cast<uint64_t>(raw_base) + raw_total;
  if (raw_end > comp || ans_total != h.ans_words || (n_ans == 0 && raw_end != comp)) err = PIVCO_E_CORRUPT;
  wave_sync_lds();
  // padding bits of raw bodies must be zero
  if (!err) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = 4 * lane + k;
      const uint64_t bits = i < I ? static_cast<uint64_t>(t.nv[i]) * (t.fd[i] ? t.fd[i] : 1u) : 0u;
      if (i < I && !t.kind[i] && (bits & 7)) {
        const uint32_t last = rd.u8(t.boff[i] + static_cast<uint32_t>(bits >> 3));
        if (last >> (bits & 7)) err = PIVCO_E_CORRUPT;
      }
    }
  }
  const bool any = __ballot(err != 0) != 0;
  if (any) {
    const uint64_t bad = __ballot(err != 0);
    const int src = __ffsll(static_cast<long long>(bad)) - 1;
    err = __shfl(err, src, kWave);
  }
  if (lane == 0) {
    h.raw_end = raw_end > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(raw_end);
    h.n_ans = n_ans;
    h.err = err;
  }
  wave_sync_lds();
}


// ---------------------------------------------------------------------------
// Kernel: rANS decode of entropy-coded node bitmaps into scratch
// ---------------------------------------------------------------------------
// The plan kernel lists every chunk of every rANS node (walk_rans); k_rans
// decodes them two at a time per wave: lanes 0-31 run one chunk's 32
// interleaved states, lanes 32-63 another's.  Per step every active lane
// decodes one bit; lanes whose state fell below 2^16 read the chunk's next
// 16-bit words in lane order (the cursor + their rank in the half-wave's
// ballot) from a window of the chunk's words staged in LDS; the half-wave's
// 32 decoded bits are its part of the ballot of the bits (bit i = lane i).
// A step is a chain of dependent operations (state, ballot, rank, LDS word);
// the step is branch-free and keeps the cursors in registers, so that the
// chain holds no scalar round trip.
constexpr int kRansNT = 256;
constexpr int kRansWin = 2048;        // u16 words per half-wave window in LDS
constexpr uint32_t kRansSteps = 32;   // steps per window check (one output word per lane)

// Lists the entropy-coded chunks of the block parsed in h/t (one lane):
// reserves the block's slots in the batch's list (their number follows
// from the node sizes), then walks the bodies that follow the raw bodies
// once, checking every size and filling the slots (on a corrupt body the
// rest become empty chunks).  A rANS body is u16 probability, u16 zero, u32
// length, then per chunk of 2^chunk_log2 bits a u32 word count, the 32 u32
// lane states and the words, padded to 4 bytes.  In a stream with flags bit
// 0 a body is the tANS marker u8 (table 1..50, 0x80: complemented), u8
// zero, u16 zero, u32 length, then per chunk the 32 u16 cursor states, the
// 32 u16 stream lengths, the streams and zero padding to 4 bytes.  Returns
// a status.
__device__ int32_t walk_rans(const JobDev &J, BlockHdr &h, const NodeTab &t, Counters *ctr,
                             RansChunk *chunks, uint64_t cap) {
  const uint8_t *bp = J.in + h.blk;
  const uint64_t comp = h.comp, C = 1ull << J.chunk_log2;
  const bool fse = J.flags & 1;
  // a node of n_v bits has ceil(n_v / C) chunks: the block's slots are
  // reserved before the walk, which then reads each chunk header once
  uint64_t want = 0;
  for (uint32_t i = 0; i < h.I; ++i)
    if (t.kind[i]) want += (static_cast<uint64_t>(t.nv[i]) + C - 1) / C;
  const uint32_t nch = want > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(want);
  const uint32_t base = atomicAdd(&ctr->rans_chunks, nch);
  if (static_cast<uint64_t>(base) + nch > cap) {
    // slots reserved past the list's capacity stay unused (k_rans reads
    // at most cap); the ones below it become empty chunks
    for (uint64_t f = base; f < cap; ++f) chunks[f] = RansChunk{0, 0, 0, 0, 1, h.job};
    return PIVCO_E_UNSUPPORTED;
  }
  h.chunk0 = base;
  h.nchunk = nch;
  uint32_t k = 0;                        // slots written
  // on a corrupt body the slots not yet written become empty chunks
  auto fail = [&]() {
    for (uint32_t f = k; f < nch; ++f) chunks[base + f] = RansChunk{0, 0, 0, 0, 1, h.job};
    return static_cast<int32_t>(PIVCO_E_CORRUPT);
  };
  uint64_t o = h.raw_end;
  for (uint32_t i = 0; i < h.I; ++i) {
    if (!t.kind[i]) continue;
    while (o & 3) {
      if (o >= comp || bp[o]) return fail();
      ++o;
    }
    if (o + 8 > comp || t.nv[i] == 0) return fail();
    const uint32_t w0 = bp[o] | (bp[o + 1] << 8);
    const uint32_t pad = bp[o + 2] | (bp[o + 3] << 8);
    const uint32_t blen = *reinterpret_cast<const uint32_t *>(bp + o + 4);
    const uint32_t tt = w0 & 0x7F;
    if (pad || o + 8 + blen > comp) return fail();
    if (fse ? ((w0 >> 8) || tt < 1 || tt > kFseTables) : (w0 < 1 || w0 > 4095)) return fail();
    const uint32_t p1q = fse ? kFseTag | w0 : w0;
    const uint64_t body = o + 8;
    uint64_t co = 0;
    const uint64_t nv = t.nv[i];
    for (uint64_t s = 0; s < nv; s += C) {
      uint32_t nw;
      uint64_t size;
      if (fse) {
        if (co + kFseChunkHdr > blen) return fail();
        const uint32_t *lens = reinterpret_cast<const uint32_t *>(bp + body + co + 2 * kFseLanes);
        nw = 0;
        for (uint32_t q = 0; q < kFseLanes / 2; ++q) {
          const uint32_t v = lens[q];
          nw += (v & 0xFFFF) + (v >> 16);
        }
        const uint64_t used = kFseChunkHdr + static_cast<uint64_t>(nw);
        size = (used + 3) & ~3ull;
        if (co + size > blen) return fail();
        for (uint64_t u = used; u < size; ++u)
          if (bp[body + co + u]) return fail();
      } else {
        if (co + kChunkHdr > blen) return fail();
        nw = *reinterpret_cast<const uint32_t *>(bp + body + co);
        size = (kChunkHdr + 2ull * nw + 3) & ~3ull;
        if (nw > C || co + size > blen) return fail();
      }
      RansChunk c;
      c.src = h.blk + body + co;
      c.dst = h.ans_word0 + t.boff[i] + s / 32;
      c.nbits = static_cast<uint32_t>(nv - s < C ? nv - s : C);
      c.nw = nw;
      c.p1q = p1q;
      c.job = h.job;
      chunks[base + k] = c;
      ++k;
      co += size;
    }
    if (co != blen) return fail();
    o = body + blen;
  }
  if (o != comp) return fail();
  return PIVCO_OK;
}

typedef __attribute__((address_space(1))) const uint16_t GlobalCU16;

// v_writelane_b32: lane `lane` of r takes the wave-uniform value v (the lane
// select goes through M0: two SGPR operands would exceed the constant bus).
__device__ __forceinline__ void write_lane(uint32_t &r, uint32_t v, uint32_t lane) {
  asm volatile("v_writelane_b32 %0, %1, m0" : "+v"(r) : "s"(v), "{m0}"(lane));
}
// The same with a lane known at compile time (an inline constant).
template <uint32_t L>
__device__ __forceinline__ void write_lane_i(uint32_t &r, uint32_t v) {
  static_assert(L < 64, "a lane of the wave");
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(r) : "s"(v), "i"(L));
}

// One decode step of both half-waves (lane hl of half h: bit 32 k + hl of
// its chunk); returns the ballot of the decoded bits (half 0 low, half 1
// high).  FULL: every lane of both halves is active.  co is the lane's
// half's cursor relative to its window (words consumed - window start).  A
// lane whose state fell below 2^16 takes the window word at co + its rank
// among the half's such lanes (mbcnt over the half's word of the ballot;
// mbcnt_hi counts nothing for lanes 0-31), and co advances by the half's
// count.  Every lane reads a word, so no branch surrounds the
// renormalisation; the window index is masked, so a corrupt chunk that runs
// past its words reads stale window words and fails the final cursor check.
template <bool FULL>
__device__ __forceinline__ uint64_t rans_step(uint32_t &x, uint32_t &co, uint32_t k, uint32_t hl,
                                              uint32_t half, uint32_t nbits, uint32_t f0, uint32_t f1,
                                              const uint16_t *w) {
  const bool act = FULL || 32 * k + hl < nbits;
  const uint32_t slot = x & (kRansM - 1);
  const bool bit = slot >= f0;
  const uint32_t xn = __umul24(bit ? f1 : f0, x >> 12) + slot - (bit ? f0 : 0u);
  x = act ? xn : x;
  const bool need = act && x < kRansL;
  const uint64_t m = __ballot(need);
  const uint32_t mlo = static_cast<uint32_t>(m), mhi = static_cast<uint32_t>(m >> 32);
  // both halves' forms in every lane, then a select (no divergent branch)
  uint32_t rlo = __builtin_amdgcn_mbcnt_lo(mlo, co), rhi = __builtin_amdgcn_mbcnt_hi(mhi, co);
  uint32_t clo = __popc(mlo) + co, chi = __popc(mhi) + co;
  asm volatile("" : "+v"(rlo), "+v"(rhi), "+v"(clo), "+v"(chi));
  uint32_t wv = w[(half ? rhi : rlo) & (kRansWin - 1)];
  asm volatile("" : "+v"(wv));
  x = need ? ((x << 16) | wv) : x;
  co = half ? chi : clo;
  return __ballot(act && bit);
}

// 32 full steps, unrolled, the ballot of step J into lanes J and 32 + J of stg.
template <size_t... J>
__device__ __forceinline__ void rans_full_group(std::index_sequence<J...>, uint32_t &x, uint32_t &stg,
                                                uint32_t &co, uint32_t hl, uint32_t half, uint32_t f0,
                                                uint32_t f1, const uint16_t *w) {
  ((void)([&] {
     const uint64_t bm = rans_step<true>(x, co, 0, hl, half, 0, f0, f1, w);
     write_lane_i<J>(stg, static_cast<uint32_t>(bm));
     write_lane_i<32 + J>(stg, static_cast<uint32_t>(bm >> 32));
   }()), ...);
}

// Decodes chunks ia (lanes 0-31) and ib (lanes 32-63) of the list; an index
// at or past `end`, or an empty chunk, leaves its half idle.  Every 32 steps
// lane j of a half holds the half's decoded word of step j (the step's
// ballot went into lane j, resp. 32 + j, with v_writelane) and the 32 words
// go out as one coalesced store.
__device__ void rans_pair(const JobDev *jobs, const RansChunk *chunks, uint32_t ia, uint32_t ib,
                          uint32_t end, uint32_t *scratch, uint16_t (*win)[kRansWin]) {
  const uint32_t lane = lane_id(), half = lane >> 5, hl = lane & 31;
  const uint32_t idx = half ? ib : ia;
  RansChunk c = RansChunk{0, 0, 0, 0, 1, 0};
  if (idx < end) c = chunks[idx];
  if (c.p1q & kFseTag) c = RansChunk{0, 0, 0, 0, 1, 0};   // a tANS chunk: k_fse's
  const bool has = c.nbits != 0;
  const uint8_t *base = has ? jobs[c.job].in + c.src : nullptr;
  uint32_t x = has ? reinterpret_cast<const uint32_t *>(base)[1 + hl] : kRansL;
  bool err = has && x < kRansL;
  GlobalCU16 *words = has ? (GlobalCU16 *)(base + kChunkHdr) : nullptr;   // C cast: generic to global
  uint16_t *w = win[half];
  const uint32_t f0 = kRansM - c.p1q, f1 = c.p1q;
  const uint32_t K = (c.nbits + 31) / 32;
  // per-half sizes, wave-uniform
  const uint32_t ka = __builtin_amdgcn_readlane(K, 0), kb = __builtin_amdgcn_readlane(K, 32);
  const uint32_t kmax = ka > kb ? ka : kb;
  const uint32_t nba = __builtin_amdgcn_readlane(c.nbits, 0), nbb = __builtin_amdgcn_readlane(c.nbits, 32);
  const uint32_t nwa = __builtin_amdgcn_readlane(c.nw, 0), nwb = __builtin_amdgcn_readlane(c.nw, 32);
  uint32_t wsa = 0, wsb = 0, wea = 0, web = 0, co = 0;
  uint32_t *dst = scratch + c.dst;
  constexpr uint32_t kAhead = kRansSteps * 32;   // most words a half takes in kRansSteps steps
  static_assert(kAhead <= static_cast<uint32_t>(kRansWin), "a group's words fit the window");
  for (uint32_t k0 = 0; k0 < kmax; k0 += kRansSteps) {
    // the halves' cursors; slide a half's window to its cursor when fewer
    // than kAhead of its words are staged ahead of it (and the chunk has more)
    const uint32_t pa = wsa + __builtin_amdgcn_readlane(co, 0), pb = wsb + __builtin_amdgcn_readlane(co, 32);
    const bool ra = pa + kAhead > wea && wea < nwa, rb = pb + kAhead > web && web < nwb;
    if (ra || rb) {
      if (ra) { wsa = pa < nwa ? pa : nwa; wea = nwa - wsa > kRansWin ? wsa + kRansWin : nwa; }
      if (rb) { wsb = pb < nwb ? pb : nwb; web = nwb - wsb > kRansWin ? wsb + kRansWin : nwb; }
      co = half ? pb - wsb : pa - wsa;
      if (half ? rb : ra) {
        const uint32_t ws = half ? wsb : wsa, nwin = (half ? web : wea) - ws;
        for (uint32_t i0 = 0; i0 < nwin; i0 += 32 * 8) {
          uint16_t v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + 32 * u + hl;
            v[u] = i < nwin ? words[ws + i] : 0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + 32 * u + hl;
            if (i < nwin) w[i] = v[u];
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    uint32_t stg = 0;
    const uint32_t full_bits = 32 * (k0 + kRansSteps);
    if (full_bits <= nba && full_bits <= nbb) {
      rans_full_group(std::make_index_sequence<kRansSteps>(), x, stg, co, hl, half, f0, f1, w);
    } else {
      const uint32_t steps = kmax - k0 < kRansSteps ? kmax - k0 : kRansSteps;
      for (uint32_t j = 0; j < steps; ++j) {
        const uint64_t bm = rans_step<false>(x, co, k0 + j, hl, half, c.nbits, f0, f1, w);
        write_lane(stg, static_cast<uint32_t>(bm), j);
        write_lane(stg, static_cast<uint32_t>(bm >> 32), 32 + j);
      }
    }
    // lane hl of half h: the half's bits of step k0 + hl (lanes past the
    // group's steps hold nothing and store nothing: k0 + hl < K <= k0 + steps)
    if (k0 + hl < K) dst[k0 + hl] = stg;
  }
  if (has) {
    if ((half ? wsb : wsa) + co != c.nw || x != kRansL) err = true;
    const uint32_t used = kChunkHdr + 2 * c.nw, size = (used + 3) & ~3u;
    if (hl < size - used && base[used + hl] != 0) err = true;
  }
  const uint64_t e = __ballot(err);
  const uint32_t eh = half ? static_cast<uint32_t>(e >> 32) : static_cast<uint32_t>(e);
  if (hl == 0 && eh) set_err(jobs[c.job].status, PIVCO_E_CORRUPT);
}

// Decodes the batch's listed chunks, a pair per wave from a shared counter;
// or, for single >= 0, only the chunks of block ritems[single] with one
// workgroup (the per-block launch mode).
__global__ __launch_bounds__(kRansNT) void k_rans(const JobDev *jobs, const ParsedBlock *recs,
                                                   const uint2 *ritems, Counters *ctr,
                                                   const RansChunk *chunks, uint64_t cap,
                                                   uint32_t *scratch, int32_t single) {
  __shared__ uint16_t win[kRansNT / kWave][2][kRansWin];
  const uint32_t wave = wave_id();
  constexpr uint32_t NW = kRansNT / kWave;
  uint32_t first = 0, end = 0;
  if (single >= 0) {
    const BlockHdr &h = recs[ritems[single].x].h;
    if (!h.err) { first = h.chunk0; end = h.chunk0 + h.nchunk; }
  } else {
    const uint32_t n = ctr->rans_chunks;
    end = n < cap ? n : static_cast<uint32_t>(cap);
  }
  for (uint32_t it = 0;; ++it) {
    uint32_t pair;
    if (single >= 0) {
      pair = wave + NW * it;
    } else {
      uint32_t p = 0;
      if (lane_id() == 0) p = atomicAdd(&ctr->rans_next, 1u);
      pair = __builtin_amdgcn_readfirstlane(p);
    }
    const uint32_t ia = first + 2 * pair;
    if (ia >= end) break;
    rans_pair(jobs, chunks, ia, ia + 1, end, scratch, win[wave]);
  }
}

// ---------------------------------------------------------------------------
// Kernel: selective tANS decode of byte-coded node bitmaps into scratch
// ---------------------------------------------------------------------------
// In a stream with flags bit 0 the entropy-coded nodes are coded as bytes
// with one of 50 static tANS tables (Sec. 5.2).  The plan kernel lists their
// chunks in the same list as rANS chunks (p1q = kFseTag | marker); k_fse
// decodes them two at a time per wave, lanes 0-31 one chunk's 32 cursors,
// lanes 32-63 another's.  Cursor l owns bytes l, l + 32, ... of its chunk
// and reads its own bit stream.  Per step a cursor looks its state up in the
// chunk's decoding table (in LDS; reloaded only when the half's table
// changes), takes the entry's bit count from a 64-bit buffer and stages its
// byte in LDS; every 32 steps the half's 1 KiB of bytes goes out as
// coalesced words.  The buffer is refilled from a queue of kFseQ words that
// every lane loads at the start of each group of kFseG steps, so a group
// waits for memory once.
constexpr int kFseNT = 256;
constexpr uint32_t kFseG = 16;   // steps per group: at most 16 * 11 = 176 bits
constexpr uint32_t kFseQ = 6;    // words queued per group: refills happen with
                                 // fewer than 11 bits left, so at most 6 a group
typedef __attribute__((address_space(1))) const uint32_t GlobalCU32;

__device__ void fse_pair(const JobDev *jobs, const RansChunk *chunks, uint32_t ia, uint32_t ib,
                         uint32_t end, const uint32_t *dec, uint32_t *scratch, uint32_t (*tab)[kFseSize],
                         uint32_t (*stage)[256], uint32_t &loaded) {
  const uint32_t lane = lane_id(), half = lane >> 5, hl = lane & 31;
  const uint32_t idx = half ? ib : ia;
  RansChunk c = RansChunk{0, 0, 0, 0, 0, 0};
  if (idx < end) c = chunks[idx];
  if (!(c.p1q & kFseTag)) c = RansChunk{0, 0, 0, 0, 0, 0};   // a rANS chunk: k_rans's
  const bool has = c.nbits != 0;
  const uint32_t tno = has ? c.p1q & 0x7F : 0u;              // 1..50, checked by the plan kernel
  const uint32_t flip = (c.p1q & 0x80) ? 0xFFu : 0u;
  // the halves' tables
  const uint32_t ta = __builtin_amdgcn_readlane(tno, 0), tb = __builtin_amdgcn_readlane(tno, 32);
  const uint32_t la = __builtin_amdgcn_readlane(loaded, 0), lb = __builtin_amdgcn_readlane(loaded, 32);
  const bool ra = ta && ta != la, rb = tb && tb != lb;
  if (ra || rb) {
    if (half ? rb : ra) {
      const uint4 *src = reinterpret_cast<const uint4 *>(dec + static_cast<uint64_t>(tno - 1) * kFseSize);
      uint4 *dst = reinterpret_cast<uint4 *>(tab[half]);
      for (uint32_t i0 = 0; i0 < kFseSize / 4; i0 += 32 * 8) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[i0 + 32 * u + hl];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[i0 + 32 * u + hl] = v[u];
      }
      loaded = tno;
    }
    wave_sync_lds();
  }
  const uint32_t *T = tab[half];
  uint8_t *sb = reinterpret_cast<uint8_t *>(stage[half]);
  // chunk header: cursor states, then stream lengths; a cursor's stream
  // starts after the 128-byte header and the streams of the cursors before it
  const uint8_t *base = has ? jobs[c.job].in + c.src : nullptr;
  GlobalCU32 *w32 = has ? (GlobalCU32 *)base : nullptr;   // C cast: generic to global
  const uint32_t hw0 = has ? w32[hl >> 1] : 0u, hw1 = has ? w32[16 + (hl >> 1)] : 0u;
  const uint32_t X0 = (hl & 1) ? hw0 >> 16 : hw0 & 0xFFFF;
  const uint32_t len = (hl & 1) ? hw1 >> 16 : hw1 & 0xFFFF;
  uint32_t incl = wave_incl_scan(len);
  if (half) incl -= __builtin_amdgcn_readlane(incl, 31);
  const uint32_t a = kFseChunkHdr + incl - len;              // first byte of the cursor's stream
  const uint32_t cw = (kFseChunkHdr + c.nw + 3) >> 2;        // the chunk's words
  const uint32_t cb = (c.nbits + 7) >> 3;                    // bytes it decodes
  const uint32_t my = cb > hl ? (cb - hl + 31) >> 5 : 0u;    // this cursor's steps
  const uint32_t K = (cb + 31) >> 5;
  const uint32_t ka = __builtin_amdgcn_readlane(K, 0), kb = __builtin_amdgcn_readlane(K, 32);
  const uint32_t kmax = ka > kb ? ka : kb;
  bool err = has && X0 >= kFseSize;
  uint32_t X = X0 & (kFseSize - 1);
  uint32_t wi = a >> 2;
  uint64_t buf = 0;
  uint32_t have = 0, p = 0, lastb = 0;
  if (has) {
    const uint32_t sh = 8 * (a & 3);
    buf = (wi < cw ? w32[wi] : 0u) >> sh;
    have = 32 - sh;
    ++wi;
  }
  const uint32_t lastk = (cb - 1) >> 5, lastl = (cb - 1) & 31;   // the bitmap's last byte
  uint32_t *dst = scratch + c.dst;
  const uint32_t ncw = (cb + 3) >> 2;                        // output words of the chunk
  for (uint32_t k0 = 0; k0 < kmax; k0 += 32) {
    for (uint32_t g = 0; g < 32 && k0 + g < kmax; g += kFseG) {
      uint32_t q[kFseQ];
#pragma unroll
      for (uint32_t u = 0; u < kFseQ; ++u) q[u] = has && wi + u < cw ? w32[wi + u] : 0u;
#pragma unroll
      for (uint32_t j = 0; j < kFseG; ++j) {
        const uint32_t k = k0 + g + j;
        const bool act = k < my;
        if (have < kFseLog) {
          buf |= static_cast<uint64_t>(q[0]) << have;
          have += 32;
          ++wi;
#pragma unroll
          for (uint32_t u = 0; u + 1 < kFseQ; ++u) q[u] = q[u + 1];
          q[kFseQ - 1] = 0;
        }
        const uint32_t e = T[X];
        const uint32_t nb = act ? (e >> 8) & 15 : 0u;
        const uint32_t v = static_cast<uint32_t>(buf) & ((1u << nb) - 1);
        buf >>= nb;
        have -= nb;
        p += nb;
        X = act ? (e >> 12) + v : X;
        const uint32_t byte = act ? (e ^ flip) & 255 : 0u;
        if (act && k == lastk && hl == lastl) lastb = byte;
        sb[32 * (g + j) + hl] = static_cast<uint8_t>(byte);
      }
    }
    wave_sync_lds();
    // the window's words: 32 steps of 32 bytes
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) {
      const uint32_t wj = 32 * u + hl;
      if (8 * k0 + wj < ncw) dst[8 * k0 + wj] = stage[half][wj];
    }
    wave_sync_lds();
  }
  if (has) {
    // every bit of the stream used and no more, its padding bits zero, the
    // cursor back at state 0; the bitmap's bits past n_v zero
    if (have < 8) buf |= static_cast<uint64_t>(wi < cw ? w32[wi] : 0u) << have;
    const uint32_t padb = 8 * len - p;
    if (X != 0 || (p + 7) >> 3 != len || (static_cast<uint32_t>(buf) & ((1u << (padb & 7)) - 1))) err = true;
    if (hl == lastl && (c.nbits & 7) && (lastb >> (c.nbits & 7))) err = true;
  }
  const uint64_t eb = __ballot(err);
  const uint32_t eh = half ? static_cast<uint32_t>(eb >> 32) : static_cast<uint32_t>(eb);
  if (hl == 0 && eh) set_err(jobs[c.job].status, PIVCO_E_CORRUPT);
}

// Decodes the batch's listed tANS chunks, a pair per wave from a shared
// counter; or, for single >= 0, only the chunks of block ritems[single] with
// one workgroup (the per-block launch mode).
__global__ __launch_bounds__(kFseNT) void k_fse(const JobDev *jobs, const ParsedBlock *recs,
                                                 const uint2 *ritems, Counters *ctr,
                                                 const RansChunk *chunks, uint64_t cap,
                                                 const uint32_t *dec, uint32_t *scratch, int32_t single) {
  __shared__ uint32_t tab[kFseNT / kWave][2][kFseSize];
  __shared__ uint32_t stage[kFseNT / kWave][2][256];
  const uint32_t wave = wave_id();
  constexpr uint32_t NW = kFseNT / kWave;
  uint32_t first = 0, end = 0;
  if (single >= 0) {
    const BlockHdr &h = recs[ritems[single].x].h;
    if (!h.err) { first = h.chunk0; end = h.chunk0 + h.nchunk; }
  } else {
    const uint32_t n = ctr->rans_chunks;
    end = n < cap ? n : static_cast<uint32_t>(cap);
  }
  uint32_t loaded = 0;
  for (uint32_t it = 0;; ++it) {
    uint32_t pair;
    if (single >= 0) {
      pair = wave + NW * it;
    } else {
      uint32_t p = 0;
      if (lane_id() == 0) p = atomicAdd(&ctr->fse_next, 1u);
      pair = __builtin_amdgcn_readfirstlane(p);
    }
    const uint32_t ia = first + 2 * pair;
    if (ia >= end) break;
    fse_pair(jobs, chunks, ia, ia + 1, end, dec, scratch, tab[wave], stage[wave], loaded);
  }
}

// ---------------------------------------------------------------------------
// Kernel: bottom-up merge decode
// ---------------------------------------------------------------------------
template <int NT_, int T_, int BODY_, int K_, int LOCK_>
struct MergeCfg {
  static constexpr int NT = NT_;
  static constexpr int T = T_;                        // output symbols per tile
  static constexpr int BODY = BODY_;                  // resident block bytes
  static constexpr int K = K_;                        // outputs per merge task (8, 16 or 32)
  static constexpr int LOCK = LOCK_;                  // windows a wave merges at once (1, 2 or 4)
  static_assert(LOCK == 1 || LOCK == 2 || LOCK == 4, "windows per wave step");
  static constexpr int NW = NT / kWave;
  static constexpr int LVL = T + (K - 1) * 128 + 64;  // bytes per level buffer (shares rounded to K)
  static constexpr int LEVELS = kMaxLenGpu;
  static constexpr int WIN = (T / K + 128 + 63) / 64 + 1;    // 64-task windows per level
  static_assert(K == 8 || K == 16 || K == 32, "task width");
  static constexpr int STG = BODY / 8;                // streaming: staged (word, rank) pairs
  static constexpr int SUP = BODY / 32 + 2;           // rank directory, per 256 bits
  static constexpr int REL = BODY / 8 + 8;            // rank directory, per 64 bits
};

// What a merge lane needs about a node with work in the current tile (16
// bytes): where its bits start (resident: LDS bit address; streaming: first
// staged word), the 1 bits before that point (a flat node: flat_tag), its
// output offset in its level buffer | its first task in the level << 16, and
// one 16-bit code per child (kid_code).
struct NodeRec {
  uint32_t x0;
  uint32_t arank;
  uint32_t ot;
  uint32_t kids;
};

template <class C>
struct MergeSmem {
  ParsedBlock pb;          // h and t of the current block
  BlockExt nxt;            // extent of the next item's block (looked ahead)
  uint2 nxt_item;          // next item: record, tile
  uint32_t cur[256];       // bits of the node consumed by earlier tiles
  uint32_t tv[256];        // node's share of the current tile
  union {
    struct {
      uint32_t abit[256];  // resident: LDS bit address of the node bitmap
      uint32_t arank[256]; // resident: 1 bits of the body before the cursor
      uint32_t r0[256];    // resident: 1 bits of the body before the node
      uint32_t aend[256];  // resident: 1 bits of the body before the share's end
    };
    struct {
      uint32_t tone[256];  // streaming: 1 bits in the tile share
      uint32_t ones[256];  // streaming: 1 bits seen so far
      uint32_t stg[256];   // streaming: first staged word of the node
      uint32_t obase[256]; // streaming: output offset in the level buffer (16-byte aligned)
    };
  };
  NodeRec rec[256];        // nodes with work, level by level (slot order)
  uint64_t smask[C::LEVELS][C::WIN];  // bit i of window w: a node's first task is 64 w + i
  uint8_t wstart[C::LEVELS][C::WIN];  // level slot of the node holding task 64 w
  uint32_t ntask[C::LEVELS];          // 16-output tasks of the level
  uint32_t nftask[C::LEVELS];         // of which belong to flat nodes (the first ones)
  uint32_t actbase[C::LEVELS];        // slots of the levels above
  uint32_t act_run;
  uint32_t warm_sink;
  const uint8_t *warm_in, *warm_rec;
  uint32_t stage_top;
  uint32_t tile;           // runtime tile size for this block
  uint32_t sel[16];
  uint32_t item;
  uint32_t scan_tot[C::NW];
  uint32_t leafrow[256];   // four copies of byte s: the "sequence" of a leaf child s
  uint32_t lvl[2][C::LVL / 4] __attribute__((aligned(16)));
  uint32_t sup[C::SUP];    // resident: 1 bits of the body before each 256-bit superblock
  uint8_t rel[C::REL];     // resident: 1 bits of the superblock before each 64-bit word
  uint32_t body[C::BODY / 4 + 16] __attribute__((aligned(16)));
};

// Code of a child in a NodeRec: the LDS byte address of its sequence / 4 in
// bits 0-14, and bit 15 set for an internal child (whose sequence advances
// with its rank) or clear for a leaf (whose constant row is read at the same
// address for every output).  `off` is the internal child's output offset in
// the level buffer of parity p.
template <class C>
__device__ __forceinline__ uint32_t kid_code(const MergeSmem<C> &sm, uint32_t c, uint32_t p, uint32_t off) {
  static_assert(offsetof(MergeSmem<C>, sup) <= (1u << 17), "leaf rows and level buffers below 128 KiB");
  const uint8_t *base = reinterpret_cast<const uint8_t *>(&sm);
  if (c & 0x8000) return static_cast<uint32_t>(reinterpret_cast<const uint8_t *>(&sm.leafrow[c & 255]) - base) >> 2;
  return 0x8000u | ((static_cast<uint32_t>(reinterpret_cast<const uint8_t *>(sm.lvl[p]) - base) + off) >> 2);
}

// In a flat node's record, in place of the rank: bit 31 set, D in bits
// 24-27, and the LDS byte address of its group's symbols (the D-bit values
// index them).
template <class C>
__device__ __forceinline__ uint32_t flat_tag(const MergeSmem<C> &sm, const NodeTab &t, uint32_t v) {
  const uint8_t *base = reinterpret_cast<const uint8_t *>(&sm);
  const uint32_t a = static_cast<uint32_t>(&t.leafsym[t.child[v][0] & 255] - base);
  return 0x80000000u | (static_cast<uint32_t>(t.fd[v]) << 24) | a;
}

// Tasks skipped after a level's nft flat tasks so that its binary tasks
// start a window of their own.
__device__ __forceinline__ uint32_t flat_pad(uint32_t nft) { return (kWave - nft % kWave) % kWave; }

// Streaming tile: largest multiple of 1024 (at most C::T) whose staged words fit.
template <class C>
__device__ uint32_t pick_tile_streaming(const BlockHdr &h, const NodeTab &t) {
  uint32_t T = C::T;
  for (; T > 1024; T -= 1024) {
    uint64_t need = h.I + h.maxlen + 1;
    for (uint32_t d = 0; d < h.maxlen; ++d) {
      // a tile's share of a level is at most T symbols, D bits each at a
      // flat node (the level's flat nodes come first; the first has the
      // largest D)
      const uint32_t dmax = h.nfl[d] ? t.fd[h.lvl[d]] : 1u;
      const uint64_t cap = static_cast<uint64_t>(T) * dmax;
      const uint64_t ld = h.lvl_total[d] < cap ? h.lvl_total[d] : cap;
      need += div_up(ld, 32) + (h.lvl[d + 1] - h.lvl[d]);
    }
    if (need <= static_cast<uint64_t>(C::STG)) break;
  }
  return T;
}

// Number of 1 bits in LDS bits [0, x) of the resident body: 256-bit
// superblock count + 64-bit word count within it + popcount of the rest.
__device__ __forceinline__ uint32_t rank_at(const uint32_t *body, const uint32_t *sup,
                                            const uint8_t *rel, uint32_t x) {
  const uint64_t w = reinterpret_cast<const uint64_t *>(body)[x >> 6];
  return sup[x >> 8] + rel[x >> 6] + static_cast<uint32_t>(__popcll(w & ((1ull << (x & 63)) - 1)));
}

// The 4 bytes at LDS byte address a (relative to lds): two aligned dword
// reads and a byte funnel shift (unaligned DS reads are much slower).
__device__ __forceinline__ uint32_t lds_win(const uint8_t *lds, uint32_t a) {
  const uint32_t *p = reinterpret_cast<const uint32_t *>(lds + (a & ~3u));
  return __builtin_amdgcn_alignbyte(p[1], p[0], a);
}

// Enters a node with work into its level's task windows: its record goes to
// its slot, its first task sets a bit of the window start mask, and the
// windows whose first task falls inside it point at its level slot.
template <class C>
__device__ __forceinline__ void list_node(MergeSmem<C> &sm, uint32_t d, uint32_t ai, uint32_t gslot,
                                          uint32_t tp, uint32_t nt, const NodeRec &r) {
  sm.rec[gslot] = r;
  atomicOr(reinterpret_cast<unsigned long long *>(&sm.smask[d][tp >> 6]), 1ull << (tp & 63));
  for (uint32_t w = (tp + 63) >> 6; kWave * w < tp + nt; ++w) sm.wstart[d][w] = static_cast<uint8_t>(ai);
}

// Exclusive prefix over the 64 lanes of a wave, and the wave total.
__device__ __forceinline__ uint64_t wave_excl_scan64(uint64_t v, uint64_t &total) {
  const uint64_t inc = wave_incl_scan64(v);
  total = __shfl(inc, kWave - 1, kWave);
  return inc - v;
}


// Streaming count for level d, run by one wave: every node's share (sm.tv)
// and its 1 bits (from the staging pass) give the children's shares; the
// node's merge record, the children's output space in the next level buffer,
// and the compacted list of the level's nodes with work (with a prefix of
// their 16-output tasks) come from wave-wide prefix sums.  Cursors advance
// here.
template <class C, bool FLAT>
__device__ void count_level_streaming(MergeSmem<C> &sm, uint32_t d) {
  const uint32_t lane = lane_id();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  uint32_t out_top = 0, task_top = 0, act_top = 0, ftask = 0;
  for (uint32_t i = lane; i < static_cast<uint32_t>(C::WIN); i += kWave) sm.smask[d][i] = 0;
  const uint32_t act_base = sm.act_run;
  wave_sync_lds();
  for (uint32_t v0 = h.lvl[d]; v0 < h.lvl[d + 1]; v0 += kWave) {
    const uint32_t v = v0 + lane;
    const bool valid = v < h.lvl[d + 1];
    uint32_t tvv = 0, ones = 0, tc[2] = {0, 0};
    uint16_t ch[2] = {0x8000, 0x8000};
    uint32_t x0 = 0;
    if (valid) {
      tvv = sm.tv[v];
      x0 = sm.stg[v];
      ones = sm.tone[v];
      ch[0] = t.child[v][0];
      ch[1] = t.child[v][1];
      tc[0] = tvv - ones;
      tc[1] = ones;
      for (int bb = 0; bb < 2; ++bb) {
        if (ch[bb] & 0x8000) { tc[bb] = 0; continue; }
        if (sm.cur[ch[bb]] + tc[bb] > t.nv[ch[bb]]) {     // more symbols than the node holds
          atomicCAS(&h.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
          tc[bb] = 0;
        }
      }
    }
    const uint32_t o0 = (tc[0] + C::K - 1) & ~(C::K - 1u), o1 = (tc[1] + C::K - 1) & ~(C::K - 1u);
    const uint32_t tasks = (tvv + C::K - 1) / C::K;
    const uint32_t isact = tvv ? 1u : 0u;
    const uint64_t pk = static_cast<uint64_t>(o0 + o1) | (static_cast<uint64_t>(tasks) << 32) |
                        (static_cast<uint64_t>(isact) << 48);
    uint64_t tot;
    const uint64_t ex = wave_excl_scan64(pk, tot);
    // the level's flat nodes are its first nfl nodes: their tasks are the
    // tasks before lane nfl of the first pass
    if (FLAT && v0 == h.lvl[d])
      ftask = static_cast<uint32_t>(__shfl(ex, static_cast<int>(h.nfl[d]), kWave) >> 32) & 0xFFFF;
    if (valid) {
      const uint32_t ob = out_top + static_cast<uint32_t>(ex & 0xFFFFFFFFu);
      uint32_t kids = 0;
      for (int bb = 0; bb < 2; ++bb) {
        uint32_t code;
        if (ch[bb] & 0x8000) {
          code = kid_code<C>(sm, ch[bb], 0, 0);
        } else {
          const uint32_t cob = ob + (bb ? o0 : 0u);
          sm.tv[ch[bb]] = tc[bb];
          sm.obase[ch[bb]] = cob;
          code = kid_code<C>(sm, ch[bb], (d + 1) & 1, cob);
        }
        kids |= code << (16 * bb);
      }
      if (isact) {
        const uint32_t ai = act_top + static_cast<uint32_t>(ex >> 48);
        const bool fl = FLAT && t.fd[v];
        const uint32_t tp = task_top + static_cast<uint32_t>((ex >> 32) & 0xFFFF) +
                            (FLAT && !fl ? flat_pad(ftask) : 0u);
        NodeRec r;
        r.x0 = x0;
        r.arank = fl ? flat_tag<C>(sm, t, v) : 0u;
        r.ot = sm.obase[v] | (tp << 16);
        r.kids = kids;
        list_node<C>(sm, d, ai, act_base + ai, tp, tasks, r);
      }
      sm.cur[v] += tvv;
    }
    out_top += static_cast<uint32_t>(tot & 0xFFFFFFFFu);
    task_top += static_cast<uint32_t>((tot >> 32) & 0xFFFF);
    act_top += static_cast<uint32_t>(tot >> 48);
    wave_sync_lds();
  }
  if (lane == 0) {
    sm.ntask[d] = task_top + (FLAT ? flat_pad(ftask) : 0u);
    sm.nftask[d] = ftask;
    sm.actbase[d] = act_base;
    sm.act_run = act_base + act_top;
  }
  wave_sync_lds();
}

// Resident count for a tile that ends inside the block, run by one wave:
// top-down, a node's share and the 1 bits in it (rank directory at the
// share's end) give the children's shares.  A child that would receive more
// symbols than it has left marks the block corrupt and gets none.  Per level
// two dependent LDS round trips: the shares, then the ranks together with
// the children's cursors and sizes (read unconditionally; a leaf reads slot
// 0 and ignores it).  The rank at the share's end equals the node's rank
// when the share is empty.
template <class C>
__device__ void count_chain(MergeSmem<C> &sm) {
  const uint32_t lane = lane_id();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  const uint32_t maxd = h.maxlen;
  const uint32_t lb = lane <= maxd ? h.lvl[lane] : 0u;    // lane d: first node of level d
  bool bad = false;
  for (uint32_t d = 0; d < maxd; ++d) {
    const uint32_t lo = __builtin_amdgcn_readlane(lb, d), hi = __builtin_amdgcn_readlane(lb, d + 1);
    for (uint32_t v = lo + lane; v < hi; v += kWave) {
      const uint32_t tvv = sm.tv[v], ar = sm.arank[v];
      const uint32_t x0 = sm.abit[v] + sm.cur[v];
      const uint32_t cc = *reinterpret_cast<const uint32_t *>(t.child[v]);
      const uint32_t cl = cc & 0xFFFF, cr = cc >> 16;
      const uint32_t il = (cl & 0x8000) ? 0u : cl, ir = (cr & 0x8000) ? 0u : cr;
      const uint32_t e = rank_at(sm.body, sm.sup, sm.rel, x0 + tvv);
      const uint32_t curl = sm.cur[il], nvl = t.nv[il], curr = sm.cur[ir], nvr = t.nv[ir];
      sm.aend[v] = e;
      const uint32_t ones = e - ar, zeros = tvv - ones;
      const bool okl = curl + zeros <= nvl, okr = curr + ones <= nvr;
      if (!(cl & 0x8000)) {
        sm.tv[cl] = okl ? zeros : 0u;
        bad |= !okl;
      }
      if (!(cr & 0x8000)) {
        sm.tv[cr] = okr ? ones : 0u;
        bad |= !okr;
      }
    }
    wave_sync_lds();
  }
  if (bad) atomicCAS(&h.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
}

// Resident count for the block's last tile (all threads): every node's
// share is what is left of it, and the rank at the node's end closes it.
template <class C>
__device__ void count_last(MergeSmem<C> &sm) {
  const NodeTab &t = sm.pb.t;
  for (uint32_t v = item_tid(); v < sm.pb.h.I; v += C::NT) {
    const uint32_t nv = t.nv[v];
    const uint32_t rest = nv - sm.cur[v];
    sm.tv[v] = rest;
    sm.aend[v] = rest ? rank_at(sm.body, sm.sup, sm.rel, sm.abit[v] + nv) : sm.arank[v];
  }
}

// Resident tile bookkeeping (all threads), from the shares in sm.tv: one
// exclusive scan over the nodes in breadth-first order, where every level is
// a contiguous range, of (share rounded up to 16 bytes | 16-output tasks <<
// 32 | has-work << 48).  Differences of the scan within a level give each
// node's output offset in its level buffer, its slot in the level's list of
// nodes with work and the tasks before it; the merge records follow, and
// the cursors advance.
template <class C, bool FLAT>
__device__ void tile_lists(MergeSmem<C> &sm) {
  const int tid = item_tid();
  const int wave = wave_id();
  const uint32_t lane = lane_id();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  const uint32_t I = h.I;
  uint64_t *pfx = reinterpret_cast<uint64_t *>(sm.lvl[0]);   // level buffers are idle here
  for (int i = tid; i < C::LEVELS * C::WIN; i += C::NT) (&sm.smask[0][0])[i] = 0;
  if (wave == 0) {                       // one wave, 4 consecutive nodes per lane
    uint64_t pk[4], loc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t v = 4 * lane + k;
      const uint32_t tvv = v < I ? sm.tv[v] : 0u;
      pk[k] = ((tvv + C::K - 1) & ~(C::K - 1u)) | (static_cast<uint64_t>((tvv + C::K - 1) / C::K) << 32) |
              (static_cast<uint64_t>(tvv ? 1u : 0u) << 48);
      loc += pk[k];
    }
    uint64_t ex = wave_incl_scan64(loc) - loc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pfx[4 * lane + k] = ex;            // pfx[I] is the total (I <= 255)
      ex += pk[k];
    }
  }
  lds_barrier();
  if (static_cast<uint32_t>(tid) < I) {
    const uint32_t v = tid;
    const uint32_t d = t.depth[v];
    const uint64_t base1 = pfx[h.lvl[d + 1]];
    const uint64_t rel = pfx[v] - pfx[h.lvl[d]];
    const uint32_t tvv = sm.tv[v];
    const uint32_t cc = *reinterpret_cast<const uint32_t *>(t.child[v]);
    uint32_t kids = 0;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const uint32_t c = (cc >> (16 * bb)) & 0xFFFF;
      const uint32_t code = kid_code<C>(sm, c, (d + 1) & 1, (c & 0x8000) ? 0u : static_cast<uint32_t>(pfx[c] - base1));
      kids |= code << (16 * bb);
    }
    if (tvv) {
      const uint32_t fdv = FLAT ? t.fd[v] : 0u;
      uint32_t tp = static_cast<uint32_t>(rel >> 32) & 0xFFFF;
      if (FLAT && !fdv && h.nfl[d])         // binary tasks start after the padded flat ones
        tp += flat_pad(static_cast<uint32_t>((pfx[h.lvl[d] + h.nfl[d]] - pfx[h.lvl[d]]) >> 32) & 0xFFFF);
      NodeRec r;
      r.x0 = sm.abit[v] + (fdv ? fdv * sm.cur[v] : sm.cur[v]);     // a flat node keeps D bits per symbol
      r.arank = fdv ? flat_tag<C>(sm, t, v) : sm.arank[v];
      r.ot = static_cast<uint32_t>(rel) | (tp << 16);
      r.kids = kids;
      list_node<C>(sm, d, static_cast<uint32_t>(rel >> 48), static_cast<uint32_t>(pfx[v] >> 48), tp,
                   (tvv + C::K - 1) / C::K, r);
    }
    sm.cur[v] += tvv;
    sm.arank[v] = sm.aend[v];
  }
  if (static_cast<uint32_t>(tid) < h.maxlen) {
    const uint64_t tot = pfx[h.lvl[tid + 1]] - pfx[h.lvl[tid]];
    if (FLAT) {
      const uint64_t ftot = pfx[h.lvl[tid] + h.nfl[tid]] - pfx[h.lvl[tid]];   // the level's flat nodes come first
      const uint32_t nft = static_cast<uint32_t>(ftot >> 32) & 0xFFFF;
      sm.ntask[tid] = (static_cast<uint32_t>(tot >> 32) & 0xFFFF) + flat_pad(nft);
      sm.nftask[tid] = nft;
    } else {
      sm.ntask[tid] = static_cast<uint32_t>(tot >> 32) & 0xFFFF;
    }
    sm.actbase[tid] = static_cast<uint32_t>(pfx[h.lvl[tid]] >> 48);
  }
  lds_barrier();
}

// Streaming count for level d: one wave per node popcounts the node's share
// straight from global memory and stages it as (word, rank) pairs.
template <class C>
__device__ void stage_level_streaming(const JobDev &J, MergeSmem<C> &sm, uint32_t d,
                                      const uint32_t *scratch, uint64_t scratch_words) {
  const int wave = wave_id();
  const uint32_t lane = lane_id();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  uint2 *stage = reinterpret_cast<uint2 *>(sm.body);
  const uint32_t *gin32 = reinterpret_cast<const uint32_t *>(J.in);
  const uint64_t in_dw = J.in_len >> 2;
  for (uint32_t v = h.lvl[d] + wave; v < h.lvl[d + 1]; v += C::NW) {
    const uint32_t tvv = sm.tv[v];
    const uint32_t dv = t.fd[v] ? t.fd[v] : 1u;     // bits per symbol
    const uint32_t nbits = dv * tvv;
    const uint32_t nwords = (nbits + 31) / 32;
    uint32_t base = 0;
    if (lane == 0 && nwords) base = atomicAdd(&sm.stage_top, nwords);
    base = __builtin_amdgcn_readfirstlane(base);
    if (base + nwords > static_cast<uint32_t>(C::STG)) {   // cannot happen: tile sized for it
      if (lane == 0) {
        atomicCAS(&h.err, 0, static_cast<int32_t>(PIVCO_E_UNSUPPORTED));
        sm.tone[v] = 0;
        sm.stg[v] = 0;
      }
      continue;
    }
    const uint64_t s0 = static_cast<uint64_t>(dv) * sm.cur[v];
    uint32_t carry = 0;
    for (uint32_t q0 = 0; q0 < nwords; q0 += kWave) {
      const uint32_t q = q0 + lane;
      uint32_t w = 0;
      if (q < nwords) {
        const uint64_t p = s0 + 32ull * q;
        if (t.kind[v]) w = bits32_glb(scratch, 32 * (h.ans_word0 + t.boff[v]) + p, scratch_words);
        else w = bits32_glb(gin32, 8 * (h.blk + t.boff[v]) + p, in_dw);
        const uint32_t rem = nbits - 32 * q;
        if (rem < 32) w &= (1u << rem) - 1;
      }
      const uint32_t pc = __popc(w);
      const uint32_t inc = wave_incl_scan(pc);
      if (q < nwords) stage[base + q] = make_uint2(w, carry + inc - pc);
      carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) { sm.stg[v] = base; sm.tone[v] = carry; sm.ones[v] += carry; }
  }
}

// Merge, bottom-up by level.  A level's work is a list of K-output tasks
// over its nodes with work; a wave takes 64 consecutive tasks (a window), and
// a lane finds its node as the window's first node plus the node starts
// inside the window up to its task (popcount of the window's start mask).
// A task reads its node record, K bitmap bits and their rank, then 4-byte
// windows of the children's sequences at the ranks (a leaf child reads its
// constant row: the offset is multiplied by 0), makes groups of 4 bytes with
// one v_perm_b32 each, and stores 16 bytes at a time (LDS, or HBM at the
// root).  All window addresses are computed before any window is read.
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) U32x4 GlobalU4;
typedef uint32_t U32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) U32x2 GlobalU2;
typedef __attribute__((address_space(1))) uint8_t GlobalU8;

// N windows of one level at once, stage by stage (records, bits and ranks,
// child windows, permutes), so that each stage's LDS reads of all N windows
// are in flight together.  Lanes without a task read from clamped addresses
// and store nothing.
// Stores the K outputs of task j0 of a node (o: K/4 words): into the level
// buffer of level d at the node's offset, or at the root into HBM (16 bytes
// at a time where aligned and inside the tile).
template <class C, bool ROOT>
__device__ __forceinline__ void store_task(MergeSmem<C> &sm, int d, uint32_t ot, uint32_t j0,
                                           const uint32_t *o, uint32_t tvv, uint8_t *out) {
  constexpr int CB = C::K < 16 ? C::K : 16;    // bytes per store
  uint8_t *ldsw = reinterpret_cast<uint8_t *>(&sm);
#pragma unroll
  for (int c = 0; c < C::K / CB; ++c) {
    if (ROOT) {
      const uint32_t j = j0 + CB * c;
      uint8_t *dst = out + j;
      if (j + CB <= tvv && !(reinterpret_cast<uintptr_t>(dst) & (CB - 1))) {
        // decoded bytes are written once and not read back here: non-temporal
        if (CB == 16) __builtin_nontemporal_store(U32x4{o[4 * c], o[4 * c + 1], o[4 * c + 2], o[4 * c + 3]},
                                                  (GlobalU4 *)(dst));   // C cast: generic to global
        else __builtin_nontemporal_store(U32x2{o[0], o[1]}, (GlobalU2 *)(dst));
      } else if (j < tvv) {
        const uint32_t kk2 = tvv - j < CB ? tvv - j : CB;
        GlobalU8 *gd = (GlobalU8 *)(dst);   // C cast: generic to global address space
        for (uint32_t e = 0; e < kk2; ++e) gd[e] = static_cast<uint8_t>(o[(CB * c + e) >> 2] >> (8 * (e & 3)));
      }
    } else {
      const uint32_t dst = static_cast<uint32_t>(reinterpret_cast<const uint8_t *>(sm.lvl[d & 1]) - ldsw) +
                           (ot & 0xFFFF) + j0 + CB * c;
      if (CB == 16) *reinterpret_cast<uint4 *>(ldsw + dst) = make_uint4(o[4 * c], o[4 * c + 1], o[4 * c + 2], o[4 * c + 3]);
      else *reinterpret_cast<uint2 *>(ldsw + dst) = make_uint2(o[0], o[1]);
    }
  }
}

// merge_flat_D (Sec. 3.2) for one window of a level's flat tasks (tasks
// [0, nft)): a task reads K D-bit values of its flat node, 4 at a time from
// one 32-bit window of the node's bits, and looks each up in the node's
// group of symbols in LDS.  Lanes without a flat task read from the node
// record's start with D = 2 and an in-range table and store nothing.
template <class C, bool RESIDENT, bool ROOT>
__device__ __forceinline__ void merge_flat_window(MergeSmem<C> &sm, int d, uint32_t w, uint32_t nft,
                                                  uint32_t abase, uint8_t *out) {
  const uint32_t lane = lane_id();
  constexpr int G = C::K / 4;
  const uint8_t *lds = reinterpret_cast<const uint8_t *>(&sm);
  const uint64_t upto = ((2ull << lane) - 1) & ~1ull;
  const uint64_t B = sm.smask[d][w];
  const uint32_t slot = sm.wstart[d][w] + static_cast<uint32_t>(__popcll(B & upto));
  const NodeRec r = sm.rec[abase + slot];
  const bool valid = kWave * w + lane < nft && (r.arank >> 31);
  const uint32_t D = valid ? (r.arank >> 24) & 15 : 2u;
  const uint32_t tab = valid ? (r.arank & 0xFFFFFFu)
                             : static_cast<uint32_t>(reinterpret_cast<const uint8_t *>(sm.pb.t.leafsym) - lds);
  const uint32_t j0 = valid ? C::K * (kWave * w + lane - (r.ot >> 16)) : 0u;
  const uint2 *stage = reinterpret_cast<const uint2 *>(sm.body);
  uint32_t bits[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const uint32_t b = D * (j0 + 4 * g);       // from the node's first bit in this tile
    if (RESIDENT) {
      bits[g] = bits32_lds(sm.body, r.x0 + b);
    } else {                                   // staged words start at the node's cursor
      const uint32_t q = r.x0 + (b >> 5);
      bits[g] = __builtin_amdgcn_alignbit(stage[q + 1].x, stage[q].x, b & 31);
    }
  }
  uint32_t o[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    uint32_t v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t q = __builtin_amdgcn_ubfe(bits[g], D * e, D);
      v |= static_cast<uint32_t>(lds[tab + q]) << (8 * e);
    }
    o[g] = v;
  }
  if (valid) store_task<C, ROOT>(sm, d, r.ot, j0, o, ROOT ? sm.tv[0] : 0u, out);
}

template <class C, bool RESIDENT, int N, bool ROOT>
__device__ __forceinline__ void merge_windows(MergeSmem<C> &sm, int d, const uint32_t *w,
                                              uint32_t ntask, uint32_t abase, uint8_t *out) {
  const uint32_t lane = lane_id();
  constexpr int G = C::K / 4;                  // groups of 4 outputs
  const uint8_t *lds = reinterpret_cast<const uint8_t *>(&sm);
  const uint64_t upto = ((2ull << lane) - 1) & ~1ull;   // window bits 1 .. lane
  bool valid[N];
  NodeRec r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    // the lane's node: the window's first slot + the node starts at window
    // bits 1 .. lane.  A lane past the level's last task gets the window's
    // last node and works on that node's first task (and stores nothing).
    const uint64_t B = sm.smask[d][w[i]];
    const uint32_t slot = sm.wstart[d][w[i]] + static_cast<uint32_t>(__popcll(B & upto));
    valid[i] = kWave * w[i] + lane < ntask;
    r[i] = sm.rec[abase + slot];
  }
  uint32_t j0[N], bits[N], r1[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    j0[i] = valid[i] ? C::K * (kWave * w[i] + lane - (r[i].ot >> 16)) : 0u;
    if (RESIDENT) {
      const uint32_t x = r[i].x0 + j0[i];
      bits[i] = bits32_lds(sm.body, x);
      r1[i] = rank_at(sm.body, sm.sup, sm.rel, x) - r[i].arank;
    } else {
      const uint2 *stage = reinterpret_cast<const uint2 *>(sm.body);
      const uint2 wr = stage[r[i].x0 + (j0[i] >> 5)];
      const uint32_t sh = j0[i] & 31;   // 0, or a multiple of K: staged words start at the node's cursor
      bits[i] = wr.x >> sh;
      r1[i] = wr.y + __popc(wr.x & ((1u << sh) - 1));
    }
  }
  uint32_t aL[N][G], aR[N][G], sel[N][G];
  uint2 wl[N][G], wr[N][G];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const uint32_t kd = r[i].kids;
    uint32_t mL = (kd >> 15) & 1u, mR = kd >> 31;
    // opaque to the compiler: a 0/1 multiplier stays one v_mad_u32_u24
    // instead of being turned into a select per group
    asm volatile("" : "+v"(mL), "+v"(mR));
    const uint32_t bL = (kd & 0x7FFFu) << 2, bR = (kd >> 14) & 0x1FFFCu;
    uint32_t r1g = r1[i], r0g = j0[i] - r1[i];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint32_t m = (bits[i] >> (4 * g)) & 15;
      aL[i][g] = bL + __umul24(mL, r0g);
      aR[i][g] = bR + __umul24(mR, r1g);
      sel[i][g] = m;
      const uint32_t pc = __popc(m);
      r1g += pc;
      r0g += 4 - pc;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint32_t *ql = reinterpret_cast<const uint32_t *>(lds + (aL[i][g] & ~3u));   // 4-byte aligned:
      const uint32_t *qr = reinterpret_cast<const uint32_t *>(lds + (aR[i][g] & ~3u));   // two dword reads
      wl[i][g] = make_uint2(ql[0], ql[1]);
      wr[i][g] = make_uint2(qr[0], qr[1]);
      sel[i][g] = sm.sel[sel[i][g]];
    }
  }
  const uint32_t tvv = ROOT ? sm.tv[0] : 0u;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    uint32_t o[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint32_t l4 = __builtin_amdgcn_alignbyte(wl[i][g].y, wl[i][g].x, aL[i][g]);
      const uint32_t r4 = __builtin_amdgcn_alignbyte(wr[i][g].y, wr[i][g].x, aR[i][g]);
      o[g] = __builtin_amdgcn_perm(r4, l4, sel[i][g]);
    }
    // the outputs exist here for every lane: otherwise the compiler moves a
    // window's LDS reads into the store branch below and waits for each one
    // in turn
#pragma unroll
    for (int g = 0; g < G; ++g) asm volatile("" ::"v"(o[g]));
    if (!valid[i]) continue;
    store_task<C, ROOT>(sm, d, r[i].ot, j0[i], o, tvv, out);
  }
}

// One level of a tile: first the windows of its flat tasks, then the binary
// tasks, a wave taking up to C::LOCK of their windows at once.  The flat
// tasks are the level's first nft tasks, and its binary tasks start at the
// next multiple of 64 (flat_pad): no window holds both kinds.
template <class C, bool RESIDENT, bool ROOT, bool FLAT>
__device__ __forceinline__ void merge_level(MergeSmem<C> &sm, int d, uint8_t *out) {
  const uint32_t wave = wave_id();
  const uint32_t ntask = sm.ntask[d], abase = sm.actbase[d];
  const uint32_t nwin = (ntask + kWave - 1) / kWave;
  uint32_t nfw = 0, wv = wave;
  if (FLAT) {
    const uint32_t nft = sm.nftask[d];
    nfw = (nft + kWave - 1) / kWave;
    for (uint32_t w = wave; w < nfw; w += C::NW) merge_flat_window<C, RESIDENT, ROOT>(sm, d, w, nft, abase, out);
    wv = (wave + C::NW - nfw % C::NW) % C::NW;   // binary windows go first to the waves after the flat ones
  }
  for (uint32_t w = nfw + wv; w < nwin; w += C::LOCK * C::NW) {
    const uint32_t left = (nwin - w + C::NW - 1) / C::NW;   // windows of this wave from w on
    const uint32_t ww[4] = {w, w + C::NW, w + 2 * C::NW, w + 3 * C::NW};
    if (C::LOCK >= 4 && left >= 4) merge_windows<C, RESIDENT, (C::LOCK >= 4 ? 4 : 1), ROOT>(sm, d, ww, ntask, abase, out);
    else if (C::LOCK >= 4 && left == 3) merge_windows<C, RESIDENT, (C::LOCK >= 4 ? 3 : 1), ROOT>(sm, d, ww, ntask, abase, out);
    else if (C::LOCK >= 2 && left >= 2) merge_windows<C, RESIDENT, (C::LOCK >= 2 ? 2 : 1), ROOT>(sm, d, ww, ntask, abase, out);
    else merge_windows<C, RESIDENT, 1, ROOT>(sm, d, ww, ntask, abase, out);
  }
  lds_barrier();
}

// All levels of the tile, deepest first (into LDS), the root last (into
// HBM); one barrier per level.  For a tile of a whole block (touch) the
// last wave, which has the fewest windows in the deep levels, first reads
// one word of every 4 KiB page of the tile's output, so that the root
// level's stores find their address translations cached (64Ki-symbol blocks
// decoding into one large buffer: 0.4% of the step).  Reading them for a
// split block's tiles too cost more than it saved, and reading them earlier
// (with the item's loads, or during the first tile's rank chain) either
// stalled the workgroup on the misses or came too early to help.
template <class C, bool RESIDENT, bool FLAT>
__device__ __forceinline__ void merge_tile(MergeSmem<C> &sm, int maxd, uint8_t *out, bool touch) {
  if (touch && wave_id() == C::NW - 1) {
    const uint32_t a = lane_id() * 4096u, troot = sm.tv[0];
    const uint32_t v = a + 4 <= troot ? *reinterpret_cast<const uint32_t *>(out + a) : 0u;
    if (v == 0x9E3779B9u) sm.warm_sink = v;   // keeps the read; the value is irrelevant
  }
  for (int d = maxd - 1; d >= 1; --d) merge_level<C, RESIDENT, false, FLAT>(sm, d, out);
  merge_level<C, RESIDENT, true, FLAT>(sm, 0, out);
}

// The block's extent and owner from the first 48 bytes of its record.
__device__ __forceinline__ BlockExt load_ext(const ParsedBlock *rec) {
  const uint4 *p = reinterpret_cast<const uint4 *>(rec);
  const uint4 a = p[0], c = p[1], o = p[2];
  BlockExt e;
  e.blk = (static_cast<uint64_t>(a.y) << 32) | a.x;
  e.end = (static_cast<uint64_t>(a.w) << 32) | a.z;
  e.ans_word0 = (static_cast<uint64_t>(c.y) << 32) | c.x;
  e.ans_words = c.z;
  e.err = static_cast<int32_t>(c.w);
  e.in = reinterpret_cast<const uint8_t *>((static_cast<uint64_t>(o.y) << 32) | o.x);
  e.job = o.z;
  e.pad = 0;
  return e;
}

// Whether block ext is decoded from LDS: the whole block (header and raw
// bodies, 16-byte aligned) plus its decoded rANS bitmaps fit.
template <class C>
__device__ __forceinline__ bool block_resident(const BlockExt &ext) {
  const uint64_t span = ((ext.end + 15) & ~15ull) - (ext.blk & ~15ull);
  return !ext.err && span + 4ull * ext.ans_words + 64 <= static_cast<uint64_t>(C::BODY);
}

// Loads the block's parsed header (its record) and, when resident, the block
// itself and its decoded rANS bitmaps into LDS with 16-byte direct-to-LDS
// reads (global_load_lds_dwordx4: lane i of a wave fills LDS bytes
// [16 i, 16 i + 16) after the wave's base); wave iterations that touch the
// end of the stream use guarded loads instead.  Ends with a barrier.
template <class C>
__device__ void load_block(const JobDev &J, const ParsedBlock *rec, const BlockExt &ext,
                           const uint32_t *scratch, uint64_t scratch_words, MergeSmem<C> &sm) {
  const int tid = item_tid();
  const int wave = wave_id();
  const uint32_t lane = lane_id();
  constexpr uint32_t kRec16 = kRecWhole16;
  const uint8_t *rb = reinterpret_cast<const uint8_t *>(rec);
  uint32_t *pbw = reinterpret_cast<uint32_t *>(&sm.pb);
  for (uint32_t base = kWave * wave; base < kRec16; base += kWave * C::NW)
    if (base + lane < kRec16)
      __builtin_amdgcn_global_load_lds(rb + 16ull * (base + lane), &pbw[4 * base], 16, 0, 0);
  if (block_resident<C>(ext)) {
    const uint64_t g0 = ext.blk & ~15ull;
    const uint64_t span = ((ext.end + 15) & ~15ull) - g0;
    // the job's stream pointer and length in registers: read from the job
    // table inside the loop, each read would wait for every direct-to-LDS
    // load issued before it (a global load's s_waitcnt vmcnt counts them)
    const uint8_t *const jin = J.in;
    const uint64_t jlen = J.in_len;
    const uint64_t in_dw = jlen >> 2;
    const uint64_t in16 = jlen >> 4;
    const uint32_t *gin = reinterpret_cast<const uint32_t *>(jin);
    const uint32_t n16 = static_cast<uint32_t>(span >> 4);
    for (uint32_t base = kWave * wave; base < n16; base += kWave * C::NW) {
      if (base + kWave <= n16 && (g0 >> 4) + base + kWave <= in16) {
        __builtin_amdgcn_global_load_lds(jin + g0 + 16ull * (base + lane), &sm.body[4 * base], 16, 0, 0);
      } else {
        const uint32_t i = base + lane;
        if (i < n16) {
          const uint64_t q = (g0 >> 2) + 4ull * i;
          uint4 v;
          v.x = q < in_dw ? gin[q] : 0u;
          v.y = q + 1 < in_dw ? gin[q + 1] : 0u;
          v.z = q + 2 < in_dw ? gin[q + 2] : 0u;
          v.w = q + 3 < in_dw ? gin[q + 3] : 0u;
          *reinterpret_cast<uint4 *>(&sm.body[4 * i]) = v;
        }
      }
    }
    const uint32_t abase = static_cast<uint32_t>(span >> 2);
    for (uint32_t i = tid; i < ext.ans_words; i += C::NT) {
      const uint64_t q = ext.ans_word0 + i;
      sm.body[abase + i] = q < scratch_words ? scratch[q] : 0u;
    }
    const uint32_t body_dw = abase + ext.ans_words;
    for (uint32_t i = body_dw + tid; i < ((body_dw + 7) & ~7u) + 8; i += C::NT) sm.body[i] = 0u;
  }
  __builtin_amdgcn_s_waitcnt(0);     // direct-to-LDS loads of this wave have landed
  __syncthreads();
}

// The look-ahead of the persistent loop: the next item, its extent, and
// where its bytes and record are (for warming the cache).  Held by one
// thread (64) from the start of a block until publish_next puts it in LDS.
struct Lookahead {
  uint32_t item;             // next work item (n_items: none)
  uint2 rt;                  // its (record, tile) pair
  BlockExt ext;              // its block's extent and job
  const uint8_t *in;         // its stream (null: nothing to warm)
  const uint8_t *rec;        // its record
};

template <class C>
__device__ __forceinline__ void publish_next(MergeSmem<C> &sm, const Lookahead &la) {
  if (threadIdx.x != kWave) return;
  sm.item = la.item;
  sm.nxt_item = la.rt;
  sm.nxt = la.ext;
  sm.warm_in = la.in;
  sm.warm_rec = la.rec;
}

// Wave 1 reads a word of every 128-byte line of the next block (if it would
// be resident) and of its record, and waits for them, so that the next
// load_block finds them in the cache.  Runs while wave 0 computes the first
// tile's shares and the other waves are idle.
template <class C>
__device__ void warm_next(MergeSmem<C> &sm) {
  const uint32_t lane = lane_id();
  const uint8_t *in = sm.warm_in;
  if (!in) return;
  const uint8_t *rec = sm.warm_rec;
  const uint64_t blk = sm.nxt.blk, end = sm.nxt.end;
  // every load is issued before any is consumed (one memory round trip)
  constexpr int NB = (C::BODY + 127) / (128 * kWave) + 1;            // lines per lane: block
  constexpr int NR = (16 * kRecWhole16 + 128 * kWave - 1) / (128 * kWave);        // and record
  uint32_t v[NB + NR];
  const bool fits = end > blk && end - blk <= static_cast<uint64_t>(C::BODY);
  const uint64_t a0 = (blk & ~127ull) + 128ull * lane;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint64_t a = a0 + 128ull * kWave * k;
    v[k] = fits && a < end ? *reinterpret_cast<const uint32_t *>(in + a) : 0u;
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const uint32_t a = 128 * (lane + kWave * k);
    v[NB + k] = a < 16 * kRecWhole16 ? *reinterpret_cast<const uint32_t *>(rec + a) : 0u;
  }
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < NB + NR; ++k) acc ^= v[k];
  if (acc == 0x9E3779B9u) sm.warm_sink = acc;   // keeps the reads; the value is irrelevant
}

// Selector for v_perm_b32(R, L, sel) per 4 bitmap bits: output byte k takes
// the left sequence's next byte (values 0-3) or the right one's (values 4-7).
template <class C>
__device__ __forceinline__ void init_sel(MergeSmem<C> &sm) {
  const uint32_t tid = threadIdx.x;
  if (tid < 16) {
    uint32_t s = 0, ones = 0;
    for (int k = 0; k < 4; ++k) {
      const uint32_t bit = (tid >> k) & 1;
      const uint32_t v = bit ? 4 + ones : k - ones;
      s |= v << (8 * k);
      ones += bit;
    }
    sm.sel[tid] = s;
  }
}

// n copies of symbol c at out (a constant block or tile).
template <class C>
__device__ void fill_constant(uint8_t *out, uint32_t n, uint32_t c) {
  const uint32_t tid = threadIdx.x;
  const uint32_t c4 = c * 0x01010101u;
  const uint32_t head = static_cast<uint32_t>((4 - (reinterpret_cast<uintptr_t>(out) & 3)) & 3);
  for (uint32_t i = tid; i < n && i < head; i += C::NT) out[i] = static_cast<uint8_t>(c);
  if (n > head) {
    uint32_t *o4 = reinterpret_cast<uint32_t *>(out + head);
    const uint32_t nd = (n - head) / 4;
    for (uint32_t i = tid; i < nd; i += C::NT) o4[i] = c4;
    for (uint32_t i = head + 4 * nd + tid; i < n; i += C::NT) out[i] = static_cast<uint8_t>(c);
  }
}

// Rank directory over the first body_dw words of sm.body: per 256-bit
// superblock the 1 bits before it, per 64-bit word the 1 bits of its
// superblock before it; then every node's rank at its first bit (sm.abit).
// Ends with a barrier only when `last` is set: otherwise the caller's next
// barrier orders the ranks before their readers.
template <class C>
__device__ void build_directory(MergeSmem<C> &sm, uint32_t body_dw, uint32_t I, bool last) {
  const uint32_t tid = item_tid();
  const uint32_t wave = wave_id();
  const uint32_t lane = lane_id();
  const uint32_t nsb = (body_dw + 7) / 8 + 1;
  const uint32_t per = (nsb + C::NT - 1) / C::NT;
  const uint32_t s0 = tid * per;
  uint32_t loc = 0;
  for (uint32_t k = s0; k < s0 + per && k < nsb; ++k) {
    const uint4 a = *reinterpret_cast<const uint4 *>(&sm.body[8 * k]);
    const uint4 c = *reinterpret_cast<const uint4 *>(&sm.body[8 * k + 4]);
    const uint32_t w0 = __popc(a.x) + __popc(a.y), w1 = __popc(a.z) + __popc(a.w);
    const uint32_t w2 = __popc(c.x) + __popc(c.y), w3 = __popc(c.z) + __popc(c.w);
    *reinterpret_cast<uint32_t *>(&sm.rel[4 * k]) = (w0 << 8) | ((w0 + w1) << 16) | ((w0 + w1 + w2) << 24);
    const uint32_t cnt = w0 + w1 + w2 + w3;
    sm.sup[k] = cnt;
    loc += cnt;
  }
  const uint32_t inc = wave_incl_scan(loc);
  if (lane == kWave - 1) sm.scan_tot[wave] = inc;
  lds_barrier();
  uint32_t run = inc - loc + sum_first(sm.scan_tot, wave);
  for (uint32_t k = s0; k < s0 + per && k < nsb; ++k) {
    const uint32_t c = sm.sup[k];
    sm.sup[k] = run;
    run += c;
  }
  lds_barrier();
  for (uint32_t i = tid; i < I; i += C::NT) {
    const uint32_t r = rank_at(sm.body, sm.sup, sm.rel, sm.abit[i]);
    sm.r0[i] = r;
    sm.arank[i] = r;
  }
  if (last) lds_barrier();
}

// Decodes the block whose record (and, when resident, body) load_block put
// into LDS, with the whole workgroup; or, for k != kWholeBlock, tile k of a
// split block that load_tile put into LDS (its shares are known: there is no
// count phase and no end-of-block check, the boundary kernel validated the
// block's bitmaps).
template <class C>
__device__ void decode_block(const JobDev &J, const BlockExt &ext, uint32_t k,
                             const uint32_t *scratch, uint64_t scratch_words, MergeSmem<C> &sm,
                             const Lookahead &la) {
  const int tid = item_tid();
  const int wave = wave_id();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  const bool tiled = k != kWholeBlock;
  const bool resident = tiled || block_resident<C>(ext);
  const uint64_t g0 = ext.blk & ~15ull;
  const uint64_t span = ((ext.end + 15) & ~15ull) - g0;
  if (h.err) {
    publish_next<C>(sm, la);
    if (tid == 0) set_err(J.status, h.err);
    return;
  }
  uint8_t *out = J.out + h.out_off;
  uint32_t n = h.n;
  if (tiled) {
    out += static_cast<uint64_t>(k) * kTileOut;
    n = n - k * kTileOut < kTileOut ? n - k * kTileOut : kTileOut;
  }
  if (h.mode == 1) {                 // constant block
    publish_next<C>(sm, la);
    fill_constant<C>(out, n, h.csym);
    return;
  }
  const uint32_t I = h.I;
  if (tiled) {
    // the tile's shares stand in for the nodes' sizes: a variant whose tiles
    // are smaller than a split block's tile walks the shares sub-tile by
    // sub-tile like a whole block
    for (uint32_t i = tid; i < I; i += C::NT) {
      sm.cur[i] = 0;
      t.nv[i] = sm.tv[i];
    }
    if (tid == 0) sm.tile = C::T;
    build_directory<C>(sm, 4 * sm.stage_top, I, n == 0);   // the tile loop's first barrier follows
  } else {
    if (resident) {
      const uint32_t lb = static_cast<uint32_t>(h.blk - g0);
      const uint32_t abase = static_cast<uint32_t>(span >> 2);
      for (uint32_t i = tid; i < I; i += C::NT)
        sm.abit[i] = 8 * (t.kind[i] ? 4 * (abase + t.boff[i]) : lb + t.boff[i]);
    }
    for (uint32_t i = tid; i < I; i += C::NT) {
      sm.cur[i] = 0;
      sm.tv[i] = 0;
      if (!resident) sm.ones[i] = 0;
    }
    if (!resident && wave == 0) {            // symbols passing each level, for the tile size
      const uint32_t lane = lane_id();
      if (lane < 17) h.lvl_total[lane] = 0;
      wave_sync_lds();
      for (uint32_t v = lane; v < I; v += kWave)
        atomicAdd(reinterpret_cast<unsigned long long *>(&h.lvl_total[t.depth[v]]),
                  static_cast<unsigned long long>(t.nv[v]) * (t.fd[v] ? t.fd[v] : 1u));
      wave_sync_lds();
    }
    if (tid == 0) {
      sm.tile = resident ? C::T : pick_tile_streaming<C>(h, t);
      if (!resident) sm.obase[0] = 0;      // shares the union with the resident arrays
    }
    // build_directory's barriers order the writes above before their readers
    if (resident) build_directory<C>(sm, static_cast<uint32_t>(span >> 2) + h.ans_words, I, n == 0);
    else lds_barrier();
  }
  const uint32_t T = sm.tile;
  const uint32_t maxd = h.maxlen;        // internal levels are 0 .. maxd-1
  const bool flat = h.nflat != 0;
  bool bad = false;

  publish_next<C>(sm, la);            // visible after the next barrier
  // a split block's tile is one pass whose shares are known: the task lists'
  // first barrier orders the rank directory's last writes before their
  // readers, and the root's share already is troot
  const bool one_tile = tiled && C::T >= static_cast<int>(kTileOut);
  for (uint32_t t0 = 0; t0 < n; t0 += T) {
    const uint32_t troot = n - t0 < T ? n - t0 : T;
    if (tid == 0) {
      sm.stage_top = 0;
      sm.act_run = 0;
      sm.tv[0] = troot;
    }
    if (!one_tile) lds_barrier();
    if (resident) {
      if (!tiled || C::T < kTileOut) {
        if (t0 + troot < n) {
          if (wave == 0) count_chain<C>(sm);
          else if (wave == 1 && t0 == 0) warm_next<C>(sm);
        } else {
          count_last<C>(sm);
        }
        lds_barrier();
      }
      if (flat) tile_lists<C, true>(sm);
      else tile_lists<C, false>(sm);
    } else {
      for (uint32_t d = 0; d < maxd; ++d) {
        stage_level_streaming<C>(J, sm, d, scratch, scratch_words);
        lds_barrier();
        if (wave == 0) {
          if (flat) count_level_streaming<C, true>(sm, d);
          else count_level_streaming<C, false>(sm, d);
        }
        lds_barrier();
      }
    }
    if (h.err) { bad = true; break; }
    // blocks without flat nodes run code with no flat paths in it
    if (resident) {
      if (flat) merge_tile<C, true, true>(sm, static_cast<int>(maxd), out + t0, !tiled);
      else merge_tile<C, true, false>(sm, static_cast<int>(maxd), out + t0, !tiled);
    } else {
      if (flat) merge_tile<C, false, true>(sm, static_cast<int>(maxd), out + t0, !tiled);
      else merge_tile<C, false, false>(sm, static_cast<int>(maxd), out + t0, !tiled);
    }
    if (!resident) {
      for (uint32_t i = tid; i < I; i += C::NT) sm.tv[i] = 0;
      lds_barrier();
    }
  }
  if (!bad && !tiled) {
    for (uint32_t i = tid; i < I; i += C::NT) {
      const uint32_t ones = resident ? sm.arank[i] - sm.r0[i] : sm.ones[i];
      if (sm.cur[i] != t.nv[i] || (!t.fd[i] && ones != t.nr[i]))    // any D-bit value is a symbol
        atomicCAS(&h.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
    }
  }
  lds_barrier();
  if (tid == 0 && h.err) set_err(J.status, h.err);
}

// A tile of a split block: the block's record and the tile's two boundary
// rows (each node's position at the tile's start and end), then every node's
// share of the tile -- the covering 16-byte chunks of its bitmap, from the
// stream or from the rANS scratch -- gathered into LDS, node after node.
// After its last barrier sm.cur and sm.tv hold the shares and sm.stage_top
// the staged words; sm.abit (the LDS bit address of each share's first bit)
// is written by thread v for node v after that barrier.
template <class C>
__device__ void load_tile(const JobDev &J, const ParsedBlock *rec, const uint2 *tab, uint32_t k,
                          const uint32_t *scratch, uint64_t scratch_words, MergeSmem<C> &sm) {
  const int tid = item_tid();
  const int wave = wave_id();
  const uint32_t lane = lane_id();
  constexpr uint32_t kRec16 = kRecTile16;
  const uint8_t *rb = reinterpret_cast<const uint8_t *>(rec);
  uint32_t *pbw = reinterpret_cast<uint32_t *>(&sm.pb);
  for (uint32_t base = kWave * wave; base < kRec16; base += kWave * C::NW)
    if (base + lane < kRec16)
      __builtin_amdgcn_global_load_lds(rb + 16ull * (base + lane), &pbw[4 * base], 16, 0, 0);
  for (uint32_t v = tid; v < kTabCols; v += C::NT) {
    const uint32_t a = tab[static_cast<uint64_t>(k) * kTabCols + v].x;
    const uint32_t b = tab[static_cast<uint64_t>(k + 1) * kTabCols + v].x;
    sm.cur[v] = a;
    sm.tv[v] = b > a ? b - a : 0u;
  }
  // the job's stream pointer and length, read with the record
  const uint8_t *const jin = reinterpret_cast<const uint8_t *>(uniform64(reinterpret_cast<uint64_t>(J.in)));
  const uint64_t jlen = uniform64(J.in_len);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  BlockHdr &h = sm.pb.h;
  NodeTab &t = sm.pb.t;
  if (h.err || h.mode == 1) return;     // decode_block reports or fills
  const uint32_t I = h.I;
  // chunk counts and their exclusive prefix over the nodes (block scan)
  uint32_t nch = 0;
  uint64_t a16 = 0, gb = 0;
  if (static_cast<uint32_t>(tid) < I && sm.tv[tid]) {
    const uint32_t dv = t.fd[tid] ? t.fd[tid] : 1u;     // bits per symbol
    gb = (t.kind[tid] ? 32ull * (h.ans_word0 + t.boff[tid]) : 8ull * (h.blk + t.boff[tid])) +
         static_cast<uint64_t>(dv) * sm.cur[tid];
    a16 = (gb >> 3) & ~15ull;
    const uint64_t b16 = (((gb + static_cast<uint64_t>(dv) * sm.tv[tid] + 7) >> 3) + 15) & ~15ull;
    nch = static_cast<uint32_t>((b16 - a16) >> 4);
  }
  const uint32_t inc = tid < 256 ? wave_incl_scan(nch) : 0u;
  if (tid < 256 && lane == kWave - 1) sm.scan_tot[wave] = inc;
  lds_barrier();
  const uint32_t before = tid < 256 ? sum_first(sm.scan_tot, static_cast<uint32_t>(wave)) : 0u;
  if (static_cast<uint32_t>(tid) < I) {
    sm.stg[tid] = inc - nch + before;   // first staged chunk of the node
    sm.ones[tid] = nch;                 // its chunks
  }
  if (wave == 0) {
    const uint32_t tot = sum_first(sm.scan_tot, 4);
    if (tid == 0) sm.stage_top = tot;
  }
  lds_barrier();
  const uint32_t total = sm.stage_top;
  if (16ull * total + 64 > static_cast<uint64_t>(C::BODY)) {   // cannot happen for 12-bit codes
    if (tid == 0) atomicCAS(&h.err, 0, static_cast<int32_t>(PIVCO_E_UNSUPPORTED));
    lds_barrier();
    return;
  }
  // copy: the staged chunks in order, C::NT per step.  Staged chunk s (of
  // node v, stg[v] <= s < stg[v] + ones[v]) goes to LDS slot s, so a wave's
  // 64 lanes fill 64 consecutive slots with one direct-to-LDS load, each lane
  // gathering from its own node's range; chunks not wholly inside their
  // buffer take guarded byte loads afterwards.  Every source address is
  // computed (LDS reads) before the first load is issued: a direct-to-LDS
  // load writes LDS, so an LDS or global read issued after it waits for
  // every such load in flight.
  constexpr uint32_t KS = (C::BODY / 16 + C::NT - 1) / C::NT;
  for (uint32_t i = 4 * total + tid; i < 4 * total + 16; i += C::NT) sm.body[i] = 0u;   // not a load target
  uint64_t qa[KS];          // source byte offset of the lane's chunk at each step
  uint32_t inb = 0, scr = 0;  // bit k: step k's chunk lies inside its buffer / comes from scratch
#pragma unroll
  for (uint32_t k = 0; k < KS; ++k) {
    const uint32_t sc = k * C::NT + static_cast<uint32_t>(tid);
    qa[k] = 0;
    if (sc < total) {
      uint32_t lo = 0, hi = I;                  // the last node whose chunks start at or before sc
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sm.stg[mid] <= sc) lo = mid; else hi = mid;
      }
      const uint32_t v = lo;
      const bool kind = t.kind[v] != 0;
      const uint64_t g = (kind ? 32ull * (h.ans_word0 + t.boff[v]) : 8ull * (h.blk + t.boff[v])) +
                         static_cast<uint64_t>(t.fd[v] ? t.fd[v] : 1u) * sm.cur[v];
      const uint64_t q = ((g >> 3) & ~15ull) + 16ull * (sc - sm.stg[v]);
      qa[k] = q;
      if (q + 16 <= (kind ? 4ull * scratch_words : jlen)) inb |= 1u << k;
      if (kind) scr |= 1u << k;
    }
  }
  const uint8_t *const sbase = reinterpret_cast<const uint8_t *>(scratch);
#pragma unroll
  for (uint32_t k = 0; k < KS; ++k) {
    const uint32_t b = k * C::NT + kWave * static_cast<uint32_t>(wave);   // the wave's first slot
    if (b < total && ((inb >> k) & 1))
      __builtin_amdgcn_global_load_lds(((scr >> k) & 1 ? sbase : jin) + qa[k], &sm.body[4 * b], 16, 0, 0);
  }
#pragma unroll
  for (uint32_t k = 0; k < KS; ++k) {
    const uint32_t sc = k * C::NT + static_cast<uint32_t>(tid);
    if (sc < total && !((inb >> k) & 1)) {
      const bool kind = (scr >> k) & 1;
      const uint8_t *src = kind ? sbase : jin;
      const uint64_t lim = kind ? 4ull * scratch_words : jlen;
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t x = 0;
        for (int by = 0; by < 4; ++by) {
          const uint64_t a = qa[k] + 4 * e + by;
          if (a < lim) x |= static_cast<uint32_t>(src[a]) << (8 * by);
        }
        w[e] = x;
      }
      *reinterpret_cast<uint4 *>(&sm.body[4 * sc]) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // LDS bit address of each share's first bit (abit shares its words with
  // tone, not with stg or ones); read after the rank directory's first
  // barrier
  if (static_cast<uint32_t>(tid) < I)
    sm.abit[tid] = sm.tv[tid] ? 128u * sm.stg[tid] + static_cast<uint32_t>(gb - 8 * a16) : 0u;
}

// Persistent merge: a workgroup takes items from the queue (largest first) --
// whole blocks, or tiles of split blocks -- looking one item ahead.  `single`
// selects the item source: kQueueItems (the persistent queue), kGridItems
// (workgroup b decodes item b and exits: one non-persistent launch with a
// workgroup per item), or an item index (one item, one workgroup).
template <class C>
__global__ __launch_bounds__(C::NT) void k_merge(const JobDev *jobs, const uint2 *items,
                                                  const ParsedBlock *recs,
                                                  const TiledBlock *tiled, const uint2 *tab,
                                                  uint32_t n_items, Counters *ctr,
                                                  const uint32_t *scratch, uint64_t scratch_words,
                                                  int32_t single) {
  __shared__ MergeSmem<C> sm;
  const int tid = threadIdx.x;
  for (int i = tid; i < 256; i += C::NT) sm.leafrow[i] = static_cast<uint32_t>(i) * 0x01010101u;
  init_sel<C>(sm);
  if (tid == 0) {
    const uint32_t it = single >= 0            ? static_cast<uint32_t>(single)
                        : single == kGridItems ? blockIdx.x
                                               : atomicAdd(&ctr->merge_next, 1u);
    sm.item = it;
    if (it < n_items) {
      const uint2 rt = items[it];
      sm.nxt_item = rt;
      sm.nxt = load_ext(recs + rt.x);
    }
  }
  lds_barrier();
  for (;;) {
    const uint32_t it = sm.item;
    if (it >= n_items) break;
    const uint2 rt = sm.nxt_item;
    const BlockExt ext = sm.nxt;
    lds_barrier();                   // the look-ahead slots are rewritten below
    // look ahead (thread 64, in a wave that is idle while wave 0 computes
    // the first tile's shares): take the next item now; its extent and
    // stream are read while this item is decoded, and published to LDS
    // before the merge (or when the item ends early)
    Lookahead la{n_items, make_uint2(0, 0), BlockExt{}, nullptr, nullptr};
    if (tid == kWave && single == kQueueItems) la.item = atomicAdd(&ctr->merge_next, 1u);
    const JobDev &J = jobs[ext.job];
    const bool whole = rt.y == kWholeBlock;
    if (whole) {
      load_block<C>(J, recs + rt.x, ext, scratch, scratch_words, sm);
    } else {
      const TiledBlock tb = tiled[rt.y >> 8];
      load_tile<C>(J, recs + rt.x, tab + tb.tab, rt.y & 255, scratch, scratch_words, sm);
    }
    if (tid == kWave && la.item < n_items) {
      la.rt = items[la.item];
      la.ext = load_ext(recs + la.rt.x);
      la.in = la.ext.err || la.rt.y != kWholeBlock ? nullptr : la.ext.in;
      la.rec = reinterpret_cast<const uint8_t *>(recs + la.rt.x);
    }
    decode_block<C>(J, ext, whole ? kWholeBlock : rt.y & 255, scratch, scratch_words, sm, la);
    lds_barrier();
  }
}

// Bits [b0, b1) of a 32-bit word whose first bit is bit wb.
__device__ __forceinline__ uint32_t range_mask(uint64_t wb, uint64_t b0, uint64_t b1) {
  const uint64_t lo = b0 > wb ? b0 - wb : 0;
  const uint64_t hi = b1 >= wb + 32 ? 32 : (b1 > wb ? b1 - wb : 0);
  if (hi <= lo) return 0u;
  const uint32_t mh = hi >= 32 ? 0xFFFFFFFFu : (1u << hi) - 1;
  return mh & ~((1u << lo) - 1);
}

// The 16-byte chunk at byte q of p (16-byte aligned): one unconditional
// load, so that a thread's chunk loads can all be in flight.  A chunk that
// is not wholly inside the nbytes readable is loaded from the last 16 bytes
// instead (the buffers hold at least 16), and chunk_popc counts only the
// bits of the chunk at q that it holds.
struct Chunk {
  uint4 x;
  uint64_t at;             // byte offset the 16 bytes were loaded from
};
__device__ __forceinline__ Chunk chunk_load(const uint8_t *p, uint64_t nbytes, uint64_t q) {
  const uint64_t at = q + 16 <= nbytes ? q : (nbytes >= 16 ? nbytes - 16 : 0);
  Chunk c;
  c.x = *reinterpret_cast<const uint4 *>(p + at);
  c.at = at;
  return c;
}
// 1 bits of the chunk at byte q inside bits [b0, b1) (bit addresses relative
// to p; b1 never past the readable bytes): the range is cut to the chunk and
// made relative to the loaded bytes, then each word's part is extracted.
__device__ __forceinline__ uint32_t chunk_popc(const Chunk &c, uint64_t q, uint64_t b0, uint64_t b1) {
  const int64_t base = 8 * static_cast<int64_t>(c.at);
  const int64_t l64 = static_cast<int64_t>(b0 > 8 * q ? b0 : 8 * q) - base;
  const int64_t h64 = static_cast<int64_t>(b1 < 8 * q + 128 ? b1 : 8 * q + 128) - base;
  const int lo = static_cast<int>(l64 < 0 ? 0 : l64 > 128 ? 128 : l64);
  const int hi = static_cast<int>(h64 < 0 ? 0 : h64 > 128 ? 128 : h64);
  const uint32_t w[4] = {c.x.x, c.x.y, c.x.z, c.x.w};
  uint32_t n = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = lo - 32 * e < 0 ? 0 : lo - 32 * e > 32 ? 32 : lo - 32 * e;
    const int h = hi - 32 * e < 0 ? 0 : hi - 32 * e > 32 ? 32 : hi - 32 * e;
    const int wd = h > l ? h - l : 0;
    const uint32_t bits = wd >= 32 ? w[e] : __builtin_amdgcn_ubfe(w[e], static_cast<uint32_t>(l) & 31u,
                                                                  static_cast<uint32_t>(wd));
    n += __popc(bits);
  }
  return n;
}

// chunk_popc with a fast path for a chunk wholly inside [b0, b1).
__device__ __forceinline__ uint32_t chunk_count(const Chunk &c, uint64_t q, uint64_t b0, uint64_t b1) {
  if (c.at == q && 8 * q >= b0 && 8 * q + 128 <= b1)
    return __popc(c.x.x) + __popc(c.x.y) + __popc(c.x.z) + __popc(c.x.w);
  return chunk_popc(c, q, b0, b1);
}

// Boundaries of a split block (one workgroup per block).  A node's rank at
// a position (its 1 bits before it) is a difference of prefix counts over
// the region its bitmap lies in: the raw bitmaps follow each other in the
// block (their padding bits are zero), and so do the decoded rANS bitmaps in
// the scratch buffer (decoded words end in zero bits).  So the kernel first
// builds one rank directory per region: the region is cut at the absolute
// G-bit boundaries of its buffer (G = 512 .. 8192: the smallest whose
// directory fits), the 1 bits of each piece are counted by spr = G/128
// consecutive lanes (one 16-byte chunk each: the region is streamed with
// coalesced loads, four steps in flight) and exclusive-scanned in two levels
// (per superblock of kTilesSB pieces a 32-bit count of the region's 1 bits
// before it, per piece a 16-bit count of the superblock's before it; the
// second region starts a superblock of its own).  Then P(x), the region's 1
// bits before bit x, is a directory entry plus or minus one popcount of at
// most half a piece (region_prefix), and node
// v's rank at position s is P(start_v + s) - P(start_v).  Top-down by level,
// every (node, boundary) pair of the level is one thread: node v's position
// at boundary k (symbols of the block before k * kTileOut that pass it)
// gives its rank there, and the rank the right child's position (position -
// rank the left child's).  The root's positions are k * kTileOut.
// Positions live in LDS when the block's table fits, else in the table
// itself.  Table row k, column v holds (position, rank).  A node whose
// bitmap holds a different number of 1 bits than its header count marks the
// job corrupt; positions are clamped to the nodes' sizes so that the tiles
// never read outside their bitmaps.  A flat node (v2 streams) has leaves
// only: its positions are all a tile needs (D bits per position).
constexpr int kTilesNT = 1024;
constexpr uint32_t kTilesDir = 32768;     // directory pieces (LDS)
constexpr uint32_t kTilesSB = 8;          // pieces per directory superblock
constexpr uint32_t kTilesPos = 16384;     // positions kept in LDS
constexpr int kTilesG = 5;                // piece sizes 512 << e, e < kTilesG

// A bit region of a split block: bits [b0, b1) of buffer p (nb readable).
struct TileRegion {
  const uint8_t *p;
  uint64_t nb, b0, b1;
  uint32_t d0;             // its first directory entry
  uint32_t np;             // its pieces
};

struct TilesSmem {
  ParsedBlock pb;
  uint16_t rel[kTilesDir];                // 1 bits of the superblock before the piece
  uint32_t sup[kTilesDir / kTilesSB + 1]; // 1 bits of the region before the superblock
  uint32_t pos[kTilesPos];                // [v * (K + 1) + k] when (K + 1) * I fits
  uint32_t pstart[256];                   // P(start of node v's bitmap)
  int32_t err;
};

// The region's 1 bits before bit x (b0 <= x <= b1), from the directory
// entry of x's piece (of the last piece when x is the region's end on a
// piece boundary): the entry plus the piece's bits before x, or, when x lies
// in the second half of a piece that is not the region's last, the next
// entry minus the piece's bits from x on.  Only the chunks that hold those
// bits are loaded (at most SPR / 2 + 1), B at a time.
template <uint32_t SPR>                            // chunks per piece: G = 128 * SPR
__device__ __forceinline__ uint32_t region_prefix(const TilesSmem &sm, const TileRegion &r, uint64_t x) {
  constexpr uint32_t LG = 31 - __builtin_clz(SPR) + 7, B = SPR < 8 ? SPR : 8;
  if (r.np == 0) return 0u;
  uint32_t j = static_cast<uint32_t>((x >> LG) - (r.b0 >> LG));
  j = j < r.np ? j : r.np - 1;
  const uint64_t sb = ((r.b0 >> LG) + j) << LG, pe = sb + (1ull << LG);
  const bool back = j + 1 < r.np && x - sb > (1ull << (LG - 1));
  // bits [lo, hi) counted; chunks from byte q0 on
  const uint64_t lo = back ? x : (sb > r.b0 ? sb : r.b0), hi = back ? pe : x;
  const uint64_t q0 = back ? (x >> 7) << 4 : sb >> 3;
  const uint32_t nck = hi > lo ? static_cast<uint32_t>((hi - 8 * q0 + 127) >> 7) : 0u;
  uint32_t n = 0;
  for (uint32_t c0 = 0; c0 < nck; c0 += B) {
    Chunk ch[B];
#pragma unroll
    for (uint32_t c = 0; c < B; ++c)       // past the last chunk: the last one again (counted once)
      ch[c] = chunk_load(r.p, r.nb, q0 + 16ull * (c0 + c < nck ? c0 + c : nck - 1));
#pragma unroll
    for (uint32_t c = 0; c < B; ++c)
      if (c0 + c < nck) n += chunk_count(ch[c], q0 + 16ull * (c0 + c), lo, hi);
  }
  const uint32_t e = r.d0 + j + (back ? 1 : 0);
  const uint32_t base = sm.sup[e / kTilesSB] + sm.rel[e];
  return back ? base - n : base + n;
}

// The level loop of k_tiles (POS_LDS: positions in sm.pos, else in the table).
template <bool POS_LDS, uint32_t SPR>
__device__ void tiles_levels(TilesSmem &sm, const TileRegion *reg, uint2 *T, uint32_t K) {
  const BlockHdr &h = sm.pb.h;
  const NodeTab &t = sm.pb.t;
  const uint32_t tid = threadIdx.x;
  for (uint32_t d = 0; d < h.maxlen; ++d) {
    const uint32_t v0 = h.lvl[d], m = h.lvl[d + 1] - v0;
    for (uint32_t q = tid; q < m * (K + 1); q += kTilesNT) {
      const uint32_t v = v0 + q / (K + 1), k = q % (K + 1);
      uint2 *row = T + static_cast<uint64_t>(k) * kTabCols;
      const uint32_t nv = t.nv[v];
      const uint32_t sp = POS_LDS ? sm.pos[v * (K + 1) + k] : row[v].x;
      const uint32_t s = sp < nv ? sp : nv;
      if (t.fd[v]) {                     // a flat node: its position only (no children, no ranks)
        row[v] = make_uint2(s, 0u);
        if (k == K && s != nv) atomicCAS(&sm.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
        continue;
      }
      const TileRegion &r = reg[t.kind[v] ? 1 : 0];
      const uint64_t gb = t.kind[v] ? 32ull * (h.ans_word0 + t.boff[v]) : 8ull * (h.blk + t.boff[v]);
      const uint32_t rk = region_prefix<SPR>(sm, r, gb + s) - sm.pstart[v];
      row[v] = make_uint2(s, rk);
      const uint32_t cc = *reinterpret_cast<const uint32_t *>(t.child[v]);
      const uint32_t c0 = cc & 0xFFFF, c1 = cc >> 16;
      if (!(c0 & 0x8000)) {
        const uint32_t x0 = s - rk < t.nv[c0] ? s - rk : t.nv[c0];
        if (POS_LDS) sm.pos[c0 * (K + 1) + k] = x0; else row[c0].x = x0;
      }
      if (!(c1 & 0x8000)) {
        const uint32_t x1 = rk < t.nv[c1] ? rk : t.nv[c1];
        if (POS_LDS) sm.pos[c1 * (K + 1) + k] = x1; else row[c1].x = x1;
      }
      if (k == K && (rk != t.nr[v] || s != nv)) atomicCAS(&sm.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
    }
    if (POS_LDS) lds_barrier();
    else __syncthreads();                          // the table's positions are read next
  }
}

// Every node's prefix at its bitmap's start, then the levels.
template <uint32_t SPR>
__device__ void tiles_prefix_levels(TilesSmem &sm, const TileRegion *reg, uint2 *T, uint32_t K,
                                    bool pos_lds) {
  const BlockHdr &h = sm.pb.h;
  const NodeTab &t = sm.pb.t;
  for (uint32_t v = threadIdx.x; v < h.I; v += kTilesNT) {
    if (t.fd[v]) { sm.pstart[v] = 0; continue; }
    const TileRegion &r = reg[t.kind[v] ? 1 : 0];
    const uint64_t gb = t.kind[v] ? 32ull * (h.ans_word0 + t.boff[v]) : 8ull * (h.blk + t.boff[v]);
    sm.pstart[v] = region_prefix<SPR>(sm, r, gb);
  }
  __syncthreads();
  if (pos_lds) tiles_levels<true, SPR>(sm, reg, T, K);
  else tiles_levels<false, SPR>(sm, reg, T, K);
}

__global__ __launch_bounds__(kTilesNT) void k_tiles(const JobDev *jobs, const TiledBlock *tiled,
                                                   uint32_t n_tiled, const ParsedBlock *recs,
                                                   const uint32_t *scratch, uint64_t scratch_words,
                                                   uint2 *tab) {
  if (blockIdx.x >= n_tiled) return;               // one workgroup per split block
  __shared__ TilesSmem sm;
  const uint32_t tid = threadIdx.x, wave = wave_id(), lane = lane_id();
  constexpr uint32_t NW = kTilesNT / kWave;
  const TiledBlock tb = tiled[blockIdx.x];
  {
    const uint4 *src = reinterpret_cast<const uint4 *>(recs + tb.rec);
    uint4 *dst = reinterpret_cast<uint4 *>(&sm.pb);
    for (uint32_t i = tid; i < sizeof(ParsedBlock) / 16; i += kTilesNT) dst[i] = src[i];
  }
  if (tid == 0) sm.err = 0;
  __syncthreads();
  const BlockHdr &h = sm.pb.h;
  const JobDev &J = jobs[h.job];
  if (h.err || h.mode == 1) return;                // the tiles report or fill
  const uint32_t K = tb.ntiles, n = h.n, I = h.I;
  uint2 *T = tab + tb.tab;
  // the two regions (the job's stream is read once: the table stores below
  // would otherwise make the compiler reload it from the job table)
  TileRegion reg[2];
  reg[0].p = J.in;
  reg[0].nb = J.in_len;
  reg[0].b0 = 8ull * (h.blk + h.raw_base);
  reg[0].b1 = 8ull * (h.blk + h.raw_end);
  reg[1].p = reinterpret_cast<const uint8_t *>(scratch);
  reg[1].nb = 4ull * scratch_words;
  reg[1].b0 = 32ull * h.ans_word0;
  reg[1].b1 = 32ull * (h.ans_word0 + h.ans_words);
  // the smallest piece size whose directory fits (the second region's
  // pieces start at a superblock boundary)
  uint32_t lg = 0, S = 0, np[2] = {0, 0};
  for (;; ++lg) {
    for (int i = 0; i < 2; ++i)
      np[i] = reg[i].b1 > reg[i].b0
                  ? static_cast<uint32_t>(((reg[i].b1 - 1) >> (9 + lg)) - (reg[i].b0 >> (9 + lg)) + 1)
                  : 0u;
    S = (np[0] + kTilesSB - 1) / kTilesSB * kTilesSB + np[1];
    if (S <= kTilesDir || lg + 1 == kTilesG) break;
  }
  if (S > kTilesDir) {                             // more than 8192 * 32Ki bitmap bits
    if (tid == 0) set_err(J.status, PIVCO_E_UNSUPPORTED);
    return;
  }
  const uint32_t LG = 9 + lg, spr = 4u << lg;      // G = 1 << LG bits = spr chunks
  reg[0].d0 = 0;
  reg[0].np = np[0];
  reg[1].d0 = S - np[1];
  reg[1].np = np[1];
  const bool pos_lds = (K + 1) * I <= kTilesPos;
  for (uint32_t k = tid; k <= K; k += kTilesNT) {
    const uint64_t s = static_cast<uint64_t>(k) * kTileOut;
    const uint32_t x = s < n ? static_cast<uint32_t>(s) : n;
    if (pos_lds) sm.pos[k] = x;
    else T[static_cast<uint64_t>(k) * kTabCols] = make_uint2(x, 0u);
  }
  // counting pass: the pieces' chunks, region after region, 64 consecutive
  // chunks a wave step (coalesced), U steps in flight; spr consecutive lanes
  // add up one piece
  {
    constexpr uint32_t U = 4, STEP = kWave * U;
    const uint32_t CT = S * spr, c0e = reg[0].np * spr, c1 = reg[1].d0 * spr;
    for (uint32_t base = wave * STEP; base < CT; base += NW * STEP) {
      Chunk x[U];
      uint64_t q[U], lo[U], hi[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t c = base + u * kWave + lane;
        const bool second = c >= c1;
        const TileRegion &r = reg[second ? 1 : 0];
        const uint32_t cr = second ? c - c1 : (c < c0e ? c : 0u);
        q[u] = ((r.b0 >> LG) << (LG - 3)) + 16ull * cr;
        lo[u] = r.b0;
        // between the regions and past the last piece: no bits
        hi[u] = c < CT && (second || c < c0e) ? r.b1 : r.b0;
        x[u] = chunk_load(second ? reg[1].p : reg[0].p, second ? reg[1].nb : reg[0].nb, q[u]);
      }
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        uint32_t m = chunk_count(x[u], q[u], lo[u], hi[u]);
        for (uint32_t sh = spr >> 1; sh >= 1; sh >>= 1) m += __shfl_xor(m, static_cast<int>(sh), static_cast<int>(spr));
        const uint32_t c = base + u * kWave + lane;
        if (c % spr == 0 && c < CT) sm.rel[c / spr] = static_cast<uint16_t>(m);   // at most 8192
      }
    }
  }
  __syncthreads();
  // exclusive scan of the directory (whole superblocks per thread): per
  // superblock the 1 bits before it, per piece those of its superblock
  // before it (at most 7 * 8192: 16 bits)
  {
    const uint32_t nsb = (S + kTilesSB - 1) / kTilesSB;
    const uint32_t per = (nsb + kTilesNT - 1) / kTilesNT;
    const uint32_t s0 = tid * per, s1 = s0 + per < nsb ? s0 + per : nsb;
    uint32_t loc = 0;
    for (uint32_t f = s0 * kTilesSB; f < s1 * kTilesSB && f < S; ++f) loc += sm.rel[f];
    const uint32_t incl = wave_incl_scan(loc);
    __shared__ uint32_t tot[kTilesNT / kWave];
    if (lane == kWave - 1) tot[wave] = incl;
    __syncthreads();
    uint32_t run = incl - loc + sum_first(tot, wave);
    __syncthreads();
    for (uint32_t sb = s0; sb < s1; ++sb) {
      sm.sup[sb] = run;
      uint32_t acc = 0;
      for (uint32_t f = sb * kTilesSB; f < (sb + 1) * kTilesSB && f < S; ++f) {
        const uint32_t c = sm.rel[f];
        sm.rel[f] = static_cast<uint16_t>(acc);
        acc += c;
      }
      run += acc;
    }
    __syncthreads();
    // the second region's prefix starts from its own first piece (the first
    // of a superblock)
    const uint32_t base1 = reg[1].np ? sm.sup[reg[1].d0 / kTilesSB] : 0u;
    __syncthreads();
    for (uint32_t sb = reg[1].d0 / kTilesSB + tid; sb < nsb; sb += kTilesNT) sm.sup[sb] -= base1;
  }
  __syncthreads();
  switch (lg) {
    case 0: tiles_prefix_levels<4>(sm, reg, T, K, pos_lds); break;
    case 1: tiles_prefix_levels<8>(sm, reg, T, K, pos_lds); break;
    case 2: tiles_prefix_levels<16>(sm, reg, T, K, pos_lds); break;
    case 3: tiles_prefix_levels<32>(sm, reg, T, K, pos_lds); break;
    default: tiles_prefix_levels<64>(sm, reg, T, K, pos_lds); break;
  }
  if (tid == 0 && sm.err) set_err(J.status, sm.err);
}

// Plan: one wave per work item parses and validates the block's header from
// a copy of its first bytes in LDS (offsets, code lengths, canonical tree,
// node table, symbol counts, body offsets, padding) and writes the result as
// the item's record.
constexpr int kPlanWaves = 4;
constexpr uint32_t kHdrMax = kBlockFixed + kLenTable + 32 + 4 * kMaxInternal;   // largest header

__global__ __launch_bounds__(kWave * kPlanWaves) void k_plan(const JobDev *jobs, const uint2 *items,
                                                             uint32_t n_items, ParsedBlock *recs,
                                                             Counters *ctr, RansChunk *chunks,
                                                             uint64_t chunk_cap) {
  __shared__ ParsedBlock pb[kPlanWaves];
  __shared__ uint32_t hdr[kPlanWaves][kHdrMax / 4 + 1];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const uint32_t it = blockIdx.x * kPlanWaves + wave;
  if (it >= n_items) return;
  const uint2 item = items[it];
  const JobDev &J = jobs[item.x];
  BlockHdr &h = pb[wave].h;
  NodeTab &t = pb[wave].t;
  if (lane == 0) {
    parse_offsets(J, item.y, h);
    h.in = J.in;
    h.job = item.x;
    h.pad = 0;
  }
  wave_sync_lds();
  const uint64_t len = h.end - h.blk;
  const uint32_t hn = h.err ? 0u : static_cast<uint32_t>(len < kHdrMax ? len : kHdrMax);
  const uint8_t *g = J.in + h.blk;
  for (uint32_t i = lane; 4 * i < hn; i += kWave) {
    uint32_t w;
    if (4 * i + 4 <= hn) {
      w = *reinterpret_cast<const uint32_t *>(g + 4 * i);      // the block is 4-byte aligned
    } else {
      w = 0;
      for (uint32_t k = 0; 4 * i + k < hn; ++k) w |= static_cast<uint32_t>(g[4 * i + k]) << (8 * k);
    }
    hdr[wave][i] = w;
  }
  wave_sync_lds();
  parse_block_wave(J, item.y, h, t, SplitBytes{reinterpret_cast<const uint8_t *>(hdr[wave]), hn, g});
  if (lane == 0) {
    h.chunk0 = 0;
    h.nchunk = 0;
    if (!h.err && h.mode == 0 && h.n_ans) {
      const int32_t e = walk_rans(J, h, t, ctr, chunks, chunk_cap);
      if (e) h.err = e;
    }
  }
  wave_sync_lds();
  const uint4 *src = reinterpret_cast<const uint4 *>(&pb[wave]);
  uint4 *dst = reinterpret_cast<uint4 *>(recs + it);
  for (uint32_t i = lane; i < sizeof(ParsedBlock) / 16; i += kWave) dst[i] = src[i];
}

// Resets the queue heads and the per-job status words (graph-safe: a kernel,
// not a memset node).
__global__ void k_init(Counters *ctr, int32_t *status, const int32_t *status0, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) { ctr->merge_next = 0; ctr->rans_next = 0; ctr->rans_chunks = 0; ctr->fse_next = 0; }
  if (i < count) status[i] = status0[i];
}

// Copies the 48-byte header of every job's stream into hdr (planning).
__global__ void k_gather_headers(const pivco_job *jobs, uint32_t count, uint8_t *hdr) {
  const uint32_t j = blockIdx.x;
  if (j >= count) return;
  const uint32_t i = threadIdx.x;
  if (i < kHeaderBytes) {
    const pivco_job jb = jobs[j];
    hdr[static_cast<uint64_t>(j) * kHeaderBytes + i] =
        i < jb.in_len ? static_cast<const uint8_t *>(jb.d_in)[i] : 0;
  }
}

// ---------------------------------------------------------------------------
// Kernel: top-down decode (ablation of the bottom-up merge)
// ---------------------------------------------------------------------------
// The decoding of Sec. 2.1, before the paper turns it bottom-up (Sec. 3): for
// a slice of output positions, the root splits the positions by its bits,
// stably, into one list per child (the partition primitive); every internal
// node does the same with the positions that reach it, reading its bitmap
// from its cursor on; a leaf writes its symbol at the positions that reach
// it (the scatter primitive).  Here a slice is kTdS outputs, the position
// lists are 16-bit entries in LDS (two level buffers), the slice's output is
// assembled in LDS and stored with 16-byte stores.  One wave per node: it
// counts the node's 1 bits in the slice, reserves its children's lists, then
// partitions with ballot + mbcnt ranks.  Work items are the merge kernel's:
// whole blocks (cursors from 0) or tiles of split blocks (cursors from the
// boundary table).
constexpr int kTdNT = 256;
constexpr uint32_t kTdS = 4096;

struct TdSmem {
  ParsedBlock pb;
  uint32_t cur[256];         // node's bits consumed so far
  uint32_t ones[256];        // of which 1 bits
  uint32_t tv[256];          // node's positions in this slice
  uint32_t seg[256];         // their list in the level buffer of the node's depth
  uint32_t top[2];           // next free entry of each level buffer
  uint32_t item;
  int32_t err;
  uint16_t pos[2][kTdS];
  uint8_t out[kTdS] __attribute__((aligned(16)));
};

// Bit x of a node's bitmap: raw bodies are read byte-wise from the stream,
// decoded rANS bitmaps word-wise from the scratch.
__device__ __forceinline__ uint32_t td_bit(const uint8_t *in, const uint32_t *scr, bool rans,
                                           uint64_t base, uint64_t x) {
  const uint64_t b = base + x;
  return rans ? (scr[b >> 5] >> (b & 31)) & 1u : (in[b >> 3] >> (b & 7)) & 1u;
}

__global__ __launch_bounds__(kTdNT) void k_topdown(const JobDev *jobs, const uint2 *items,
                                                   const ParsedBlock *recs, const TiledBlock *tiled,
                                                   const uint2 *tab, uint32_t n_items, Counters *ctr,
                                                   const uint32_t *scratch, int32_t single) {
  __shared__ TdSmem sm;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  constexpr uint32_t NW = kTdNT / kWave;
  const uint64_t lt = (1ull << lane) - 1;
  for (uint32_t round = 0;; ++round) {
    if (tid == 0)
      sm.item = single >= 0 ? (round == 0 ? static_cast<uint32_t>(single) : n_items)
                : single == kGridItems ? (round == 0 ? blockIdx.x : n_items)
                                       : atomicAdd(&ctr->merge_next, 1u);
    __syncthreads();
    const uint32_t it = sm.item;
    if (it >= n_items) break;
    const uint2 rt = items[it];
    {
      const uint4 *src = reinterpret_cast<const uint4 *>(recs + rt.x);
      uint4 *dst = reinterpret_cast<uint4 *>(&sm.pb);
      for (uint32_t i = tid; i < sizeof(ParsedBlock) / 16; i += kTdNT) dst[i] = src[i];
    }
    if (tid == 0) sm.err = 0;
    __syncthreads();
    const BlockHdr &h = sm.pb.h;
    const NodeTab &t = sm.pb.t;
    const JobDev &J = jobs[h.job];
    const bool whole = rt.y == kWholeBlock;
    const uint32_t k = whole ? 0u : (rt.y & 255);
    const uint32_t lo = whole ? 0u : k * kTileOut;
    const uint32_t hi = whole ? h.n : (h.n - lo < kTileOut ? h.n : lo + kTileOut);
    uint8_t *out = J.out + h.out_off;
    if (h.err) {
      if (tid == 0) set_err(J.status, h.err);
      __syncthreads();
      continue;
    }
    if (h.mode == 1) {
      for (uint32_t i = lo + tid; i < hi; i += kTdNT) out[i] = static_cast<uint8_t>(h.csym);
      __syncthreads();
      continue;
    }
    if (J.version != 1) {                // the ablation decodes canonical trees only
      if (tid == 0) set_err(J.status, PIVCO_E_UNSUPPORTED);
      __syncthreads();
      continue;
    }
    const uint32_t I = h.I;
    for (uint32_t v = tid; v < I; v += kTdNT) {
      sm.cur[v] = whole ? 0u : tab[tiled[rt.y >> 8].tab + static_cast<uint64_t>(k) * kTabCols + v].x;
      sm.ones[v] = 0;
    }
    __syncthreads();
    for (uint32_t s0 = lo; s0 < hi; s0 += kTdS) {
      const uint32_t S = hi - s0 < kTdS ? hi - s0 : kTdS;
      for (uint32_t v = tid; v < I; v += kTdNT) sm.tv[v] = 0;
      for (uint32_t i = tid; i < S; i += kTdNT) sm.pos[0][i] = static_cast<uint16_t>(i);
      if (tid == 0) { sm.tv[0] = S; sm.seg[0] = 0; }
      __syncthreads();
      for (uint32_t d = 0; d < h.maxlen; ++d) {
        if (tid == 0) sm.top[(d + 1) & 1] = 0;
        __syncthreads();
        const uint16_t *lp = sm.pos[d & 1];
        uint16_t *cp = sm.pos[(d + 1) & 1];
        for (uint32_t v = h.lvl[d] + wave; v < h.lvl[d + 1]; v += NW) {
          const uint32_t tvv = sm.tv[v];
          if (tvv == 0) continue;
          const bool rans = t.kind[v] != 0;
          const uint64_t base = rans ? 32ull * (h.ans_word0 + t.boff[v]) : 8ull * (h.blk + t.boff[v]);
          const uint32_t c0 = sm.cur[v];
          // the node's 1 bits in this slice
          uint32_t ones = 0;
          for (uint32_t c = 0; c < tvv; c += kWave) {
            const bool act = c + lane < tvv;
            const uint32_t b = act ? td_bit(J.in, scratch, rans, base, c0 + c + lane) : 0u;
            ones += __popcll(__ballot(b));
          }
          // the children's lists (a child may not receive more than it has left)
          const uint32_t ch[2] = {t.child[v][0], t.child[v][1]};
          const uint32_t want[2] = {tvv - ones, ones};
          bool bad = false;
          for (int bb = 0; bb < 2; ++bb)
            if (!(ch[bb] & 0x8000) && sm.cur[ch[bb]] + want[bb] > t.nv[ch[bb]]) bad = true;
          if (bad) {                       // its children get no positions: the item fails
            if (lane == 0) atomicCAS(&sm.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
            continue;
          }
          uint32_t cseg[2] = {0, 0};
          for (int bb = 0; bb < 2; ++bb) {
            if (ch[bb] & 0x8000) continue;
            uint32_t sg = 0;
            if (lane == 0) {
              sg = atomicAdd(&sm.top[(d + 1) & 1], want[bb]);
              sm.seg[ch[bb]] = sg;
              sm.tv[ch[bb]] = want[bb];
            }
            cseg[bb] = __builtin_amdgcn_readfirstlane(sg);
          }
          // partition: positions with a 0 bit to the left child, 1 to the right
          // (a leaf child takes its symbol at them)
          const uint32_t lseg = sm.seg[v];
          uint32_t r[2] = {0, 0};
          for (uint32_t c = 0; c < tvv; c += kWave) {
            const bool act = c + lane < tvv;
            const uint32_t p = act ? lp[lseg + c + lane] : 0u;
            const uint32_t b = act ? td_bit(J.in, scratch, rans, base, c0 + c + lane) : 0u;
            const uint64_t m1 = __ballot(b), m0 = __ballot(act && !b);
            if (act) {
              const uint32_t bb = b;
              const uint32_t rank = r[bb] + static_cast<uint32_t>(__popcll((bb ? m1 : m0) & lt));
              if (ch[bb] & 0x8000) sm.out[p] = static_cast<uint8_t>(ch[bb] & 255);
              else cp[cseg[bb] + rank] = static_cast<uint16_t>(p);
            }
            r[0] += __popcll(m0);
            r[1] += __popcll(m1);
          }
          if (lane == 0) {
            sm.cur[v] = c0 + tvv;
            sm.ones[v] += ones;
          }
        }
        __syncthreads();
      }
      if (sm.err) break;
      // the slice's output: 16-byte stores where the destination allows
      uint8_t *dst = out + s0;
      const uint32_t head = static_cast<uint32_t>((16 - (reinterpret_cast<uintptr_t>(dst) & 15)) & 15);
      const uint32_t h0 = head < S ? head : S;
      for (uint32_t i = tid; i < h0; i += kTdNT) dst[i] = sm.out[i];
      const uint32_t n16 = (S - h0) / 16;
      for (uint32_t i = tid; i < n16; i += kTdNT) {
        const uint8_t *sp = sm.out + h0 + 16 * i;
        uint4 q;
        q.x = sp[0] | (sp[1] << 8) | (sp[2] << 16) | (static_cast<uint32_t>(sp[3]) << 24);
        q.y = sp[4] | (sp[5] << 8) | (sp[6] << 16) | (static_cast<uint32_t>(sp[7]) << 24);
        q.z = sp[8] | (sp[9] << 8) | (sp[10] << 16) | (static_cast<uint32_t>(sp[11]) << 24);
        q.w = sp[12] | (sp[13] << 8) | (sp[14] << 16) | (static_cast<uint32_t>(sp[15]) << 24);
        *reinterpret_cast<uint4 *>(dst + h0 + 16 * i) = q;
      }
      for (uint32_t i = h0 + 16 * n16 + tid; i < S; i += kTdNT) dst[i] = sm.out[i];
      __syncthreads();
    }
    // a whole block must consume every node's bits, with its count of 1 bits
    if (whole && !sm.err)
      for (uint32_t v = tid; v < I; v += kTdNT)
        if (sm.cur[v] != t.nv[v] || sm.ones[v] != t.nr[v]) atomicCAS(&sm.err, 0, static_cast<int32_t>(PIVCO_E_CORRUPT));
    __syncthreads();
    if (tid == 0 && sm.err) set_err(J.status, sm.err);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host-side launch table
// ---------------------------------------------------------------------------
// Merge-kernel variants: workgroup size, tile of a whole block, resident
// block bytes, outputs per task, windows per wave step.
using Cfg0 = MergeCfg<1024, 32768, 57344, 16, 2>;
using Cfg1 = MergeCfg<1024, 32768, 56320, 8, 2>;
using Cfg2 = MergeCfg<1024, 32768, 55296, 32, 1>;
using Cfg3 = MergeCfg<1024, 16384, 57344, 16, 2>;
using Cfg4 = MergeCfg<512, 32768, 57344, 16, 2>;
using Cfg5 = MergeCfg<512, 16384, 57344, 16, 2>;

template <class C>
static hipError_t launch_merge_t(dim3 grid, hipStream_t s, const JobDev *jobs,
                                 const uint2 *items, const ParsedBlock *recs,
                                 const TiledBlock *tiled, const uint2 *tab, uint32_t n_items,
                                 Counters *ctr, const uint32_t *scratch, uint64_t scratch_words,
                                 int32_t single) {
  hipLaunchKernelGGL(k_merge<C>, grid, dim3(C::NT), 0, s, jobs, items, recs, tiled, tab,
                     n_items, ctr, scratch, scratch_words, single);
  return hipGetLastError();
}

template <class C>
static int occupancy_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_merge<C>, C::NT, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace pivco

// ---- entry points used by the host library (C++ linkage, internal) -------
namespace pivco {

uint32_t merge_variant_count() { return 6; }

const char *merge_variant_name(uint32_t v) {
  switch (v) {
    case 0: return "wg1024_tile32k_body56k_k16_x2";
    case 1: return "wg1024_tile32k_body55k_k8_x2";
    case 2: return "wg1024_tile32k_body54k_k32_x1";
    case 3: return "wg1024_tile16k_body56k_k16_x2";
    case 4: return "wg512_tile32k_body56k_k16_x2";
    case 5: return "wg512_tile16k_body56k_k16_x2";
    default: return "?";
  }
}

int merge_variant_occupancy(uint32_t v) {
  switch (v) {
    case 0: return occupancy_t<Cfg0>();
    case 1: return occupancy_t<Cfg1>();
    case 2: return occupancy_t<Cfg2>();
    case 3: return occupancy_t<Cfg3>();
    case 4: return occupancy_t<Cfg4>();
    default: return occupancy_t<Cfg5>();
  }
}

hipError_t launch_merge(uint32_t variant, uint32_t grid, hipStream_t s, const JobDev *jobs,
                        const uint2 *items, const void *recs,
                        const TiledBlock *tiled, const uint2 *tab, uint32_t n_items,
                        Counters *ctr, const uint32_t *scratch, uint64_t scratch_words,
                        int32_t single) {
  const ParsedBlock *r = static_cast<const ParsedBlock *>(recs);
  switch (variant) {
    case 0: return launch_merge_t<Cfg0>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
    case 1: return launch_merge_t<Cfg1>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
    case 2: return launch_merge_t<Cfg2>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
    case 3: return launch_merge_t<Cfg3>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
    case 4: return launch_merge_t<Cfg4>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
    default: return launch_merge_t<Cfg5>(dim3(grid), s, jobs, items, r, tiled, tab, n_items, ctr, scratch, scratch_words, single);
  }
}

hipError_t launch_plan(hipStream_t s, const JobDev *jobs, const uint2 *blocks, uint32_t n_blocks,
                       void *recs, Counters *ctr, RansChunk *chunks, uint64_t chunk_cap) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan, dim3((n_blocks + kPlanWaves - 1) / kPlanWaves), dim3(kWave * kPlanWaves), 0,
                     s, jobs, blocks, n_blocks, static_cast<ParsedBlock *>(recs), ctr, chunks, chunk_cap);
  return hipGetLastError();
}

hipError_t launch_topdown(uint32_t grid, hipStream_t s, const JobDev *jobs, const uint2 *items,
                          const void *recs, const TiledBlock *tiled, const uint2 *tab,
                          uint32_t n_items, Counters *ctr, const uint32_t *scratch, int32_t single) {
  hipLaunchKernelGGL(k_topdown, dim3(grid), dim3(kTdNT), 0, s, jobs, items,
                     static_cast<const ParsedBlock *>(recs), tiled, tab, n_items, ctr, scratch, single);
  return hipGetLastError();
}

int topdown_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_topdown, kTdNT, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_tiles(hipStream_t s, const JobDev *jobs, const TiledBlock *tiled,
                        uint32_t n_tiled, const void *recs, const uint32_t *scratch,
                        uint64_t scratch_words, uint2 *tab) {
  if (n_tiled == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tiles, dim3(n_tiled), dim3(kTilesNT), 0, s, jobs, tiled, n_tiled,
                     static_cast<const ParsedBlock *>(recs), scratch, scratch_words, tab);
  return hipGetLastError();
}

hipError_t launch_rans(uint32_t grid, hipStream_t s, const JobDev *jobs, const void *recs,
                       const uint2 *ritems, Counters *ctr, const RansChunk *chunks,
                       uint64_t chunk_cap, uint32_t *scratch, int32_t single, uint32_t coders) {
  if (coders & 1) {
    hipLaunchKernelGGL(k_rans, dim3(grid), dim3(kRansNT), 0, s, jobs,
                       static_cast<const ParsedBlock *>(recs), ritems, ctr, chunks, chunk_cap, scratch,
                       single);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (coders & 2) {
    const FseTables *ft = fse_tables();
    if (!ft) return hipErrorNotInitialized;
    hipLaunchKernelGGL(k_fse, dim3(grid), dim3(kFseNT), 0, s, jobs,
                       static_cast<const ParsedBlock *>(recs), ritems, ctr, chunks, chunk_cap, ft->dec,
                       scratch, single);
    return hipGetLastError();
  }
  return hipSuccess;
}

int rans_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rans, kRansNT, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_init(hipStream_t s, Counters *ctr, int32_t *status, const int32_t *status0,
                       uint32_t count) {
  const uint32_t n = count > 0 ? count : 1;
  hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, s, ctr, status, status0, count);
  return hipGetLastError();
}

hipError_t launch_gather_headers(hipStream_t s, const pivco_job *jobs, uint32_t count, uint8_t *hdr) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_headers, dim3(count), dim3(64), 0, s, jobs, count, hdr);
  return hipGetLastError();
}

}  // namespace pivco
