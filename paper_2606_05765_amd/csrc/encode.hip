// encode.hip -- gfx950 kernels and host driver for PivCo-Huffman encoding.
//
// Encoding (Sec. 4 of the paper) uses the same tree as decoding and walks it
// top-down: each internal node receives the codes of the symbols passing
// through it, emits one bit per symbol (its bitmap) and partitions the
// symbols between its children (the enc_partition primitives of Table 11).
// The driver:
//   1. k_hist      symbol histogram of every block (end-to-end encode time is
//                  dominated by this count, Sec. 4);
//   2. host        optimal length-limited lengths per block (package-merge),
//                  canonical codes, breadth-first node table, n_v / n_right
//                  from the counts, the rANS selection rule;
//   3. k_split     per block, tiles of input symbols: per level, one wave per
//                  node turns 64 symbols at a time into a 64-bit ballot of
//                  code bits (LSB first = stream order), ORs it into the
//                  node's bitmap and scatters the symbols to the children's
//                  segments in LDS with ballot + mbcnt ranks (stable);
//   4. k_rans_enc  32-lane interleaved binary rANS of the selected bitmaps,
//                  one wave per chunk, steps in reverse order;
//   5. host        final layout (block and scratch offsets, headers);
//   6. k_copy      place headers, raw bitmaps and rANS chunks in the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "pivco_int.h"

namespace pivco {

pivco_status lengths_from_counts(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]);
pivco_status canonical_codes(const uint8_t len[256], uint16_t code[256]);
bool tree_is_complete(const uint8_t len[256], uint32_t max_len);

namespace {

constexpr int kWaveE = 64;
constexpr uint32_t kHistSlice = 1u << 16;
constexpr int kSplitNT = 256;
constexpr uint32_t kSplitT = 4096;      // input symbols per tile

// Per-block description for the split kernel (device copy).
struct EncBlock {
  uint64_t in_off;        // first input symbol
  uint64_t bmp_word;      // first bitmap scratch word of the block
  uint32_t n;             // symbols
  uint32_t I;             // internal nodes (0: constant block, nothing to split)
  uint32_t maxlen;
  uint32_t pad;
  uint32_t lvl[16];       // first node id of each depth
  uint32_t fc[17];        // first canonical code of each length
  uint32_t cnt[17];       // symbols of each length
  uint32_t code[256];     // (len << 16) | code
  uint16_t child[256][2]; // internal id or 0x8000 | symbol
  uint32_t word[256];     // node's first bitmap word, relative to bmp_word
};

struct RansJob {
  uint64_t bmp_word;      // absolute scratch word of the chunk's first bit
  uint64_t slot;          // byte offset of the chunk's output slot
  uint32_t nbits;
  uint32_t p1q;
};

struct CopyDesc {
  uint64_t src;           // byte offset in the workspace
  uint64_t dst;           // byte offset in the stream
  uint64_t len;
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint32_t *p, uint64_t nwords) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nwords;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// Histogram of every block, one workgroup per slice of kHistSlice symbols:
// the slice's counts go to its own row of slh (the split kernel's slices
// start at the same boundaries) and are added to the block's row of hist.
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
  if (v) atomicAdd(&hist[b * 256 + tid], v);
}

// Per block, the slice histograms become exclusive prefixes: row k holds the
// count of each symbol in the block's slices before slice k (one thread per
// symbol, one workgroup per block).
__global__ __launch_bounds__(256) void k_slice_prefix(uint32_t *slh, uint32_t spb) {
  uint32_t *row = slh + static_cast<uint64_t>(blockIdx.x) * spb * 256 + threadIdx.x;
  uint32_t run = 0;
  for (uint32_t k = 0; k < spb; ++k) {
    const uint32_t c = row[256ull * k];
    row[256ull * k] = run;
    run += c;
  }
}

static_assert(kSplitNT == 256, "the split kernel's prefix walk has one thread per symbol");
static_assert(kHistSlice % kSplitT == 0, "split tiles never cross a slice");

struct SplitSmem {
  EncBlock B;
  uint32_t cur[256];      // bits written by earlier tiles
  uint32_t tv[256];       // node's symbols in this tile
  uint32_t seg[256];      // node's segment in its level buffer
  uint32_t top[16];
  uint32_t hist[256];
  uint8_t buf[2][kSplitT];
};

// One workgroup per slice of kHistSlice symbols of a block (slice k of block
// b is workgroup b * spb + k), so that large blocks are split by many
// workgroups.  A node's bits from this slice start at the number of the
// block's symbols before the slice that pass the node: the sum, over the
// symbols on whose path the node lies, of their counts before the slice
// (the slice's row of the prefix histograms).  Slices share bitmap words at
// their edges: every word is written with atomicOr into zeroed scratch.
__global__ __launch_bounds__(kSplitNT) void k_split(const uint8_t *in, const EncBlock *blocks,
                                                    uint32_t nblocks, uint32_t spb,
                                                    const uint32_t *pre, uint32_t *bmp) {
  __shared__ SplitSmem sm;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const uint32_t lane = __lane_id();
  const uint32_t b = blockIdx.x / spb, slice = blockIdx.x % spb;
  if (b >= nblocks) return;
  {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&blocks[b]);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&sm.B);
    for (uint32_t i = tid; i < sizeof(EncBlock) / 4; i += kSplitNT) dst[i] = src[i];
  }
  __syncthreads();
  const EncBlock &B = sm.B;
  const uint32_t s_lo = slice * kHistSlice;
  if (B.I == 0 || s_lo >= B.n) return;
  const uint32_t s_hi = B.n - s_lo < kHistSlice ? B.n : s_lo + kHistSlice;
  for (uint32_t i = tid; i < 256; i += kSplitNT) sm.cur[i] = 0;
  __syncthreads();
  if (slice) {   // bits of each node before this slice
    const uint32_t s = tid;
    const uint32_t c = pre[static_cast<uint64_t>(blockIdx.x) * 256 + s];
    const uint32_t cl = B.code[s], len = cl >> 16, code = cl & 0xFFFF;
    if (c && len)
      for (uint32_t d = 0; d < len; ++d) {
        const uint32_t p = code >> (len - d);
        atomicAdd(&sm.cur[B.lvl[d] + (p - (B.fc[d] + B.cnt[d]))], c);
      }
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
      const uint32_t cl = B.code[s], len = cl >> 16, code = cl & 0xFFFF;
      if (c && len) {
        for (uint32_t d = 0; d < len; ++d) {
          const uint32_t p = code >> (len - d);
          const uint32_t id = B.lvl[d] + (p - (B.fc[d] + B.cnt[d]));
          atomicAdd(&sm.tv[id], c);
        }
      }
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
        uint32_t *nb = bmp + B.bmp_word + B.word[v];
        const uint32_t base_bit = sm.cur[v];
        for (uint32_t c = 0; c < tvv; c += kWaveE) {
          const bool act = c + lane < tvv;
          const uint32_t s = act ? lb[seg + c + lane] : 0u;
          const uint32_t cl = B.code[s], len = cl >> 16, code = cl & 0xFFFF;
          const bool bit = act && ((code >> (len - 1 - d)) & 1);
          const uint64_t m1 = __ballot(bit);
          const uint64_t m0 = __ballot(act && !bit);
          const uint64_t lt = (1ull << lane) - 1;
          // bitmap: 64 bits at bit position base_bit + c
          const uint64_t P = static_cast<uint64_t>(base_bit) + c;
          const uint32_t q = static_cast<uint32_t>(P >> 5), sh = static_cast<uint32_t>(P & 31);
          const uint32_t lo = static_cast<uint32_t>(m1), hi = static_cast<uint32_t>(m1 >> 32);
          uint32_t wv = 0;
          if (lane == 0) wv = lo << sh;
          if (lane == 1) wv = sh ? (lo >> (32 - sh)) | (hi << sh) : hi;
          if (lane == 2) wv = sh ? hi >> (32 - sh) : 0u;
          if (lane < 3 && wv) atomicOr(&nb[q + lane], wv);
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

// One wave per chunk: encode steps k = K-1 .. 0; within a step the lanes
// push their renormalisation words in the order lane 31 .. 0, the reverse of
// the decoder's read order, so the decoder reads the pushed words backwards.
__global__ __launch_bounds__(256) void k_rans_enc(const RansJob *jobs, uint32_t njobs,
                                                  const uint32_t *bmp, uint8_t *slots,
                                                  uint32_t *sizes) {
  const uint32_t lane = __lane_id();
  const uint32_t j = blockIdx.x * (256 / kWaveE) + (threadIdx.x >> 6);
  if (j >= njobs) return;
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
}

// One wave per descriptor: byte copy from the workspace into the stream.
__global__ __launch_bounds__(256) void k_copy(const CopyDesc *desc, uint64_t ndesc,
                                              const uint8_t *ws, uint8_t *out) {
  const uint32_t lane = __lane_id();
  for (uint64_t d = blockIdx.x * 4ull + (threadIdx.x >> 6); d < ndesc; d += gridDim.x * 4ull) {
    const CopyDesc c = desc[d];
    const uint8_t *s = ws + c.src;
    uint8_t *o = out + c.dst;
    for (uint64_t i = lane; i < c.len; i += kWaveE) o[i] = s[i];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

void put16(uint8_t *p, uint32_t v) { p[0] = uint8_t(v); p[1] = uint8_t(v >> 8); }
void put32(uint8_t *p, uint32_t v) { for (int i = 0; i < 4; ++i) p[i] = uint8_t(v >> (8 * i)); }
void put64(uint8_t *p, uint64_t v) { for (int i = 0; i < 8; ++i) p[i] = uint8_t(v >> (8 * i)); }

bool opts_ok(const pivco_encode_opts *o) {
  return o && o->block_size >= 1 && o->max_len >= 1 && o->max_len <= kMaxLenGpu &&
         o->ans_mode <= 2 && o->rans_chunk_log2 >= 5 && o->rans_chunk_log2 <= 24;
}

struct WsLayout {
  uint64_t hist, slh, blocks, bmp, rjobs, rsizes, slots, staging, desc, total;
};

// Generous sizes derived from n alone (the data is not known yet).
WsLayout ws_layout(uint64_t n, const pivco_encode_opts *o) {
  WsLayout L{};
  const uint64_t nb = div_up(n, o->block_size);
  const uint64_t C = 1ull << o->rans_chunk_log2;
  const uint64_t bits = n * o->max_len;
  const uint64_t nodes = nb * std::min<uint64_t>(255, std::max<uint64_t>(1, o->block_size));
  const uint64_t chunks = o->ans_mode ? bits / C + nodes + 1 : 0;
  uint64_t x = 0;
  L.hist = x; x = align_up(x + nb * 1024 + 16, 256);
  L.slh = x; x = align_up(x + nb * div_up(o->block_size, kHistSlice) * 1024 + 16, 256);
  L.blocks = x; x = align_up(x + nb * sizeof(EncBlock), 256);
  L.bmp = x; x = align_up(x + 4 * (bits / 32 + nodes + 16), 256);
  L.rjobs = x; x = align_up(x + chunks * sizeof(RansJob), 256);
  L.rsizes = x; x = align_up(x + 4 * chunks, 256);
  L.slots = x; x = align_up(x + (o->ans_mode ? 136 * chunks + 2 * bits + 64 : 0), 256);
  L.staging = x; x = align_up(x + kHeaderBytes + 16 * (nb + 1) + nb * (12 + 128 + 32 + 4 * 255 + 8 * 255 + 16), 256);
  L.desc = x; x = align_up(x + sizeof(CopyDesc) * (nb * (1 + 2 * 255) + chunks + 4), 256);
  L.total = x;
  return L;
}

struct HostNode {
  uint64_t nv = 0, nr = 0;
  uint16_t child[2] = {0, 0};
  uint8_t kind = 0;
};

struct HostBlock {
  uint64_t n = 0;
  int mode = 0;              // 0 coded, 1 constant
  uint8_t csym = 0;
  uint8_t len[256];
  std::vector<HostNode> nodes;
  uint64_t bmp_word = 0;     // first bitmap word
  std::vector<uint32_t> word;  // per node, relative
  // filled after rANS: per rANS node, chunk ids
  std::vector<std::vector<uint32_t>> chunks;
  std::vector<uint32_t> p1q;
};

uint32_t p1q_of(uint64_t nv, uint64_t nr) {
  if (nv == 0) return 2048;
  uint64_t q = (nr * 4096 + nv / 2) / nv;
  return static_cast<uint32_t>(std::min<uint64_t>(4095, std::max<uint64_t>(1, q)));
}

bool select_ans(uint32_t mode, uint64_t nv, uint64_t nr) {
  if (nv == 0) return false;
  if (mode == 1) return 10 * nr < nv || 10 * nr > 9 * nv;
  return mode == 2;
}

// Builds the breadth-first node table of a canonical code and the device
// description of the block.  Internal nodes at depth d are the prefixes
// [fc(d) + cnt(d), 2^d) of a complete canonical code.
void make_block(HostBlock &hb, const uint64_t counts[256], uint32_t ans_mode, EncBlock &eb) {
  std::memset(&eb, 0, sizeof(eb));
  uint16_t code[256];
  canonical_codes(hb.len, code);
  uint32_t cnt[17] = {0}, maxlen = 0;
  for (int s = 0; s < 256; ++s)
    if (hb.len[s]) { cnt[hb.len[s]]++; maxlen = std::max<uint32_t>(maxlen, hb.len[s]); }
  uint32_t fc[18] = {0}, lvl[18] = {0};
  cnt[0] = 0;
  for (uint32_t d = 0; d <= 16; ++d) {
    fc[d + 1] = 2 * (fc[d] + (d < 17 ? cnt[d] : 0));
    const uint32_t Id = d < maxlen ? (1u << d) - fc[d] - cnt[d] : 0;
    lvl[d + 1] = lvl[d] + Id;
  }
  const uint32_t I = lvl[maxlen];
  hb.nodes.assign(I, HostNode{});
  // symbols of each length in symbol order
  std::vector<int> bylen[17];
  for (int s = 0; s < 256; ++s)
    if (hb.len[s]) bylen[hb.len[s]].push_back(s);
  for (uint32_t d = 0; d < maxlen; ++d) {
    for (uint32_t i = lvl[d]; i < lvl[d + 1]; ++i) {
      const uint32_t p = fc[d] + cnt[d] + (i - lvl[d]);
      const uint32_t leafend = fc[d + 1] + cnt[d + 1];
      for (int b = 0; b < 2; ++b) {
        const uint32_t q = 2 * p + b;
        hb.nodes[i].child[b] = q < leafend ? uint16_t(0x8000 | bylen[d + 1][q - fc[d + 1]])
                                           : uint16_t(lvl[d + 1] + (q - leafend));
      }
    }
  }
  for (int s = 0; s < 256; ++s) {
    const uint32_t L = hb.len[s];
    if (!L || !counts[s]) continue;
    for (uint32_t d = 0; d < L; ++d) {
      const uint32_t p = code[s] >> (L - d);
      const uint32_t id = lvl[d] + (p - (fc[d] + cnt[d]));
      hb.nodes[id].nv += counts[s];
      if ((code[s] >> (L - 1 - d)) & 1) hb.nodes[id].nr += counts[s];
    }
  }
  hb.word.assign(I, 0);
  uint32_t w = 0;
  for (uint32_t i = 0; i < I; ++i) {
    hb.nodes[i].kind = select_ans(ans_mode, hb.nodes[i].nv, hb.nodes[i].nr) ? 1 : 0;
    hb.word[i] = w;
    w += static_cast<uint32_t>(div_up(hb.nodes[i].nv, 32));
  }
  eb.n = static_cast<uint32_t>(hb.n);
  eb.I = I;
  eb.maxlen = maxlen;
  for (uint32_t d = 0; d < 16; ++d) eb.lvl[d] = lvl[d];
  for (uint32_t d = 0; d < 17; ++d) { eb.fc[d] = fc[d]; eb.cnt[d] = cnt[d]; }
  for (int s = 0; s < 256; ++s) eb.code[s] = (uint32_t(hb.len[s]) << 16) | code[s];
  for (uint32_t i = 0; i < I; ++i) {
    eb.child[i][0] = hb.nodes[i].child[0];
    eb.child[i][1] = hb.nodes[i].child[1];
    eb.word[i] = hb.word[i];
  }
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

pivco_status encode_stream(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                           uint64_t *h_out_len, const pivco_encode_opts *o, void *d_ws,
                           uint64_t ws_bytes, hipStream_t s) {
  if (!opts_ok(o) || !h_out_len || (n && !d_in) || !d_out) return PIVCO_E_ARG;
  if ((reinterpret_cast<uintptr_t>(d_in) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 15))
    return PIVCO_E_ARG;
  if (o->tree && !tree_is_complete(o->tree->code_len, o->max_len)) return PIVCO_E_ARG;
  const uint64_t bs = o->block_size;
  const uint64_t nb64 = div_up(n, bs);
  if (nb64 > 0xFFFFFFFFull) return PIVCO_E_ARG;
  const uint32_t nb = static_cast<uint32_t>(nb64);
  const WsLayout L = ws_layout(n, o);
  if (ws_bytes < L.total || !d_ws) return PIVCO_E_CAPACITY;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  const uint8_t *in = static_cast<const uint8_t *>(d_in);
  uint8_t *out = static_cast<uint8_t *>(d_out);

  // 1. histograms
  std::vector<uint32_t> hist(static_cast<size_t>(nb) * 256, 0);
  if (nb) {
    uint32_t *dh = reinterpret_cast<uint32_t *>(ws + L.hist);
    hipLaunchKernelGGL(k_fill_zero, dim3(std::min<uint64_t>(4096, div_up(nb64 * 256, 256))), dim3(256), 0, s,
                       dh, nb64 * 256);
    const uint32_t spb = static_cast<uint32_t>(div_up(bs, kHistSlice));
    const uint64_t grid = nb64 * spb;
    if (grid > 0x7FFFFFFFull) return PIVCO_E_UNSUPPORTED;
    uint32_t *dslh = reinterpret_cast<uint32_t *>(ws + L.slh);
    hipLaunchKernelGGL(k_hist, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, s, in, n,
                       static_cast<uint32_t>(bs), spb, dh, dslh);
    HIPCHK(hipGetLastError());
    if (spb > 1) {
      hipLaunchKernelGGL(k_slice_prefix, dim3(nb), dim3(256), 0, s, dslh, spb);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(hist.data(), dh, hist.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  // 2. trees and node tables
  std::vector<HostBlock> hb(nb);
  std::vector<EncBlock> eb(nb);
  uint64_t bmp_words = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    HostBlock &B = hb[b];
    B.n = std::min<uint64_t>(bs, n - static_cast<uint64_t>(b) * bs);
    uint64_t counts[256];
    int m = 0, last = 0;
    for (int k = 0; k < 256; ++k) {
      counts[k] = hist[static_cast<size_t>(b) * 256 + k];
      if (counts[k]) { ++m; last = k; }
    }
    std::memset(B.len, 0, 256);
    if (!o->tree && m == 1) {
      B.mode = 1;
      B.csym = static_cast<uint8_t>(last);
      std::memset(&eb[b], 0, sizeof(EncBlock));
      eb[b].n = static_cast<uint32_t>(B.n);
      eb[b].in_off = static_cast<uint64_t>(b) * bs;
      continue;
    }
    if (o->tree) {
      std::memcpy(B.len, o->tree->code_len, 256);
      for (int k = 0; k < 256; ++k)
        if (counts[k] && !B.len[k]) return PIVCO_E_ARG;
    } else {
      const pivco_status st = lengths_from_counts(counts, o->max_len, B.len);
      if (st) return st;
    }
    make_block(B, counts, o->ans_mode, eb[b]);
    eb[b].in_off = static_cast<uint64_t>(b) * bs;
    B.bmp_word = bmp_words;
    eb[b].bmp_word = bmp_words;
    for (auto &nd : B.nodes) bmp_words += div_up(nd.nv, 32);
    bmp_words = align_up(bmp_words, 4);
  }
  if ((L.rjobs - L.bmp) < 4 * bmp_words + 64) return PIVCO_E_CAPACITY;

  // 3. split: node bitmaps into zeroed scratch
  uint32_t *dbmp = reinterpret_cast<uint32_t *>(ws + L.bmp);
  if (nb) {
    HIPCHK(hipMemcpyAsync(ws + L.blocks, eb.data(), sizeof(EncBlock) * nb, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_zero, dim3(std::min<uint64_t>(8192, div_up(bmp_words + 16, 256))), dim3(256), 0, s,
                       dbmp, bmp_words + 16);
    const uint32_t spb = static_cast<uint32_t>(div_up(bs, kHistSlice));
    hipLaunchKernelGGL(k_split, dim3(static_cast<uint32_t>(nb64 * spb)), dim3(kSplitNT), 0, s, in,
                       reinterpret_cast<const EncBlock *>(ws + L.blocks), nb, spb,
                       reinterpret_cast<const uint32_t *>(ws + L.slh), dbmp);
    HIPCHK(hipGetLastError());
  }

  // 4. rANS of the selected bitmaps
  const uint64_t C = 1ull << o->rans_chunk_log2;
  std::vector<RansJob> rj;
  uint64_t slot_bytes = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    HostBlock &B = hb[b];
    if (B.mode) continue;
    B.chunks.assign(B.nodes.size(), {});
    B.p1q.assign(B.nodes.size(), 0);
    for (size_t i = 0; i < B.nodes.size(); ++i) {
      if (!B.nodes[i].kind) continue;
      B.p1q[i] = p1q_of(B.nodes[i].nv, B.nodes[i].nr);
      for (uint64_t st = 0; st < B.nodes[i].nv; st += C) {
        const uint64_t cl = std::min<uint64_t>(C, B.nodes[i].nv - st);
        RansJob r;
        r.bmp_word = B.bmp_word + B.word[i] + st / 32;
        r.slot = slot_bytes;
        r.nbits = static_cast<uint32_t>(cl);
        r.p1q = B.p1q[i];
        B.chunks[i].push_back(static_cast<uint32_t>(rj.size()));
        rj.push_back(r);
        slot_bytes += align_up(kChunkHdr + 2 * cl + 4, 16);
      }
    }
  }
  std::vector<uint32_t> rsize(rj.size(), 0);
  if (!rj.empty()) {
    if ((L.rsizes - L.rjobs) < sizeof(RansJob) * rj.size() || (L.staging - L.slots) < slot_bytes)
      return PIVCO_E_CAPACITY;
    HIPCHK(hipMemcpyAsync(ws + L.rjobs, rj.data(), sizeof(RansJob) * rj.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_rans_enc, dim3(static_cast<uint32_t>(div_up(rj.size(), 4))), dim3(256), 0, s,
                       reinterpret_cast<const RansJob *>(ws + L.rjobs), static_cast<uint32_t>(rj.size()),
                       dbmp, ws + L.slots, reinterpret_cast<uint32_t *>(ws + L.rsizes));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(rsize.data(), ws + L.rsizes, 4 * rsize.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }

  // 5. final layout: headers in a host staging buffer, copy descriptors
  std::vector<uint8_t> stg;
  std::vector<CopyDesc> desc;
  const uint64_t tab = kHeaderBytes + 16ull * (nb + 1);
  stg.resize(tab, 0);
  put32(&stg[0], kMagic);
  put16(&stg[4], 1);
  put16(&stg[6], 0);
  put64(&stg[8], n);
  put32(&stg[16], static_cast<uint32_t>(bs));
  put32(&stg[20], nb);
  stg[24] = static_cast<uint8_t>(o->max_len);
  stg[25] = static_cast<uint8_t>(o->rans_chunk_log2);
  desc.push_back({L.staging, 0, tab});
  uint64_t off = tab, ans_total = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    HostBlock &B = hb[b];
    put64(&stg[kHeaderBytes + 8ull * b], off);
    put64(&stg[kHeaderBytes + 8ull * (nb + 1) + 8ull * b], ans_total);
    const uint32_t cw = B.n <= 65535 ? 2 : 4;
    const uint64_t hstart = stg.size();
    if (B.mode == 1) {
      stg.resize(hstart + 12, 0);
      put32(&stg[hstart], 12);
      put32(&stg[hstart + 4], static_cast<uint32_t>(B.n));
      stg[hstart + 8] = 1;
      stg[hstart + 9] = B.csym;
      stg[hstart + 10] = static_cast<uint8_t>(cw);
      desc.push_back({L.staging + hstart, off, 12});
      off = align_up(off + 12, 4);
      continue;
    }
    const uint32_t I = static_cast<uint32_t>(B.nodes.size());
    const uint32_t kb = (I + 7) / 8;
    const uint64_t hlen = 12 + 128 + kb + uint64_t(cw) * I;
    stg.resize(hstart + hlen, 0);
    uint8_t *h = &stg[hstart];
    put32(h + 4, static_cast<uint32_t>(B.n));
    h[10] = static_cast<uint8_t>(cw);
    for (int j = 0; j < 128; ++j) h[12 + j] = static_cast<uint8_t>(B.len[2 * j] | (B.len[2 * j + 1] << 4));
    for (uint32_t i = 0; i < I; ++i) {
      if (B.nodes[i].kind) h[140 + i / 8] |= static_cast<uint8_t>(1u << (i % 8));
      if (cw == 2) put16(h + 140 + kb + 2 * i, static_cast<uint32_t>(B.nodes[i].nr));
      else put32(h + 140 + kb + 4 * i, static_cast<uint32_t>(B.nodes[i].nr));
    }
    uint64_t o2 = hlen;               // offset within the block
    for (uint32_t i = 0; i < I; ++i) {
      if (B.nodes[i].kind) continue;
      const uint64_t nbytes = div_up(B.nodes[i].nv, 8);
      if (nbytes) desc.push_back({L.bmp + 4 * (B.bmp_word + B.word[i]), off + o2, nbytes});
      o2 += nbytes;
    }
    for (uint32_t i = 0; i < I; ++i) {
      if (!B.nodes[i].kind) continue;
      o2 = align_up(o2, 4);
      uint64_t blen = 0;
      for (uint32_t c : B.chunks[i]) blen += rsize[c];
      const uint64_t bh = stg.size();
      stg.resize(bh + 8, 0);
      put16(&stg[bh], B.p1q[i]);
      put32(&stg[bh + 4], static_cast<uint32_t>(blen));
      desc.push_back({L.staging + bh, off + o2, 8});
      o2 += 8;
      for (uint32_t c : B.chunks[i]) {
        desc.push_back({L.slots + rj[c].slot, off + o2, rsize[c]});
        o2 += rsize[c];
      }
      ans_total += div_up(B.nodes[i].nv, 32);
    }
    put32(&stg[hstart], static_cast<uint32_t>(o2));
    desc.push_back({L.staging + hstart, off, hlen});
    off = align_up(off + o2, 4);
  }
  put64(&stg[kHeaderBytes + 8ull * nb], off);
  put64(&stg[kHeaderBytes + 8ull * (nb + 1) + 8ull * nb], ans_total);
  put64(&stg[32], ans_total);
  // the header table was queued first with the final values now in place
  if (off > out_cap) return PIVCO_E_CAPACITY;
  if (stg.size() > L.desc - L.staging || sizeof(CopyDesc) * desc.size() > L.total - L.desc)
    return PIVCO_E_CAPACITY;

  // 6. assemble
  HIPCHK(hipMemcpyAsync(ws + L.staging, stg.data(), stg.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ws + L.desc, desc.data(), sizeof(CopyDesc) * desc.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fill_zero, dim3(std::min<uint64_t>(8192, div_up(off / 4 + 1, 256))), dim3(256), 0, s,
                     reinterpret_cast<uint32_t *>(out), off / 4);
  hipLaunchKernelGGL(k_copy, dim3(static_cast<uint32_t>(std::min<uint64_t>(65535, div_up(desc.size(), 4)))),
                     dim3(256), 0, s, reinterpret_cast<const CopyDesc *>(ws + L.desc),
                     static_cast<uint64_t>(desc.size()), ws, out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  *h_out_len = off;
  return PIVCO_OK;
}

}  // namespace pivco
