// pivco_int.h -- definitions shared by the host planner and the gfx950
// kernels of the PivCo-Huffman library.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/pivco.h"

namespace pivco {

// Stream format v1 constants.
constexpr uint32_t kMagic = 0x31435650u;   // "PVC1"
constexpr uint32_t kHeaderBytes = 48;
constexpr uint32_t kBlockFixed = 12;       // comp_size, n, mode, const_sym, cnt_width, pad
constexpr uint32_t kLenTable = 128;        // 256 nibbles (App. D)
constexpr uint32_t kMaxInternal = 255;
constexpr uint32_t kMaxLenGpu = 12;        // deepest code the GPU decoder accepts
constexpr uint32_t kRansM = 4096;          // 12-bit probabilities
constexpr uint32_t kRansL = 65536;         // lower state bound, 16-bit words
constexpr uint32_t kRansLanes = 32;
constexpr uint32_t kChunkHdr = 4 + 4 * 32; // n_words u32 + 32 lane states
constexpr uint32_t kParsedBlockBytes = 5984; // per-block record written by the plan kernel

// A block of more than split_min symbols (never fewer than kSplitMin) and at
// most kMaxTiles tiles is decoded as independent tiles of kTileOut symbols,
// each its own work item; the others as one work item each.  A split block's boundary table holds,
// per tile boundary k = 0..ntiles, one row of kTabCols (position, rank) pairs:
// the symbols of the block before boundary k that pass node v, and the 1
// bits among them.
constexpr uint32_t kTileOut = 32768;
constexpr uint32_t kSplitMin = 65536;
constexpr uint32_t kMaxTiles = 128;
constexpr uint32_t kTabCols = 256;
constexpr uint32_t kWholeBlock = 0xFFFFFFFFu;
static_assert(kMaxTiles <= 256, "tile index fits the low 8 bits of an item");

__host__ __device__ inline uint32_t tiles_of_block(uint64_t n, uint64_t split_min = kSplitMin) {
  const uint64_t k = (n + kTileOut - 1) / kTileOut;
  return n > kSplitMin && n > split_min && k <= kMaxTiles ? static_cast<uint32_t>(k) : 0u;
}

// Split threshold of a batched job.  A whole block decodes fastest when its
// bytes and decoded rANS bitmaps fit in the merge kernel's LDS (estimated
// from the job's average block); splitting then only adds the boundary pass.
// Blocks that do not fit, and blocks large enough to hold back the batch
// (more than half a compute unit's share of its symbols), are split.
constexpr uint64_t kResidentGuess = 48 << 10;
inline uint64_t split_threshold(uint64_t in_len, uint64_t ans_words, uint32_t n_blocks,
                                uint64_t batch_symbols, int cus) {
  if (n_blocks && (in_len + 4 * ans_words) / n_blocks > kResidentGuess) return kSplitMin;
  const uint64_t share = batch_symbols / (2ull * static_cast<uint64_t>(cus > 0 ? cus : 1));
  return share > kSplitMin ? share : kSplitMin;
}

// A split block: its record, tile count, and first boundary-table entry.
struct TiledBlock {
  uint32_t rec;
  uint32_t ntiles;
  uint64_t tab;
};

// One job as the kernels see it (80 bytes, read through the scalar cache).
struct JobDev {
  const uint8_t *in;
  uint64_t in_len;
  uint8_t *out;
  uint64_t out_cap;
  uint64_t n_total;
  uint64_t scratch_base;   // first scratch word (u32) of this job
  uint32_t n_blocks;
  uint32_t block_size;
  uint16_t max_len;
  uint16_t chunk_log2;
  uint16_t version;        // 1: canonical trees; 2: flat-subtree trees
  uint16_t flags;          // bit 0: entropy-coded nodes use the byte tANS tables
  int32_t *status;
  uint64_t ans_words;      // scratch words of this job (its stream header's total)
};
static_assert(sizeof(JobDev) == 80, "JobDev layout");

// Counters at the head of the decode workspace.
struct Counters {
  uint32_t merge_next;     // next merge work item
  uint32_t rans_next;      // next pair of rANS chunks to decode
  uint32_t rans_chunks;    // entropy-coded chunks listed by the plan kernel
  uint32_t fse_next;       // next pair of chunks for the tANS kernel
  uint32_t pad[12];
};

// One entropy-coded chunk of a node's bitmap, listed by the plan kernel:
// where its coded data is, where its decoded bits go, how many.  A binary
// rANS chunk holds 32 lane states and 16-bit words; a tANS chunk (p1q =
// kFseTag | marker) 32 cursor states, 32 stream lengths and the streams.
struct RansChunk {
  uint64_t src;            // byte offset of the chunk in the job's stream
  uint64_t dst;            // scratch word of its first decoded word
  uint32_t nbits;          // bits it decodes (<= 2^chunk_log2)
  uint32_t nw;             // rANS: 16-bit renormalisation words; tANS: stream bytes
  uint32_t p1q;            // rANS: 12-bit probability of a 1 bit; tANS: kFseTag | marker
  uint32_t job;
};

// Selective tANS of bitmap bytes (Sec. 5.2): 50 static tables of 2^11
// states, table t for bitmaps whose majority bit has fraction (t + 49)%.
// A node body is marker u8 (t | 0x80 when the bitmap is coded complemented)
// | 0 u8 | 0 u16 | body_len u32 | chunks; a chunk of 2^chunk_log2 bits is
// X0 u16[32] | nbytes u16[32] | 32 cursor streams | zero padding to 4 bytes.
constexpr uint32_t kFseTag = 0x10000u;
constexpr uint32_t kFseTables = 50;
constexpr uint32_t kFseLog = 11;
constexpr uint32_t kFseSize = 1u << kFseLog;
constexpr uint32_t kFseLanes = 32;
constexpr uint32_t kFseChunkHdr = 4 * kFseLanes;
constexpr uint32_t kFseEncWords = 256 + 256 + kFseSize;   // norm | first | state (u16)
// Device addresses of the tables on one GPU: decoding entries (symbol |
// bits << 8 | base << 12, per table and state), encoding tables (norm,
// first state of each byte, states in increasing order, per table), and per
// table one more than the deepest node the selection rule codes with it.
struct FseTables {
  const uint32_t *dec;
  const uint16_t *enc;
  const uint8_t *dmax;
};
// The current device's tables, built on the host and copied into static
// device arrays on the first call for the device (synchronous; call it
// before any stream capture); null on a runtime error.
const FseTables *fse_tables();
static_assert(sizeof(RansChunk) == 32, "RansChunk layout");

// Upper bound on the rANS chunks of a job: a rANS node of n_v bits has
// ceil(n_v / 2^chunk_log2) chunks and ceil(n_v / 32) scratch words, and a
// block has at most 255 nodes.
inline uint64_t rans_chunk_bound(uint64_t ans_words, uint32_t n_blocks, uint32_t chunk_log2) {
  if (ans_words == 0) return 0;
  const uint64_t per_bits = chunk_log2 >= 5 ? (ans_words << 5) >> chunk_log2 : ans_words << 5;
  const uint64_t nodes = std::min<uint64_t>(255ull * n_blocks, ans_words);
  return per_bits + nodes;
}

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Work lists of one batched decode (host): blocks (job, block) for the plan
// and rANS kernels, split blocks for the boundary kernel, and merge items
// (record = index into blocks, kWholeBlock or split-block index << 8 | tile)
// largest first.
struct WorkLists {
  std::vector<uint2> blocks, ritems, items;
  std::vector<TiledBlock> tiled;
  uint64_t tab_entries = 0;
  std::vector<std::pair<uint64_t, uint2>> sized;   // (symbols, item) before ordering

  void clear() {
    blocks.clear(); ritems.clear(); items.clear(); tiled.clear(); sized.clear();
    tab_entries = 0;
  }
  // Adds the blocks of job j (n_total symbols in blocks of block_size).
  void add_job(uint32_t j, uint64_t n_total, uint32_t n_blocks, uint32_t block_size, bool ans,
               uint64_t split_min = kSplitMin) {
    for (uint32_t b = 0; b < n_blocks; ++b) {
      const uint64_t start = static_cast<uint64_t>(b) * block_size;
      const uint64_t sz = std::min<uint64_t>(block_size, n_total - start);
      const uint32_t rec = static_cast<uint32_t>(blocks.size());
      blocks.push_back(make_uint2(j, b));
      if (ans) ritems.push_back(make_uint2(rec, 0u));   // record of a block with rANS nodes
      const uint32_t nt = tiles_of_block(sz, split_min);
      if (nt == 0) {
        sized.push_back({sz, make_uint2(rec, kWholeBlock)});
      } else {
        tiled.push_back(TiledBlock{rec, nt, tab_entries});
        tab_entries += static_cast<uint64_t>(nt + 1) * kTabCols;
        const uint32_t ti = static_cast<uint32_t>(tiled.size() - 1);
        for (uint32_t k = 0; k < nt; ++k)   // item.y = split-block index << 8 | tile
          sized.push_back({std::min<uint64_t>(kTileOut, sz - static_cast<uint64_t>(k) * kTileOut),
                           make_uint2(rec, (ti << 8) | k)});
      }
    }
  }
  // What one job adds to the lists (for admission checks).
  struct Need {
    uint64_t items = 0, tiles = 0, split = 0, tab_entries = 0;
  };
  static Need need_of(uint64_t n_total, uint32_t n_blocks, uint32_t block_size) {
    Need n;
    for (uint32_t b = 0; b < n_blocks; ++b) {
      const uint64_t sz = std::min<uint64_t>(block_size, n_total - static_cast<uint64_t>(b) * block_size);
      const uint32_t nt = tiles_of_block(sz);
      n.items += nt ? nt : 1;
      if (nt) {
        n.tiles += nt;
        n.split += 1;
        n.tab_entries += static_cast<uint64_t>(nt + 1) * kTabCols;
      }
    }
    return n;
  }
  // Orders the split blocks by decreasing tile count (the boundary kernel
  // takes them in list order: longest first) and the merge items by
  // decreasing size (longest first).
  void finish() {
    if (tiled.size() > 1) {
      std::vector<uint32_t> order(tiled.size()), pos(tiled.size());
      for (uint32_t i = 0; i < order.size(); ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [this](uint32_t a, uint32_t b) {
        return tiled[a].ntiles > tiled[b].ntiles;
      });
      std::vector<TiledBlock> sorted;
      sorted.reserve(tiled.size());
      for (uint32_t i = 0; i < order.size(); ++i) {
        sorted.push_back(tiled[order[i]]);
        pos[order[i]] = i;
      }
      tiled.swap(sorted);
      for (auto &x : sized)
        if (x.second.y != kWholeBlock) x.second.y = (pos[x.second.y >> 8] << 8) | (x.second.y & 255);
    }
    std::stable_sort(sized.begin(), sized.end(),
                     [](const std::pair<uint64_t, uint2> &a, const std::pair<uint64_t, uint2> &b) {
                       return a.first > b.first;
                     });
    items.clear();
    items.reserve(sized.size());
    for (auto &x : sized) items.push_back(x.second);
  }
};

// Item source of the merge kernel (its `single` argument): the persistent
// queue, or one workgroup per item; values >= 0 decode that one item.
constexpr int32_t kQueueItems = -1;
constexpr int32_t kGridItems = -2;

// Decode launchers (decode.hip), used by the batch planner and the server.
// A launch is k_init, k_plan over the blocks (records: kParsedBlockBytes per
// block), k_rans when some block has rANS nodes, k_tiles over the split
// blocks (boundary tables), then k_merge over the items.
uint32_t merge_variant_count();
const char *merge_variant_name(uint32_t v);
int merge_variant_occupancy(uint32_t v);
hipError_t launch_plan(hipStream_t s, const JobDev *jobs, const uint2 *blocks, uint32_t n_blocks,
                       void *recs, Counters *ctr, RansChunk *chunks, uint64_t chunk_cap);
hipError_t launch_tiles(hipStream_t s, const JobDev *jobs, const TiledBlock *tiled,
                        uint32_t n_tiled, const void *recs, const uint32_t *scratch,
                        uint64_t scratch_words, uint2 *tab);
hipError_t launch_merge(uint32_t variant, uint32_t grid, hipStream_t s, const JobDev *jobs,
                        const uint2 *items, const void *recs,
                        const TiledBlock *tiled, const uint2 *tab, uint32_t n_items,
                        Counters *ctr, const uint32_t *scratch, uint64_t scratch_words,
                        int32_t single);
// coders: bit 0, some job has rANS nodes; bit 1, some job has tANS nodes
// (then fse_tables() has been called for the device).
hipError_t launch_rans(uint32_t grid, hipStream_t s, const JobDev *jobs, const void *recs,
                       const uint2 *ritems, Counters *ctr, const RansChunk *chunks,
                       uint64_t chunk_cap, uint32_t *scratch, int32_t single, uint32_t coders);
int rans_occupancy();
// Top-down decode of the same work items (ablation of the merge kernel).
hipError_t launch_topdown(uint32_t grid, hipStream_t s, const JobDev *jobs, const uint2 *items,
                          const void *recs, const TiledBlock *tiled, const uint2 *tab,
                          uint32_t n_items, Counters *ctr, const uint32_t *scratch, int32_t single);
int topdown_occupancy();
hipError_t launch_init(hipStream_t s, Counters *ctr, int32_t *status, const int32_t *status0,
                       uint32_t count);
hipError_t launch_gather_headers(hipStream_t s, const pivco_job *jobs, uint32_t count, uint8_t *hdr);

}  // namespace pivco
