// api.cpp -- C ABI of the PivCo-Huffman library: argument checks, host-side
// planning of batched decodes (stream headers -> job table and a work queue
// ordered by decreasing block size), HIP-graph plans, the autotuner, and the
// encode driver.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pivco_int.h"

namespace pivco {
// tree.cpp
pivco_status lengths_from_counts(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]);
// encode.hip
pivco_status encode_stream(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                           uint64_t *h_out_len, const pivco_encode_opts *o, void *d_ws,
                           uint64_t ws_bytes, hipStream_t s);
pivco_status encode_stream_async(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                                 uint64_t *d_out_len, int32_t *d_status, const pivco_encode_opts *o,
                                 void *d_ws, uint64_t ws_bytes, hipStream_t s);
uint64_t encode_bound(uint64_t n, const pivco_encode_opts *o);
uint64_t encode_workspace(uint64_t n, const pivco_encode_opts *o);
}  // namespace pivco

using namespace pivco;

namespace {

inline uint64_t rd64(const uint8_t *p) {
  uint64_t v;
  std::memcpy(&v, p, 8);
  return v;
}
inline uint32_t rd32(const uint8_t *p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
inline uint16_t rd16(const uint8_t *p) {
  uint16_t v;
  std::memcpy(&v, p, 2);
  return v;
}
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

struct StreamHdr {
  uint64_t n_total = 0, ans_words = 0;
  uint32_t block_size = 0, n_blocks = 0, max_len = 0, chunk_log2 = 0, version = 1, flags = 0;
};

// Parses the 48-byte stream header; returns PIVCO_OK or PIVCO_E_CORRUPT.
pivco_status parse_stream_header(const uint8_t *h, uint64_t avail, StreamHdr *o) {
  if (avail < kHeaderBytes) return PIVCO_E_CORRUPT;
  const uint32_t ver = rd16(h + 4), flags = rd16(h + 6);
  if (rd32(h) != kMagic || (ver != 1 && ver != 2) || flags > 1) return PIVCO_E_CORRUPT;
  o->version = ver;
  o->flags = flags;
  o->n_total = rd64(h + 8);
  o->block_size = rd32(h + 16);
  o->n_blocks = rd32(h + 20);
  o->max_len = h[24];
  o->chunk_log2 = h[25];
  o->ans_words = rd64(h + 32);
  if (o->block_size == 0 || o->max_len < 1 || o->max_len > 15 || o->chunk_log2 < 5 ||
      o->chunk_log2 > 24 || (o->flags && o->chunk_log2 < 8))   // a tANS chunk holds whole 32-byte steps
    return PIVCO_E_CORRUPT;
  if (div_up(o->n_total, o->block_size) != o->n_blocks) return PIVCO_E_CORRUPT;
  return PIVCO_OK;
}

// Everything the device needs for one batched decode.
struct HostPlan {
  uint32_t count = 0;
  std::vector<JobDev> jobs;
  WorkLists w;                 // blocks, rANS blocks, split blocks, merge items
  std::vector<int32_t> status0;
  uint64_t scratch_words = 0;
  uint64_t chunk_cap = 0;      // entropy-coded chunk list capacity (bound over the jobs)
  uint32_t coders = 0;         // bit 0: some job has rANS nodes; bit 1: tANS nodes
  // workspace layout (byte offsets)
  uint64_t off_ctr = 0, off_jobs = 0, off_blocks = 0, off_items = 0, off_ritems = 0,
           off_tiled = 0, off_status0 = 0, off_recs = 0, off_tab = 0, off_chunks = 0, off_scratch = 0,
           total = 0;
};

void layout(HostPlan &p) {
  uint64_t o = 0;
  p.off_ctr = o; o += 256;
  p.off_jobs = o; o = align_up(o + sizeof(JobDev) * p.count, 256);
  p.off_blocks = o; o = align_up(o + 8 * p.w.blocks.size(), 256);
  p.off_items = o; o = align_up(o + 8 * p.w.items.size(), 256);
  p.off_ritems = o; o = align_up(o + 8 * p.w.ritems.size(), 256);
  p.off_tiled = o; o = align_up(o + sizeof(TiledBlock) * p.w.tiled.size(), 256);
  p.off_status0 = o; o = align_up(o + 4ull * p.count, 256);
  p.off_recs = o; o = align_up(o + static_cast<uint64_t>(kParsedBlockBytes) * p.w.blocks.size(), 256);
  p.off_tab = o; o = align_up(o + 8 * p.w.tab_entries, 256);
  p.off_chunks = o; o = align_up(o + sizeof(RansChunk) * p.chunk_cap, 256);
  p.off_scratch = o; o = align_up(o + 4 * p.scratch_words + 64, 256);
  // header gathering reuses the start of the workspace before the upload
  const uint64_t gather = align_up(sizeof(pivco_job) * p.count, 256) + kHeaderBytes * p.count;
  p.total = std::max(o, gather);
}

pivco_status read_headers(const pivco_job *h_jobs, uint32_t count, void *d_ws, uint64_t ws_bytes,
                          hipStream_t s, std::vector<uint8_t> &hdr) {
  hdr.assign(static_cast<size_t>(count) * kHeaderBytes, 0);
  if (count == 0) return PIVCO_OK;
  const uint64_t jb = align_up(sizeof(pivco_job) * count, 256);
  if (d_ws && ws_bytes >= jb + kHeaderBytes * count) {
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    if (hipMemcpyAsync(ws, h_jobs, sizeof(pivco_job) * count, hipMemcpyHostToDevice, s) != hipSuccess)
      return PIVCO_E_DEVICE;
    if (launch_gather_headers(s, reinterpret_cast<const pivco_job *>(ws), count, ws + jb) != hipSuccess)
      return PIVCO_E_DEVICE;
    if (hipMemcpyAsync(hdr.data(), ws + jb, kHeaderBytes * count, hipMemcpyDeviceToHost, s) != hipSuccess)
      return PIVCO_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PIVCO_E_DEVICE;
    return PIVCO_OK;
  }
  for (uint32_t j = 0; j < count; ++j) {
    const uint64_t nbytes = std::min<uint64_t>(kHeaderBytes, h_jobs[j].in_len);
    if (nbytes && h_jobs[j].d_in &&
        hipMemcpy(&hdr[static_cast<size_t>(j) * kHeaderBytes], h_jobs[j].d_in, nbytes,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return PIVCO_E_DEVICE;
  }
  return PIVCO_OK;
}

pivco_status check_jobs(const pivco_job *h_jobs, uint32_t count) {
  if (count && !h_jobs) return PIVCO_E_ARG;
  for (uint32_t j = 0; j < count; ++j) {
    if (h_jobs[j].in_len && (!h_jobs[j].d_in || (reinterpret_cast<uintptr_t>(h_jobs[j].d_in) & 15)))
      return PIVCO_E_ARG;
    if (h_jobs[j].out_cap && !h_jobs[j].d_out) return PIVCO_E_ARG;
  }
  return PIVCO_OK;
}

pivco_status build_plan(const pivco_job *h_jobs, uint32_t count, const std::vector<uint8_t> &hdr,
                        int32_t *d_status, HostPlan &p) {
  p.count = count;
  p.jobs.assign(count, JobDev{});
  p.status0.assign(count, PIVCO_OK);
  p.w.clear();
  p.chunk_cap = 0;
  p.coders = 0;
  uint64_t sw = 0;
  std::vector<StreamHdr> hs(count);
  std::vector<pivco_status> sts(count);
  uint64_t batch_symbols = 0;
  for (uint32_t j = 0; j < count; ++j) {
    const pivco_job &jb = h_jobs[j];
    StreamHdr &sh = hs[j];
    pivco_status st = parse_stream_header(&hdr[static_cast<size_t>(j) * kHeaderBytes],
                                          std::min<uint64_t>(jb.in_len, kHeaderBytes), &sh);
    if (st == PIVCO_OK && jb.in_len < kHeaderBytes + 16ull * (sh.n_blocks + 1ull)) st = PIVCO_E_CORRUPT;
    if (st == PIVCO_OK && sh.n_total > jb.out_cap) st = PIVCO_E_CAPACITY;
    sts[j] = st;
    if (st == PIVCO_OK) batch_symbols += sh.n_total;
  }
  for (uint32_t j = 0; j < count; ++j) {
    const pivco_job &jb = h_jobs[j];
    const StreamHdr &sh = hs[j];
    const pivco_status st = sts[j];
    JobDev &d = p.jobs[j];
    d.in = static_cast<const uint8_t *>(jb.d_in);
    d.in_len = jb.in_len;
    d.out = static_cast<uint8_t *>(jb.d_out);
    d.out_cap = jb.out_cap;
    d.status = d_status + j;
    p.status0[j] = st;
    if (st != PIVCO_OK) continue;
    d.n_total = sh.n_total;
    d.n_blocks = sh.n_blocks;
    d.block_size = sh.block_size;
    d.max_len = static_cast<uint16_t>(sh.max_len);
    d.chunk_log2 = static_cast<uint16_t>(sh.chunk_log2);
    d.version = static_cast<uint16_t>(sh.version);
    d.flags = static_cast<uint16_t>(sh.flags);
    if (sh.ans_words) p.coders |= sh.flags ? 2u : 1u;
    d.scratch_base = sw;
    d.ans_words = sh.ans_words;
    sw = align_up(sw + sh.ans_words, 4);
    p.chunk_cap += rans_chunk_bound(sh.ans_words, sh.n_blocks, sh.chunk_log2);
    p.w.add_job(j, sh.n_total, sh.n_blocks, sh.block_size, sh.ans_words != 0,
                split_threshold(jb.in_len, sh.ans_words, sh.n_blocks, batch_symbols, device_cus()));
  }
  p.w.finish();
  if (p.w.items.size() > 0xFFFFFFF0ull || p.w.blocks.size() > 0xFFFFFFF0ull) return PIVCO_E_UNSUPPORTED;
  if ((p.coders & 2) && !fse_tables()) return PIVCO_E_DEVICE;   // tables on this device, before any launch
  p.scratch_words = sw;
  layout(p);
  return PIVCO_OK;
}

pivco_status upload_plan(const HostPlan &p, void *d_ws, hipStream_t s) {
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  auto cp = [&](uint64_t off, const void *src, uint64_t n) {
    return n == 0 || hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  if (!cp(p.off_jobs, p.jobs.data(), sizeof(JobDev) * p.count) ||
      !cp(p.off_blocks, p.w.blocks.data(), 8 * p.w.blocks.size()) ||
      !cp(p.off_items, p.w.items.data(), 8 * p.w.items.size()) ||
      !cp(p.off_ritems, p.w.ritems.data(), 8 * p.w.ritems.size()) ||
      !cp(p.off_tiled, p.w.tiled.data(), sizeof(TiledBlock) * p.w.tiled.size()) ||
      !cp(p.off_status0, p.status0.data(), 4ull * p.count))
    return PIVCO_E_DEVICE;
  return PIVCO_OK;
}

struct Dev {
  Counters *ctr;
  const JobDev *jobs;
  const uint2 *blocks, *items, *ritems;
  const TiledBlock *tiled;
  const int32_t *status0;
  void *recs;
  uint2 *tab;
  RansChunk *chunks;
  uint32_t *scratch;
};

Dev dev_ptrs(const HostPlan &p, void *d_ws) {
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  Dev d;
  d.ctr = reinterpret_cast<Counters *>(ws + p.off_ctr);
  d.jobs = reinterpret_cast<const JobDev *>(ws + p.off_jobs);
  d.blocks = reinterpret_cast<const uint2 *>(ws + p.off_blocks);
  d.items = reinterpret_cast<const uint2 *>(ws + p.off_items);
  d.ritems = reinterpret_cast<const uint2 *>(ws + p.off_ritems);
  d.tiled = reinterpret_cast<const TiledBlock *>(ws + p.off_tiled);
  d.tab = reinterpret_cast<uint2 *>(ws + p.off_tab);
  d.status0 = reinterpret_cast<const int32_t *>(ws + p.off_status0);
  d.recs = ws + p.off_recs;
  d.chunks = reinterpret_cast<RansChunk *>(ws + p.off_chunks);
  d.scratch = reinterpret_cast<uint32_t *>(ws + p.off_scratch);
  return d;
}

// rans_grid: workgroups of 4 waves, each wave decoding two chunks at a time;
// two workgroups per CU, so that no SIMD runs more than two decoding waves
// (a chunk is a chain of dependent steps: the waves that hold one set the
// kernel's length, and more of them on one SIMD only slow each other).
pivco_tune default_tune(uint32_t n_items, uint64_t chunk_cap) {
  pivco_tune t{};
  t.merge_variant = 0;
  const uint32_t g = static_cast<uint32_t>(device_cus() * merge_variant_occupancy(0));
  t.merge_grid = std::max<uint32_t>(1, std::min<uint32_t>(g, n_items ? n_items : 1));
  const uint64_t rg = 2ull * device_cus();
  t.rans_grid = static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(rg, (chunk_cap + 7) / 8)));
  return t;
}

// Enqueue one batched decode (kernels only; capturable).
pivco_status enqueue_batch(const HostPlan &p, void *d_ws, int32_t *d_status, const pivco_tune &t,
                           hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  Dev d = dev_ptrs(p, d_ws);
  const WorkLists &w = p.w;
  if (launch_init(s, d.ctr, d_status, d.status0, p.count) != hipSuccess) return PIVCO_E_DEVICE;
  if (launch_plan(s, d.jobs, d.blocks, static_cast<uint32_t>(w.blocks.size()), d.recs, d.ctr,
                  d.chunks, p.chunk_cap) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (!w.ritems.empty() &&
      launch_rans(t.rans_grid, s, d.jobs, d.recs, d.ritems, d.ctr, d.chunks, p.chunk_cap, d.scratch,
                  -1, p.coders) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (launch_tiles(s, d.jobs, d.tiled, static_cast<uint32_t>(w.tiled.size()), d.recs,
                   d.scratch, p.scratch_words, d.tab) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (ev0 && hipEventRecord(ev0, s) != hipSuccess) return PIVCO_E_DEVICE;
  const uint32_t ni = static_cast<uint32_t>(w.items.size());
  if (ni && launch_merge(t.merge_variant, t.grid_mode ? ni : t.merge_grid, s, d.jobs, d.items, d.recs,
                         d.tiled, d.tab, ni, d.ctr, d.scratch, p.scratch_words,
                         t.grid_mode ? kGridItems : kQueueItems) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (ev1 && hipEventRecord(ev1, s) != hipSuccess) return PIVCO_E_DEVICE;
  return PIVCO_OK;
}

pivco_status prepare(const pivco_job *h_jobs, uint32_t count, int32_t *d_status, void *d_ws,
                     uint64_t ws_bytes, hipStream_t s, HostPlan &p) {
  pivco_status st = check_jobs(h_jobs, count);
  if (st) return st;
  if (count && (!d_status || !d_ws)) return PIVCO_E_ARG;
  std::vector<uint8_t> hdr;
  st = read_headers(h_jobs, count, d_ws, ws_bytes, s, hdr);
  if (st) return st;
  st = build_plan(h_jobs, count, hdr, d_status, p);
  if (st) return st;
  if (p.total > ws_bytes) return PIVCO_E_CAPACITY;
  return upload_plan(p, d_ws, s);
}

}  // namespace

namespace {

// Autotuner cache: one choice per device architecture and workload bucket
// (items per CU, mean symbols per item, share of tile items, rANS present),
// so that batches of the same shape reuse a configuration without timing.
struct TuneKey {
  std::string arch;
  uint32_t items_per_cu, mean_log2, tile_share, rans;
  bool operator<(const TuneKey &o) const {
    return std::tie(arch, items_per_cu, mean_log2, tile_share, rans) <
           std::tie(o.arch, o.items_per_cu, o.mean_log2, o.tile_share, o.rans);
  }
};

std::mutex &tune_cache_mu() {
  static std::mutex m;
  return m;
}
std::map<TuneKey, pivco_tune> &tune_cache() {
  static std::map<TuneKey, pivco_tune> c;
  return c;
}

uint32_t log2_bucket(uint64_t x) {
  uint32_t b = 0;
  while (x > 1) { x >>= 1; ++b; }
  return b;
}

TuneKey tune_key(const HostPlan &p) {
  TuneKey k;
  int dev = 0;
  hipDeviceProp_t prop{};
  k.arch = hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess
               ? std::string(prop.gcnArchName)
               : std::string("?");
  uint64_t symbols = 0, tiles = 0;
  for (auto &x : p.w.sized) {
    symbols += x.first;
    if (x.second.y != kWholeBlock) ++tiles;
  }
  const uint64_t ni = std::max<uint64_t>(1, p.w.items.size());
  k.items_per_cu = log2_bucket(ni / static_cast<uint64_t>(device_cus()) + 1);
  k.mean_log2 = log2_bucket(symbols / ni + 1);
  k.tile_share = static_cast<uint32_t>(4 * tiles / ni);   // quarters
  k.rans = p.w.ritems.empty() ? 0u : 1u;
  return k;
}

}  // namespace

struct pivco_batch_plan {
  HostPlan plan;
  void *ws = nullptr;
  int32_t *status = nullptr;
  pivco_tune tune{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char *pivco_strerror(pivco_status st) {
  switch (st) {
    case PIVCO_OK: return "ok";
    case PIVCO_E_ARG: return "invalid argument";
    case PIVCO_E_CAPACITY: return "output or workspace too small";
    case PIVCO_E_CORRUPT: return "corrupt stream";
    case PIVCO_E_UNSUPPORTED: return "stream outside this library's limits";
    case PIVCO_E_DEVICE: return "HIP runtime error";
    case PIVCO_E_BUDGET: return "request exceeds the memory budget";
  }
  return "unknown status";
}

pivco_status pivco_build_tree(const uint64_t counts[256], uint32_t max_len, pivco_tree *out) {
  if (!counts || !out) return PIVCO_E_ARG;
  return lengths_from_counts(counts, max_len, out->code_len);
}

pivco_status pivco_stream_info(const void *h_hdr, uint64_t hdr_len, uint64_t *n_total,
                               uint32_t *n_blocks, uint32_t *block_size, uint64_t *ans_words) {
  if (!h_hdr) return PIVCO_E_ARG;
  StreamHdr sh;
  const pivco_status st = parse_stream_header(static_cast<const uint8_t *>(h_hdr), hdr_len, &sh);
  if (st) return st;
  if (n_total) *n_total = sh.n_total;
  if (n_blocks) *n_blocks = sh.n_blocks;
  if (block_size) *block_size = sh.block_size;
  if (ans_words) *ans_words = sh.ans_words;
  return PIVCO_OK;
}

uint64_t pivco_decode_workspace(const pivco_job *h_jobs, uint32_t count, hipStream_t s) {
  if (check_jobs(h_jobs, count)) return 0;
  std::vector<uint8_t> hdr;
  if (read_headers(h_jobs, count, nullptr, 0, s, hdr)) return 0;
  HostPlan p;
  if (build_plan(h_jobs, count, hdr, nullptr, p)) return 0;
  return p.total;
}

pivco_status pivco_decode_batch(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  HostPlan p;
  pivco_status st = prepare(h_jobs, count, d_status, d_ws, ws_bytes, s, p);
  if (st) return st;
  if (count == 0) return PIVCO_OK;
  const pivco_tune t = default_tune(static_cast<uint32_t>(p.w.items.size()), p.chunk_cap);
  return enqueue_batch(p, d_ws, d_status, t, s, nullptr, nullptr);
}

pivco_status pivco_decode(const void *d_in, uint64_t in_len, void *d_out, uint64_t out_cap,
                          int32_t *d_status, void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  pivco_job j{d_in, in_len, d_out, out_cap};
  return pivco_decode_batch(&j, 1, d_status, d_ws, ws_bytes, s);
}

pivco_status pivco_decode_plain(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  HostPlan p;
  pivco_status st = prepare(h_jobs, count, d_status, d_ws, ws_bytes, s, p);
  if (st) return st;
  if (count == 0) return PIVCO_OK;
  Dev d = dev_ptrs(p, d_ws);
  const WorkLists &w = p.w;
  if (launch_init(s, d.ctr, d_status, d.status0, p.count) != hipSuccess) return PIVCO_E_DEVICE;
  if (launch_plan(s, d.jobs, d.blocks, static_cast<uint32_t>(w.blocks.size()), d.recs, d.ctr,
                  d.chunks, p.chunk_cap) != hipSuccess)
    return PIVCO_E_DEVICE;
  // one launch per block (rANS), then the boundaries of split blocks, then
  // one merge launch per item, in stream order
  for (size_t r = 0; r < w.ritems.size(); ++r)
    if (launch_rans(1, s, d.jobs, d.recs, d.ritems, d.ctr, d.chunks, p.chunk_cap, d.scratch,
                    static_cast<int32_t>(r), p.coders) != hipSuccess)
      return PIVCO_E_DEVICE;
  if (launch_tiles(s, d.jobs, d.tiled, static_cast<uint32_t>(w.tiled.size()), d.recs,
                   d.scratch, p.scratch_words, d.tab) != hipSuccess)
    return PIVCO_E_DEVICE;
  std::vector<uint32_t> idx(w.items.size());
  for (uint32_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return w.items[a].x != w.items[b].x ? w.items[a].x < w.items[b].x
                                        : (w.items[a].y & 255) < (w.items[b].y & 255);
  });
  for (uint32_t i : idx)
    if (launch_merge(0, 1, s, d.jobs, d.items, d.recs, d.tiled, d.tab,
                     static_cast<uint32_t>(w.items.size()), d.ctr, d.scratch, p.scratch_words,
                     static_cast<int32_t>(i)) != hipSuccess)
      return PIVCO_E_DEVICE;
  return PIVCO_OK;
}

pivco_status pivco_decode_topdown(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                  void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  HostPlan p;
  pivco_status st = prepare(h_jobs, count, d_status, d_ws, ws_bytes, s, p);
  if (st) return st;
  if (count == 0) return PIVCO_OK;
  Dev d = dev_ptrs(p, d_ws);
  const WorkLists &w = p.w;
  const pivco_tune t = default_tune(static_cast<uint32_t>(w.items.size()), p.chunk_cap);
  if (launch_init(s, d.ctr, d_status, d.status0, p.count) != hipSuccess) return PIVCO_E_DEVICE;
  if (launch_plan(s, d.jobs, d.blocks, static_cast<uint32_t>(w.blocks.size()), d.recs, d.ctr,
                  d.chunks, p.chunk_cap) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (!w.ritems.empty() &&
      launch_rans(t.rans_grid, s, d.jobs, d.recs, d.ritems, d.ctr, d.chunks, p.chunk_cap, d.scratch,
                  kQueueItems, p.coders) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (launch_tiles(s, d.jobs, d.tiled, static_cast<uint32_t>(w.tiled.size()), d.recs,
                   d.scratch, p.scratch_words, d.tab) != hipSuccess)
    return PIVCO_E_DEVICE;
  const uint32_t ni = static_cast<uint32_t>(w.items.size());
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(ni, device_cus() * topdown_occupancy()));
  if (ni && launch_topdown(grid, s, d.jobs, d.items, d.recs, d.tiled, d.tab, ni, d.ctr, d.scratch,
                           kQueueItems) != hipSuccess)
    return PIVCO_E_DEVICE;
  return PIVCO_OK;
}

uint32_t pivco_merge_variants(void) { return merge_variant_count(); }
const char *pivco_merge_variant_name(uint32_t v) { return merge_variant_name(v); }

pivco_status pivco_batch_plan_create(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                     void *d_ws, uint64_t ws_bytes, const pivco_tune *tune,
                                     hipStream_t s, pivco_batch_plan **out) {
  if (!out) return PIVCO_E_ARG;
  *out = nullptr;
  pivco_batch_plan *bp = new pivco_batch_plan();
  pivco_status st = prepare(h_jobs, count, d_status, d_ws, ws_bytes, s, bp->plan);
  if (st) { delete bp; return st; }
  bp->ws = d_ws;
  bp->status = d_status;
  bp->tune = tune ? *tune : default_tune(static_cast<uint32_t>(bp->plan.w.items.size()),
                                         bp->plan.chunk_cap);
  if (bp->tune.merge_variant >= merge_variant_count() || bp->tune.merge_grid == 0 ||
      bp->tune.rans_grid == 0 || bp->tune.grid_mode > 1) {
    delete bp;
    return PIVCO_E_ARG;
  }
  if (hipStreamSynchronize(s) != hipSuccess) { delete bp; return PIVCO_E_DEVICE; }
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { delete bp; return PIVCO_E_DEVICE; }
  st = PIVCO_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = PIVCO_E_DEVICE;
  if (!st) {
    const pivco_status e = enqueue_batch(bp->plan, d_ws, d_status, bp->tune, cs, nullptr, nullptr);
    const hipError_t ce = hipStreamEndCapture(cs, &bp->graph);
    if (e) st = e;
    else if (ce != hipSuccess) st = PIVCO_E_DEVICE;
  }
  if (!st && hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) != hipSuccess)
    st = PIVCO_E_DEVICE;
  (void)hipStreamDestroy(cs);
  if (st) {
    pivco_batch_plan_destroy(bp);
    return st;
  }
  *out = bp;
  return PIVCO_OK;
}

pivco_status pivco_batch_plan_launch(pivco_batch_plan *p, hipStream_t s) {
  if (!p || !p->exec) return PIVCO_E_ARG;
  return hipGraphLaunch(p->exec, s) == hipSuccess ? PIVCO_OK : PIVCO_E_DEVICE;
}

pivco_status pivco_batch_plan_launch_timed(pivco_batch_plan *p, hipStream_t s,
                                           hipEvent_t merge_begin, hipEvent_t merge_end) {
  if (!p) return PIVCO_E_ARG;
  return enqueue_batch(p->plan, p->ws, p->status, p->tune, s, merge_begin, merge_end);
}

void pivco_batch_plan_destroy(pivco_batch_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

pivco_status pivco_autotune(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                            void *d_ws, uint64_t ws_bytes, hipStream_t s, pivco_tune *out) {
  if (!out) return PIVCO_E_ARG;
  HostPlan p;
  pivco_status st = prepare(h_jobs, count, d_status, d_ws, ws_bytes, s, p);
  if (st) return st;
  pivco_tune best = default_tune(static_cast<uint32_t>(p.w.items.size()), p.chunk_cap);
  if (p.w.items.empty()) { *out = best; return PIVCO_OK; }
  const TuneKey key = tune_key(p);
  {
    std::lock_guard<std::mutex> lk(tune_cache_mu());
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) { *out = it->second; return PIVCO_OK; }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PIVCO_E_DEVICE;
  const int cus = device_cus();
  const uint32_t ni = static_cast<uint32_t>(p.w.items.size());
  // rANS grids: only when the batch has rANS chunks (one, two or four
  // workgroups of four waves per CU)
  std::vector<uint32_t> rgrids{best.rans_grid};
  if (!p.w.ritems.empty())
    for (uint32_t f : {1u, 4u}) rgrids.push_back(static_cast<uint32_t>(std::max<uint64_t>(
        1, std::min<uint64_t>(static_cast<uint64_t>(f) * cus, (p.chunk_cap + 7) / 8))));
  auto time_of = [&](const pivco_tune &t, float *ms_out) -> pivco_status {
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) return PIVCO_E_DEVICE;
      const pivco_status e = enqueue_batch(p, d_ws, d_status, t, s, nullptr, nullptr);
      if (e) return e;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return PIVCO_E_DEVICE;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    *ms_out = ms_min;
    return PIVCO_OK;
  };
  float best_ms = 1e30f;
  // merge variant (tile size, workgroup size, task width) x persistent grid
  for (uint32_t v = 0; v < merge_variant_count(); ++v) {
    const uint32_t occ = static_cast<uint32_t>(merge_variant_occupancy(v));
    for (uint32_t frac : {4u, 3u, 2u}) {
      pivco_tune t = best;
      t.merge_variant = v;
      t.merge_grid = std::max<uint32_t>(1, std::min<uint32_t>(cus * occ * frac / 4, ni));
      float ms = 0;
      st = time_of(t, &ms);
      if (st) return st;
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
  }
  // then the rANS grid for the chosen merge configuration
  for (uint32_t rg : rgrids) {
    pivco_tune t = best;
    t.rans_grid = rg;
    float ms = 0;
    st = time_of(t, &ms);
    if (st) return st;
    if (ms < best_ms) { best_ms = ms; best = t; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(tune_cache_mu());
    tune_cache()[key] = best;
  }
  *out = best;
  return PIVCO_OK;
}

void pivco_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(tune_cache_mu());
  tune_cache().clear();
}

uint64_t pivco_encode_bound(uint64_t n, const pivco_encode_opts *o) {
  return o ? encode_bound(n, o) : 0;
}

uint64_t pivco_encode_workspace(uint64_t n, const pivco_encode_opts *o) {
  return o ? encode_workspace(n, o) : 0;
}

pivco_status pivco_encode(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                          uint64_t *h_out_len, const pivco_encode_opts *o, void *d_ws,
                          uint64_t ws_bytes, hipStream_t s) {
  return encode_stream(d_in, n, d_out, out_cap, h_out_len, o, d_ws, ws_bytes, s);
}

pivco_status pivco_encode_async(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                                uint64_t *d_out_len, int32_t *d_status, const pivco_encode_opts *o,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s) {
  return encode_stream_async(d_in, n, d_out, out_cap, d_out_len, d_status, o, d_ws, ws_bytes, s);
}

}  // extern "C"
