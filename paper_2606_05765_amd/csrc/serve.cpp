// serve.cpp -- continuous-batching decode server.
//
// Streams (already encoded, resident in device memory) are registered once;
// their headers are read at registration, so planning a batch later needs no
// device round trip.  run() replays a trace of (arrival time, request) pairs
// in real time on the host clock:
//   * arrivals join a FIFO;
//   * a request is admitted when an execution slot is free and its output
//     buffer fits in the device-memory budget (a first-fit allocator over a
//     caller-provided pool); a request larger than the whole budget fails
//     with PIVCO_E_BUDGET;
//   * each admission round packs the admitted requests into one batch:
//     job table + LPT work queue uploaded from pinned memory, then the same
//     init / rANS / merge kernels as pivco_decode_batch, on the slot's own
//     stream, so batches on different slots overlap on the device;
//   * completion is polled with hipEventQuery; latency = completion time on
//     the host clock minus arrival time; the output space is released.
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "pivco_int.h"

using namespace pivco;

namespace {

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Registered {
  const uint8_t *d_in;
  uint64_t in_len;
  uint64_t n_total, ans_words;
  uint32_t n_blocks, block_size, max_len, chunk_log2, version, flags;
  WorkLists::Need need;           // merge items, tiles and boundary-table entries
  uint64_t chunks;                // bound on its rANS chunks
};

// First-fit allocator over [0, size) with coalescing on free.
class PoolAlloc {
 public:
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(uint64_t n, uint64_t *off) {
    n = align_up(std::max<uint64_t>(n, 1), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = align_up(std::max<uint64_t>(n, 1), 256);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t *ws = nullptr;          // device workspace of this slot
  uint8_t *pinned = nullptr;      // host staging of job table + queue
  bool busy = false;
  std::vector<uint32_t> reqs;     // trace indices in this batch
};

}  // namespace

struct pivco_server {
  pivco_server_opts opts{};
  std::vector<Registered> reg;
  std::vector<Slot> slots;
  uint64_t ws_bytes_per_slot = 0, pinned_bytes = 0;
  // workspace layout inside a slot
  uint64_t off_ctr = 0, off_jobs = 0, off_status = 0, off_recs = 0, off_tab = 0, off_chunks = 0,
           off_scratch = 0;
  uint64_t off_pstatus = 0;
  uint32_t max_blocks = 0;
  uint64_t max_tiles = 0, max_split = 0, max_tab = 0, max_scratch_words = 0;
  uint64_t max_chunks = 1u << 16;   // rANS chunks per batch (32 B each)
  WorkLists w;                    // reused by every admission round
};

extern "C" {

pivco_status pivco_server_create(const pivco_server_opts *o, pivco_server **out) {
  if (!o || !out || o->slots == 0 || o->slots > 16 || o->max_batch == 0 || o->max_blocks == 0)
    return PIVCO_E_ARG;
  pivco_server *sv = new pivco_server();
  sv->opts = *o;
  sv->max_blocks = o->max_blocks;
  sv->max_scratch_words = o->max_scratch_words;
  // a split block has at least three tiles, so max_tiles / 3 split blocks
  sv->max_tiles = o->max_tiles ? o->max_tiles : 8192;
  sv->max_split = sv->max_tiles / 3 + 1;
  sv->max_tab = (sv->max_tiles + sv->max_split) * kTabCols;
  const uint64_t max_items = o->max_blocks + sv->max_tiles;
  uint64_t x = 0;
  sv->off_ctr = x; x += 256;
  sv->off_jobs = x; x = align_up(x + sizeof(JobDev) * o->max_batch, 256);
  // blocks, items, rANS blocks, split blocks and initial statuses follow the
  // job table, packed per batch (capacity for the largest batch)
  x = align_up(x + 8ull * o->max_blocks + 64, 64);
  x = align_up(x + 8ull * max_items + 64, 64);
  x = align_up(x + 8ull * o->max_blocks + 64, 64);
  x = align_up(x + sizeof(TiledBlock) * sv->max_split + 64, 64);
  x = align_up(x + 4ull * o->max_batch + 64, 256);
  const uint64_t pinned = x;          // counters .. statuses staged from pinned memory
  sv->off_status = x; x = align_up(x + 4ull * o->max_batch, 256);
  sv->off_pstatus = pinned;           // statuses copied back into pinned memory
  sv->off_recs = x; x = align_up(x + static_cast<uint64_t>(kParsedBlockBytes) * o->max_blocks, 256);
  sv->off_tab = x; x = align_up(x + 8ull * sv->max_tab, 256);
  sv->off_chunks = x; x = align_up(x + sizeof(RansChunk) * sv->max_chunks, 256);
  sv->off_scratch = x; x = align_up(x + 4ull * o->max_scratch_words + 64, 256);
  sv->ws_bytes_per_slot = x;
  sv->pinned_bytes = pinned;
  sv->slots.resize(o->slots);
  for (auto &s : sv->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&s.ws, sv->ws_bytes_per_slot) != hipSuccess ||
        hipHostMalloc(&s.pinned, pinned + 4ull * o->max_batch, hipHostMallocDefault) != hipSuccess) {
      pivco_server_destroy(sv);
      return PIVCO_E_DEVICE;
    }
  }
  *out = sv;
  return PIVCO_OK;
}

void pivco_server_destroy(pivco_server *sv) {
  if (!sv) return;
  for (auto &s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.ws) (void)hipFree(s.ws);
    if (s.pinned) (void)hipHostFree(s.pinned);
  }
  delete sv;
}

uint64_t pivco_server_workspace_bytes(const pivco_server *sv) {
  return sv ? sv->ws_bytes_per_slot * sv->slots.size() : 0;
}

pivco_status pivco_server_register(pivco_server *sv, const void *d_stream, uint64_t len,
                                   uint32_t *id) {
  if (!sv || !d_stream || !id || (reinterpret_cast<uintptr_t>(d_stream) & 15) || len < kHeaderBytes)
    return PIVCO_E_ARG;
  uint8_t h[kHeaderBytes];
  if (hipMemcpy(h, d_stream, kHeaderBytes, hipMemcpyDeviceToHost) != hipSuccess) return PIVCO_E_DEVICE;
  uint64_t n_total, ans;
  uint32_t nb, bs;
  pivco_status st = pivco_stream_info(h, kHeaderBytes, &n_total, &nb, &bs, &ans);
  if (st) return st;
  if (len < kHeaderBytes + 16ull * (nb + 1ull)) return PIVCO_E_CORRUPT;
  // a batch reserves its jobs' scratch in multiples of 4 words
  if (nb > sv->max_blocks || align_up(ans, 4) > sv->max_scratch_words) return PIVCO_E_UNSUPPORTED;
  const WorkLists::Need need = WorkLists::need_of(n_total, nb, bs);
  if (need.tiles > sv->max_tiles) return PIVCO_E_UNSUPPORTED;
  const uint64_t chunks = rans_chunk_bound(ans, nb, h[25]);
  if (chunks > sv->max_chunks) return PIVCO_E_UNSUPPORTED;
  Registered r;
  r.d_in = static_cast<const uint8_t *>(d_stream);
  r.in_len = len;
  r.n_total = n_total;
  r.ans_words = ans;
  r.n_blocks = nb;
  r.block_size = bs;
  r.max_len = h[24];
  r.chunk_log2 = h[25];
  r.version = static_cast<uint32_t>(h[4]) | (static_cast<uint32_t>(h[5]) << 8);
  r.flags = static_cast<uint32_t>(h[6]) | (static_cast<uint32_t>(h[7]) << 8);
  if (r.flags && ans && !fse_tables()) return PIVCO_E_DEVICE;   // tables on this device, before serving
  r.need = need;
  r.chunks = chunks;
  *id = static_cast<uint32_t>(sv->reg.size());
  sv->reg.push_back(r);
  return PIVCO_OK;
}

pivco_status pivco_server_run(pivco_server *sv, const pivco_request *reqs, uint32_t n_req,
                              void *d_pool, uint64_t pool_bytes, pivco_request_result *res,
                              pivco_server_stats *stats) {
  if (!sv || (n_req && (!reqs || !res)) || (pool_bytes && !d_pool)) return PIVCO_E_ARG;
  for (uint32_t i = 0; i < n_req; ++i)
    if (reqs[i].id >= sv->reg.size()) return PIVCO_E_ARG;
  if (pool_bytes > sv->opts.mem_budget) pool_bytes = sv->opts.mem_budget;
  PoolAlloc pool;
  pool.reset(pool_bytes);
  uint8_t *pool_base = static_cast<uint8_t *>(d_pool);
  const int cus = [] {
    int dev = 0, c = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      c = 256;
    return c > 0 ? c : 256;
  }();
  const uint32_t variant = sv->opts.merge_variant < merge_variant_count() ? sv->opts.merge_variant : 0;
  const uint32_t mgrid_full = static_cast<uint32_t>(cus * merge_variant_occupancy(variant));
  const uint32_t rgrid_full = static_cast<uint32_t>(2 * cus);   // two rANS workgroups per CU
  std::vector<uint64_t> out_off(n_req, 0);
  std::deque<uint32_t> pending;
  uint32_t next = 0, done = 0;
  uint64_t peak = 0, bytes_done = 0, batches = 0, max_batch_seen = 0, max_busy = 0;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_s = [&] { return std::chrono::duration<double>(clk::now() - t0).count(); };
  for (uint32_t i = 0; i < n_req; ++i) {
    res[i].status = PIVCO_OK;
    res[i].d_out = nullptr;
    res[i].n_out = sv->reg[reqs[i].id].n_total;
    res[i].t_admit = res[i].t_done = -1.0;
  }
  while (done < n_req) {
    const double now = now_s();
    while (next < n_req && reqs[next].arrival_s <= now) pending.push_back(next++);
    bool progressed = false;
    // completions
    for (auto &s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return PIVCO_E_DEVICE;
      const double t = now_s();
      const int32_t *st = reinterpret_cast<const int32_t *>(s.pinned + sv->off_pstatus);
      for (size_t k = 0; k < s.reqs.size(); ++k) {
        const uint32_t r = s.reqs[k];
        res[r].t_done = t;
        res[r].status = st[k];
        bytes_done += res[r].n_out;
        if (!sv->opts.keep_outputs) pool.release(out_off[r], res[r].n_out);
        ++done;
      }
      s.reqs.clear();
      s.busy = false;
      progressed = true;
    }
    // admissions: one batch per free slot
    for (auto &s : sv->slots) {
      if (s.busy || pending.empty()) continue;
      std::vector<uint32_t> batch;
      uint64_t blocks = 0, tiles = 0, split = 0, tab = 0, scratch = 0, chunks = 0;
      while (!pending.empty() && batch.size() < sv->opts.max_batch) {
        const uint32_t r = pending.front();
        const Registered &g = sv->reg[reqs[r].id];
        const uint64_t need = g.n_total;
        if (align_up(std::max<uint64_t>(need, 1), 256) > pool_bytes) {   // can never fit
          res[r].status = PIVCO_E_BUDGET;
          res[r].t_admit = res[r].t_done = now_s();
          pending.pop_front();
          ++done;
          progressed = true;
          continue;
        }
        if (blocks + g.n_blocks > sv->max_blocks || tiles + g.need.tiles > sv->max_tiles ||
            split + g.need.split > sv->max_split || tab + g.need.tab_entries > sv->max_tab ||
            chunks + g.chunks > sv->max_chunks ||
            align_up(scratch + g.ans_words, 4) > sv->max_scratch_words)
          break;
        uint64_t off = 0;
        if (!pool.alloc(need, &off)) break;          // wait for memory to free up
        out_off[r] = off;
        res[r].d_out = pool_base + off;
        res[r].t_admit = now_s();
        blocks += g.n_blocks;
        tiles += g.need.tiles;
        split += g.need.split;
        tab += g.need.tab_entries;
        chunks += g.chunks;
        scratch = align_up(scratch + g.ans_words, 4);
        batch.push_back(r);
        pending.pop_front();
      }
      if (batch.empty()) continue;
      peak = std::max(peak, pool.used());
      // plan the batch in pinned memory, then upload and launch
      JobDev *jobs = reinterpret_cast<JobDev *>(s.pinned + sv->off_jobs);
      WorkLists &w = sv->w;
      w.clear();
      uint64_t sw = 0;
      uint32_t coders = 0;
      for (uint32_t k = 0; k < batch.size(); ++k) {
        const Registered &g = sv->reg[reqs[batch[k]].id];
        JobDev d{};
        d.in = g.d_in;
        d.in_len = g.in_len;
        d.out = static_cast<uint8_t *>(res[batch[k]].d_out);
        d.out_cap = g.n_total;
        d.n_total = g.n_total;
        d.scratch_base = sw;
        d.ans_words = g.ans_words;
        d.n_blocks = g.n_blocks;
        d.block_size = g.block_size;
        d.max_len = static_cast<uint16_t>(g.max_len);
        d.chunk_log2 = static_cast<uint16_t>(g.chunk_log2);
        d.version = static_cast<uint16_t>(g.version);
        d.flags = static_cast<uint16_t>(g.flags);
        if (g.ans_words) coders |= g.flags ? 2u : 1u;
        d.status = reinterpret_cast<int32_t *>(s.ws + sv->off_status) + k;
        jobs[k] = d;
        sw = align_up(sw + g.ans_words, 4);
        w.add_job(k, g.n_total, g.n_blocks, g.block_size, g.ans_words != 0);
      }
      w.finish();
      const uint32_t nb = static_cast<uint32_t>(w.blocks.size());
      const uint32_t ni = static_cast<uint32_t>(w.items.size());
      const uint32_t nr = static_cast<uint32_t>(w.ritems.size());
      const uint32_t nt = static_cast<uint32_t>(w.tiled.size());
      // the lists packed behind the job table: one upload of what this batch uses
      const uint64_t o_blocks = align_up(sv->off_jobs + sizeof(JobDev) * batch.size(), 64);
      const uint64_t o_items = align_up(o_blocks + 8ull * nb, 64);
      const uint64_t o_ritems = align_up(o_items + 8ull * ni, 64);
      const uint64_t o_tiled = align_up(o_ritems + 8ull * nr, 64);
      const uint64_t o_status0 = align_up(o_tiled + sizeof(TiledBlock) * nt, 64);
      const uint64_t staged = o_status0 + 4ull * batch.size();
      if (staged > sv->pinned_bytes) return PIVCO_E_UNSUPPORTED;   // admission keeps this false
      std::memcpy(s.pinned + o_blocks, w.blocks.data(), 8ull * nb);
      std::memcpy(s.pinned + o_items, w.items.data(), 8ull * ni);
      std::memcpy(s.pinned + o_ritems, w.ritems.data(), 8ull * nr);
      std::memcpy(s.pinned + o_tiled, w.tiled.data(), sizeof(TiledBlock) * nt);
      int32_t *st0 = reinterpret_cast<int32_t *>(s.pinned + o_status0);
      for (uint32_t k = 0; k < batch.size(); ++k) st0[k] = PIVCO_OK;
      if (hipMemcpyAsync(s.ws, s.pinned, staged, hipMemcpyHostToDevice, s.stream) != hipSuccess)
        return PIVCO_E_DEVICE;
      Counters *ctr = reinterpret_cast<Counters *>(s.ws + sv->off_ctr);
      const JobDev *dj = reinterpret_cast<const JobDev *>(s.ws + sv->off_jobs);
      uint32_t *scr = reinterpret_cast<uint32_t *>(s.ws + sv->off_scratch);
      if (launch_init(s.stream, ctr, reinterpret_cast<int32_t *>(s.ws + sv->off_status),
                      reinterpret_cast<const int32_t *>(s.ws + o_status0),
                      static_cast<uint32_t>(batch.size())) != hipSuccess)
        return PIVCO_E_DEVICE;
      void *recs = s.ws + sv->off_recs;
      const uint2 *d_blocks = reinterpret_cast<const uint2 *>(s.ws + o_blocks);
      const TiledBlock *d_tiled = reinterpret_cast<const TiledBlock *>(s.ws + o_tiled);
      uint2 *d_tab = reinterpret_cast<uint2 *>(s.ws + sv->off_tab);
      RansChunk *d_chunks = reinterpret_cast<RansChunk *>(s.ws + sv->off_chunks);
      if (launch_plan(s.stream, dj, d_blocks, nb, recs, ctr, d_chunks, chunks) != hipSuccess)
        return PIVCO_E_DEVICE;
      if (nr && launch_rans(std::max<uint32_t>(1, std::min<uint32_t>(rgrid_full, static_cast<uint32_t>((chunks + 7) / 8))),
                            s.stream, dj, recs, reinterpret_cast<const uint2 *>(s.ws + o_ritems), ctr,
                            d_chunks, chunks, scr, -1, coders) != hipSuccess)
        return PIVCO_E_DEVICE;
      if (launch_tiles(s.stream, dj, d_tiled, nt, recs, scr, sw, d_tab) != hipSuccess)
        return PIVCO_E_DEVICE;
      if (ni && launch_merge(variant, std::max<uint32_t>(1, std::min(mgrid_full, ni)), s.stream, dj,
                             reinterpret_cast<const uint2 *>(s.ws + o_items), recs,
                             d_tiled, d_tab, ni, ctr, scr, sw, -1) != hipSuccess)
        return PIVCO_E_DEVICE;
      if (hipMemcpyAsync(s.pinned + sv->off_pstatus, s.ws + sv->off_status, 4 * batch.size(),
                         hipMemcpyDeviceToHost, s.stream) != hipSuccess)
        return PIVCO_E_DEVICE;
      if (hipEventRecord(s.done, s.stream) != hipSuccess) return PIVCO_E_DEVICE;
      s.reqs = batch;
      s.busy = true;
      ++batches;
      max_batch_seen = std::max<uint64_t>(max_batch_seen, batch.size());
      progressed = true;
    }
    const uint64_t busy = static_cast<uint64_t>(
        std::count_if(sv->slots.begin(), sv->slots.end(), [](const Slot &s) { return s.busy; }));
    max_busy = std::max(max_busy, busy);
    if (busy == 0 && !pending.empty()) {
      // nothing is in flight, so no output space will be released: the head
      // request does not fit in what is left of the pool (kept outputs of
      // earlier requests hold the rest) and never will
      const uint32_t r = pending.front();
      pending.pop_front();
      res[r].status = PIVCO_E_BUDGET;
      res[r].t_admit = res[r].t_done = now_s();
      ++done;
      progressed = true;
    }
    if (!progressed) {
      // nothing to do right now: wait for the next arrival or a completion
      const bool any_busy = std::any_of(sv->slots.begin(), sv->slots.end(), [](const Slot &s) { return s.busy; });
      if (!any_busy && next < n_req && pending.empty()) {
        const double wait = reqs[next].arrival_s - now_s();
        if (wait > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
      } else {
        std::this_thread::yield();
      }
    }
  }
  if (stats) {
    stats->wall_s = now_s();
    stats->bytes_decoded = bytes_done;
    stats->peak_pool_bytes = peak;
    stats->batches = batches;
    stats->max_batch = max_batch_seen;
    stats->max_busy_slots = max_busy;
  }
  return PIVCO_OK;
}

}  // extern "C"
