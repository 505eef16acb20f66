// pivco_int.h -- definitions shared by the host planner and the gfx950
// kernels of the PivCo-Huffman library.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

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
constexpr uint32_t kParsedBlockBytes = 5632; // per-item record written by the plan kernel

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
  uint32_t max_len;
  uint32_t chunk_log2;
  int32_t *status;
  uint64_t pad;
};
static_assert(sizeof(JobDev) == 80, "JobDev layout");

// Counters at the head of the decode workspace.
struct Counters {
  uint32_t merge_next;     // next merge work item
  uint32_t rans_next;      // next rANS work item
  uint32_t pad[14];
};

__host__ __device__ inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Decode launchers (decode.hip), used by the batch planner and the server.
// A launch is k_init, k_plan (records: kParsedBlockBytes per item), k_rans
// when some block has rANS nodes, then k_merge.
uint32_t merge_variant_count();
const char *merge_variant_name(uint32_t v);
int merge_variant_occupancy(uint32_t v);
hipError_t launch_plan(hipStream_t s, const JobDev *jobs, const uint2 *items, uint32_t n_items,
                       void *recs);
hipError_t launch_merge(uint32_t variant, uint32_t grid, hipStream_t s, const JobDev *jobs,
                        const uint2 *items, const void *recs, uint32_t n_items, Counters *ctr,
                        const uint32_t *scratch, uint64_t scratch_words, int32_t single);
hipError_t launch_rans(uint32_t grid, hipStream_t s, const JobDev *jobs, const uint2 *items,
                       uint32_t n_items, Counters *ctr, uint32_t *scratch, int32_t single);
int rans_occupancy();
hipError_t launch_init(hipStream_t s, Counters *ctr, int32_t *status, const int32_t *status0,
                       uint32_t count);
hipError_t launch_gather_headers(hipStream_t s, const pivco_job *jobs, uint32_t count, uint8_t *hdr);

}  // namespace pivco
