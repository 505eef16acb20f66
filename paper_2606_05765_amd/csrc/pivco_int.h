// pivco_int.h -- definitions shared by the host planner and the gfx950
// kernels of the PivCo-Huffman library.  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "../../include/pivco.h"

namespace pivco {

// Stream format v1 constants (see the format notes in format.md).
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

// One job as the kernels see it (64 bytes, read through the scalar cache).
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

}  // namespace pivco
