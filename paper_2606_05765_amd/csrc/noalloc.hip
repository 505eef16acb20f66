// noalloc.hip -- the decode entry point for callers that cannot allocate
// device memory.
//
// pivco_decode takes its workspace (job table, work queue, per-block
// records, rANS chunk list and scratch, boundary tables of split blocks)
// from the caller.  pivco_decode_noalloc runs the same decode with that
// workspace in a fixed array in device memory, `scratch`, which the library
// holds on every GPU it runs on until the process ends.  Nothing here calls
// hipMalloc, hipFree or an allocating library routine.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels and copies.  Every
// call on a GPU reuses the GPU's array; the decode writes every byte it later
// reads within the same call (the launch begins by resetting its counters),
// so the last call's contents never leak into the next one.  Two calls that
// overlap in time on one GPU (other streams, other threads) would share the
// array and race: callers serialise them.
#include <mutex>

#include "pivco_int.h"

namespace {

constexpr uint64_t kScratchBytes = PIVCO_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "whole 256-byte units");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up on the
// first call with the device current), or null on a runtime error.
void *scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

pivco_status pivco_decode_noalloc(const void *d_in, uint64_t in_len, void *d_out, uint64_t out_cap,
                                  int32_t *d_status, hipStream_t s) {
  void *ws = scratch_ptr();
  if (!ws) return PIVCO_E_DEVICE;
  // pivco_decode returns E_CAPACITY before any device work when the decode
  // needs more workspace than the array holds
  return pivco_decode(d_in, in_len, d_out, out_cap, d_status, ws, kScratchBytes, s);
}

}  // extern "C"
