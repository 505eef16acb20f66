// fse.hip -- the static tables of the selective tANS coding of node bitmaps
// as bytes (Sec. 5.2 of the paper: 50 precomputed tables for bitmap skews
// 50..99%, chosen per node; App. D's FSE marker).
//
// Table t (1..50) serves bitmaps whose majority bit has fraction s = (t +
// 49)%.  It is built for bytes of independent bits: P(b) = s^k (1 - s)^(8-k),
// k = popcount(b).  2^11 states.  Counts by largest remainder, in exact
// integers: floor(P(b) 2^11), at least 1; the missing units to the bytes with
// the largest remainders (lower byte first on equal ones); an excess from the
// forced 1s off the largest count.  Symbols are spread in byte order with a
// step of 2^10 + 2^8 + 3.  In state X the decoder emits b = spread[X]; the
// k-th state of b (k = n_b, n_b + 1, ... in increasing X) reads 11 -
// floor(log2 k) bits and moves to (k << bits) - 2^11 + those bits.
//
// The tables live in static device arrays, one copy per GPU, filled once
// per device from the host (hipMemcpy to the arrays' addresses, no device
// allocation).  Kernels get their addresses as arguments.
#include <cmath>
#include <cstring>
#include <mutex>

#include "pivco_int.h"

namespace pivco {
namespace {

static __device__ uint32_t g_dec[kFseTables][kFseSize];      // sym | bits << 8 | base << 12
static __device__ uint16_t g_enc[kFseTables][kFseEncWords];  // norm[256] | first[256] | state[2048]
static __device__ uint8_t g_dmax[64];                        // deepest node a table is chosen for (+1; 0: never)

struct HostTables {
  uint32_t dec[kFseTables][kFseSize];
  uint16_t enc[kFseTables][kFseEncWords];
  uint8_t dmax[64];
};

uint64_t ipow(uint64_t a, int e) {
  uint64_t r = 1;
  for (int i = 0; i < e; ++i) r *= a;
  return r;
}

void build_norm(uint32_t t, uint16_t norm[256]) {
  const uint64_t s = t + 49, q = 100 - s;
  const unsigned __int128 den = static_cast<unsigned __int128>(ipow(100, 8));
  unsigned __int128 rem[256];
  int32_t sum = 0;
  for (int b = 0; b < 256; ++b) {
    const int k = __builtin_popcount(b);
    const unsigned __int128 num = static_cast<unsigned __int128>(ipow(s, k) * ipow(q, 8 - k)) * kFseSize;
    uint32_t n = static_cast<uint32_t>(num / den);
    rem[b] = n ? num % den : 0;
    if (!n) n = 1;
    norm[b] = static_cast<uint16_t>(n);
    sum += static_cast<int32_t>(n);
  }
  for (; sum < static_cast<int32_t>(kFseSize); ++sum) {
    int best = -1;
    for (int b = 0; b < 256; ++b)
      if (rem[b] && (best < 0 || rem[b] > rem[best])) best = b;
    norm[best]++;
    rem[best] = 0;
  }
  if (sum > static_cast<int32_t>(kFseSize)) {
    int big = 0;
    for (int b = 1; b < 256; ++b)
      if (norm[b] > norm[big]) big = b;
    norm[big] = static_cast<uint16_t>(norm[big] - (sum - static_cast<int32_t>(kFseSize)));
  }
}

void build(HostTables &H) {
  std::memset(&H, 0, sizeof(H));
  for (uint32_t t = 1; t <= kFseTables; ++t) {
    uint16_t *norm = H.enc[t - 1], *first = norm + 256, *state = norm + 512;
    build_norm(t, norm);
    uint8_t spread[kFseSize];
    const uint32_t step = (kFseSize >> 1) + (kFseSize >> 3) + 3;
    uint32_t pos = 0;
    for (int b = 0; b < 256; ++b)
      for (uint32_t i = 0; i < norm[b]; ++i) {
        spread[pos] = static_cast<uint8_t>(b);
        pos = (pos + step) & (kFseSize - 1);
      }
    uint32_t next[256], at = 0;
    for (int b = 0; b < 256; ++b) {
      next[b] = norm[b];
      first[b] = static_cast<uint16_t>(at);
      at += norm[b];
    }
    for (uint32_t X = 0; X < kFseSize; ++X) {
      const uint32_t b = spread[X];
      const uint32_t k = next[b]++;
      const uint32_t nb = kFseLog - (31 - __builtin_clz(k));
      H.dec[t - 1][X] = b | (nb << 8) | (((k << nb) - kFseSize) << 12);
      state[first[b] + (k - norm[b])] = static_cast<uint16_t>(X);
    }
    // the selection's benefit ratio (depth + H) / (depth + 1) < 0.95, with H
    // the table's expected bits per bitmap bit at its own skew
    const double sk = static_cast<double>(t + 49) / 100.0;
    double h = 0.0;
    for (int b = 0; b < 256; ++b) {
      const int k = __builtin_popcount(b);
      h += std::pow(sk, k) * std::pow(1.0 - sk, 8 - k) * (static_cast<double>(kFseLog) - std::log2(static_cast<double>(norm[b]))) / 8.0;
    }
    uint8_t dm = 0;
    for (uint32_t d = 0; d < 16; ++d)
      if (static_cast<double>(d) + h < 0.95 * (static_cast<double>(d) + 1.0)) dm = static_cast<uint8_t>(d + 1);
    H.dmax[t] = dm;
  }
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
FseTables g_ptrs[kMaxDevices] = {};
HostTables *g_host = nullptr;

}  // namespace

// The tables' device addresses on the current device, uploading them the
// first time (synchronous); null on a runtime error.
const FseTables *fse_tables() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  FseTables &P = g_ptrs[dev];
  if (P.dec) return &P;
  if (!g_host) {
    g_host = new HostTables;
    build(*g_host);
  }
  void *dec = nullptr, *enc = nullptr, *dmax = nullptr;
  if (hipGetSymbolAddress(&dec, HIP_SYMBOL(g_dec)) != hipSuccess ||
      hipGetSymbolAddress(&enc, HIP_SYMBOL(g_enc)) != hipSuccess ||
      hipGetSymbolAddress(&dmax, HIP_SYMBOL(g_dmax)) != hipSuccess)
    return nullptr;
  if (hipMemcpy(dec, g_host->dec, sizeof(g_host->dec), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(enc, g_host->enc, sizeof(g_host->enc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dmax, g_host->dmax, sizeof(g_host->dmax), hipMemcpyHostToDevice) != hipSuccess)
    return nullptr;
  P.dec = static_cast<const uint32_t *>(dec);
  P.enc = static_cast<const uint16_t *>(enc);
  P.dmax = static_cast<const uint8_t *>(dmax);
  return &P;
}

}  // namespace pivco
