// golomb.hip -- PivCo-Golomb (App. G of the paper) on gfx950.
//
// The pivoted layout applied to a unary code: instead of a tree, a list of
// bitmaps, one per code-bit position.  A value v (0..255) is v 0-bits and a
// 1-bit; bitmap k holds, in stream order, the k-th code bit of every value
// >= k, so its 1 bits mark the values equal to k.  Decoding walks the list
// bottom-up, from the last bitmap to the first: at bitmap k a 1 bit gives 0
// and a 0 bit gives 1 + the value the next bitmap holds at that position
// (the appendix's merge_vec_cst_plus1 with constant 0xFF).  Stream format
// "PVG1": a 32-byte header, block offsets, then per block comp_size, n, K
// (bitmaps), the sizes n_1 .. n_{K-1}, and the bitmaps (LSB first).
//
// Encode: k_ghist (block histograms) -> host layout (the bitmap sizes follow
// from the histograms) -> k_gbits, one workgroup per (block, bitmap): a
// stable compaction of the block's values >= k gives each value's bit
// position, and the values equal to k set their bit.
// Decode: k_gdecode, one workgroup per block, tiles of kGT values: a
// top-down count gives each bitmap's share of the tile (the 0 bits of one
// bitmap's share are the next one's), then the bottom-up merge: a lane makes
// 16 values from 16 bits, their rank (a workgroup scan), 4-byte windows of
// the next bitmap's values and one v_perm_b32 per 4 values (selector 0x0C
// gives the constant 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "pivco_int.h"

namespace pivco {
namespace {

constexpr uint32_t kGMagic = 0x31475650u;   // "PVG1"
constexpr uint32_t kGHdr = 32;
constexpr int kGW = 64;
constexpr int kGNT = 1024;                  // decode workgroup
constexpr uint32_t kGT = 16 * kGNT;         // values per decode tile
constexpr uint32_t kGSlice = 1u << 16;      // histogram slice

// One Golomb job as the decode kernel sees it.
struct GJob {
  const uint8_t *in;
  uint64_t in_len;
  uint8_t *out;
  uint64_t out_cap;
  uint64_t n_total;
  uint32_t n_blocks, block_size;
  int32_t *status;
  uint64_t pad;
};

__device__ __forceinline__ void gset_err(int32_t *status, int32_t e) {
  atomicCAS(reinterpret_cast<int *>(status), 0, e);
}

__device__ __forceinline__ uint32_t g_incl_scan(uint32_t v) {
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, false));
  return v;
}

// ---------------------------------------------------------------------------
// encode kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ghist(const uint8_t *in, uint64_t n, uint32_t bs, uint32_t spb,
                                               uint32_t *hist) {
  __shared__ uint32_t h[256];
  const uint32_t tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint64_t b = blockIdx.x / spb, sl = blockIdx.x % spb;
  const uint64_t b0 = b * bs, b1 = b0 + bs < n ? b0 + bs : n;
  const uint64_t s0 = b0 + sl * kGSlice, s1 = s0 + kGSlice < b1 ? s0 + kGSlice : b1;
  for (uint64_t i = s0 + tid; i < s1; i += 256) atomicAdd(&h[in[i]], 1u);
  __syncthreads();
  if (h[tid]) atomicAdd(&hist[b * 256 + tid], h[tid]);
}

// One workgroup per (block, bitmap k): the block's values in order, 1024 at
// a time; a value >= k takes the next bit of bitmap k (wave ballot ranks +
// the waves before it + the running count), and a value equal to k sets it.
// The stream was zeroed, so bits are only ever ORed in.
struct GLevel {
  uint64_t in_off;        // first value of the block
  uint64_t bit0;          // first bit of bitmap k in the stream
  uint32_t n;             // values of the block
  uint32_t k;
};

__global__ __launch_bounds__(256) void k_gbits(const uint8_t *in, const GLevel *lv, uint32_t nlv,
                                               uint32_t *out) {
  if (blockIdx.x >= nlv) return;
  __shared__ uint32_t wcnt[4];
  __shared__ uint32_t run;
  const GLevel L = lv[blockIdx.x];
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
  if (tid == 0) run = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < L.n; c0 += 1024) {
    uint32_t v[4];
    bool ge[4];
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = c0 + 4 * tid + u;
      v[u] = i < L.n ? in[L.in_off + i] : 0u;
      ge[u] = i < L.n && v[u] >= L.k;
      mine += ge[u];
    }
    // exclusive prefix of the thread's count over the workgroup
    const uint32_t inc = g_incl_scan(mine);
    if (lane == kGW - 1) wcnt[wave] = inc;
    __syncthreads();
    uint32_t before = run + inc - mine;
    for (uint32_t w = 0; w < wave; ++w) before += wcnt[w];
    const uint32_t total = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (ge[u]) {
        if (v[u] == L.k) {
          const uint64_t bit = L.bit0 + before;
          atomicOr(&out[bit >> 5], 1u << (bit & 31));
        }
        ++before;
      }
    }
    __syncthreads();
    if (tid == 0) run += total;
    __syncthreads();
  }
}

__global__ void k_gcopy(const uint8_t *src, uint64_t n, uint8_t *dst) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_gzero(uint32_t *p, uint64_t nw) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nw;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// decode kernel
// ---------------------------------------------------------------------------
struct GSmem {
  uint32_t nk[257];          // values reaching bitmap k (n_0 = n, n_K = 0)
  uint32_t cur[257];         // of which decoded by earlier tiles
  uint32_t tv[257];          // of which in this tile
  uint64_t boff[256];        // bitmap k's first byte in the stream
  uint32_t wsum[kGNT / kGW];
  uint32_t sel[16];
  uint32_t K, n, err;
  uint32_t lvl[2][kGT / 4 + 32] __attribute__((aligned(16)));
};

// 16 bits at bit x of a bitmap (bytes p[0 .. nbytes)), zero past its end.
__device__ __forceinline__ uint32_t g_bits16(const uint8_t *p, uint64_t nbytes, uint64_t x) {
  const uint64_t q = x >> 3;
  uint32_t w = 0;
#pragma unroll
  for (int e = 0; e < 3; ++e) w |= (q + e < nbytes ? static_cast<uint32_t>(p[q + e]) : 0u) << (8 * e);
  return (w >> (x & 7)) & 0xFFFF;
}

__global__ __launch_bounds__(kGNT) void k_gdecode(const GJob *jobs, const uint2 *blocks, uint32_t nblocks) {
  __shared__ GSmem sm;
  const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = __lane_id();
  if (blockIdx.x >= nblocks) return;
  const uint2 jb = blocks[blockIdx.x];
  const GJob &J = jobs[jb.x];
  const uint32_t b = jb.y;
  if (tid < 16) {            // v_perm selectors: byte e takes the next value of
    uint32_t s = 0, z = 0;   // the next bitmap (0 bit) or the constant 0 (1 bit)
    for (int e = 0; e < 4; ++e) {
      const uint32_t bit = (tid >> e) & 1;
      s |= (bit ? 0x0Cu : z) << (8 * e);
      z += 1 - bit;
    }
    sm.sel[tid] = s;
  }
  if (tid == 0) {
    int32_t err = 0;
    const uint64_t *tab = reinterpret_cast<const uint64_t *>(J.in + kGHdr);
    const uint64_t off = tab[b], end = tab[b + 1];
    const uint64_t want = J.n_total - static_cast<uint64_t>(b) * J.block_size < J.block_size
                              ? J.n_total - static_cast<uint64_t>(b) * J.block_size : J.block_size;
    uint32_t K = 0, n = 0;
    if (off < kGHdr + 8ull * (J.n_blocks + 1) || end < off || end > J.in_len || (off & 3) || end - off < 12) {
      err = PIVCO_E_CORRUPT;
    } else {
      const uint8_t *p = J.in + off;
      const uint32_t comp = *reinterpret_cast<const uint32_t *>(p);
      n = *reinterpret_cast<const uint32_t *>(p + 4);
      K = p[8] | (p[9] << 8);
      const uint64_t hlen = 12 + 4ull * (K ? K - 1 : 0);
      if (n != want || p[10] || p[11] || K > 256 || (n == 0) != (K == 0) || comp < hlen ||
          comp > end - off || ((comp + 3ull) & ~3ull) != end - off) {
        err = PIVCO_E_CORRUPT;
      } else {
        uint64_t o = off + hlen;
        for (uint32_t k = 0; k < K; ++k) {
          const uint32_t nk = k ? *reinterpret_cast<const uint32_t *>(p + 12 + 4 * (k - 1)) : n;
          if (k && nk > sm.nk[k - 1]) err = PIVCO_E_CORRUPT;
          sm.nk[k] = nk;
          sm.boff[k] = o;
          o += (nk + 7) / 8;
        }
        if (o != off + comp) err = PIVCO_E_CORRUPT;
      }
    }
    if (err) K = 0;
    sm.nk[K] = 0;
    sm.K = K;
    sm.n = n;
    sm.err = err;
  }
  __syncthreads();
  const uint32_t K = sm.K, n = sm.n;
  if (sm.err) {
    if (tid == 0) gset_err(J.status, static_cast<int32_t>(sm.err));
    return;
  }
  for (uint32_t k = tid; k <= K; k += kGNT) sm.cur[k] = 0;
  __syncthreads();
  uint8_t *out = J.out + static_cast<uint64_t>(b) * J.block_size;
  const uint8_t *lds = reinterpret_cast<const uint8_t *>(&sm);
  for (uint32_t t0 = 0; t0 < n; t0 += kGT) {
    const uint32_t S = n - t0 < kGT ? n - t0 : kGT;
    // count, top-down: the 0 bits of bitmap k's share are bitmap k+1's share
    if (tid == 0) sm.tv[0] = S;
    __syncthreads();
    uint32_t kmax = 0;                       // bitmaps with a share in this tile
    for (uint32_t k = 0; k < K; ++k) {
      const uint32_t tvk = sm.tv[k];
      if (tvk == 0) break;
      kmax = k + 1;
      const uint32_t x = 16 * tid;
      const uint32_t bits = x < tvk ? g_bits16(J.in + sm.boff[k], (sm.nk[k] + 7) / 8, sm.cur[k] + x) &
                                          (tvk - x >= 16 ? 0xFFFFu : (1u << (tvk - x)) - 1)
                                    : 0u;
      const uint32_t inc = g_incl_scan(__popc(bits));
      if (lane == kGW - 1) sm.wsum[wave] = inc;
      __syncthreads();
      if (tid == 0) {
        uint32_t ones = 0;
        for (uint32_t w = 0; w < kGNT / kGW; ++w) ones += sm.wsum[w];
        const uint32_t zeros = tvk - ones;
        if (sm.cur[k + 1] + zeros > sm.nk[k + 1]) { sm.err = PIVCO_E_CORRUPT; sm.tv[k + 1] = 0; }
        else sm.tv[k + 1] = zeros;
      }
      __syncthreads();
    }
    if (sm.err) break;
    // merge, bottom-up; level k's values go to buffer k & 1, plus one for
    // every level but the first (its parent reads them as "1 + value")
    for (int k = static_cast<int>(kmax) - 1; k >= 0; --k) {
      const uint32_t tvk = sm.tv[k];
      const uint32_t x = 16 * tid;
      const bool act = x < tvk;
      const uint32_t bits = act ? g_bits16(J.in + sm.boff[k], (sm.nk[k] + 7) / 8, sm.cur[k] + x) &
                                      (tvk - x >= 16 ? 0xFFFFu : (1u << (tvk - x)) - 1)
                                : 0u;
      const uint32_t pc = __popc(bits);
      const uint32_t inc = g_incl_scan(pc);
      if (lane == kGW - 1) sm.wsum[wave] = inc;
      __syncthreads();
      uint32_t r1 = inc - pc;
      for (uint32_t w = 0; w < wave; ++w) r1 += sm.wsum[w];
      uint32_t r0 = x - r1;                  // values of the next bitmap before this task
      const uint32_t cb = static_cast<uint32_t>(reinterpret_cast<const uint8_t *>(sm.lvl[(k + 1) & 1]) - lds);
      uint32_t o[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t m = (bits >> (4 * g)) & 15;
        const uint32_t a = cb + r0;
        const uint32_t *q = reinterpret_cast<const uint32_t *>(lds + (a & ~3u));
        const uint32_t win = __builtin_amdgcn_alignbyte(q[1], q[0], a);
        o[g] = __builtin_amdgcn_perm(0u, win, sm.sel[m]);
        r0 += 4 - __popc(m);
      }
      if (act) {
        if (k > 0) {
          uint4 *dst = reinterpret_cast<uint4 *>(sm.lvl[k & 1]) + tid;
          *dst = make_uint4(o[0] + 0x01010101u, o[1] + 0x01010101u, o[2] + 0x01010101u, o[3] + 0x01010101u);
        } else {
          uint8_t *d = out + t0 + x;
          const uint32_t cnt = tvk - x < 16 ? tvk - x : 16;
          if (cnt == 16 && !(reinterpret_cast<uintptr_t>(d) & 15)) {
            *reinterpret_cast<uint4 *>(d) = make_uint4(o[0], o[1], o[2], o[3]);
          } else {
            for (uint32_t e = 0; e < cnt; ++e) d[e] = static_cast<uint8_t>(o[e >> 2] >> (8 * (e & 3)));
          }
        }
      }
      __syncthreads();
    }
    for (uint32_t k = tid; k < kmax; k += kGNT) sm.cur[k] += sm.tv[k];
    __syncthreads();
  }
  // the whole block consumed every bitmap, and the last one had no 0 bit
  if (!sm.err)
    for (uint32_t k = tid; k < K; k += kGNT)
      if (sm.cur[k] != sm.nk[k]) atomicCAS(&sm.err, 0u, static_cast<uint32_t>(PIVCO_E_CORRUPT));
  __syncthreads();
  if (tid == 0 && sm.err) gset_err(J.status, static_cast<int32_t>(sm.err));
}

inline uint64_t galign(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace
}  // namespace pivco

using namespace pivco;

extern "C" {

uint64_t pivco_golomb_encode_bound(uint64_t n, uint32_t block_size) {
  if (block_size == 0) return 0;
  const uint64_t nb = div_up(n, block_size);
  return kGHdr + 8 * (nb + 1) + nb * (12 + 4 * 255 + 256 + 4) + 32 * n;
}

uint64_t pivco_golomb_encode_workspace(uint64_t n, uint32_t block_size) {
  if (block_size == 0) return 0;
  const uint64_t nb = div_up(n, block_size);
  // histograms, the (block, bitmap) list, staged headers
  return galign(nb * 1024 + 16, 256) + galign(nb * 256 * sizeof(GLevel), 256) +
         galign(kGHdr + 8 * (nb + 1) + nb * (12 + 4 * 255) + 64, 256);
}

pivco_status pivco_golomb_encode(const void *d_in, uint64_t n, uint32_t block_size, void *d_out,
                                 uint64_t out_cap, uint64_t *h_out_len, void *d_ws, uint64_t ws_bytes,
                                 hipStream_t s) {
  if (!h_out_len || block_size == 0 || (n && !d_in) || !d_out || (reinterpret_cast<uintptr_t>(d_out) & 15))
    return PIVCO_E_ARG;
  const uint64_t nb = div_up(n, block_size);
  if (nb > 0xFFFFFFFFull) return PIVCO_E_ARG;
  if (!d_ws || ws_bytes < pivco_golomb_encode_workspace(n, block_size)) return PIVCO_E_CAPACITY;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  uint32_t *dh = reinterpret_cast<uint32_t *>(ws);
  GLevel *dlv = reinterpret_cast<GLevel *>(ws + galign(nb * 1024 + 16, 256));
  uint8_t *dstg = ws + galign(nb * 1024 + 16, 256) + galign(nb * 256 * sizeof(GLevel), 256);
  std::vector<uint32_t> hist(nb * 256, 0);
  if (nb) {
    const uint32_t spb = static_cast<uint32_t>(div_up(block_size, kGSlice));
    if (nb * spb > 0x7FFFFFFFull) return PIVCO_E_ARG;
    hipLaunchKernelGGL(k_gzero, dim3(static_cast<uint32_t>(std::min<uint64_t>(4096, div_up(nb * 256, 256)))),
                       dim3(256), 0, s, dh, nb * 256);
    hipLaunchKernelGGL(k_ghist, dim3(static_cast<uint32_t>(nb * spb)), dim3(256), 0, s,
                       static_cast<const uint8_t *>(d_in), n, block_size, spb, dh);
    if (hipGetLastError() != hipSuccess) return PIVCO_E_DEVICE;
    if (hipMemcpyAsync(hist.data(), dh, hist.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PIVCO_E_DEVICE;
  }
  // layout from the histograms: bitmap k of a block holds its values >= k
  std::vector<uint8_t> stg(kGHdr + 8 * (nb + 1), 0);
  std::vector<GLevel> lv;
  const uint32_t w0[6] = {kGMagic, 1u, static_cast<uint32_t>(n), static_cast<uint32_t>(n >> 32), block_size,
                          static_cast<uint32_t>(nb)};
  std::memcpy(stg.data(), w0, sizeof(w0));
  uint64_t off = stg.size();
  std::vector<std::pair<uint64_t, uint64_t>> hdrs;   // (staging offset, stream offset) of block headers
  for (uint64_t b = 0; b < nb; ++b) {
    const uint32_t bn = static_cast<uint32_t>(std::min<uint64_t>(block_size, n - b * block_size));
    const uint32_t *h = &hist[b * 256];
    uint32_t K = 0;
    for (uint32_t v = 0; v < 256; ++v) if (h[v]) K = v + 1;
    uint64_t nk[257] = {0};
    for (int v = 255; v >= 0; --v) nk[v] = nk[v + 1] + h[v];
    const uint64_t hlen = 12 + 4ull * (K ? K - 1 : 0);
    uint64_t body = 0;
    for (uint32_t k = 0; k < K; ++k) {
      lv.push_back(GLevel{b * block_size, 8 * (off + hlen + body), bn, k});
      body += (nk[k] + 7) / 8;
    }
    const uint64_t comp = hlen + body;
    std::memcpy(&stg[kGHdr + 8 * b], &off, 8);
    const uint64_t hs = stg.size();
    stg.resize(hs + hlen, 0);
    const uint32_t c32 = static_cast<uint32_t>(comp);
    std::memcpy(&stg[hs], &c32, 4);
    std::memcpy(&stg[hs + 4], &bn, 4);
    stg[hs + 8] = static_cast<uint8_t>(K);
    stg[hs + 9] = static_cast<uint8_t>(K >> 8);
    for (uint32_t k = 1; k < K; ++k) {
      const uint32_t v = static_cast<uint32_t>(nk[k]);
      std::memcpy(&stg[hs + 12 + 4 * (k - 1)], &v, 4);
    }
    hdrs.push_back({hs, off});
    off += galign(comp, 4);
  }
  std::memcpy(&stg[kGHdr + 8 * nb], &off, 8);
  if (off > out_cap) return PIVCO_E_CAPACITY;
  uint8_t *out = static_cast<uint8_t *>(d_out);
  if (hipMemcpyAsync(dstg, stg.data(), stg.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      (lv.size() && hipMemcpyAsync(dlv, lv.data(), lv.size() * sizeof(GLevel), hipMemcpyHostToDevice, s) != hipSuccess))
    return PIVCO_E_DEVICE;
  hipLaunchKernelGGL(k_gzero, dim3(static_cast<uint32_t>(std::min<uint64_t>(8192, div_up(off / 4 + 1, 256)))),
                     dim3(256), 0, s, reinterpret_cast<uint32_t *>(out), off / 4);
  // stream header and tables, then every block header (one copy each)
  hipLaunchKernelGGL(k_gcopy, dim3(static_cast<uint32_t>(std::min<uint64_t>(4096, div_up(kGHdr + 8 * (nb + 1), 256)))),
                     dim3(256), 0, s, dstg, kGHdr + 8 * (nb + 1), out);
  // block headers (small): one device-to-device copy each
  for (size_t i = 0; i < hdrs.size(); ++i) {
    const uint64_t hs = hdrs[i].first;
    const uint64_t he = i + 1 < hdrs.size() ? hdrs[i + 1].first : stg.size();
    if (hipMemcpyAsync(out + hdrs[i].second, dstg + hs, he - hs, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return PIVCO_E_DEVICE;
  }
  if (!lv.empty()) {
    hipLaunchKernelGGL(k_gbits, dim3(static_cast<uint32_t>(lv.size())), dim3(256), 0, s,
                       static_cast<const uint8_t *>(d_in), dlv, static_cast<uint32_t>(lv.size()),
                       reinterpret_cast<uint32_t *>(out));
    if (hipGetLastError() != hipSuccess) return PIVCO_E_DEVICE;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return PIVCO_E_DEVICE;
  *h_out_len = off;
  return PIVCO_OK;
}

uint64_t pivco_golomb_decode_workspace(const pivco_job *h_jobs, uint32_t count, hipStream_t s) {
  if (count && !h_jobs) return 0;
  uint64_t nb = 0;
  for (uint32_t j = 0; j < count; ++j) {
    uint8_t h[kGHdr];
    if (h_jobs[j].in_len < kGHdr || !h_jobs[j].d_in) continue;
    if (hipMemcpy(h, h_jobs[j].d_in, kGHdr, hipMemcpyDeviceToHost) != hipSuccess) return 0;
    uint32_t m = 0, b = 0;
    std::memcpy(&m, h, 4);
    std::memcpy(&b, h + 20, 4);
    if (m == kGMagic) nb += b;
  }
  (void)s;
  return galign(count * sizeof(GJob) + 16, 256) + galign(8 * nb + 16, 256);
}

pivco_status pivco_golomb_decode(const pivco_job *h_jobs, uint32_t count, int32_t *d_status, void *d_ws,
                                 uint64_t ws_bytes, hipStream_t s) {
  if (count && (!h_jobs || !d_status || !d_ws)) return PIVCO_E_ARG;
  std::vector<GJob> jobs(count);
  std::vector<uint2> blocks;
  std::vector<int32_t> st0(count, PIVCO_OK);
  for (uint32_t j = 0; j < count; ++j) {
    const pivco_job &jb = h_jobs[j];
    GJob &g = jobs[j];
    std::memset(&g, 0, sizeof(g));
    g.in = static_cast<const uint8_t *>(jb.d_in);
    g.in_len = jb.in_len;
    g.out = static_cast<uint8_t *>(jb.d_out);
    g.out_cap = jb.out_cap;
    g.status = d_status + j;
    if (jb.in_len && (!jb.d_in || (reinterpret_cast<uintptr_t>(jb.d_in) & 15))) return PIVCO_E_ARG;
    uint8_t h[kGHdr] = {0};
    if (jb.in_len < kGHdr || hipMemcpy(h, jb.d_in, kGHdr, hipMemcpyDeviceToHost) != hipSuccess) {
      st0[j] = PIVCO_E_CORRUPT;
      continue;
    }
    uint32_t m = 0, bs = 0, nb = 0;
    uint64_t n = 0;
    std::memcpy(&m, h, 4);
    std::memcpy(&n, h + 8, 8);
    std::memcpy(&bs, h + 16, 4);
    std::memcpy(&nb, h + 20, 4);
    if (m != kGMagic || h[4] != 1 || h[5] || h[6] || h[7] || bs == 0 || div_up(n, bs) != nb ||
        jb.in_len < kGHdr + 8ull * (nb + 1ull)) {
      st0[j] = PIVCO_E_CORRUPT;
      continue;
    }
    if (n > jb.out_cap) { st0[j] = PIVCO_E_CAPACITY; continue; }
    g.n_total = n;
    g.n_blocks = nb;
    g.block_size = bs;
    for (uint32_t b = 0; b < nb; ++b) blocks.push_back(make_uint2(j, b));
  }
  const uint64_t need = galign(count * sizeof(GJob) + 16, 256) + galign(8 * blocks.size() + 16, 256);
  if (ws_bytes < need) return PIVCO_E_CAPACITY;
  if (count == 0) return PIVCO_OK;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  GJob *dj = reinterpret_cast<GJob *>(ws);
  uint2 *db = reinterpret_cast<uint2 *>(ws + galign(count * sizeof(GJob) + 16, 256));
  if (hipMemcpyAsync(dj, jobs.data(), count * sizeof(GJob), hipMemcpyHostToDevice, s) != hipSuccess ||
      (blocks.size() && hipMemcpyAsync(db, blocks.data(), 8 * blocks.size(), hipMemcpyHostToDevice, s) != hipSuccess) ||
      hipMemcpyAsync(d_status, st0.data(), 4ull * count, hipMemcpyHostToDevice, s) != hipSuccess)
    return PIVCO_E_DEVICE;
  if (!blocks.empty()) {
    hipLaunchKernelGGL(k_gdecode, dim3(static_cast<uint32_t>(blocks.size())), dim3(kGNT), 0, s, dj, db,
                       static_cast<uint32_t>(blocks.size()));
    if (hipGetLastError() != hipSuccess) return PIVCO_E_DEVICE;
  }
  // the host buffers above must outlive the copies
  if (hipStreamSynchronize(s) != hipSuccess) return PIVCO_E_DEVICE;
  return PIVCO_OK;
}

}  // extern "C"
