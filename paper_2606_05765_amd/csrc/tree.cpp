// tree.cpp -- host-side code-tree construction for the encoder.
//
// App. D of the paper limits code lengths to 11 bits and stores only the
// lengths; codes are canonical (ref. [5]).  Optimal length-limited lengths
// come from package-merge (Larmore & Hirschberg, "coin collector"): the
// symbols are coins of every denomination 2^-1 .. 2^-L, packages of two
// cheapest items are formed level by level from the deepest denomination up,
// and the 2m-2 cheapest items at denomination 2^-1 are bought; a symbol's
// code length is the number of bought items containing it.
//
// Determinism rules (every encoder of the format follows them so that a
// stream is a function of its input):
//   * items are ordered by weight; on equal weight a single symbol comes
//     before a package, symbols by id, packages in creation order;
//   * the resulting multiset of lengths is handed out again in ascending
//     order to the symbols sorted by (count desc, id asc).
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "pivco_int.h"

namespace pivco {

// Rows are built from the deepest denomination (2^-L) up.  Every row is the
// merge of the m single coins with the packages formed from consecutive pairs
// of the row below, so a row only needs, per position, its weight and whether
// it is a single coin.  Buying the first k items of a row buys a prefix of its
// singles (they appear in sorted order) and a prefix of its packages (they
// appear in creation order); p bought packages buy the first 2p items of the
// row below.  A symbol's length is the number of rows whose bought singles
// include it.
pivco_status lengths_from_counts(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]) {
  std::memset(len, 0, 256);
  // symbols by (count asc, id asc): one key per symbol (counts of a block
  // stay far below 2^56)
  uint64_t key[256];
  size_t m = 0;
  for (int s = 0; s < 256; ++s) {
    if (counts[s] >> 56) return PIVCO_E_ARG;
    if (counts[s]) key[m++] = (counts[s] << 8) | static_cast<uint64_t>(s);
  }
  if (m < 2 || max_len < 1 || max_len > 15 || (size_t(1) << max_len) < m) return PIVCO_E_ARG;
  std::sort(key, key + m);
  uint64_t w[257];
  for (size_t i = 0; i < m; ++i) w[i] = key[i] >> 8;
  w[m] = ~uint64_t(0);                        // past the last single: never taken
  // rows r = 1 (2^-1) .. max_len (2^-L): weights and single-coin flags; a
  // row holds the m singles and at most m - 1 packages
  uint64_t weight[16][512];
  uint8_t single[16][512];
  size_t rlen[16] = {0};
  for (size_t i = 0; i < m; ++i) { weight[max_len][i] = w[i]; single[max_len][i] = 1; }
  rlen[max_len] = m;
  for (uint32_t r = max_len; r > 1; --r) {
    const uint64_t *below = weight[r];
    uint64_t *wr = weight[r - 1];
    uint8_t *sr = single[r - 1];
    const size_t np = rlen[r] / 2;
    // branch-free merge (the comparison is data dependent): a single is
    // taken when it weighs no more than the next package or no package is left
    size_t a = 0, p = 0;
    const size_t total = m + np;
    for (size_t o = 0; o < total; ++o) {
      const uint64_t pw = p < np ? below[2 * p] + below[2 * p + 1] : ~uint64_t(0);
      const bool take = w[a] <= pw;
      wr[o] = take ? w[a] : pw;
      sr[o] = take;
      a += take;
      p += !take;
    }
    rlen[r - 1] = total;
  }
  uint32_t depth[256] = {0};
  size_t k = 2 * m - 2;                       // items bought in row 1
  for (uint32_t r = 1; r <= max_len && k; ++r) {
    if (k > rlen[r]) return PIVCO_E_ARG;
    size_t singles = 0;
    for (size_t i = 0; i < k; ++i) singles += single[r][i];
    const size_t packs = k - singles;
    for (size_t i = 0; i < singles; ++i) depth[i]++;
    k = 2 * packs;
  }
  std::sort(depth, depth + m);
  // symbols by (count desc, id asc)
  for (size_t i = 0; i < m; ++i) {
    const uint64_t c = key[i] >> 8, sid = key[i] & 255;
    key[i] = (((uint64_t(1) << 56) - 1 - c) << 8) | sid;
  }
  std::sort(key, key + m);
  for (size_t i = 0; i < m; ++i) {
    if (depth[i] < 1 || depth[i] > max_len) return PIVCO_E_ARG;
    len[key[i] & 255] = static_cast<uint8_t>(depth[i]);
  }
  return PIVCO_OK;
}

// Canonical codes: ordered by (length, symbol); each next code is the
// previous plus one, shifted left by the length difference.
pivco_status canonical_codes(const uint8_t len[256], uint16_t code[256]) {
  uint32_t cnt[17] = {0};
  for (int s = 0; s < 256; ++s) {
    if (len[s] > 15) return PIVCO_E_ARG;
    cnt[len[s]]++;
  }
  cnt[0] = 0;
  uint32_t next[17] = {0};
  uint32_t c = 0;
  for (int l = 1; l <= 15; ++l) {
    c = (c + cnt[l - 1]) << 1;
    next[l] = c;
  }
  for (int s = 0; s < 256; ++s) {
    code[s] = 0;
    if (!len[s]) continue;
    const uint32_t v = next[len[s]]++;
    if (v >> len[s]) return PIVCO_E_ARG;
    code[s] = static_cast<uint16_t>(v);
  }
  return PIVCO_OK;
}

// Complete prefix code (Kraft sum exactly 1) with at least two symbols?
bool tree_is_complete(const uint8_t len[256], uint32_t max_len) {
  uint64_t k = 0;
  int m = 0;
  for (int s = 0; s < 256; ++s) {
    if (len[s] > max_len) return false;
    if (len[s]) {
      k += uint64_t(1) << (15 - len[s]);
      ++m;
    }
  }
  return m >= 2 && k == (uint64_t(1) << 15);
}

}  // namespace pivco
