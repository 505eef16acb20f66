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
// include it.  No row is ever bought beyond its first 2m - 2 items, so rows
// stop there.
//
// The sorts are stable counting/radix passes (the data decide the branches of
// a comparison sort): symbols by (count asc, id asc) from a radix sort of the
// counts over the ids in order, then (count desc, id asc) by walking the runs
// of equal counts backwards.
pivco_status lengths_from_counts(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]) {
  std::memset(len, 0, 256);
  uint32_t sym[256], tmp[256];
  uint64_t maxc = 0;
  size_t m = 0;
  for (uint32_t s = 0; s < 256; ++s)
    if (counts[s]) {
      sym[m++] = s;
      maxc = counts[s] > maxc ? counts[s] : maxc;
    }
  if (m < 2 || max_len < 1 || max_len > 15 || (size_t(1) << max_len) < m) return PIVCO_E_ARG;
  // LSD radix sort of the present symbols by count, 8 bits a pass (stable)
  for (uint32_t shift = 0; shift < 64 && (maxc >> shift); shift += 8) {
    uint32_t hist[257] = {0};
    for (size_t i = 0; i < m; ++i) hist[((counts[sym[i]] >> shift) & 255) + 1]++;
    for (int d = 0; d < 256; ++d) hist[d + 1] += hist[d];
    for (size_t i = 0; i < m; ++i) tmp[hist[(counts[sym[i]] >> shift) & 255]++] = sym[i];
    std::memcpy(sym, tmp, m * sizeof(uint32_t));
  }
  uint64_t w[257];
  for (size_t i = 0; i < m; ++i) w[i] = counts[sym[i]];
  w[m] = ~uint64_t(0);                        // past the last single: never taken
  const size_t cap = 2 * m - 2;               // items ever bought in a row
  // rows r = 1 (2^-1) .. max_len (2^-L): weights and single-coin flags
  uint64_t weight[16][512];
  uint8_t single[16][512];
  size_t rlen[16] = {0};
  const size_t top = m < cap ? m : cap;
  for (size_t i = 0; i < top; ++i) { weight[max_len][i] = w[i]; single[max_len][i] = 1; }
  rlen[max_len] = top;
  uint64_t pk[257];
  for (uint32_t r = max_len; r > 1; --r) {
    const uint64_t *below = weight[r];
    const size_t np = rlen[r] / 2;
    for (size_t j = 0; j < np; ++j) pk[j] = below[2 * j] + below[2 * j + 1];
    pk[np] = ~uint64_t(0);
    uint64_t *wr = weight[r - 1];
    uint8_t *sr = single[r - 1];
    // branch-free merge: a single is taken when it weighs no more than the
    // next package (both lists end in a sentinel that is never taken first)
    const size_t total = m + np < cap ? m + np : cap;
    size_t a = 0, p = 0;
    for (size_t o = 0; o < total; ++o) {
      const uint64_t x = w[a], y = pk[p];
      const bool take = x <= y;
      wr[o] = take ? x : y;
      sr[o] = static_cast<uint8_t>(take);
      a += take;
      p += !take;
    }
    rlen[r - 1] = total;
  }
  // bought items row by row: the first k of row r, k = 2m - 2 in row 1
  uint32_t nlen[17] = {0};                    // symbols of each length, from the singles bought
  uint32_t depth[256] = {0};
  size_t k = cap;
  for (uint32_t r = 1; r <= max_len && k; ++r) {
    if (k > rlen[r]) return PIVCO_E_ARG;
    size_t singles = 0;
    for (size_t i = 0; i < k; ++i) singles += single[r][i];
    for (size_t i = 0; i < singles; ++i) depth[i]++;
    k = 2 * (k - singles);
  }
  // the lengths, ascending, go to the symbols by (count desc, id asc): runs
  // of equal counts of the ascending order, taken from the last run back
  for (size_t i = 0; i < m; ++i) {
    if (depth[i] < 1 || depth[i] > max_len) return PIVCO_E_ARG;
    nlen[depth[i]]++;
  }
  uint32_t l = 1;
  size_t given = 0;
  for (size_t end = m; end > 0;) {
    size_t beg = end - 1;
    while (beg > 0 && counts[sym[beg - 1]] == counts[sym[end - 1]]) --beg;
    for (size_t i = beg; i < end; ++i) {
      while (given == nlen[l]) { given = 0; ++l; }
      len[sym[i]] = static_cast<uint8_t>(l);
      ++given;
    }
    end = beg;
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
