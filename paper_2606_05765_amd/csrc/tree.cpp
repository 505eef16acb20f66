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
#include <vector>

#include "pivco_int.h"

namespace pivco {

namespace {

struct Coin {
  uint64_t weight;
  bool single;                 // one symbol (true) or a package (false)
  std::vector<uint8_t> mult;   // how often each of the m symbols occurs in it
};

}  // namespace

pivco_status lengths_from_counts(const uint64_t counts[256], uint32_t max_len, uint8_t len[256]) {
  std::memset(len, 0, 256);
  std::vector<int> sym;
  for (int s = 0; s < 256; ++s)
    if (counts[s]) sym.push_back(s);
  const size_t m = sym.size();
  if (m < 2 || max_len < 1 || max_len > 15 || (size_t(1) << max_len) < m) return PIVCO_E_ARG;
  std::stable_sort(sym.begin(), sym.end(), [&](int a, int b) { return counts[a] < counts[b]; });
  std::vector<Coin> singles(m);
  for (size_t i = 0; i < m; ++i) {
    singles[i].weight = counts[sym[i]];
    singles[i].single = true;
    singles[i].mult.assign(m, 0);
    singles[i].mult[i] = 1;
  }
  // deepest denomination first: the row holds only single coins
  std::vector<Coin> row = singles;
  for (uint32_t level = max_len; level > 1; --level) {
    std::vector<Coin> packs;
    packs.reserve(row.size() / 2);
    for (size_t i = 0; i + 1 < row.size(); i += 2) {
      Coin p;
      p.weight = row[i].weight + row[i + 1].weight;
      p.single = false;
      p.mult.resize(m);
      for (size_t k = 0; k < m; ++k) p.mult[k] = row[i].mult[k] + row[i + 1].mult[k];
      packs.push_back(std::move(p));
    }
    std::vector<Coin> next;
    next.reserve(m + packs.size());
    size_t a = 0, b = 0;
    while (a < m || b < packs.size()) {
      const bool take_single =
          b >= packs.size() || (a < m && singles[a].weight <= packs[b].weight);
      next.push_back(take_single ? singles[a++] : std::move(packs[b++]));
    }
    row.swap(next);
  }
  std::vector<uint32_t> depth(m, 0);
  for (size_t i = 0; i < 2 * m - 2 && i < row.size(); ++i)
    for (size_t k = 0; k < m; ++k) depth[k] += row[i].mult[k];
  std::vector<uint32_t> pool(depth.begin(), depth.end());
  std::sort(pool.begin(), pool.end());
  std::vector<int> order(sym.begin(), sym.end());
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return counts[x] != counts[y] ? counts[x] > counts[y] : x < y;
  });
  for (size_t i = 0; i < m; ++i) {
    if (pool[i] < 1 || pool[i] > max_len) return PIVCO_E_ARG;
    len[order[i]] = static_cast<uint8_t>(pool[i]);
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
