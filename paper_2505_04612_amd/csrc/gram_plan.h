// Work decomposition of the Gram pass, computed on the host from the pair
// offsets at set-up (plain C++, no device code, so it can be checked on its
// own).
//
// A pair with more than `small` matches is cut into chunks of lanes * rows
// matches (one wavefront each: lane l takes matches l + lanes r of the
// chunk); a pair with 0..small matches is bucketed by its number of
// 16-match rows and packed four to a wavefront (16 lanes each; the last
// group of a bucket is padded with -1; a pair without matches is a group
// slot of zero rows, which writes its zero Gram).  Chunks are ordered by row
// count, longest first, and so are the groups, so that the work items still
// waiting for a free slot at the end of the pass are short ones.  A pair
// that spans several chunks gets one partial slot per chunk (consecutive, in
// chunk order) and an arrival counter; the chunk that arrives last adds the
// partials.  Which wavefront runs an item does not change a pair's result
// (each pair's sums use a fixed lane/row assignment and reduction order).
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

struct GramPlan {
  std::vector<int32_t> big_pair, big_chunk;  // chunk work items: pair, chunk index within the pair
  std::vector<int32_t> big_slot;             // partial slot of the chunk (-1: the chunk is its whole pair)
  std::vector<int32_t> groups;               // [4 n_groups] pair ids, -1 = unused slot
  std::vector<int32_t> multi;                // pairs spanning several chunks
  std::vector<int64_t> multi_first;          // first partial slot of each multi-chunk pair
  int64_t n_multi = 0, n_empty = 0, n_partials = 0;
};

inline GramPlan make_gram_plan(const int64_t* off, int64_t P, int64_t lanes, int64_t rows, int64_t small) {
  struct Chunk {
    int32_t pair, chunk, slot, rows;
  };
  const int64_t chunk = lanes * rows;
  const int64_t max_group_rows = (small + 15) / 16;
  GramPlan g;
  std::vector<Chunk> chunks;
  std::vector<std::vector<int32_t>> bucket(max_group_rows + 1);
  for (int64_t n = 0; n < P; ++n) {
    const int64_t c = off[n + 1] - off[n];
    if (c <= small) {
      if (c == 0) ++g.n_empty;
      bucket[(c + 15) / 16].push_back((int32_t)n);
    } else {
      const int64_t nch = (c + chunk - 1) / chunk;
      if (nch > 1) {
        g.multi.push_back((int32_t)n);
        g.multi_first.push_back(g.n_partials);
      }
      for (int64_t j = 0; j < nch; ++j) {
        const int64_t cnt = std::min<int64_t>(chunk, c - j * chunk);
        chunks.push_back({(int32_t)n, (int32_t)j, nch > 1 ? (int32_t)(g.n_partials + j) : -1,
                          (int32_t)((cnt + lanes - 1) / lanes)});
      }
      if (nch > 1) g.n_partials += nch;
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& x, const Chunk& y) { return x.rows > y.rows; });
  for (const Chunk& ch : chunks) {
    g.big_pair.push_back(ch.pair);
    g.big_chunk.push_back(ch.chunk);
    g.big_slot.push_back(ch.slot);
  }
  for (int64_t r = max_group_rows; r >= 0; --r) {
    for (int32_t n : bucket[r]) g.groups.push_back(n);
    while (g.groups.size() % 4) g.groups.push_back(-1);
  }
  g.n_multi = (int64_t)g.multi.size();
  return g;
}
