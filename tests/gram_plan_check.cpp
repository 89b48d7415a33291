// Checks the invariants of the Gram pass's work plan (make_gram_plan) on pair
// sizes read from stdin: "P s_0 ... s_{P-1}".  Prints "OK ..." and exits 0,
// or prints the first violated invariant and exits 1.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

#include "gram_plan.h"

static int fail(const char* what, long a = 0, long b = 0) {
  std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

static int check(const std::vector<int64_t>& off, int64_t lanes, int64_t rows, int64_t small) {
  const int64_t P = (int64_t)off.size() - 1, chunk = lanes * rows;
  const GramPlan g = make_gram_plan(off.data(), P, lanes, rows, small);
  std::vector<int> seen(P, 0);
  std::vector<int64_t> covered(P, 0);
  std::map<int32_t, int64_t> first;  // multi pair -> first slot
  for (size_t i = 0; i < g.multi.size(); ++i) first[g.multi[i]] = g.multi_first[i];
  if ((int64_t)g.multi_first.size() != g.n_multi || (int64_t)g.multi.size() != g.n_multi)
    return fail("multi sizes", (long)g.multi_first.size(), g.n_multi);
  if (g.big_slot.size() != g.big_pair.size() || g.big_chunk.size() != g.big_pair.size())
    return fail("chunk table sizes", (long)g.big_slot.size(), (long)g.big_pair.size());
  std::vector<int> slot_used(g.n_partials, 0);
  int32_t prev_rows = 1 << 30;
  for (size_t i = 0; i < g.big_pair.size(); ++i) {
    const int32_t n = g.big_pair[i], j = g.big_chunk[i], s = g.big_slot[i];
    if (n < 0 || n >= P) return fail("big pair out of range", n);
    const int64_t c = off[n + 1] - off[n];
    if (c <= small) return fail("small pair in a chunk", n, c);
    const int64_t nch = (c + chunk - 1) / chunk;
    if (j < 0 || j >= nch) return fail("chunk index", n, j);
    const int64_t cnt = std::min<int64_t>(chunk, c - (int64_t)j * chunk);
    const int32_t r = (int32_t)((cnt + lanes - 1) / lanes);
    if (r > rows) return fail("chunk rows", n, r);
    if (r > prev_rows) return fail("chunks not longest first", (long)i, r);
    prev_rows = r;
    covered[n] += cnt;
    ++seen[n];
    if (nch == 1) {
      if (s != -1) return fail("single-chunk pair has a slot", n, s);
    } else {
      auto it = first.find(n);
      if (it == first.end()) return fail("multi pair not listed", n);
      if (s != it->second + j) return fail("slot not first + chunk", n, s);
      if (s < 0 || s >= g.n_partials || slot_used[s]++) return fail("slot reused or out of range", n, s);
    }
  }
  prev_rows = 1 << 30;
  if (g.groups.size() % 4) return fail("groups not a multiple of 4", (long)g.groups.size());
  for (size_t q = 0; q < g.groups.size(); q += 4) {
    int32_t r = -1;
    bool pad = false;
    for (int k = 0; k < 4; ++k) {
      const int32_t n = g.groups[q + k];
      if (n < 0) {
        pad = true;
        continue;
      }
      if (pad) return fail("live pair after an empty slot", (long)q, n);
      if (n >= P) return fail("group pair out of range", n);
      const int64_t c = off[n + 1] - off[n];
      if (c < 0 || c > small) return fail("group pair size", n, c);
      const int32_t rr = (int32_t)((c + 15) / 16);
      if (r >= 0 && rr != r) return fail("group rows differ", (long)q, rr);
      r = rr;
      covered[n] += c;
      ++seen[n];
    }
    if (r < 0) return fail("group without a pair", (long)q);
    if (r > prev_rows) return fail("groups not longest first", (long)q, r);
    prev_rows = r;
  }
  int64_t empty = 0;
  for (int64_t n = 0; n < P; ++n) empty += off[n + 1] == off[n];
  if (empty != g.n_empty) return fail("empty count", (long)empty, (long)g.n_empty);
  for (int64_t n = 0; n < P; ++n) {
    const int64_t c = off[n + 1] - off[n];
    const int expect = c <= small ? 1 : (int)((c + chunk - 1) / chunk);
    if (seen[n] != expect) return fail("pair covered a wrong number of times", n, seen[n]);
    if (covered[n] != c) return fail("pair matches not covered exactly", n, covered[n]);
  }
  for (int64_t s = 0; s < g.n_partials; ++s)
    if (!slot_used[s]) return fail("partial slot unused", s);
  std::printf("OK rows=%ld chunks=%zu groups=%zu partials=%ld multi=%ld empty=%ld\n", (long)rows, g.big_pair.size(),
              g.groups.size() / 4, (long)g.n_partials, (long)g.n_multi, (long)g.n_empty);
  return 0;
}

int main() {
  long P;
  if (std::scanf("%ld", &P) != 1 || P < 0) return fail("input");
  std::vector<int64_t> off(P + 1, 0);
  for (long n = 0; n < P; ++n) {
    long c;
    if (std::scanf("%ld", &c) != 1 || c < 0) return fail("input size", n);
    off[n + 1] = off[n] + c;
  }
  // the two shapes the library uses: chunks of 16 rows and groups of pairs
  // up to 256 matches (FP32/FP64), chunks of 64 rows and groups of pairs up
  // to 1024 matches (BF16)
  return check(off, 64, 16, 256) || check(off, 64, 64, 1024);
}
