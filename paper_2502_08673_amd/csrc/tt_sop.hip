// tt_sop.hip -- two-level minimisation of a packed plane on the host (the
// downstream step after enumeration; no device code): Quine-McCluskey prime
// implicants, essential primes, then a branch-and-bound cover search for
// the fewest terms and, among those, the fewest literals; and the text of a
// four-variable Karnaugh map in the layout of the paper's map template.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "tt.h"

namespace {

struct Cube {
  uint32_t care, value;  // covers row r iff (r & care) == value
  bool operator==(const Cube& o) const { return care == o.care && value == o.value; }
};
struct CubeHash {
  size_t operator()(const Cube& c) const { return ((size_t)c.care << 32) ^ c.value; }
};

int popc(uint32_t x) { return __builtin_popcount(x); }

// Quine-McCluskey: merge cubes that differ in one cared digit, level by
// level; cubes never merged are prime.
std::vector<Cube> prime_implicants(const uint64_t* plane, int n) {
  const uint32_t full = (n == 32) ? ~0u : ((1u << n) - 1u);
  std::vector<Cube> level, primes;
  for (uint32_t r = 0; r < (1u << n); ++r)
    if ((plane[r >> 6] >> (r & 63)) & 1ull) level.push_back({full, r});
  while (!level.empty()) {
    std::unordered_set<Cube, CubeHash> next_set, merged;
    std::unordered_set<Cube, CubeHash> present(level.begin(), level.end());
    for (const Cube& c : level) {
      bool any = false;
      for (int j = 0; j < n; ++j) {
        const uint32_t bit = 1u << j;
        if (!(c.care & bit)) continue;
        const Cube o{c.care, c.value ^ bit};
        if (present.count(o)) {
          any = true;
          next_set.insert({c.care & ~bit, c.value & ~bit});
        }
      }
      if (!any) primes.push_back(c);
    }
    level.assign(next_set.begin(), next_set.end());
  }
  return primes;
}

struct Search {
  int n_min = 0;
  std::vector<std::vector<int>> by_minterm;  // primes covering each on-set row (index)
  std::vector<std::vector<uint32_t>> prime_rows;  // rows (indices) each prime covers
  std::vector<int> prime_lits;
  std::vector<int> count;  // how many chosen primes cover each row
  std::vector<int> chosen, best;
  int best_terms = 1 << 30, best_lits = 1 << 30;
  long nodes = 0, budget = 0;
  bool exhausted = false;

  void take(int p, int d) {
    for (uint32_t m : prime_rows[p]) count[m] += d;
  }
  void run(int terms, int lits) {
    if (++nodes > budget) {
      exhausted = true;
      return;
    }
    int pick = -1;
    size_t fewest = ~size_t(0);
    for (int m = 0; m < n_min; ++m)
      if (count[m] == 0 && by_minterm[m].size() < fewest) {
        fewest = by_minterm[m].size();
        pick = m;
      }
    if (pick < 0) {
      if (terms < best_terms || (terms == best_terms && lits < best_lits)) {
        best_terms = terms;
        best_lits = lits;
        best = chosen;
      }
      return;
    }
    if (terms + 1 > best_terms) return;  // one more term is needed at least
    std::vector<int> cand = by_minterm[pick];
    std::sort(cand.begin(), cand.end(), [&](int a, int b) {
      return prime_rows[a].size() != prime_rows[b].size() ? prime_rows[a].size() > prime_rows[b].size()
                                                          : prime_lits[a] < prime_lits[b];
    });
    for (int p : cand) {
      if (terms + 1 == best_terms && lits + prime_lits[p] >= best_lits) continue;
      chosen.push_back(p);
      take(p, +1);
      run(terms + 1, lits + prime_lits[p]);
      take(p, -1);
      chosen.pop_back();
      if (exhausted) return;
    }
  }
};

}  // namespace

extern "C" {

int tt_sop_minimize(const uint64_t* h_plane, int n_vars, long node_budget, int max_terms, uint32_t* h_care,
                    uint32_t* h_value, int* n_terms, int* n_literals, int* exact) {
  if (!h_plane || n_vars < 0 || n_vars > 12 || max_terms < 0 || !n_terms || !n_literals || !exact) return TT_EINVAL;
  if (max_terms > 0 && (!h_care || !h_value)) return TT_EINVAL;
  const uint32_t rows = 1u << n_vars;
  // the plane's rows (bits past 2^n_vars in a one-word plane are ignored)
  std::vector<uint64_t> plane((rows + 63) / 64, 0);
  for (uint32_t w = 0; w < plane.size(); ++w) plane[w] = h_plane[w];
  if (rows < 64) plane[0] &= (1ull << rows) - 1ull;
  std::vector<Cube> primes = prime_implicants(plane.data(), n_vars);
  Search S;
  std::vector<uint32_t> on;
  std::vector<int32_t> index(rows, -1);
  for (uint32_t r = 0; r < rows; ++r)
    if ((plane[r >> 6] >> (r & 63)) & 1ull) {
      index[r] = (int32_t)on.size();
      on.push_back(r);
    }
  S.n_min = (int)on.size();
  S.by_minterm.assign(S.n_min, {});
  S.prime_rows.assign(primes.size(), {});
  S.prime_lits.assign(primes.size(), 0);
  for (size_t p = 0; p < primes.size(); ++p) {
    S.prime_lits[p] = popc(primes[p].care);
    // rows of the cube: enumerate the free digits
    const uint32_t free_mask = ((rows - 1u)) & ~primes[p].care;
    uint32_t sub = 0;
    do {
      const uint32_t r = primes[p].value | sub;
      S.prime_rows[p].push_back((uint32_t)index[r]);
      S.by_minterm[index[r]].push_back((int)p);
      sub = (sub - free_mask) & free_mask;
    } while (sub != 0);
  }
  S.count.assign(S.n_min, 0);
  // essential primes first (a row only one prime covers)
  std::vector<char> taken(primes.size(), 0);
  int terms = 0, lits = 0;
  for (int m = 0; m < S.n_min; ++m)
    if (S.by_minterm[m].size() == 1 && !taken[S.by_minterm[m][0]]) {
      const int p = S.by_minterm[m][0];
      taken[p] = 1;
      S.chosen.push_back(p);
      S.take(p, +1);
      ++terms;
      lits += S.prime_lits[p];
    }
  S.budget = node_budget > 0 ? node_budget : 1000000;
  S.run(terms, lits);
  if (S.best_terms == (1 << 30)) return TT_ERANGE;  // no cover found within the budget
  *n_terms = S.best_terms;
  *n_literals = S.best_lits;
  *exact = S.exhausted ? 0 : 1;
  for (int t = 0; t < S.best_terms && t < max_terms; ++t) {
    h_care[t] = primes[S.best[t]].care;
    h_value[t] = primes[S.best[t]].value;
  }
  return TT_OK;
}

int tt_kmap_text(const uint64_t* h_plane, char* buf, int size) {
  // rows x1 x2 and columns x3 x4 in Gray order; cell = row 8 x1 + 4 x2 + 2 x3 + x4
  if (!h_plane || !buf || size < 128) return TT_EINVAL;
  static const int gray[4] = {0, 1, 3, 2};
  static const char* lab[4] = {"00", "01", "11", "10"};
  int o = snprintf(buf, size, "x1x2\\x3x4  00 01 11 10\n");
  for (int i = 0; i < 4; ++i) {
    o += snprintf(buf + o, size - o, "%8s   ", lab[i]);
    for (int k = 0; k < 4; ++k) {
      const int r = 8 * (gray[i] >> 1) + 4 * (gray[i] & 1) + 2 * (gray[k] >> 1) + (gray[k] & 1);
      o += snprintf(buf + o, size - o, " %d ", (int)((h_plane[0] >> r) & 1ull));
    }
    o += snprintf(buf + o, size - o, "\n");
  }
  return TT_OK;
}

}  // extern "C"
