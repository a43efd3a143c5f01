// tt_sop.hip -- two-level minimisation of a packed plane on the host (the
// downstream step after enumeration; no device code): Quine-McCluskey prime
// implicants, essential primes, then a branch-and-bound cover search for
// the fewest terms, then the fewest literals, then (a fixed rule among equal
// covers) the smallest sorted list of term keys; the text of a four-variable
// Karnaugh map in the layout of the paper's map template; and the Simplify
// step of the transformation (Algorithm 1), which writes a found
// expression's table as a short program of logical operators.
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

// Key of a term: its literals in ascending variable order, x_j coded 2j and
// NOT x_j coded 2j + 1.  Covers of equal cost are ordered by the sorted list
// of their terms' keys (lexicographic, a shorter prefix first).
std::vector<int> term_key(const Cube& c, int n) {
  std::vector<int> k;
  for (int j = 0; j < n; ++j)
    if ((c.care >> j) & 1u) k.push_back(2 * j + (((c.value >> j) & 1u) ? 0 : 1));
  return k;
}

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
  int n_min = 0, n_vars = 0;
  const std::vector<Cube>* primes = nullptr;
  std::vector<std::vector<int>> by_minterm;  // primes covering each on-set row (index)
  std::vector<std::vector<uint32_t>> prime_rows;  // rows (indices) each prime covers
  std::vector<int> prime_lits;
  std::vector<int> count;  // how many chosen primes cover each row
  std::vector<int> chosen, best;
  std::vector<std::vector<int>> best_keys;  // sorted term keys of best
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
      if (terms > best_terms || (terms == best_terms && lits > best_lits)) return;
      std::vector<std::vector<int>> keys;
      for (int p : chosen) keys.push_back(term_key((*primes)[p], n_vars));
      std::sort(keys.begin(), keys.end());
      if (terms == best_terms && lits == best_lits && !(keys < best_keys)) return;
      best_terms = terms;
      best_lits = lits;
      best = chosen;
      best_keys = std::move(keys);
      return;
    }
    if (terms + 1 > best_terms) return;  // one more term is needed at least
    std::vector<int> cand = by_minterm[pick];
    std::sort(cand.begin(), cand.end(), [&](int a, int b) {
      return prime_rows[a].size() != prime_rows[b].size() ? prime_rows[a].size() > prime_rows[b].size()
                                                          : prime_lits[a] < prime_lits[b];
    });
    for (int p : cand) {
      if (terms + 1 == best_terms && lits + prime_lits[p] > best_lits) continue;
      chosen.push_back(p);
      take(p, +1);
      run(terms + 1, lits + prime_lits[p]);
      take(p, -1);
      chosen.pop_back();
      if (exhausted) return;
    }
  }
};

// A cover of the plane's ones by prime implicants with the fewest terms,
// then literals, then the smallest sorted list of term keys, returned sorted
// by term key.  Returns TT_ERANGE when the search found no cover within the
// node budget; *exact = 0 when it stopped early with one.
int minimize(const uint64_t* h_plane, int n_vars, long node_budget, std::vector<Cube>& cover, int* n_literals,
             int* exact) {
  const uint32_t rows = 1u << n_vars;
  // the plane's rows (bits past 2^n_vars in a one-word plane are ignored)
  std::vector<uint64_t> plane((rows + 63) / 64, 0);
  for (uint32_t w = 0; w < plane.size(); ++w) plane[w] = h_plane[w];
  if (rows < 64) plane[0] &= (1ull << rows) - 1ull;
  std::vector<Cube> primes = prime_implicants(plane.data(), n_vars);
  Search S;
  S.n_vars = n_vars;
  S.primes = &primes;
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
  // essential primes first (a row only one prime covers: in every cover)
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
  cover.clear();
  for (int p : S.best) cover.push_back(primes[p]);
  std::sort(cover.begin(), cover.end(),
            [&](const Cube& a, const Cube& b) { return term_key(a, n_vars) < term_key(b, n_vars); });
  *n_literals = S.best_lits;
  *exact = S.exhausted ? 0 : 1;
  return TT_OK;
}

// The gate program of one form (Simplify): a tree of operators written in
// post-order, every gate but the last into a fresh temporary.
struct FormWriter {
  std::vector<tt_gate> g;
  int32_t lit(int digit, bool neg) const { return digit | (neg ? TT_OPD_NEG : 0); }
  int32_t emit(int op, int32_t a, int32_t b) {
    const int32_t t = (int32_t)g.size();
    g.push_back({op, a, b, t});
    return t | TT_OPD_TEMP;
  }
  // a chain op(op(op(x0, x1), x2), ...) over operands already written
  int32_t chain(int op, const std::vector<int32_t>& xs) {
    int32_t acc = xs[0];
    for (size_t i = 1; i < xs.size(); ++i) acc = emit(op, acc, xs[i]);
    return acc;
  }
  void finish(int32_t root) {
    if (g.empty() || root != (((int32_t)g.size() - 1) | TT_OPD_TEMP))
      g.push_back({TT_GATE_COPY, root, 0, 0});  // a lone literal: a buffer or NOT
    g.back().dst = -1;
  }
};

}  // namespace

extern "C" {

int tt_sop_minimize(const uint64_t* h_plane, int n_vars, long node_budget, int max_terms, uint32_t* h_care,
                    uint32_t* h_value, int* n_terms, int* n_literals, int* exact) {
  if (!h_plane || n_vars < 0 || n_vars > 12 || max_terms < 0 || !n_terms || !n_literals || !exact) return TT_EINVAL;
  if (max_terms > 0 && (!h_care || !h_value)) return TT_EINVAL;
  std::vector<Cube> cover;
  const int st = minimize(h_plane, n_vars, node_budget, cover, n_literals, exact);
  if (st != TT_OK) return st;
  *n_terms = (int)cover.size();
  for (int t = 0; t < (int)cover.size() && t < max_terms; ++t) {
    h_care[t] = cover[t].care;
    h_value[t] = cover[t].value;
  }
  return TT_OK;
}

int tt_simplify(const uint64_t* h_table, int n_vars, int max_gates, tt_gate* h_gates, int* n_gates, int* exact) {
  if (!h_table || n_vars < 0 || n_vars > 12 || max_gates < 0 || !n_gates || !exact) return TT_EINVAL;
  if (max_gates > 0 && !h_gates) return TT_EINVAL;
  const uint32_t rows = 1u << n_vars;
  auto bit = [&](uint32_t r) { return (int)((h_table[r >> 6] >> (r & 63)) & 1ull); };
  // the support: digits some pair of rows differing only there tells apart
  std::vector<int> S;
  for (int j = 0; j < n_vars; ++j) {
    bool dep = false;
    for (uint32_t r = 0; r < rows && !dep; ++r) dep = bit(r) != bit(r ^ (1u << j));
    if (dep) S.push_back(j);
  }
  // the table restricted to its support (other digits at 0)
  const int k = (int)S.size();
  std::vector<uint64_t> t(((1u << k) + 63) / 64, 0);
  bool parity = k >= 2, coparity = k >= 2;
  for (uint32_t r = 0; r < (1u << k); ++r) {
    uint32_t row = 0;
    for (int i = 0; i < k; ++i) row |= ((r >> i) & 1u) << S[i];
    const int v = bit(row), odd = popc(r) & 1;
    t[r >> 6] |= (uint64_t)v << (r & 63);
    parity = parity && v == odd;
    coparity = coparity && v != odd;
  }
  FormWriter w;
  *exact = 1;
  if (k == 0) {
    w.g.push_back({TT_GATE_CONST, bit(0), 0, -1});
  } else if (parity || coparity) {  // XOR chained in ascending digit, XNOR last for the complement
    int32_t acc = w.lit(S[0], false);
    for (int i = 1; i < k; ++i) acc = w.emit(i == k - 1 && coparity ? TT_GATE_XNOR : TT_GATE_XOR, acc, w.lit(S[i], false));
    w.finish(acc);
  } else {
    std::vector<Cube> cover;
    int lits = 0;
    const int st = minimize(t.data(), k, 0, cover, &lits, exact);
    if (st != TT_OK) return st;
    std::vector<int32_t> terms;
    for (const Cube& c : cover) {  // each term an AND chain of its literals, ascending digit
      std::vector<int32_t> ls;
      for (int i = 0; i < k; ++i)
        if ((c.care >> i) & 1u) ls.push_back(w.lit(S[i], !((c.value >> i) & 1u)));
      terms.push_back(w.chain(TT_GATE_AND, ls));
    }
    w.finish(w.chain(TT_GATE_OR, terms));
  }
  *n_gates = (int)w.g.size();
  if (*n_gates > max_gates) return TT_ERANGE;
  std::memcpy(h_gates, w.g.data(), sizeof(tt_gate) * w.g.size());
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
