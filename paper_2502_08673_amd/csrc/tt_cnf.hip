// tt_cnf.hip -- the CNF-to-circuit transformation (Section "Transformation
// Algorithm", Algorithm 1) on packed truth tables, one wave per CNF instance
// (gfx950).
//
// A wave walks its instance's clauses in order, growing the sub-clause list
// SC (a contiguous clause range, since SC is emptied whenever an expression
// is found).  After each clause it tries the variables of SC that are
// neither primary inputs nor intermediate, in decreasing index: lane w
// builds word w (rows 64w .. 64w + 63) of f (the conjunction of the clauses
// holding -v, that literal removed) and of g (the same for +v) over the
// other variables of SC, ascending index = ascending row digit, straight
// from literal bit patterns; the complement test is an XOR per word and one
// ballot.  A found expression is written with its table and its support
// (digit j is in the support when some pair of rows differing in digit j
// differs: a shifted XOR inside a word for j < 6, a lane exchange for
// j >= 6).  An SC with no output whose variables occur in no later clause
// becomes an auxiliary output constrained to 1 (the conjunction of SC).
#include "tt_internal.h"

namespace tt {

namespace {

constexpr uint8_t kClsPI = 1, kClsIV = 2, kClsPO = 4;

// rows whose digit j is 1, for j < 6 (inside one 64-row word)
__device__ __forceinline__ uint64_t digit_pattern(int j) {
  switch (j) {
    case 0: return 0xAAAAAAAAAAAAAAAAull;
    case 1: return 0xCCCCCCCCCCCCCCCCull;
    case 2: return 0xF0F0F0F0F0F0F0F0ull;
    case 3: return 0xFF00FF00FF00FF00ull;
    case 4: return 0xFFFF0000FFFF0000ull;
    default: return 0xFFFFFFFF00000000ull;
  }
}

// word w of the literal on digit j (negated when neg)
__device__ __forceinline__ uint64_t literal_word(int j, int w, bool neg) {
  const uint64_t p = j < 6 ? digit_pattern(j) : (((w >> (j - 6)) & 1) ? ~0ull : 0ull);
  return neg ? ~p : p;
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

// Support over k digits of a table held as words (lane w < W holds word w,
// valid = the rows that exist in a one-word table).
__device__ uint32_t table_support(uint64_t t, int k, int W, uint64_t valid) {
  const int lane = threadIdx.x;
  uint32_t sup = 0;
  for (int j = 0; j < k; ++j) {
    bool d;
    if (j < 6) {
      const int s = 1 << j;
      d = lane < W && (((t ^ (t >> s)) & ~digit_pattern(j) & valid) != 0);
    } else {
      const uint64_t o = shfl_xor64(t, 1 << (j - 6));
      d = lane < W && t != o;
    }
    if (__ballot(d) != 0) sup |= 1u << j;
  }
  return sup;
}

}  // namespace

// STAGED: the instance's clause offsets, literals and clause reaches are
// copied into LDS first (every later read is an LDS read), when the largest
// instance of the batch fits; else they are read from global memory.
template <bool STAGED>
__global__ __launch_bounds__(64) void cnf_transform_kernel(CnfArgs a) {
  extern __shared__ int32_t smem[];  // [staged clause offsets, reaches, literals] then the class bytes
  const int inst = a.order[blockIdx.x], lane = threadIdx.x;  // longest instances first
  const int nvar = a.n_vars[inst];
  const int c0 = a.inst_off[inst], nc = a.inst_off[inst + 1] - c0;
  const int32_t* coff;   // clause c of the instance: literals lits[coff[c] .. coff[c + 1] - 1]
  const int32_t* lits;
  const int32_t* creach;
  uint8_t* cls;          // variable classes of this instance, [n_vars + 1]
  if constexpr (STAGED) {
    int32_t* so = smem;
    int32_t* sr = so + a.stage_clauses + 1;
    int32_t* sl = sr + a.stage_clauses;
    const int l0 = a.clause_off[c0], nl = a.clause_off[c0 + nc] - l0;
    for (int c = lane; c <= nc; c += 64) so[c] = a.clause_off[c0 + c] - l0;
    for (int c = lane; c < nc; c += 64) sr[c] = a.clause_reach[c0 + c];
    for (int q = lane; q < nl; q += 64) sl[q] = a.lits[l0 + q];
    coff = so;
    creach = sr;
    lits = sl;
    cls = reinterpret_cast<uint8_t*>(sl + a.stage_lits);
  } else {
    coff = a.clause_off + c0;
    creach = a.clause_reach + c0;
    lits = a.lits;
    cls = reinterpret_cast<uint8_t*>(smem);
  }
  for (int x = lane; x <= nvar; x += 64) cls[x] = 0;
  __syncthreads();
  // SC's variables, ascending, one per lane: lane q holds the q-th (lanes at
  // or past nsc hold INT_MAX), so finding a variable's place is one ballot
  int my = INT_MAX, nsc = 0;
  // with each variable, what SC says of it: bit 0 it occurs as +v, bit 1 as
  // -v, bit 2 in a clause of its own, bit 3 in two clauses or more (bit 4:
  // in an earlier clause, bit 5: in the current one).  A variable that
  // occurs with one sign only, in a single clause with other literals, is
  // never SC's output: f (or g) is then true and the other is that clause
  // without v, which some row satisfies.  Such variables are skipped
  // without a walk.
  int occ = 0;
  int start = 0, nexpr = 0, status = 0, reach = -1;
  for (int i = 0; i < nc; ++i) {
    reach = max(reach, creach[i]);
    const bool unit = coff[i + 1] - coff[i] == 1;
    for (int p = coff[i]; p < coff[i + 1]; ++p) {  // merge the clause's variables
      const int L = lits[p], x = abs(L);
      if (__ballot(my == x) == 0) {
        const int pos = __popcll(__ballot(my < x));
        const int up = __shfl_up(my, 1), occ_up = __shfl_up(occ, 1);
        my = lane < pos ? my : (lane == pos ? x : up);
        occ = lane < pos ? occ : (lane == pos ? 0 : occ_up);
        ++nsc;
      }
      if (my == x) occ |= (L > 0 ? 1 : 2) | (unit ? 4 : 0) | 32;
    }
    if (occ & 32) occ = ((occ & 16) ? occ | 8 : occ | 16) & ~32;
    if (nsc > kCnfMaxVars) {
      status = 1;
      break;
    }
    bool found = false;
    for (int ci = nsc - 1; ci >= 0 && !found; --ci) {
      const int v = __shfl(my, ci);
      if (cls[v] & (kClsPI | kClsIV)) continue;
      const int ov = __shfl(occ, ci);
      if ((ov & 3) != 3 && !(ov & 12)) continue;
      const int k = nsc - 1;
      const int W = k > 6 ? 1 << (k - 6) : 1;
      const uint64_t valid = k >= 6 ? ~0ull : ((1ull << (1u << k)) - 1ull);
      // every lane runs the clause walk (the slot lookups are ballots); lanes
      // at or past W build words that are never used
      uint64_t f = ~0ull, g = ~0ull;
      for (int c = start; c <= i; ++c) {
        bool negv = false, posv = false;
        uint64_t word = 0;
        for (int p = coff[c]; p < coff[c + 1]; ++p) {
          const int L = lits[p], x = abs(L);
          if (x == v) {
            negv = negv || L < 0;
            posv = posv || L > 0;
            continue;
          }
          const int q = __ffsll((unsigned long long)__ballot(my == x)) - 1;
          word |= literal_word(q > ci ? q - 1 : q, lane, L < 0);
        }
        if (negv) f &= word;
        if (posv) g &= word;
      }
      const bool ok = lane >= W || ((f ^ g) & valid) == valid;
      if (__ballot(!ok) != 0) continue;
      found = true;
      f &= valid;
      const bool all1 = __ballot(lane < W && f != valid) == 0;
      const bool all0 = __ballot(lane < W && f != 0) == 0;
      const uint32_t sup = table_support(f, k, W, valid);
      tt_cnf_expr* e = a.expr + c0 + nexpr;
      e->table[lane] = lane < W ? f : 0ull;
      const int next = __shfl_down(my, 1);
      if (lane < kCnfMaxVars) e->vars[lane] = lane < ci ? my : (lane < k ? next : 0);
      if (lane == 0) {
        e->out = v;
        e->kind = (all1 || all0) ? TT_CNF_PO : TT_CNF_IV;
        e->first = start;
        e->last = i;
        e->n_vars = k;
        e->support = sup;
      }
      // classes: lane ci marks v, the other lanes of SC their own variable
      if (lane == ci) cls[v] |= (all1 || all0) ? kClsPO : kClsIV;
      if (lane < nsc && lane != ci && !(cls[my] & kClsIV)) cls[my] |= kClsPI;
      ++nexpr;
      start = i + 1;
      reach = -1;
      my = INT_MAX;
      occ = 0;
      nsc = 0;
    }
    if (!found && reach <= i) {
      // under-specified: the conjunction of SC over all its variables,
      // an auxiliary output constrained to 1
      const int W = nsc > 6 ? 1 << (nsc - 6) : 1;
      const uint64_t valid = nsc >= 6 ? ~0ull : ((1ull << (1u << nsc)) - 1ull);
      uint64_t t = ~0ull;
      for (int c = start; c <= i; ++c) {
        uint64_t word = 0;
        for (int p = coff[c]; p < coff[c + 1]; ++p) {
          const int L = lits[p];
          const int q = __ffsll((unsigned long long)__ballot(my == abs(L))) - 1;
          word |= literal_word(q, lane, L < 0);
        }
        t &= word;
      }
      t &= valid;
      const uint32_t sup = table_support(t, nsc, W, valid);
      tt_cnf_expr* e = a.expr + c0 + nexpr;
      e->table[lane] = lane < W ? t : 0ull;
      if (lane < kCnfMaxVars) e->vars[lane] = lane < nsc ? my : 0;
      if (lane == 0) {
        e->out = 0;
        e->kind = TT_CNF_AUX;
        e->first = start;
        e->last = i;
        e->n_vars = nsc;
        e->support = sup;
      }
      if (lane < nsc && !(cls[my] & kClsIV)) cls[my] |= kClsPI;
      ++nexpr;
      start = i + 1;
      reach = -1;
      my = INT_MAX;
      occ = 0;
      nsc = 0;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int x = lane; x <= nvar; x += 64) a.var_class[a.var_off[inst] + x] = cls[x];
  if (lane == 0) {
    a.n_expr[inst] = nexpr;
    a.status[inst] = status;
  }
}

hipError_t launch_cnf_transform(const CnfArgs& a, int max_vars, hipStream_t s) {
  if (a.n_inst <= 0) return hipSuccess;
  const size_t cls_bytes = ((size_t)max_vars + 1 + 3) / 4 * 4;
  const size_t staged = 4 * (2 * (size_t)a.stage_clauses + 1 + (size_t)a.stage_lits) + cls_bytes;
  if (staged <= 64 * 1024)
    hipLaunchKernelGGL(cnf_transform_kernel<true>, dim3((unsigned)a.n_inst), dim3(64), staged, s, a);
  else
    hipLaunchKernelGGL(cnf_transform_kernel<false>, dim3((unsigned)a.n_inst), dim3(64), cls_bytes, s, a);
  return hipGetLastError();
}

}  // namespace tt
