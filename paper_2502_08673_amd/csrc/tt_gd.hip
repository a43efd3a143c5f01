// tt_gd.hip -- gradient-descent sampling of a transformed CNF (the paper's
// probabilistic model: Table 1, the sigmoid embedding, the L2 loss, GD, then
// hardening and the satisfiable / non-redundant filter), one sample per lane
// (gfx950).
//
// Every expression of the circuit is a truth table over at most twelve
// variables; its probabilistic value is the table's multilinear extension
// (the probability that it outputs 1 for independent inputs).  Up to six
// inputs it is built by contracting the 2^k table bits one digit at a time,
// and its derivative in input j is the extension with p_j = 1 minus the one
// with p_j = 0; wider tables sum products over their rows.  A wave
// keeps its 64 samples' probabilities and adjoints in LDS as [slot][lane]
// (one bank per lane; the LDS this takes per wave bounds the waves per CU);
// the program (expressions, clauses) is wave-uniform and read with scalar
// loads.  Circuits with more variables keep the same arrays in a global
// workspace, one column per sample.
#include "tt_internal.h"

namespace tt {

namespace {

template <int K>
__device__ __forceinline__ float mlext(uint64_t t, const float* p) {
  float v[1 << K];
#pragma unroll
  for (int r = 0; r < (1 << K); ++r) v[r] = (float)((t >> r) & 1ull);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int half = 1 << (K - 1 - j);
#pragma unroll
    for (int r = 0; r < half; ++r) v[r] = v[2 * r] * (1.f - p[j]) + v[2 * r + 1] * p[j];
  }
  return v[0];
}

// value and derivatives of a K-input table at p
template <int K>
__device__ __forceinline__ float mlext_grad(uint64_t t, const float* p, float* d) {
  float q[6];
#pragma unroll
  for (int j = 0; j < K; ++j) q[j] = p[j];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    q[j] = 1.f;
    const float hi = mlext<K>(t, q);
    q[j] = 0.f;
    const float lo = mlext<K>(t, q);
    q[j] = p[j];
    d[j] = hi - lo;
  }
  return mlext<K>(t, q);
}

// Tables over 7 to 12 inputs: a sum over the rows that carry a 1 of the
// product of the inputs' probabilities, derivatives from prefix and suffix
// products (no division, so inputs at exactly 0 or 1 are fine).
__device__ float ext_wide(int k, const uint64_t* tab, const float* p, float* d, bool grad) {
  float P = 0.f;
#pragma unroll
  for (int j = 0; j < 12; ++j) d[j] = 0.f;
  for (int r = 0; r < (1 << k); ++r) {
    if (!((tab[r >> 6] >> (r & 63)) & 1ull)) continue;
    float pre[13];
    pre[0] = 1.f;
#pragma unroll
    for (int j = 0; j < 12; ++j) pre[j + 1] = j < k ? pre[j] * (((r >> j) & 1) ? p[j] : 1.f - p[j]) : pre[j];
    P += pre[12];
    if (grad) {
      float suf = 1.f;
#pragma unroll
      for (int j = 11; j >= 0; --j) {
        if (j < k) {
          const bool one = (r >> j) & 1;
          d[j] += (one ? 1.f : -1.f) * pre[j] * suf;
          suf *= one ? p[j] : 1.f - p[j];
        }
      }
    }
  }
  return P;
}

__device__ __forceinline__ float ext_dispatch(int k, uint64_t t, const float* p, float* d, bool grad) {
  switch (k) {
    case 0: return (float)(t & 1ull);
    case 1: return grad ? mlext_grad<1>(t, p, d) : mlext<1>(t, p);
    case 2: return grad ? mlext_grad<2>(t, p, d) : mlext<2>(t, p);
    case 3: return grad ? mlext_grad<3>(t, p, d) : mlext<3>(t, p);
    case 4: return grad ? mlext_grad<4>(t, p, d) : mlext<4>(t, p);
    case 5: return grad ? mlext_grad<5>(t, p, d) : mlext<5>(t, p);
    default: return grad ? mlext_grad<6>(t, p, d) : mlext<6>(t, p);
  }
}

}  // namespace

// GLOBAL: probabilities, adjoints and logits in a global workspace, each
// wave's own contiguous [2 n_slots + n_pi][64] block (a few pages per wave, where one
// column per sample across the whole batch would spread a wave's accesses
// over a page per slot), for circuits whose variables do not fit a wave's
// LDS; else the same block in LDS.
template <bool GLOBAL, bool WIDE>
__global__ __launch_bounds__(64) void gd_sample_kernel(GdArgs a) {
  constexpr int KM = WIDE ? 12 : 6;  // most inputs of an expression
  extern __shared__ float lds[];
  const int lane = threadIdx.x;
  const long s = (long)blockIdx.x * 64 + lane;
  const bool live = s < a.batch;
  constexpr long RS = 64;  // row stride of a slot
  const long col = lane;   // this sample's column
  float* P = GLOBAL ? a.state + (size_t)blockIdx.x * (2 * a.n_slots + a.n_pi) * 64 : lds;  // [n_slots][64]
  float* Gr = P + a.n_slots * RS;                                                         // [n_slots][64]
  // the logits: in the global form a [n_pi][64] part of the wave's block
  // (copied from and back to the caller's rows), in the LDS form the
  // caller's rows themselves (a lane reads and updates its own), which
  // leaves the LDS to the probabilities and adjoints
  float* Vr = a.V + (live ? s : 0) * a.n_pi;
  float* Vp = GLOBAL ? Gr + a.n_slots * RS + col : Vr;
  constexpr long VS = GLOBAL ? 64 : 1;
  if (GLOBAL)
    for (int q = 0; q < a.n_pi; ++q) Vp[q * VS] = live ? Vr[q] : 0.f;
  for (int q = a.n_pi; q < a.n_slots; ++q) P[q * RS + col] = a.slot_const[q];  // constants; others overwritten
  float pin[12], d[12];  // entries KM .. 11 unused
  for (int it = 0; it < a.iters; ++it) {
    for (int q = 0; q < a.n_pi; ++q) P[q * RS + col] = 1.f / (1.f + __expf(-(live ? Vp[q * VS] : 0.f)));
    for (int q = 0; q < a.n_slots; ++q) Gr[q * RS + col] = 0.f;
    // forward through the intermediate variables; loss adjoints of the
    // constrained outputs
    for (int x = 0; x < a.n_expr; ++x) {
      const GdExpr e = a.expr[x];
#pragma unroll
      for (int j = 0; j < KM; ++j) pin[j] = j < e.k ? P[e.in[j] * RS + col] : 0.f;
      if (e.kind == TT_CNF_IV) {
        P[e.out * RS + col] = WIDE && e.k > 6 ? ext_wide(e.k, a.wide_tab + 64 * e.wide, pin, d, false)
                                              : ext_dispatch(e.k, e.table, pin, d, false);
      } else if (e.kind == TT_CNF_AUX) {
        const float y = WIDE && e.k > 6 ? ext_wide(e.k, a.wide_tab + 64 * e.wide, pin, d, true)
                                        : ext_dispatch(e.k, e.table, pin, d, true);
#pragma unroll
        for (int j = 0; j < KM; ++j)
          if (j < e.k) Gr[e.in[j] * RS + col] += 2.f * (y - 1.f) * d[j];
      } else if (e.out < a.n_pi) {  // a constant expression on a primary input
        Gr[e.out * RS + col] += 2.f * (P[e.out * RS + col] - (float)(e.table & 1ull));
      }
    }
    // chain rule back through the intermediate variables
    for (int x = a.n_expr - 1; x >= 0; --x) {
      const GdExpr e = a.expr[x];
      if (e.kind != TT_CNF_IV || e.k == 0) continue;
#pragma unroll
      for (int j = 0; j < KM; ++j) pin[j] = j < e.k ? P[e.in[j] * RS + col] : 0.f;
      if (WIDE && e.k > 6)
        (void)ext_wide(e.k, a.wide_tab + 64 * e.wide, pin, d, true);
      else
        (void)ext_dispatch(e.k, e.table, pin, d, true);
      const float go = Gr[e.out * RS + col];
#pragma unroll
      for (int j = 0; j < KM; ++j)
        if (j < e.k) Gr[e.in[j] * RS + col] += go * d[j];
    }
    for (int q = 0; q < a.n_pi && live; ++q) {
      const float pq = P[q * RS + col];
      Vp[q * VS] -= a.lr * Gr[q * RS + col] * pq * (1.f - pq);
    }
  }
  // harden (P now holds 0/1), check every clause, write the solution
  if (GLOBAL && live)
    for (int q = 0; q < a.n_pi; ++q) Vr[q] = Vp[q * VS];
  for (int q = 0; q < a.n_pi; ++q) P[q * RS + col] = live && Vp[q * VS] > 0.f ? 1.f : 0.f;
  for (int q = a.n_pi; q < a.n_slots; ++q) P[q * RS + col] = a.slot_const[q];
  for (int x = 0; x < a.n_expr; ++x) {
    const GdExpr e = a.expr[x];
    if (e.kind != TT_CNF_IV) continue;
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < e.k) r |= (P[e.in[j] * RS + col] > 0.5f ? 1u : 0u) << j;
    const uint64_t word = WIDE && e.k > 6 ? a.wide_tab[64 * e.wide + (r >> 6)] : e.table;
    P[e.out * RS + col] = (float)((word >> (r & 63)) & 1ull);
  }
  bool ok = true;
  for (int c = 0; c < a.n_clauses; ++c) {
    bool sat = false;
    for (int q = a.clause_off[c]; q < a.clause_off[c + 1]; ++q) {
      const int L = a.lits[q];
      sat = sat || ((P[(L >> 1) * RS + col] > 0.5f) != (bool)(L & 1));
    }
    ok = ok && sat;
  }
  if (!live) return;
  a.valid[s] = ok ? 1 : 0;
  for (int w = 0; w < a.words; ++w) {
    uint64_t bits = 0;
    for (int b = 0; b < 64 && 64 * w + b < a.n_pi; ++b)
      bits |= (uint64_t)(P[(64 * w + b) * RS + col] > 0.5f) << b;
    a.sol[s * a.words + w] = bits;
  }
}

// Distinct solutions: open addressing on sample indices (capacity a power
// of two at least twice the batch, so every probe sequence ends); a sample's
// place is claimed with one compare-and-swap and a taken place is compared
// word by word.
__global__ __launch_bounds__(256) void gd_unique_kernel(const uint8_t* valid, const uint64_t* sol, int words,
                                                        int batch, int32_t* table, uint32_t cap_mask,
                                                        uint8_t* first, uint32_t* count) {
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  if (!valid[s]) {
    first[s] = 0;
    return;
  }
  uint64_t h = 0x9E3779B97F4A7C15ull;
  for (int w = 0; w < words; ++w) {
    h ^= sol[s * words + w];
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  uint32_t at = (uint32_t)h & cap_mask;
  for (uint32_t probe = 0; probe <= cap_mask; ++probe) {
    const int32_t cur = atomicCAS(&table[at], -1, (int32_t)s);
    if (cur == -1) {
      first[s] = 1;
      atomicAdd(count, 1u);
      return;
    }
    bool same = true;
    for (int w = 0; w < words && same; ++w) same = sol[(long)cur * words + w] == sol[s * words + w];
    if (same) {
      first[s] = 0;
      return;
    }
    at = (at + 1) & cap_mask;
  }
  first[s] = 0;  // not reached: the table has more places than samples
}

__global__ void fill_i32_kernel(int32_t* p, long n, int32_t v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_gd_sample(const GdArgs& a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.batch + 63) / 64));
  const size_t lds = a.state ? 0 : (size_t)(2 * a.n_slots) * 64 * sizeof(float);
  if (a.state && a.has_wide)
    hipLaunchKernelGGL((gd_sample_kernel<true, true>), grid, dim3(64), 0, s, a);
  else if (a.state)
    hipLaunchKernelGGL((gd_sample_kernel<true, false>), grid, dim3(64), 0, s, a);
  else if (a.has_wide)
    hipLaunchKernelGGL((gd_sample_kernel<false, true>), grid, dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((gd_sample_kernel<false, false>), grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_gd_unique(const uint8_t* valid, const uint64_t* sol, int words, int batch, int32_t* table,
                            uint32_t cap, uint8_t* first, uint32_t* count, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(std::min<uint32_t>(4096, (cap + 255) / 256)), dim3(256), 0, s, table,
                     (long)cap, -1);
  hipLaunchKernelGGL(gd_unique_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, valid, sol, words,
                     batch, table, cap - 1, first, count);
  return hipGetLastError();
}

}  // namespace tt
