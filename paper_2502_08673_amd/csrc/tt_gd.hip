// tt_gd.hip -- gradient-descent sampling of a transformed CNF (the paper's
// probabilistic model: Table 1, the sigmoid embedding, the L2 loss, GD, then
// hardening and the satisfiable / non-redundant filter), one sample per lane
// (gfx950).
//
// Every expression of the circuit comes as its simplified form, a short
// program of Table 1's operators (AND, OR, XOR, XNOR over operands that may
// be negated, NOT being 1 - p), so the probabilistic value of an expression
// is the composition of its gates, as in the paper's generated module.  The
// forward pass runs the intermediate expressions in order; the loss terms
// (auxiliary outputs constrained to 1, constants on primary inputs) seed the
// adjoints; the backward pass walks the intermediate expressions in reverse,
// recomputing each one's temporaries and applying Table 1's derivatives
// gate by gate in reverse (a variable read twice collects both reads).
// A wave keeps its 64 samples' probabilities and adjoints as [slot][lane]
// (one bank per lane) in LDS, or for larger circuits in its own block of a
// global workspace; the gate program and the clauses are wave-uniform and
// read with scalar loads.  Hardening runs the same gates on 0/1 values,
// where Table 1's operators are exactly the Boolean gates.
#include "tt_gd.h"

namespace tt {

namespace {

struct Lane {
  float* P;    // [variable slots][64] probabilities
  float* Gr;   // [variable slots][64] adjoints
  float* Pt;   // [temporaries][64] probabilities of the current form's temporaries (LDS)
  float* Grt;  // [temporaries][64] their adjoints (LDS)
  long col;
  int32_t nv;  // variable slots; slot nv + t is temporary t

  // a slot's cells (the branch is wave-uniform: slots come from the gate records)
  __device__ __forceinline__ float* p_at(int32_t slot) const {
    return slot >= nv ? Pt + (slot - nv) * 64L + col : P + slot * 64L + col;
  }
  __device__ __forceinline__ float* g_at(int32_t slot) const {
    return slot >= nv ? Grt + (slot - nv) * 64L + col : Gr + slot * 64L + col;
  }
  __device__ __forceinline__ float val(int32_t o) const {
    const float v = *p_at(o & kGdSlot);
    return (o & kGdNeg) ? 1.f - v : v;
  }
  // Table 1: the operator's value at (x, y)
  __device__ __forceinline__ void forward(const GdGate& g) const {
    float z;
    if (g.op == TT_GATE_CONST) {
      z = (float)g.a;
    } else {
      const float x = val(g.a);
      if (g.op == TT_GATE_COPY) {
        z = x;
      } else {
        const float y = val(g.b);
        if (g.op == TT_GATE_AND)
          z = x * y;
        else if (g.op == TT_GATE_OR)
          z = 1.f - (1.f - x) * (1.f - y);
        else if (g.op == TT_GATE_XOR)
          z = (1.f - x) * y + x * (1.f - y);
        else
          z = x * y + (1.f - x) * (1.f - y);
      }
    }
    *p_at(g.dst) = z;
  }
  // adds c to an operand's adjoint (a temporary is read by one gate only,
  // so its adjoint is set); a negated operand takes -c
  __device__ __forceinline__ void give(int32_t o, float c) const {
    float* q = g_at(o & kGdSlot);
    if (o & kGdNeg) c = -c;
    *q = (o & kGdTemp) ? c : *q + c;
  }
  // Table 1's derivatives times the gate's adjoint, to its operands
  __device__ __forceinline__ void backward(const GdGate& g) const {
    if (g.op == TT_GATE_CONST) return;
    const float adj = *g_at(g.dst);
    if (g.op == TT_GATE_COPY) {
      give(g.a, adj);
      return;
    }
    const float x = val(g.a), y = val(g.b);
    float dx, dy;
    if (g.op == TT_GATE_AND) {
      dx = y;
      dy = x;
    } else if (g.op == TT_GATE_OR) {
      dx = 1.f - y;
      dy = 1.f - x;
    } else if (g.op == TT_GATE_XOR) {
      dx = 1.f - 2.f * y;
      dy = 1.f - 2.f * x;
    } else {
      dx = 2.f * y - 1.f;
      dy = 2.f * x - 1.f;
    }
    give(g.a, adj * dx);
    give(g.b, adj * dy);
  }
};

}  // namespace

// GLOBAL: the variables' probabilities and adjoints and the logits in a
// global workspace, each wave's own contiguous [2 n_vslots + n_pi][64] block
// (a few pages per wave, where one column per sample across the whole batch
// would spread a wave's accesses over a page per slot), and the forms'
// temporaries in LDS: a temporary lives inside one form, and on this
// hardware a global load also waits for the wave's earlier stores, so
// keeping the temporaries out of global memory removes most of those waits.
// For circuits whose slots all fit a wave's LDS, the whole
// [2][n_slots][64] block is in LDS.
template <bool GLOBAL>
__global__ __launch_bounds__(64) void gd_sample_kernel(GdArgs a) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x;
  const long s = (long)blockIdx.x * 64 + lane;
  const bool live = s < a.batch;
  const long col = lane;  // this sample's column
  const int nv = a.n_vslots, nt = a.n_slots - a.n_vslots;
  const int blk = 2 * nv + a.n_pi + (a.temps_lds ? 0 : 2 * nt);  // global block rows
  float* P = GLOBAL ? a.state + (size_t)blockIdx.x * blk * 64 : lds;
  float* Gr = GLOBAL ? P + nv * 64L : P + a.n_slots * 64L;
  float* Pt = !GLOBAL ? P + nv * 64L : a.temps_lds ? lds : P + (2 * nv + a.n_pi) * 64L;
  const Lane L{P, Gr, Pt, !GLOBAL ? Gr + nv * 64L : Pt + nt * 64L, col, nv};
  // the logits: in the global form a [n_pi][64] part of the wave's block
  // (copied from and back to the caller's rows), in the LDS form the
  // caller's rows themselves (a lane reads and updates its own), which
  // leaves the LDS to the probabilities and adjoints
  float* Vr = a.V + (live ? s : 0) * a.n_pi;
  float* Vp = GLOBAL ? Gr + nv * 64L + col : Vr;
  constexpr long VS = GLOBAL ? 64 : 1;
  if (GLOBAL)
    for (int q = 0; q < a.n_pi; ++q) Vp[q * VS] = live ? Vr[q] : 0.f;
  for (int q = a.n_pi; q < a.n_vslots; ++q) P[q * 64L + col] = a.slot_const[q];  // constants; others overwritten
  for (int it = 0; it < a.iters; ++it) {
    for (int q = 0; q < a.n_pi; ++q) P[q * 64L + col] = 1.f / (1.f + __expf(-(live ? Vp[q * VS] : 0.f)));
    for (int q = 0; q < a.n_vslots; ++q) L.Gr[q * 64L + col] = 0.f;
    // forward through the intermediate variables
    for (int g = 0; g < a.iv_rng[a.n_iv]; ++g) L.forward(a.gate[g]);
    // loss: an auxiliary output's form must be 1, a constant on a primary
    // input its constant; the adjoint 2 (P - target) goes back through the
    // auxiliary output's gates at once
    for (int x = 0; x < a.n_aux; ++x) {
      const int g0 = a.aux_rng[x], g1 = a.aux_rng[x + 1];
      for (int g = g0; g < g1; ++g) L.forward(a.gate[g]);
      const int32_t out = a.gate[g1 - 1].dst;
      *L.g_at(out) = 2.f * (*L.p_at(out) - 1.f);
      for (int g = g1 - 1; g >= g0; --g) L.backward(a.gate[g]);
    }
    for (int x = 0; x < a.n_po; ++x) {
      const int32_t q = a.po[2 * x];
      L.Gr[q * 64L + col] += 2.f * (P[q * 64L + col] - (float)a.po[2 * x + 1]);
    }
    // chain rule back through the intermediate variables, last first: the
    // expression's temporaries again, then its gates in reverse
    for (int x = a.n_iv - 1; x >= 0; --x) {
      const int g0 = a.iv_rng[x], g1 = a.iv_rng[x + 1];
      for (int g = g0; g < g1 - 1; ++g) L.forward(a.gate[g]);
      for (int g = g1 - 1; g >= g0; --g) L.backward(a.gate[g]);
    }
    for (int q = 0; q < a.n_pi && live; ++q) {
      const float pq = P[q * 64L + col];
      Vp[q * VS] -= a.lr * L.Gr[q * 64L + col] * pq * (1.f - pq);
    }
  }
  // harden: primary inputs from the logits' signs, the intermediate
  // variables through their gates on 0/1 values; check every clause
  if (GLOBAL && live)
    for (int q = 0; q < a.n_pi; ++q) Vr[q] = Vp[q * VS];
  for (int q = 0; q < a.n_pi; ++q) P[q * 64L + col] = live && Vp[q * VS] > 0.f ? 1.f : 0.f;
  for (int q = a.n_pi; q < a.n_vslots; ++q) P[q * 64L + col] = a.slot_const[q];
  for (int g = 0; g < a.iv_rng[a.n_iv]; ++g) L.forward(a.gate[g]);
  bool ok = true;
  for (int c = 0; c < a.n_clauses; ++c) {
    bool sat = false;
    for (int q = a.clause_off[c]; q < a.clause_off[c + 1]; ++q) {
      const int lit = a.lits[q];
      sat = sat || ((P[(lit >> 1) * 64L + col] > 0.5f) != (bool)(lit & 1));
    }
    ok = ok && sat;
  }
  if (!live) return;
  a.valid[s] = ok ? 1 : 0;
  for (int w = 0; w < a.words; ++w) {
    uint64_t bits = 0;
    for (int b = 0; b < 64 && 64 * w + b < a.n_pi; ++b)
      bits |= (uint64_t)(P[(64 * w + b) * 64L + col] > 0.5f) << b;
    a.sol[s * a.words + w] = bits;
  }
}

// Distinct solutions.  Nearly every sample of a batch has a solution of its
// own, so claiming places by compare-and-swap costs one device-scope atomic
// per sample.  Instead each valid sample first stores its index at its
// solution's place in a large table (a plain store: one of the writers
// stays), and reads the place back: the sample found there is the first of
// its solution when the two solutions are equal (only that sample sees
// itself), and a different solution there means a hash collision -- those
// samples, about one in sixteen, take the open-addressing table (capacity a
// power of two at least twice the batch, so every probe sequence ends),
// where a place is claimed with one compare-and-swap and a taken place is
// compared word by word.  Every place read back was written in this call by
// a valid sample, so the large table is never cleared.  The count of first
// samples is added once per block of a grid of at most 1024 blocks.
__device__ __forceinline__ uint64_t solution_hash(const uint64_t* sol, int words, long s) {
  uint64_t h = kGdHashSeed;
  for (int w = 0; w < words; ++w) {
    h ^= sol[s * words + w];
    h *= kGdHashMul;
    h ^= h >> 31;
  }
  return h;
}

__device__ __forceinline__ bool same_solution(const uint64_t* sol, int words, long a, long b) {
  bool same = true;
  for (int w = 0; w < words && same; ++w) same = sol[a * words + w] == sol[b * words + w];
  return same;
}

__global__ __launch_bounds__(256) void gd_unique_place_kernel(const uint8_t* valid, const uint64_t* sol, int words,
                                                              int batch, int32_t* primary, uint32_t pmask) {
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch || !valid[s]) return;
  primary[(uint32_t)solution_hash(sol, words, s) & pmask] = (int32_t)s;
}

__global__ __launch_bounds__(256) void gd_unique_kernel(const uint8_t* valid, const uint64_t* sol, int words,
                                                        int batch, const int32_t* primary, uint32_t pmask,
                                                        int32_t* table, uint32_t cap_mask, uint8_t* first,
                                                        uint32_t* count) {
  __shared__ uint32_t s_firsts[4];
  uint32_t firsts = 0;
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < batch; s += (long)gridDim.x * blockDim.x) {
    bool is_first = false;
    if (valid[s]) {
      const uint64_t h = solution_hash(sol, words, s);
      const int32_t w = primary[(uint32_t)h & pmask];
      if (w == (int32_t)s || same_solution(sol, words, w, s)) {
        is_first = w == (int32_t)s;
      } else {
        // another solution holds the place: the other half of the hash
        // picks the open-addressing place; the loop always ends by a claim
        // or a match (the table has more places than samples)
        uint32_t at = (uint32_t)(h >> 32) & cap_mask;
        for (uint32_t probe = 0; probe <= cap_mask; ++probe) {
          const int32_t cur = atomicCAS(&table[at], -1, (int32_t)s);
          if (cur == -1) {
            is_first = true;
            break;
          }
          if (same_solution(sol, words, cur, s)) break;
          at = (at + 1) & cap_mask;
        }
      }
    }
    first[s] = is_first ? 1 : 0;
    firsts += is_first ? 1u : 0u;
  }
  // one add per block: adds to one address from every wave of a large grid
  // serialise (about 12 ns each here)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) firsts += (uint32_t)__shfl_xor((int)firsts, off, 64);
  if ((threadIdx.x & 63) == 0) s_firsts[threadIdx.x >> 6] = firsts;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t total = s_firsts[0] + s_firsts[1] + s_firsts[2] + s_firsts[3];
    if (total) atomicAdd(count, total);
  }
}

uint32_t gd_unique_primary_places(int batch) {
  // about sixteen places per sample: a place is taken by another solution
  // for about one sample in sixteen
  uint32_t cap = 1024;
  while ((uint64_t)cap < 16ull * (uint64_t)batch && cap < (1u << 24)) cap <<= 1;
  return cap;
}

__global__ void fill_i32_kernel(int32_t* p, long n, int32_t v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_gd_sample(const GdArgs& a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.batch + 63) / 64));
  // LDS: the temporaries (global state, if they fit) or the whole state
  const size_t lds = !a.state ? (size_t)(2 * a.n_slots) * 64 * sizeof(float)
                              : a.temps_lds ? (size_t)(2 * (a.n_slots - a.n_vslots)) * 64 * sizeof(float) : 0;
  if (a.state)
    hipLaunchKernelGGL((gd_sample_kernel<true>), grid, dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((gd_sample_kernel<false>), grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_gd_unique_placed(const uint8_t* valid, const uint64_t* sol, int words, int batch,
                                   const int32_t* primary, uint32_t primary_places, int32_t* table, uint32_t cap,
                                   uint8_t* first, uint32_t* count, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  // a grid of at most 1024 blocks (one count add each), samples in a stride loop
  const unsigned blocks = (unsigned)std::min<long>(((long)batch + 255) / 256, 1024);
  hipLaunchKernelGGL(gd_unique_kernel, dim3(blocks), dim3(256), 0, s, valid, sol, words, batch, primary,
                     primary_places - 1, table, cap - 1, first, count);
  return hipGetLastError();
}

hipError_t launch_gd_unique(const uint8_t* valid, const uint64_t* sol, int words, int batch, int32_t* primary,
                            int32_t* table, uint32_t cap, uint8_t* first, uint32_t* count, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const uint32_t pcap = gd_unique_primary_places(batch);
  const dim3 grid((unsigned)((batch + 255) / 256));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(std::min<uint32_t>(4096, (cap + 255) / 256)), dim3(256), 0, s, table,
                     (long)cap, -1);
  hipLaunchKernelGGL(gd_unique_place_kernel, grid, dim3(256), 0, s, valid, sol, words, batch, primary, pcap - 1);
  return launch_gd_unique_placed(valid, sol, words, batch, primary, pcap, table, cap, first, count, s);
}

}  // namespace tt
