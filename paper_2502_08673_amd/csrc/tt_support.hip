// tt_support.hip -- input support and code histogram of packed tables, and
// packing of per-row codes into planes (gfx950).
//
// Support.  Input j is in the support iff two rows that differ only in digit
// j carry different codes.  Walking from one digit value to another one bit
// at a time shows that this holds iff flipping some single row bit inside
// digit j changes the code of some row, so the kernels test single-bit flips:
//  - row bits 0..5 (inside a 64-row word): XOR of a plane word with itself
//    shifted by 2^i, restricted to positions whose bit i is 0;
//  - row bits 6+k: word h against word h ^ 2^k.
// A row bit is recorded in found[n] (bit = row bit); a digit is in the
// support iff any of its b row bits is, and a digit is no longer tested once
// one of its bits is found.  Only the tables are read.  (For tables that are
// the enumeration of their descriptors, support_params_kernel below decides
// the support from the parameters instead.)
#include "tt_internal.h"

namespace tt {

__device__ __forceinline__ uint64_t words_per_plane(int Fb) {
  return Fb >= 6 ? (1ull << (Fb - 6)) : 1ull;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}


__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Support from the tables alone (no histogram), in two launches of one
// kernel after the found bits are cleared.  Checks come in two kinds:
//  - near items, up to 512 contiguous words (lane = word bits 0..5, register
//    k = word bits 6..8): in-word row bits and word bits 0..8;
//  - far items, for a digit with row bits from 15 (word bit 9) up: 64 x 2^c
//    words, lanes varying word bits 0..5 and register k the digit's word
//    bits s .. s + c - 1 (c <= 3; a 4-bit digit takes two groups), so each
//    load still reads 512 contiguous bytes.
// The probe launch gives kProbes units per neuron; unit k takes item
// k * items / kProbes of every check (spread over the table, so that a digit
// that only matters in part of the table is likely seen) and resets the list
// counter.  A list kernel then collects the neurons with bits still unknown,
// and the work launch gives each listed neuron U units (part = u % U) that
// take items part, part + U, ... of each check whose bits are still unknown,
// re-reading the found bits as they go.  Every new bit is published with one
// atomic OR.
constexpr int kProbes = 4;
constexpr int kTaskR = 8;

// Pair tests over the registers P0..P2 (planes, O of them; zero registers
// compare equal), each true if some pair of rows differs in some plane in
// some lane of the wave.
//  - in-word row bit q < 6: rows l and l + 2^q of a word (bit q of l clear).
//    For q < 5 both rows of a pair lie in the same 32-bit half, so the test
//    runs on the halves with 32-bit shifts; for q = 5 the pairs are the halves.
template <int O>
__device__ __forceinline__ bool inword_differs(const uint64_t* P0, const uint64_t* P1, const uint64_t* P2, int q) {
  uint32_t x = 0;
  if (q == 5) {
#pragma unroll
    for (int k = 0; k < kTaskR; ++k) {
      x |= (uint32_t)P0[k] ^ (uint32_t)(P0[k] >> 32);
      if (O > 1) x |= (uint32_t)P1[k] ^ (uint32_t)(P1[k] >> 32);
      if (O > 2) x |= (uint32_t)P2[k] ^ (uint32_t)(P2[k] >> 32);
    }
  } else {
    const int sh = 1 << q;
#pragma unroll
    for (int k = 0; k < kTaskR; ++k) {
      uint32_t lo = (uint32_t)P0[k], hi = (uint32_t)(P0[k] >> 32);
      x |= (lo ^ (lo >> sh)) | (hi ^ (hi >> sh));
      if (O > 1) {
        lo = (uint32_t)P1[k];
        hi = (uint32_t)(P1[k] >> 32);
        x |= (lo ^ (lo >> sh)) | (hi ^ (hi >> sh));
      }
      if (O > 2) {
        lo = (uint32_t)P2[k];
        hi = (uint32_t)(P2[k] >> 32);
        x |= (lo ^ (lo >> sh)) | (hi ^ (hi >> sh));
      }
      __builtin_amdgcn_sched_barrier(0);  // one register's temporaries at a time
    }
    x &= (uint32_t)low_flip_select(q);
  }
  return __any(x != 0u);
}

//  - lane bit t (word bit t of a 64-word run): lanes l and l ^ 2^t.
template <int O>
__device__ __forceinline__ bool lane_differs(const uint64_t* P0, const uint64_t* P1, const uint64_t* P2, int t) {
  bool df = false;
#pragma unroll
  for (int k = 0; k < kTaskR; ++k) {
    df |= shfl_xor_u64(P0[k], 1 << t) != P0[k];
    if (O > 1) df |= shfl_xor_u64(P1[k], 1 << t) != P1[k];
    if (O > 2) df |= shfl_xor_u64(P2[k], 1 << t) != P2[k];
    __builtin_amdgcn_sched_barrier(0);
  }
  return __any(df);
}

//  - register bit i: registers k and k + 2^i (bit i of k clear, k + 2^i < nreg).
template <int O>
__device__ __forceinline__ bool reg_differs(const uint64_t* P0, const uint64_t* P1, const uint64_t* P2, int i,
                                            int nreg) {
  bool df = false;
  const int u = 1 << i;
#pragma unroll
  for (int k = 0; k < kTaskR; ++k) {
    if (!(k & u) && (k | u) < nreg) {
      df |= P0[k] != P0[k | u];
      if (O > 1) df |= P1[k] != P1[k | u];
      if (O > 2) df |= P2[k] != P2[k | u];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return __any(df);
}

// One check item: registers k < 2^c hold words base + lane + (k << s) of
// each of the o planes (lanes below `nw` only: fewer words than a full
// item; absent planes stay zero and compare equal).  Near items (s = 6) also
// test in-word row bits and the lane word bits.  Returns the row bits of
// `need` it finds.  (The probe's few items per neuron take this one
// variant for every o, which keeps its register use down.)
__device__ __forceinline__ uint32_t check_item(const uint64_t* t0, uint64_t W, int o, int b, int Fb, bool near,
                                               uint64_t base, int s, int c, int nw, uint32_t need) {
  const int lane = threadIdx.x & 63;
  uint64_t P0[kTaskR], P1[kTaskR], P2[kTaskR];
#pragma unroll
  for (int k = 0; k < kTaskR; ++k) {
    P0[k] = P1[k] = P2[k] = 0ull;
    if (k < (1 << c)) {  // uniform
      // a wave-uniform row pointer plus the lane: scalar base, small vector offset
      const uint64_t* q = t0 + base + ((uint64_t)k << s);
      if (!near || lane + 64 * k < nw) {
        P0[k] = q[lane];
        if (o > 1) P1[k] = q[W + lane];
        if (o > 2) P2[k] = q[2 * W + lane];
      }
    }
  }
  // testable row bits: in-word (near), lane word bits (near) and register
  // word bits s .. s + c - 1 = row bits s + 6 ..
  const int lowbits = Fb < 6 ? Fb : 6;
  int lb = 0;
  while ((1 << lb) < nw && lb < 6) ++lb;
  uint32_t todo = (((1u << c) - 1u) << (s + 6));
  if (near) todo |= ((1u << lowbits) - 1u) | (((1u << lb) - 1u) << 6);
  todo &= need;
  uint32_t fl = 0;
  while (todo) {  // uniform; a digit is done once one of its bits differs
    const int bit = __ffs(todo) - 1;
    todo &= todo - 1u;
    bool d;
    if (near && bit < 6)
      d = inword_differs<3>(P0, P1, P2, bit);
    else if (near && bit < 12)
      d = lane_differs<3>(P0, P1, P2, bit - 6);
    else
      d = reg_differs<3>(P0, P1, P2, bit - (s + 6), 1 << c);
    if (d) {
      fl |= 1u << bit;
      todo &= ~(((1u << b) - 1u) << ((bit / b) * b));
    }
  }
  return fl;
}

// Far group g (g = 0, 1, ...) of a neuron: the digit j and its first row
// bit s0 (>= 15) and bit count c <= 3; false when there is no such group.
__device__ __forceinline__ bool far_group(int F, int b, int g, int& j, int& s0, int& c) {
  for (j = 0; j < F; ++j) {
    const int lo = j * b > 15 ? j * b : 15, hi = (j + 1) * b;
    for (s0 = lo; s0 < hi; s0 += 3) {
      if (g-- == 0) {
        c = hi - s0 < 3 ? hi - s0 : 3;
        return true;
      }
    }
  }
  return false;
}

__device__ __forceinline__ uint64_t far_base(uint64_t it, int s, int c) {
  const uint64_t lowb = it & ((1ull << (s - 6)) - 1ull);
  return ((it >> (s - 6)) << (s + c)) | (lowb << 6);
}

// Probe: unit (n, k), k < kProbes, checks item k * items / kProbes of the
// near check and of every far group; also resets the pending-list counter.
__global__ __launch_bounds__(256) void support_probe_kernel(SupportArgs a, uint32_t* count) {
  const int lane = threadIdx.x & 63;
  const int wave_in_grid = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  if (wave_in_grid == 0 && lane == 0) *count = 0u;
  const long units = (long)a.n_large * kProbes;
  const long nwv = (long)((gridDim.x * blockDim.x) >> 6);
  for (long u = wave_in_grid; u < units; u += nwv) {
    const int n = a.large[u / kProbes], part = (int)(u % kProbes);
    const tt_neuron* dp = a.desc + n;
    const int F = __builtin_amdgcn_readfirstlane(dp->F), b = __builtin_amdgcn_readfirstlane(dp->b);
    const int o = __builtin_amdgcn_readfirstlane(dp->o);
    const uint64_t* t0 = a.tables + dp->word_off;
    const int Fb = F * b, Wb = Fb > 6 ? Fb - 6 : 0;
    const uint64_t W = 1ull << Wb;
    uint32_t mine = 0;
    // near: one item of up to 512 words
    {
      const long items = Wb > 9 ? 1L << (Wb - 9) : 1L;
      const long it = (long)part * items / kProbes;
      const bool fresh = part == 0 || it != (long)(part - 1) * items / kProbes;
      if (fresh) {
        const int nw = Wb < 9 ? 1 << Wb : 512;
        const int c = Wb < 9 ? (Wb > 6 ? Wb - 6 : 0) : 3;
        mine |= check_item(t0, W, o, b, Fb, true, (uint64_t)it << 9, 6, c, nw,
                           unknown_row_bits(0u, F, b) & ((1u << 15) - 1u));
      }
    }
    int j, s0, c;
    for (int g = 0; far_group(F, b, g, j, s0, c); ++g) {
      const uint32_t D = ((1u << b) - 1u) << (j * b);
      if (mine & D) continue;
      const long items = (long)(W >> (6 + c));
      const long it = (long)part * items / kProbes;
      if (part > 0 && it == (long)(part - 1) * items / kProbes) continue;
      mine |= check_item(t0, W, o, b, Fb, false, far_base((uint64_t)it, s0 - 6, c), s0 - 6, c, 0, D);
    }
    if (lane == 0 && mine) atomicOr(&a.found[n], mine);
  }
}

// Work: unit (listed neuron, part) takes items part + 1, part + 1 + U, ... of
// the near check (full 512-word items) and part, part + U, ... of each far
// group whose digit is still unknown; found bits are published per item and
// re-read as it goes.
template <int O>
__device__ __forceinline__ void work_unit(const SupportArgs& a, int n, int part, int U, int F, int b,
                                          const uint64_t* t0, int Wb) {
  const int lane = threadIdx.x & 63;
  const uint64_t W = 1ull << Wb;
  uint32_t fnd = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.found[n]);
  uint64_t P0[kTaskR], P1[kTaskR], P2[kTaskR];
  if (Wb > 9) {
    const int items = 1 << (Wb - 9);
    for (int it = 1 + part; it < items; it += U) {
      const uint32_t need = unknown_row_bits(fnd, F, b) & ((1u << 15) - 1u);
      if (!need) break;
      const uint64_t* q0 = t0 + ((uint64_t)it << 9);
#pragma unroll
      for (int k = 0; k < kTaskR; ++k) {
        P0[k] = q0[64 * k + lane];
        P1[k] = P2[k] = 0ull;
        if (O > 1) P1[k] = q0[W + 64 * k + lane];
        if (O > 2) P2[k] = q0[2 * W + 64 * k + lane];
      }
      const uint32_t fnow = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.found[n]);
      uint32_t fl = 0;
      for (uint32_t todo = need; todo;) {  // uniform; a digit is done once one of its bits differs
        const int bit = __ffs(todo) - 1;
        todo &= todo - 1u;
        bool d;
        if (bit < 6)
          d = inword_differs<O>(P0, P1, P2, bit);
        else if (bit < 12)
          d = lane_differs<O>(P0, P1, P2, bit - 6);
        else
          d = reg_differs<O>(P0, P1, P2, bit - 12, kTaskR);
        if (d) {
          fl |= 1u << bit;
          todo &= ~(((1u << b) - 1u) << ((bit / b) * b));
        }
      }
      if (fl && lane == 0) atomicOr(&a.found[n], fl);
      fnd |= fl | fnow;
    }
  }
  int j, s0, c;
  for (int g = 0; far_group(F, b, g, j, s0, c); ++g) {
    const uint32_t D = ((1u << b) - 1u) << (j * b);
    const int s = s0 - 6;
    const long items = (long)(W >> (6 + c));
    for (long it = part; it < items; it += U) {
      if (fnd & D) break;
      const uint64_t* q0 = t0 + far_base((uint64_t)it, s, c);
#pragma unroll
      for (int k = 0; k < kTaskR; ++k) {
        P0[k] = P1[k] = P2[k] = 0ull;
        if (k < (1 << c)) {  // uniform
          const uint64_t* q = q0 + ((uint64_t)k << s);
          P0[k] = q[lane];
          if (O > 1) P1[k] = q[W + lane];
          if (O > 2) P2[k] = q[2 * W + lane];
        }
      }
      const uint32_t fnow = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.found[n]);
      uint32_t fl = 0;
      for (int i = 0; i < c; ++i)  // bits of one digit: the first that differs settles it
        if (reg_differs<O>(P0, P1, P2, i, 1 << c)) {
          fl |= 1u << (s0 + i);
          break;
        }
      if (fl && lane == 0) atomicOr(&a.found[n], fl);
      fnd |= fl | fnow;
    }
  }
}

__global__ __launch_bounds__(256) void support_work_kernel(SupportArgs a, int U, const int32_t* list,
                                                           const uint32_t* count) {
  const int wave_in_grid = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const long listed = (long)(uint32_t)__builtin_amdgcn_readfirstlane((int)*count);
  const long units = listed * U;
  const long nwv = (long)((gridDim.x * blockDim.x) >> 6);
  for (long u = wave_in_grid; u < units; u += nwv) {
    const int n = __builtin_amdgcn_readfirstlane(list[u / U]);
    const int part = (int)(u % U);
    const tt_neuron* dp = a.desc + n;
    const int F = __builtin_amdgcn_readfirstlane(dp->F), b = __builtin_amdgcn_readfirstlane(dp->b);
    const int o = __builtin_amdgcn_readfirstlane(dp->o);
    const uint64_t* t0 = a.tables + dp->word_off;
    const int Fb = F * b, Wb = Fb > 6 ? Fb - 6 : 0;
    switch (o) {
      case 1: work_unit<1>(a, n, part, U, F, b, t0, Wb); break;
      case 2: work_unit<2>(a, n, part, U, F, b, t0, Wb); break;
      default: work_unit<3>(a, n, part, U, F, b, t0, Wb); break;
    }
  }
}

// Histogram of packed tables: unit (n, part) takes the 512-word chunks
// part, part + U, ... of neuron n (a table of fewer words is one chunk),
// counts the rows of every code with popcounts of plane combinations, sums
// its lanes and adds the totals to hist[n] (zeroed beforehand).
__global__ __launch_bounds__(256) void hist_tables_kernel(SupportArgs a, int U) {
  const int lane = threadIdx.x & 63;
  const int wave_in_grid = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const long units = (long)a.n_large * U;
  const long nwv = (long)((gridDim.x * blockDim.x) >> 6);
  for (long u = wave_in_grid; u < units; u += nwv) {
    const int n = a.large[u / U], part = (int)(u % U);
    const tt_neuron* dp = a.desc + n;
    const int F = __builtin_amdgcn_readfirstlane(dp->F), b = __builtin_amdgcn_readfirstlane(dp->b);
    const int o = __builtin_amdgcn_readfirstlane(dp->o);
    const uint64_t* t0 = a.tables + dp->word_off;
    const int Fb = F * b, Wb = Fb > 6 ? Fb - 6 : 0;
    const uint64_t W = 1ull << Wb;
    const int nw = Wb < 9 ? 1 << Wb : 512;  // words per chunk
    const long items = Wb > 9 ? 1L << (Wb - 9) : 1L;
    if (part >= items) continue;
    // rows past 2^(F b) in a single-word table are not counted
    const uint64_t validw = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
    uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long it = part; it < items; it += U) {
      const uint64_t* q0 = t0 + ((uint64_t)it << 9);
#pragma unroll
      for (int k = 0; k < kTaskR; ++k) {
        if (64 * k < nw) {  // uniform
          const bool in = lane + 64 * k < nw;
          uint64_t p0 = 0, p1 = 0, p2 = 0;
          if (in) {
            p0 = q0[64 * k + lane];
            if (o > 1) p1 = q0[W + 64 * k + lane];
            if (o > 2) p2 = q0[2 * W + 64 * k + lane];
          }
          const uint64_t m = in ? validw : 0ull;
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            uint64_t x = m & ((v & 1) ? p0 : ~p0);
            x &= (v & 2) ? p1 : ~p1;  // planes at or above o read as zero
            x &= (v & 4) ? p2 : ~p2;
            hv[v] += (uint32_t)__popcll(x);
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      if (v < (1 << o)) {  // uniform
        uint32_t x = hv[v];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off, 64);
        if (lane == 0 && x) atomicAdd(&a.hist[(size_t)n * 8 + v], x);
      }
    }
  }
}

hipError_t launch_hist_tables(const SupportArgs& a, int units_per_neuron, hipStream_t s) {
  if (a.n_large <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const long units = (long)a.n_large * units_per_neuron;
  const long waves = units < 32L * cus ? units : 32L * cus;
  hipLaunchKernelGGL(hist_tables_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a, units_per_neuron);
  return hipGetLastError();
}

// Neurons with a digit not yet known to matter (order not kept).
__global__ void support_pending_kernel(SupportArgs a, int32_t* list, uint32_t* count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_large) return;
  const int n = a.large[k];
  const tt_neuron* dp = a.desc + n;
  if (unknown_row_bits(a.found[n], dp->F, dp->b)) list[atomicAdd(count, 1u)] = n;
}

hipError_t launch_support_tasks(const SupportArgs& a, int units_per_neuron, int32_t* list, uint32_t* count,
                                hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (a.n_large <= 0) return hipSuccess;
  const long pu = (long)a.n_large * kProbes;
  const long pw = pu < 32L * cus ? pu : 32L * cus;
  hipLaunchKernelGGL(support_probe_kernel, dim3((unsigned)((pw + 3) / 4)), dim3(256), 0, s, a, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(support_pending_kernel, dim3((a.n_large + 255) / 256), dim3(256), 0, s, a, list, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long units = (long)a.n_large * units_per_neuron;  // at most
  const long waves = units < 32L * cus ? units : 32L * cus;
  hipLaunchKernelGGL(support_work_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a, units_per_neuron,
                     list, count);
  return hipGetLastError();
}

__global__ void support_finish_kernel(SupportArgs a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n_large) return;
  const int n = a.large[k];
  const tt_neuron* dp = a.desc + n;
  const int F = dp->F, b = dp->b;
  const uint32_t f = a.found[n];
  uint32_t s = 0;
  for (int j = 0; j < F; ++j)
    if (f & (((1u << b) - 1u) << (j * b))) s |= 1u << j;
  a.support[n] = (uint8_t)s;
}

// Support and/or histogram of the small tables (at most kSmallTableWords
// words per plane), one lane per neuron holding its whole table: in-word row
// bits by shifted XOR, word bits by comparing word pairs, codes by popcounts.
__global__ __launch_bounds__(256) void small_tables_kernel(SupportArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n) return;
  const tt_neuron* dp = a.desc + n;
  const int F = dp->F, b = dp->b, o = dp->o;
  const int Fb = F * b, Wb = Fb > 6 ? Fb - 6 : 0;
  const int W = 1 << Wb;
  if (W > kSmallTableWords) return;
  const uint64_t* t0 = a.tables + dp->word_off;
  uint64_t P0[kSmallTableWords], P1[kSmallTableWords], P2[kSmallTableWords];
#pragma unroll
  for (int h = 0; h < kSmallTableWords; ++h) {
    P0[h] = P1[h] = P2[h] = 0ull;
    if (h < W) {
      P0[h] = t0[h];
      if (o > 1) P1[h] = t0[W + h];
      if (o > 2) P2[h] = t0[2 * W + h];
    }
  }
  if (a.hist) {
    const uint64_t validw = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
    uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < kSmallTableWords; ++h) {
      const uint64_t m0 = h < W ? validw : 0ull;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        uint64_t x = m0 & ((v & 1) ? P0[h] : ~P0[h]);
        x &= (v & 2) ? P1[h] : ~P1[h];
        x &= (v & 4) ? P2[h] : ~P2[h];
        hv[v] += (uint32_t)__popcll(x);
      }
    }
    uint4* hd = reinterpret_cast<uint4*>(a.hist + (size_t)n * 8);
    hd[0] = make_uint4(hv[0], hv[1], hv[2], hv[3]);
    hd[1] = make_uint4(hv[4], hv[5], hv[6], hv[7]);
  }
  if (a.support) {
    uint32_t fl = 0;
    const int lowbits = Fb < 6 ? Fb : 6;
    for (int q = 0; q < lowbits; ++q) {
      const int sh = 1 << q;
      uint64_t x = 0;
#pragma unroll
      for (int h = 0; h < kSmallTableWords; ++h)
        x |= (P0[h] ^ (P0[h] >> sh)) | (P1[h] ^ (P1[h] >> sh)) | (P2[h] ^ (P2[h] >> sh));
      if (x & low_flip_select(q)) fl |= 1u << q;
    }
    for (int t = 0; t < Wb; ++t) {
      bool df = false;
#pragma unroll
      for (int h = 0; h < kSmallTableWords; ++h) {
#pragma unroll
        for (int u = 0; u < 4; ++u)  // h ^ 2^t for the t of this iteration
          if (u == t && !(h & (1 << u)) && (h | (1 << u)) < kSmallTableWords)
            df |= P0[h] != P0[h | (1 << u)] || P1[h] != P1[h | (1 << u)] || P2[h] != P2[h | (1 << u)];
      }
      if (df) fl |= 1u << (6 + t);
    }
    uint32_t sres = 0;
    for (int j = 0; j < F; ++j)
      if (fl & (((1u << b) - 1u) << (j * b))) sres |= 1u << j;
    a.support[n] = (uint8_t)sres;
  }
}

// Support of a neuron from its parameters, for tables that are its own
// enumeration.  q is a non-decreasing function of the pre-activation a
// (ReLU and the threshold count are both monotone), with jumps exactly at
// the thresholds (identity) or at the thresholds >= 1 (ReLU: q is constant
// for a <= 0).  Fix the other digits: their sum s (bias included) runs over
// the set S_j = bias + { sum_{i != j} w_i x_i }, and as x_j runs over
// 0 .. 2^b - 1 the pre-activation takes every value of s + w_j x_j, whose
// two ends are s and s + w_j (2^b - 1).  So digit j changes some code iff
// some jump point t has lo < t <= hi for the ends lo < hi of that range,
// for some s in S_j: exactly the definition of the support.  Offsets of S_j
// from its minimum form the set of sums of |w_i| x_i, a subset-sum bitset
// built by shift-ORs: x_i = sum of its bits 2^m, so b shifts by 2^m |w_i|
// per digit.  One wave per digit; the bitset (at most 8 * 128 * 15 + 1
// values) lives in registers, word k = lane + 64 m in register m of the
// lane; a shift is at most 8 * 128 bits (16 words), so each word takes
// its parts from registers m and m - 1 of another lane (shuffles).
constexpr int kSumRegs = 4;  // 4 x 64 words: 16384 values

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Word k - d of the bitset, for the word k = lane + 64 m of this lane (0 < d < 64).
__device__ __forceinline__ uint64_t word_back(const uint64_t (&S)[kSumRegs], int m, int d, int lane) {
  const int src = (lane - d) & 63;
  const uint64_t same = shfl64(S[m], src);
  const uint64_t prev = m > 0 ? shfl64(S[m > 0 ? m - 1 : 0], src) : 0ull;
  return lane >= d ? same : prev;
}

// S |= S << a (a <= 1024) over the first nr registers.
__device__ __forceinline__ void shift_or(uint64_t (&S)[kSumRegs], int a, int nr, int lane) {
  const int q = a >> 6, r = a & 63;
  uint64_t out[kSumRegs];
#pragma unroll
  for (int m = 0; m < kSumRegs; ++m) {
    out[m] = S[m];
    if (m < nr) {  // uniform
      const uint64_t v1 = q == 0 ? S[m] : word_back(S, m, q, lane);
      const uint64_t v2 = word_back(S, m, q + 1, lane);
      out[m] |= (v1 << r) | (r ? (v2 >> (64 - r)) : 0ull);
    }
  }
#pragma unroll
  for (int m = 0; m < kSumRegs; ++m) S[m] = out[m];
}

// Whether any bit of S in [lo, hi] is set (wave-uniform).
__device__ __forceinline__ bool any_in_range(const uint64_t (&S)[kSumRegs], int64_t lo, int64_t hi, int lane) {
  bool hit = false;
#pragma unroll
  for (int m = 0; m < kSumRegs; ++m) {
    const int64_t k0 = (int64_t)(lane + 64 * m) * 64;
    const int64_t a = lo > k0 ? lo : k0, e = hi < k0 + 63 ? hi : k0 + 63;
    if (a <= e) {
      const int sa = (int)(a - k0), se = (int)(e - k0);
      const uint64_t mask = (se == 63 ? ~0ull : ((1ull << (se + 1)) - 1ull)) & ~((1ull << sa) - 1ull);
      hit |= (S[m] & mask) != 0ull;
    }
  }
  return __any(hit);
}

// One block of eight waves per neuron (grid-strided), wave j deciding digit j.
__global__ __launch_bounds__(512) void support_params_kernel(const tt_neuron* desc, const int32_t* list, int n,
                                                             uint8_t* support) {
  __shared__ uint32_t s_bits[8];
  const int lane = threadIdx.x & 63;
  const int j = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int c = blockIdx.x; c < n; c += gridDim.x) {
    const int i = list ? list[c] : c;
    const tt_neuron* dp = desc + i;
    const int F = dp->F, b = dp->b, o = dp->o, act = dp->act;
    const int K = (1 << o) - 1, dmax = (1 << b) - 1;
    int w[8];
    int Rall = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      w[k] = k < F ? (int)dp->w[k] : 0;
      Rall += (w[k] < 0 ? -w[k] : w[k]) * dmax;
    }
    const int nr = Rall / 4096 + 1;  // registers in use (64 words each)
    bool found = false;
    if (j < F && w[j] != 0) {  // uniform per wave
      // S_j as offsets from its minimum base
      int64_t base = dp->bias;
      int R = 0;
      uint64_t S[kSumRegs];
#pragma unroll
      for (int m = 0; m < kSumRegs; ++m) S[m] = (lane == 0 && m == 0) ? 1ull : 0ull;
      for (int i2 = 0; i2 < F; ++i2) {
        if (i2 == j || w[i2] == 0) continue;
        const int aw = w[i2] < 0 ? -w[i2] : w[i2];
        base += (int64_t)(w[i2] < 0 ? w[i2] : 0) * dmax;
        R += aw * dmax;
        for (int m = 0; m < b; ++m) shift_or(S, aw << m, nr, lane);
      }
      const int64_t D = (int64_t)(w[j] < 0 ? -w[j] : w[j]) * dmax;
      for (int k = 0; k < K && !found; ++k) {
        const int64_t t = dp->thr[k];
        if (act == TT_ACT_RELU && t < 1) continue;
        // s with s < t <= s + D (w_j > 0) or s - D < t <= s (w_j < 0)
        int64_t lo = w[j] > 0 ? t - D : t, hi = w[j] > 0 ? t - 1 : t + D - 1;
        lo -= base;
        hi -= base;
        if (lo < 0) lo = 0;
        if (hi > R) hi = R;
        if (lo <= hi) found = any_in_range(S, lo, hi, lane);
      }
    }
    if (lane == 0) s_bits[j] = found ? 1u << j : 0u;
    __syncthreads();
    if (threadIdx.x == 0)
      support[i] = (uint8_t)(s_bits[0] | s_bits[1] | s_bits[2] | s_bits[3] | s_bits[4] | s_bits[5] | s_bits[6] |
                             s_bits[7]);
    __syncthreads();  // s_bits is reused by the next neuron
  }
}

// Neurons whose sums span at most 512 values (sum_j |w_j| (2^b - 1) < 512,
// e.g. |w| <= 7 and b <= 3): one wave per neuron, lane group g (8 lanes,
// 8 words = 512 bits) deciding digit g; every shift is below 8 words and
// stays inside the group.
__global__ __launch_bounds__(256) void support_params_small_kernel(const tt_neuron* desc, const int32_t* list,
                                                                  int count, uint8_t* support) {
  const int gw = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  for (int c = gw; c < count; c += nw) {
    const int i = __builtin_amdgcn_readfirstlane(list[c]);
    const NeuronRegs d = load_neuron(desc + i);
    const uint32_t sup = small_support_wave(d, neuron_sum_range(d));
    if ((threadIdx.x & 63) == 0) support[i] = (uint8_t)sup;
  }
}

hipError_t launch_support_params_small(const tt_neuron* desc, const int32_t* list, int count, uint8_t* support,
                                       hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (count + 3) / 4 < 4096 ? (count + 3) / 4 : 4096;
  hipLaunchKernelGGL(support_params_small_kernel, dim3(blocks), dim3(256), 0, s, desc, list, count, support);
  return hipGetLastError();
}

hipError_t launch_support_params(const tt_neuron* desc, const int32_t* list, int n, uint8_t* support,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = n < 8192 ? n : 8192;
  hipLaunchKernelGGL(support_params_kernel, dim3(blocks), dim3(512), 0, s, desc, list, n, support);
  return hipGetLastError();
}

hipError_t launch_small_tables(const SupportArgs& a, hipStream_t s) {
  if (a.n <= 0 || a.n_large >= a.n) return hipSuccess;
  hipLaunchKernelGGL(small_tables_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Pack: one wave per 64 words of one neuron.  Row r's code is read by lane
// r % 64; a ballot per plane bit gives the word, which lane (word index)
// keeps until the wave stores its 64 words in one coalesced run per plane.
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
  const int lane = threadIdx.x & 63;
  const int it = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (it >= a.n_items) return;
  const int n = a.item_neuron[it];
  const int h0 = a.item_h0[it];
  const tt_neuron d = a.desc[n];
  const int o = d.o, Fb = d.F * d.b;
  const uint64_t W = words_per_plane(Fb);
  const uint64_t R = 1ull << Fb;
  const int nw = (int)min((uint64_t)64, W - (uint64_t)h0);
  const uint8_t* codes = a.codes + a.code_off[n];
  uint64_t mine0 = 0, mine1 = 0, mine2 = 0;
  for (int i = 0; i < nw; ++i) {
    const uint64_t row = ((uint64_t)(h0 + i) << 6) + (uint64_t)lane;
    const uint32_t c = row < R ? codes[row] : 0u;
    const uint64_t m0 = __ballot(c & 1u);
    const uint64_t m1 = __ballot(c & 2u);
    const uint64_t m2 = __ballot(c & 4u);
    if (lane == i) {
      mine0 = m0;
      mine1 = m1;
      mine2 = m2;
    }
  }
  if (lane < nw) {
    uint64_t* dst = a.tables + d.word_off + (uint64_t)h0 + (uint64_t)lane;
    dst[0] = mine0;
    if (o > 1) dst[W] = mine1;
    if (o > 2) dst[2 * W] = mine2;
  }
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_support_finish(const SupportArgs& a, hipStream_t s) {
  if (a.n_large <= 0) return hipSuccess;
  hipLaunchKernelGGL(support_finish_kernel, dim3((a.n_large + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3((a.n_items + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tt
