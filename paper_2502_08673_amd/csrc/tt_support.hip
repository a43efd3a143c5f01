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
// support iff any of its b row bits is.  Pass-0 items stage contiguous
// chunks of 2^11 words in LDS and handle row bits 0..5 and the word bits
// inside the chunk (and the histogram); later items stage 16-word runs whose
// high word bits vary, covering the word bits beyond one chunk.  A bit is
// skipped as soon as its digit is known to be in the support.
#include "tt_internal.h"

namespace tt {

__device__ __forceinline__ uint64_t low_flip_select(int i) {
  switch (i) {
    case 0: return 0x5555555555555555ull;
    case 1: return 0x3333333333333333ull;
    case 2: return 0x0F0F0F0F0F0F0F0Full;
    case 3: return 0x00FF00FF00FF00FFull;
    case 4: return 0x0000FFFF0000FFFFull;
    default: return 0x00000000FFFFFFFFull;
  }
}

__device__ __forceinline__ uint64_t words_per_plane(int Fb) {
  return Fb >= 6 ? (1ull << (Fb - 6)) : 1ull;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Local index t of an item -> word bit.
__device__ __forceinline__ int item_word_bit(const SupportItem& it, int t) {
  return t < it.a ? t : it.s + (t - it.a);
}

// Row bits of the digits that have no found bit yet.
__device__ __forceinline__ uint32_t unknown_row_bits(uint32_t found, int F, int b) {
  uint32_t need = 0;
  for (int j = 0; j < F; ++j) {
    const uint32_t D = ((1u << b) - 1u) << (j * b);
    if (!(found & D)) need |= D;
  }
  return need;
}

// Local bits of an item that still need a flip check, given unknown row bits.
// Pass-0 items check all their local bits; later items only the bits beyond
// the contiguous run (the run's bits were covered by pass 0).
__device__ __forceinline__ uint32_t item_local_need(const SupportItem& it, uint32_t need) {
  uint32_t ln = 0;
  for (int t = it.hist ? 0 : it.a; t < it.c; ++t)
    if ((need >> (6 + item_word_bit(it, t))) & 1u) ln |= 1u << t;
  return ln;
}

// Register-resident words of one item: thread t holds local words
// t + 256k, k < kPer (every load is issued before any is used).
constexpr int kPer = kSupChunk / 256;

__device__ __forceinline__ void load_item(const SupportArgs& a, const SupportItem& it, uint64_t* P0, uint64_t* P1,
                                          uint64_t* P2) {
  const int cnt = 1 << it.c;
  const int amask = (1 << it.a) - 1;
  const uint64_t* src = a.tables + it.word_off;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = (int)threadIdx.x + k * 256;
    P0[k] = P1[k] = P2[k] = 0ull;
    if (i < cnt) {
      const uint64_t w = (uint64_t)it.base + (uint64_t)(i & amask) + ((uint64_t)(i >> it.a) << it.s);
      P0[k] = src[w];
      if (it.o > 1) P1[k] = src[it.W + w];
      if (it.o > 2) P2[k] = src[2 * it.W + w];
    }
  }
}

// Stage the item's words in LDS (planes at s_pl + p * kSupChunk) and check
// the flips of the local bits in `local_need`; returns the row bits found
// by this thread.  Contains one barrier: call uniformly.
__device__ __forceinline__ uint32_t stage_and_check(const SupportItem& it, uint32_t local_need, uint64_t* s_pl,
                                                    const uint64_t* P0, const uint64_t* P1, const uint64_t* P2) {
  const int cnt = 1 << it.c;
  const int o = it.o;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = (int)threadIdx.x + k * 256;
    if (i < cnt) {
      s_pl[i] = P0[k];
      if (o > 1) s_pl[kSupChunk + i] = P1[k];
      if (o > 2) s_pl[2 * kSupChunk + i] = P2[k];
    }
  }
  __syncthreads();
  uint32_t fb = 0;
  for (int i = threadIdx.x; i < cnt; i += 256) {
    for (uint32_t q = local_need & ~fb; q; q &= q - 1) {
      const int t = __ffs(q) - 1;
      if ((i >> t) & 1) continue;
      const int j = i | (1 << t);
      bool diff = s_pl[i] != s_pl[j];
      if (o > 1) diff |= s_pl[kSupChunk + i] != s_pl[kSupChunk + j];
      if (o > 2) diff |= s_pl[2 * kSupChunk + i] != s_pl[2 * kSupChunk + j];
      if (diff) fb |= 1u << t;
    }
  }
  uint32_t rows = 0;
  for (uint32_t q = fb; q; q &= q - 1) rows |= 1u << (6 + item_word_bit(it, __ffs(q) - 1));
  return rows;
}

__device__ __forceinline__ void publish_found(const SupportArgs& a, int n, uint32_t fl) {
  for (int off = 32; off >= 1; off >>= 1) fl |= __shfl_xor(fl, off, 64);
  if ((threadIdx.x & 63) == 0 && fl) atomicOr(&a.found[n], fl);
}

// Pass 0, grid-stride over contiguous chunks: histogram (always, if asked),
// in-word row bits and in-chunk word bits of digits not yet in the support.
__global__ __launch_bounds__(256) void support_p0_kernel(SupportArgs a) {
  extern __shared__ uint64_t s_pl[];
  __shared__ uint32_t s_f[2];
  const int lane = threadIdx.x & 63;
  int iter = 0;
  for (int idx = blockIdx.x; idx < a.n_items; idx += gridDim.x, ++iter) {
    const SupportItem it = a.items[idx];
    const int n = it.neuron;
    const int Fb = it.F * it.b;
    const bool do_hist = a.hist != nullptr;
    uint64_t P0[kPer], P1[kPer], P2[kPer];
    if (do_hist || a.want_support) load_item(a, it, P0, P1, P2);
    if (threadIdx.x == 0) s_f[iter & 1] = a.want_support ? a.found[n] : 0u;
    __syncthreads();  // also retires the previous item's use of the LDS stage
    const uint32_t need = a.want_support ? unknown_row_bits(s_f[iter & 1], it.F, it.b) : 0u;
    const uint32_t local_need = item_local_need(it, need);
    const int lowbits = Fb < 6 ? Fb : 6;
    const uint32_t low_need = need & ((1u << lowbits) - 1u);
    if (!do_hist && !local_need && !low_need) continue;  // uniform
    const int cnt = 1 << it.c;
    const int o = it.o;
    const uint64_t valid = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
    uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t fl = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = (int)threadIdx.x + k * 256;
      if (i >= cnt) break;
      if (do_hist) {
        for (int v = 0; v < (1 << o); ++v) {
          uint64_t m = valid & ((v & 1) ? P0[k] : ~P0[k]);
          if (o > 1) m &= (v & 2) ? P1[k] : ~P1[k];
          if (o > 2) m &= (v & 4) ? P2[k] : ~P2[k];
          hv[v] += (uint32_t)__popcll(m);
        }
      }
      for (uint32_t q = low_need & ~fl; q; q &= q - 1) {
        const int bit = __ffs(q) - 1;
        const int sh = 1 << bit;
        const uint64_t x = ((P0[k] ^ (P0[k] >> sh)) | (P1[k] ^ (P1[k] >> sh)) | (P2[k] ^ (P2[k] >> sh))) &
                           low_flip_select(bit);
        if (x) fl |= 1u << bit;
      }
    }
    if (do_hist) {
      for (int v = 0; v < (1 << o); ++v) {
        uint32_t x = hv[v];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0 && x) atomicAdd(&a.hist[(size_t)n * 8 + v], x);
      }
    }
    if (local_need) fl |= stage_and_check(it, local_need, s_pl, P0, P1, P2);
    if (a.want_support) publish_found(a, n, fl);
  }
}

// Word bits beyond one chunk, in batches of 64 items: wave 0 decides from
// the found bits which items of the batch still have work (settled items
// cost almost nothing); the block then runs the rest one after another.
__global__ __launch_bounds__(256) void support_far_kernel(SupportArgs a) {
  extern __shared__ uint64_t s_pl[];
  __shared__ uint64_t s_mask[2];
  const int lane = threadIdx.x & 63;
  const int nb = (a.n_items + 63) >> 6;
  int iter = 0;
  for (int bt = blockIdx.x; bt < nb; bt += gridDim.x, ++iter) {
    if (threadIdx.x < 64) {
      const int idx = (bt << 6) + lane;
      bool work = false;
      if (idx < a.n_items) {
        const SupportItem it = a.items[idx];
        work = item_local_need(it, unknown_row_bits(a.found[it.neuron], it.F, it.b)) != 0u;
      }
      const uint64_t m = __ballot(work);
      if (lane == 0) s_mask[iter & 1] = m;
    }
    __syncthreads();
    uint64_t m = s_mask[iter & 1];
    while (m) {
      const int k = __ffsll((long long)m) - 1;
      m &= m - 1;
      const SupportItem it = a.items[(bt << 6) + k];
      uint64_t P0[kPer], P1[kPer], P2[kPer];
      load_item(a, it, P0, P1, P2);
      // Bits settled since the batch was screened are skipped here (the
      // mask below is uniform: every thread reads the same found word
      // after the barrier inside the previous item or the screen).
      const uint32_t local_need = item_local_need(it, unknown_row_bits(a.found[it.neuron], it.F, it.b));
      __syncthreads();  // the previous item is done with the LDS stage
      const uint32_t fl = stage_and_check(it, local_need | 0u, s_pl, P0, P1, P2);
      publish_found(a, it.neuron, fl);
    }
  }
}

__global__ void support_finish_kernel(SupportArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n) return;
  const tt_neuron d = a.desc[n];
  const uint32_t f = a.found[n];
  uint32_t s = 0;
  for (int j = 0; j < d.F; ++j)
    if (f & (((1u << d.b) - 1u) << (j * d.b))) s |= 1u << j;
  a.support[n] = (uint8_t)s;
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

hipError_t launch_support(const SupportArgs& a, int far, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int o_max = a.o_max < 1 ? 1 : a.o_max;
  const size_t lds = sizeof(uint64_t) * (size_t)kSupChunk * (size_t)o_max;
  const int per_cu = (int)((160 * 1024) / (lds + 1024));
  const int blocks = (per_cu < 1 ? 1 : per_cu) * cus;
  if (far) {
    const int nb = (a.n_items + 63) / 64;
    hipLaunchKernelGGL(support_far_kernel, dim3(nb < blocks ? nb : blocks), dim3(256), lds, s, a);
  } else {
    hipLaunchKernelGGL(support_p0_kernel, dim3(a.n_items < blocks ? a.n_items : blocks), dim3(256), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_support_finish(const SupportArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(support_finish_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3((a.n_items + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tt
