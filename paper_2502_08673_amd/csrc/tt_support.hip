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

// One item: stage 2^c words per plane, histogram (pass 0), in-word flips
// (pass 0) and flips of the item's local word bits, for unknown digits only.
__device__ void support_item(const SupportArgs& a, const SupportItem& it, uint64_t (*s_pl)[kSupChunk],
                             uint32_t* s_found, uint32_t* s_new, uint32_t* s_hist) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = it.neuron;
  const tt_neuron d = a.desc[n];
  const int b = d.b, o = d.o, Fb = d.F * d.b;
  const uint64_t W = words_per_plane(Fb);
  __syncthreads();  // the previous item is done with the shared state
  if (tid == 0) {
    *s_found = a.want_support ? a.found[n] : 0u;
    *s_new = 0u;
  }
  if (tid < 8) s_hist[tid] = 0u;
  __syncthreads();
  const uint32_t need = a.want_support ? unknown_row_bits(*s_found, d.F, b) : 0u;
  const uint32_t local_need = item_local_need(it, need);
  const int lowbits = Fb < 6 ? Fb : 6;
  const uint32_t low_need = it.hist ? (need & ((1u << lowbits) - 1u)) : 0u;
  const bool do_hist = it.hist && a.hist != nullptr;
  const bool stage = local_need != 0u;
  if (!stage && !low_need && !do_hist) return;  // uniform

  const int cnt = 1 << it.c;
  const int amask = (1 << it.a) - 1;
  const uint64_t* src = a.tables + d.word_off;
  const uint64_t valid = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
  uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t fl = 0;
  // Every load of this thread is issued before any of them is used.
  constexpr int kPer = kSupChunk / 256;
  uint64_t P0[kPer], P1[kPer], P2[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid + k * 256;
    P0[k] = P1[k] = P2[k] = 0ull;
    if (i < cnt) {
      const uint64_t w = (uint64_t)it.base + (uint64_t)(i & amask) + ((uint64_t)(i >> it.a) << it.s);
      P0[k] = src[w];
      if (o > 1) P1[k] = src[W + w];
      if (o > 2) P2[k] = src[2 * W + w];
    }
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid + k * 256;
    if (i >= cnt) break;
    if (stage) {
      s_pl[0][i] = P0[k];
      if (o > 1) s_pl[1][i] = P1[k];
      if (o > 2) s_pl[2][i] = P2[k];
    }
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
      if (lane == 0 && x) atomicAdd(&s_hist[v], x);
    }
  }
  if (stage) {
    __syncthreads();
    uint32_t fb = 0;  // local bits found by this thread
    for (int i = tid; i < cnt; i += blockDim.x) {
      for (uint32_t q = local_need & ~fb; q; q &= q - 1) {
        const int t = __ffs(q) - 1;
        if ((i >> t) & 1) continue;
        const int j = i | (1 << t);
        bool diff = s_pl[0][i] != s_pl[0][j];
        if (o > 1) diff |= s_pl[1][i] != s_pl[1][j];
        if (o > 2) diff |= s_pl[2][i] != s_pl[2][j];
        if (diff) fb |= 1u << t;
      }
    }
    for (uint32_t q = fb; q; q &= q - 1) fl |= 1u << (6 + item_word_bit(it, __ffs(q) - 1));
  }
  for (int off = 32; off >= 1; off >>= 1) fl |= __shfl_xor(fl, off, 64);
  if (lane == 0 && fl) atomicOr(s_new, fl);
  __syncthreads();
  if (tid == 0) {
    if (*s_new) atomicOr(&a.found[n], *s_new);
    if (do_hist)
      for (int v = 0; v < 8; ++v)
        if (s_hist[v]) atomicAdd(&a.hist[(size_t)n * 8 + v], s_hist[v]);
  }
}

// Persistent over batches of 64 items: wave 0 decides from the found bits
// which items of the batch still have work, so settled items cost almost
// nothing; the block then runs the remaining items one after another.
__global__ __launch_bounds__(256) void support_kernel(SupportArgs a) {
  static_assert(kSupChunk % 256 == 0, "items are split evenly over 256 threads");
  __shared__ uint64_t s_pl[3][kSupChunk];
  __shared__ uint32_t s_found, s_new;
  __shared__ uint32_t s_hist[8];
  __shared__ uint64_t s_mask;
  const int lane = threadIdx.x & 63;
  const int nb = (a.n_items + 63) >> 6;
  for (int bt = blockIdx.x; bt < nb; bt += gridDim.x) {
    __syncthreads();
    if (threadIdx.x < 64) {
      const int idx = (bt << 6) + lane;
      bool work = false;
      if (idx < a.n_items) {
        const SupportItem it = a.items[idx];
        if (it.hist && a.hist) {
          work = true;
        } else if (a.want_support) {
          const tt_neuron& d = a.desc[it.neuron];
          const uint32_t need = unknown_row_bits(a.found[it.neuron], d.F, d.b);
          const int fb = d.F * d.b;
          const uint32_t lown = it.hist ? (need & ((1u << (fb < 6 ? fb : 6)) - 1u)) : 0u;
          work = item_local_need(it, need) != 0u || lown != 0u;
        }
      }
      const uint64_t m = __ballot(work);
      if (lane == 0) s_mask = m;
    }
    __syncthreads();
    uint64_t m = s_mask;
    while (m) {
      const int k = __ffsll((long long)m) - 1;
      m &= m - 1;
      const SupportItem it = a.items[(bt << 6) + k];
      support_item(a, it, s_pl, &s_found, &s_new, s_hist);
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

hipError_t launch_support(const SupportArgs& a, hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int nb = (a.n_items + 63) / 64;
  const int grid = nb < 3 * cus ? nb : 3 * cus;
  hipLaunchKernelGGL(support_kernel, dim3(grid), dim3(256), 0, s, a);
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
