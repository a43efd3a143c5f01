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
// support iff any of its b row bits is.  Pass 0 stages a chunk of words in
// LDS and handles row bits 0..5 and the word bits inside the chunk; pass 1
// pairs words across chunks for the remaining word bits.  Both skip a bit as
// soon as its digit is already known to be in the support.
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

// Row bits of the digit that contains row bit rb.
__device__ __forceinline__ uint32_t digit_row_bits(int rb, int b) {
  const int j = rb / b;
  return ((1u << b) - 1u) << (j * b);
}

__device__ __forceinline__ uint64_t words_per_plane(int Fb) {
  return Fb >= 6 ? (1ull << (Fb - 6)) : 1ull;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Pass 0: one block per (neuron, chunk of words); histogram, in-word bits and
// in-chunk word bits.
__global__ __launch_bounds__(256) void support_chunk_kernel(SupportArgs a) {
  __shared__ uint64_t s_pl[3][kSupChunk];
  __shared__ uint32_t s_found;
  __shared__ uint32_t s_hist[8];
  const SupportItem it = a.items[blockIdx.x];
  const int n = it.neuron;
  const tt_neuron d = a.desc[n];
  const int b = d.b, o = d.o, Fb = d.F * d.b;
  const uint64_t W = words_per_plane(Fb);
  const int cnt = it.count;
  const uint64_t* src = a.tables + d.word_off + (uint64_t)it.h0;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  if (tid == 0) s_found = a.want_support ? a.found[n] : 0u;
  if (tid < 8) s_hist[tid] = 0u;
  for (int p = 0; p < o; ++p)
    for (int i = tid; i < cnt; i += blockDim.x) s_pl[p][i] = src[(uint64_t)p * W + i];
  __syncthreads();

  const uint64_t valid = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
  const int lowbits = Fb < 6 ? Fb : 6;
  uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t fl = 0;
  for (int i = tid; i < cnt; i += blockDim.x) {
    const uint64_t P0 = s_pl[0][i];
    const uint64_t P1 = o > 1 ? s_pl[1][i] : 0ull;
    const uint64_t P2 = o > 2 ? s_pl[2][i] : 0ull;
    if (a.hist) {
      for (int v = 0; v < (1 << o); ++v) {
        uint64_t m = valid & ((v & 1) ? P0 : ~P0);
        if (o > 1) m &= (v & 2) ? P1 : ~P1;
        if (o > 2) m &= (v & 4) ? P2 : ~P2;
        hv[v] += (uint32_t)__popcll(m);
      }
    }
    if (a.want_support) {
      for (int q = 0; q < lowbits; ++q) {
        const int s = 1 << q;
        const uint64_t x = ((P0 ^ (P0 >> s)) | (P1 ^ (P1 >> s)) | (P2 ^ (P2 >> s))) & low_flip_select(q);
        if (x) fl |= 1u << q;
      }
    }
  }
  if (a.hist) {
    for (int v = 0; v < 8; ++v) {
      uint32_t x = hv[v];
      for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0 && x) atomicAdd(&s_hist[v], x);
    }
  }
  if (a.want_support) {
    for (int off = 32; off >= 1; off >>= 1) fl |= __shfl_xor(fl, off, 64);
    if (lane == 0 && fl) atomicOr(&s_found, fl);
  }
  __syncthreads();

  if (a.want_support) {
    const int cbits = __ffs(cnt) - 1;  // cnt is a power of two
    for (int k = 0; k < cbits; ++k) {
      const uint32_t f = s_found;
      __syncthreads();
      if (!(f & digit_row_bits(6 + k, b))) {
        bool diff = false;
        const int half = cnt >> 1;
        const int lo = (1 << k) - 1;
        for (int i = tid; i < half; i += blockDim.x) {
          const int h = ((i >> k) << (k + 1)) | (i & lo);
          const int h2 = h | (1 << k);
          for (int p = 0; p < o; ++p) diff |= s_pl[p][h] != s_pl[p][h2];
        }
        if (__any(diff) && lane == 0) atomicOr(&s_found, 1u << (6 + k));
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (a.want_support && s_found) atomicOr(&a.found[n], s_found);
    if (a.hist)
      for (int v = 0; v < 8; ++v)
        if (s_hist[v]) atomicAdd(&a.hist[(size_t)n * 8 + v], s_hist[v]);
  }
}

// Pass 1: one block per (neuron, word bit k beyond the chunk, range of word
// pairs).  Words are read straight from HBM: consecutive pair indices map to
// consecutive words inside runs of 2^k.
__global__ __launch_bounds__(256) void support_far_kernel(SupportArgs a) {
  const SupportItem it = a.items[blockIdx.x];
  const int n = it.neuron;
  const tt_neuron d = a.desc[n];
  const int b = d.b, o = d.o, Fb = d.F * d.b;
  const int k = it.bit;
  const int rb = 6 + k;
  if (a.found[n] & digit_row_bits(rb, b)) return;
  const uint64_t W = words_per_plane(Fb);
  const uint64_t* src = a.tables + d.word_off;
  const int lo = (1 << k) - 1;
  bool diff = false;
  for (int i = it.h0 + threadIdx.x; i < it.h0 + it.count; i += blockDim.x) {
    const uint64_t h = ((uint64_t)(i >> k) << (k + 1)) | (uint64_t)(i & lo);
    const uint64_t h2 = h | (1ull << k);
    for (int p = 0; p < o; ++p) diff |= src[(uint64_t)p * W + h] != src[(uint64_t)p * W + h2];
  }
  if (__any(diff) && (threadIdx.x & 63) == 0) atomicOr(&a.found[n], 1u << rb);
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

hipError_t launch_support(const SupportArgs& a, int pass, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (pass == 0)
    hipLaunchKernelGGL(support_chunk_kernel, dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(support_far_kernel, dim3(grid), dim3(256), 0, s, a);
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
