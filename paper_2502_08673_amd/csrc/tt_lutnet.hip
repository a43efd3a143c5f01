// tt_lutnet.hip -- a layered network of enumerated neurons evaluated through
// its packed truth tables (gfx950): lookups only, no arithmetic.
//
// Signals 0 .. n_inputs - 1 are primary input codes (uint8 per sample), and
// signal n_inputs + i is the output code of neuron i.  A neuron gathers its
// F input codes, forms the row r from their low b bits, and reads bit
// r % 64 of word r / 64 of each of its o planes.  Two forms: the whole
// network per block with the samples' signals in LDS (when a few dozen
// samples' signals fit), else one launch per level (a level reads only the
// primary inputs and earlier levels) with the signals in global memory.
#include <algorithm>

#include "tt_internal.h"

namespace tt {

__global__ __launch_bounds__(256) void lutnet_level_kernel(LutnetArgs a) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)a.batch * a.count) return;
  const int s = (int)(t / a.count);
  const int i = a.level[t % a.count];
  const tt_neuron* dp = a.desc + i;
  const int F = dp->F, b = dp->b, o = dp->o;
  const uint32_t mask = (1u << b) - 1u;
  const int32_t* fi = a.fanin + 8 * (long)i;
  const uint8_t* in = a.inputs + (long)s * a.n_inputs;
  const uint8_t* prev = a.out + (long)s * a.n - a.n_inputs;  // prev[sig] for sig >= n_inputs
  uint32_t r = 0;
  for (int j = 0; j < F; ++j) {
    const int sig = fi[j];
    const uint32_t code = sig < a.n_inputs ? in[sig] : prev[sig];
    r |= (code & mask) << (j * b);
  }
  const int Fb = F * b;
  const uint64_t W = Fb >= 6 ? (1ull << (Fb - 6)) : 1ull;
  const uint64_t* t0 = a.tables + dp->word_off + (r >> 6);
  uint32_t q = 0;
  for (int p = 0; p < o; ++p) q |= (uint32_t)((t0[(uint64_t)p * W] >> (r & 63u)) & 1ull) << p;
  a.out[(long)s * a.n + i] = (uint8_t)q;
}

// Whole network per block: a block takes up to 64 samples, one per lane, and
// keeps their signal rows (n_inputs + n codes and one zero byte, the stride
// an odd number of dwords so that the 64 rows fall in distinct LDS banks) in
// LDS through all levels, with a barrier between levels.  A wave takes
// kNetStep neurons at a time: their records are wave-uniform (scalar loads,
// no chain of dependent loads), each lane reads the fan-in codes from its
// own row (FMAX reads, unused slots pointing at the zero byte, so no branch
// on F), and one load per lane returns the row's group of interleaved plane
// dwords, all inside the neuron's table, which stays in cache.  The block
// writes its output rows at the end.
constexpr int kNetSamples = 64;
constexpr int kNetStep = 8;
constexpr int kNetThreads = 512;
constexpr long kNetMaxLds = 64 * 1024;
constexpr int kCopyRows = 8;  // rows per wave with their loads in flight together while staging

// Rows [0, rows) of `per_row` elements, contiguous at src, into LDS rows of
// `stride` bytes at dst, each element ANDed with its column's entry of
// colmask (when given).  Wave w takes rows w, w + waves, ... and lane l the
// columns l, l + 64, ...; a wave issues kCopyRows rows' loads before its
// first LDS store.
template <typename T>
__device__ __forceinline__ void rows_to_lds(const T* src, int rows, int per_row, uint8_t* dst, int stride,
                                            const T* colmask) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = blockDim.x >> 6;
  for (int c0 = 0; c0 < per_row; c0 += 64) {
    const int c = c0 + lane;
    const bool cok = c < per_row;
    const T m = colmask && cok ? colmask[c] : (T)~T(0);
    for (int r0 = wave; r0 < rows; r0 += nw * kCopyRows) {
      T v[kCopyRows];
#pragma unroll
      for (int u = 0; u < kCopyRows; ++u) {
        const int r = r0 + u * nw;
        v[u] = cok && r < rows ? src[(long)r * per_row + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kCopyRows; ++u) {
        const int r = r0 + u * nw;
        if (cok && r < rows) reinterpret_cast<T*>(dst + r * stride)[c] = (T)(v[u] & m);
      }
    }
  }
}

// the reverse: LDS rows of `stride` bytes at src to contiguous rows at dst
template <typename T>
__device__ __forceinline__ void lds_to_rows(const uint8_t* src, int stride, int rows, int per_row, T* dst) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = blockDim.x >> 6;
  for (int c0 = 0; c0 < per_row; c0 += 64) {
    const int c = c0 + lane;
    const bool cok = c < per_row;
    for (int r0 = wave; r0 < rows; r0 += nw * kCopyRows) {
      T v[kCopyRows];
#pragma unroll
      for (int u = 0; u < kCopyRows; ++u) {
        const int r = r0 + u * nw;
        v[u] = cok && r < rows ? reinterpret_cast<const T*>(src + r * stride)[c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kCopyRows; ++u) {
        const int r = r0 + u * nw;
        if (cok && r < rows) dst[(long)r * per_row + c] = v[u];
      }
    }
  }
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output number k >= 1 of the stream seeded with
// seed, i.e. the finaliser applied to seed + k * golden gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int FMAX, int OMAX, bool MASK>
__global__ __launch_bounds__(kNetThreads) void lutnet_fused_kernel(NetArgs a, const NetSample smp) {
  extern __shared__ uint8_t sig[];  // [kNetSamples][stride]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nwaves = blockDim.x >> 6;
  const long s0 = (long)blockIdx.x * kNetSamples;
  const int ns = (int)min((long)kNetSamples, (long)a.batch - s0);
  // the samples' input rows into LDS, each code reduced to the digits its
  // readers take when they all take the same number (then no reader masks)
  if (a.sample) {
    // drawn: bytes 8m .. 8m + 7 of row r are the bytes of output
    // (first + s0 + r) Q + m + 1 of the stream, masked per column.  With
    // Q < 64 draws per row a wave takes 64 / Q rows per pass (lane = sub Q +
    // m) and each lane's column mask is one 8-byte load, taken once; a whole
    // draw goes to LDS as two dword stores (rows are dword aligned)
    const int Q = (a.n_inputs + 7) >> 3;
    const bool wide = Q >= 64 || Q == 0;  // (no inputs: nothing to draw)
    const int RP = wide ? 1 : 64 / Q;  // rows per wave and pass
    const int sub = wide ? 0 : lane / Q;
    const int m0 = lane - sub * Q;
    if (sub < RP) {
      uint64_t mk0 = 0;
      if (m0 < Q && 8 * m0 + 8 <= a.n_inputs) mk0 = *reinterpret_cast<const uint64_t*>(a.in_mask + 8 * m0);
      for (int r = wave * RP + sub; r < ns; r += nwaves * RP)
        for (int m = m0; m < Q; m += 64) {
          const uint64_t z = splitmix64_at(smp.seed, (smp.first + (uint64_t)(s0 + r)) * (uint64_t)Q + m + 1);
          uint8_t* dst = sig + r * a.stride + 8 * m;
          if (8 * m + 8 <= a.n_inputs) {
            const uint64_t v = z & (m == m0 ? mk0 : *reinterpret_cast<const uint64_t*>(a.in_mask + 8 * m));
            reinterpret_cast<uint32_t*>(dst)[0] = (uint32_t)v;
            reinterpret_cast<uint32_t*>(dst)[1] = (uint32_t)(v >> 32);
          } else {
            for (int t = 0; 8 * m + t < a.n_inputs; ++t) dst[t] = (uint8_t)(z >> (8 * t)) & a.in_mask[8 * m + t];
          }
        }
    }
  } else if ((a.n_inputs & 3) == 0 && ((uintptr_t)a.inputs & 3) == 0) {
    rows_to_lds<uint32_t>(reinterpret_cast<const uint32_t*>(a.inputs + s0 * a.n_inputs), ns, a.n_inputs / 4, sig,
                          a.stride, reinterpret_cast<const uint32_t*>(a.in_mask));
  } else {
    rows_to_lds<uint8_t>(a.inputs + s0 * a.n_inputs, ns, a.n_inputs, sig, a.stride, a.in_mask);
  }
  if (threadIdx.x < kNetSamples) sig[threadIdx.x * a.stride + a.n_inputs + a.n] = 0;
  __syncthreads();
  const uint32_t rowb = (uint32_t)(lane * a.stride);
  for (int lv = 0; lv < a.depth; ++lv) {
    const int kb = a.level_begin[lv], count = a.level_begin[lv + 1] - kb;
    for (int k0 = wave * kNetStep; k0 < count; k0 += nwaves * kNetStep) {
      const NetRec* R[kNetStep];
#pragma unroll
      for (int u = 0; u < kNetStep; ++u) R[u] = a.rec + kb + min(k0 + u, count - 1);  // a repeat is not written
      uint32_t c[kNetStep][FMAX];
#pragma unroll
      for (int u = 0; u < kNetStep; ++u)
#pragma unroll
        for (int j = 0; j < FMAX; ++j) c[u][j] = sig[rowb + R[u]->sig[j]];
      constexpr int G = OMAX <= 1 ? 1 : OMAX == 2 ? 2 : 4;
      uint32_t r[kNetStep], d[kNetStep][G];
#pragma unroll
      for (int u = 0; u < kNetStep; ++u) {
        const uint32_t mask = R[u]->mask, b = R[u]->b;
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < FMAX; ++j) x |= (MASK ? c[u][j] & mask : c[u][j]) << (j * b);
        r[u] = x;
        const uint32_t* tb = a.tables + R[u]->tab;  // group x >> 5 holds bit x & 31 of every plane
        if constexpr (G == 1) {
          d[u][0] = tb[x >> 5];
        } else if constexpr (G == 2) {
          const uint2 v = reinterpret_cast<const uint2*>(tb)[x >> 5];
          d[u][0] = v.x;
          d[u][G - 1] = v.y;
        } else {
          const uint4 v = reinterpret_cast<const uint4*>(tb)[x >> 5];
          d[u][0] = v.x;
          d[u][1 % G] = v.y;
          d[u][2 % G] = v.z;
        }
      }
#pragma unroll
      for (int u = 0; u < kNetStep; ++u) {
        const uint32_t sh = r[u] & 31u;
        uint32_t q = (d[u][0] >> sh) & 1u;
#pragma unroll
        for (int p = 1; p < OMAX; ++p) q |= ((d[u][p] >> sh) & 1u) << p;
        // unconditional: a repeated neuron writes the value its first copy
        // writes, and lanes past the batch write rows that are never read out
        sig[rowb + R[u]->out] = (uint8_t)q;
      }
    }
    __syncthreads();
  }
  if (a.sample) {
    // wave 0 checks the targets of its lanes' draws, reserves places for the
    // kept ones with one atomic, and copies their input rows out together
    if (wave != 0) return;
    bool ok = lane < ns;
    for (int t = 0; t < smp.n_targets; ++t) ok = ok && sig[rowb + smp.tsig[t]] == smp.tval[t];
    const uint64_t kept = __ballot(ok);
    if (kept == 0) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(smp.count, (uint32_t)__popcll(kept));
    base = __shfl(base, 0);
    uint64_t rest = kept;
    for (uint64_t pos = base; rest != 0 && pos < (uint64_t)smp.max_found; ++pos) {
      const int l = __ffsll((unsigned long long)rest) - 1;
      rest &= rest - 1;
      for (int j = lane; j < a.n_inputs; j += 64) smp.found_inputs[pos * a.n_inputs + j] = sig[l * a.stride + j];
      if (lane == 0) smp.found_draw[pos] = smp.first + (uint64_t)(s0 + l);
    }
    return;
  }
  // output rows back: the block's rows are one contiguous run of the output
  if ((a.n & 3) == 0 && (a.n_inputs & 3) == 0 && ((uintptr_t)a.out & 3) == 0)
    lds_to_rows<uint32_t>(sig + a.n_inputs, a.stride, ns, a.n / 4, reinterpret_cast<uint32_t*>(a.out + s0 * a.n));
  else
    lds_to_rows<uint8_t>(sig + a.n_inputs, a.stride, ns, a.n, a.out + s0 * a.n);
}

__global__ __launch_bounds__(256) void lutnet_repack_kernel(const RepackItem* items, int n, int G,
                                                            const uint64_t* tables, uint32_t* il) {
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const RepackItem it = items[k];
    const uint32_t* src = reinterpret_cast<const uint32_t*>(tables + it.src_word);
    for (uint32_t g = threadIdx.x; g < it.groups; g += blockDim.x)
      for (int p = 0; p < G; ++p)
        il[it.dst_dword + (uint64_t)g * G + p] = p < (int)it.o ? src[(uint64_t)p * 2 * it.W + g] : 0u;
  }
}

hipError_t launch_lutnet_repack(const RepackItem* items, int n, int G, const uint64_t* tables, uint32_t* il,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lutnet_repack_kernel, dim3((unsigned)std::min(n, 4096)), dim3(256), 0, s, items, n, G, tables,
                     il);
  return hipGetLastError();
}

long lutnet_fused_stride(int n_inputs, int n) {
  // the signals and the zero byte, rounded to an odd number of dwords
  long stride = ((long)n_inputs + n + 1 + 3) / 4 * 4;
  if ((stride / 4) % 2 == 0) stride += 4;
  return kNetSamples * stride <= kNetMaxLds ? stride : 0;
}

hipError_t launch_lutnet_fused(const NetArgs& a, const NetSample& smp, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  const long blocks = ((long)a.batch + kNetSamples - 1) / kNetSamples;
  const size_t lds = (size_t)kNetSamples * a.stride;
  const int fk = (a.fmax + 1) / 2;  // FMAX rounded up to even: 2, 4, 6, 8
#define TT_NET_LAUNCH(FM, OM)                                                                          \
  if (a.mask)                                                                                          \
    hipLaunchKernelGGL((lutnet_fused_kernel<FM, OM, true>), dim3((unsigned)blocks), dim3(kNetThreads), \
                       lds, s, a, smp);                                                                     \
  else                                                                                                 \
    hipLaunchKernelGGL((lutnet_fused_kernel<FM, OM, false>), dim3((unsigned)blocks), dim3(kNetThreads), \
                       lds, s, a, smp);                                                                     \
  break
#define TT_NET_O(FM)                \
  switch (a.omax) {                 \
    case 1: TT_NET_LAUNCH(FM, 1);   \
    case 2: TT_NET_LAUNCH(FM, 2);   \
    default: TT_NET_LAUNCH(FM, 3);  \
  }                                 \
  break
  switch (fk) {
    case 1: TT_NET_O(2);
    case 2: TT_NET_O(4);
    case 3: TT_NET_O(6);
    default: TT_NET_O(8);
  }
#undef TT_NET_O
#undef TT_NET_LAUNCH
  return hipGetLastError();
}

hipError_t launch_lutnet_level(const LutnetArgs& a, hipStream_t s) {
  const long threads = (long)a.batch * a.count;
  if (threads <= 0) return hipSuccess;
  hipLaunchKernelGGL(lutnet_level_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace tt
