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
// on F), and the lanes' lookups all land in the neuron's planes, one dword
// per plane (OMAX loads, planes past the neuron's o aliasing plane 0 and
// masked off).  The block writes its output rows at the end.
constexpr int kNetSamples = 64;
constexpr int kNetStep = 4;
constexpr int kNetThreads = 512;
constexpr long kNetMaxLds = 64 * 1024;
constexpr int kCopyBatch = 16;  // loads in flight per thread while staging rows

// rows [0, rows) of `per_row` elements each, contiguous at src, into LDS
// rows of `stride` bytes at dst
template <typename T>
__device__ __forceinline__ void rows_to_lds(const uint8_t* src_b, int rows, int per_row, uint8_t* dst, int stride) {
  const T* src = reinterpret_cast<const T*>(src_b);
  const int total = rows * per_row;
  for (int base = threadIdx.x; base < total; base += kCopyBatch * blockDim.x) {
    T v[kCopyBatch];
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int e = base + u * blockDim.x;
      v[u] = e < total ? src[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int e = base + u * blockDim.x;
      if (e < total) {
        const int r = e / per_row, c = e - r * per_row;
        reinterpret_cast<T*>(dst + r * stride)[c] = v[u];
      }
    }
  }
}

// the reverse: LDS rows of `stride` bytes at src to contiguous rows at dst
template <typename T>
__device__ __forceinline__ void lds_to_rows(const uint8_t* src, int stride, int rows, int per_row, uint8_t* dst_b) {
  T* dst = reinterpret_cast<T*>(dst_b);
  const int total = rows * per_row;
  for (int base = threadIdx.x; base < total; base += kCopyBatch * blockDim.x) {
    T v[kCopyBatch];
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int e = base + u * blockDim.x;
      if (e < total) {
        const int r = e / per_row, c = e - r * per_row;
        v[u] = reinterpret_cast<const T*>(src + r * stride)[c];
      }
    }
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int e = base + u * blockDim.x;
      if (e < total) dst[e] = v[u];
    }
  }
}

template <int FMAX, int OMAX>
__global__ __launch_bounds__(kNetThreads) void lutnet_fused_kernel(NetArgs a) {
  extern __shared__ uint8_t sig[];  // [kNetSamples][stride]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nwaves = blockDim.x >> 6;
  const long s0 = (long)blockIdx.x * kNetSamples;
  const int ns = (int)min((long)kNetSamples, (long)a.batch - s0);
  // the samples' input rows into LDS; the rows are contiguous in memory, so
  // the block walks them as one flat run, every thread issuing all of its
  // loads before its first LDS store (one memory latency, not one per row)
  if ((a.n_inputs & 3) == 0 && ((uintptr_t)a.inputs & 3) == 0)
    rows_to_lds<uint32_t>(a.inputs + s0 * a.n_inputs, ns, a.n_inputs / 4, sig, a.stride);
  else
    rows_to_lds<uint8_t>(a.inputs + s0 * a.n_inputs, ns, a.n_inputs, sig, a.stride);
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
      uint32_t r[kNetStep], d[kNetStep][OMAX];
#pragma unroll
      for (int u = 0; u < kNetStep; ++u) {
        const uint32_t mask = R[u]->mask, b = R[u]->b;
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < FMAX; ++j) x |= (c[u][j] & mask) << (j * b);
        r[u] = x;
        const uint32_t off = (x >> 5) << 2;  // the dword holding bit x of each plane
        const uint8_t* p0 = reinterpret_cast<const uint8_t*>(a.tables + R[u]->plane0);
        d[u][0] = *reinterpret_cast<const uint32_t*>(p0 + off);
        if (OMAX > 1) d[u][1 % OMAX] = *reinterpret_cast<const uint32_t*>(p0 + R[u]->plane_off[0] + off);
        if (OMAX > 2) d[u][2 % OMAX] = *reinterpret_cast<const uint32_t*>(p0 + R[u]->plane_off[1] + off);
      }
#pragma unroll
      for (int u = 0; u < kNetStep; ++u) {
        const uint32_t sh = r[u] & 31u;
        uint32_t q = (d[u][0] >> sh) & 1u;
#pragma unroll
        for (int p = 1; p < OMAX; ++p) q |= ((d[u][p] >> sh) & 1u) << p;
        q &= R[u]->qmask;
        // unconditional: a repeated neuron writes the value its first copy
        // writes, and lanes past the batch write rows that are never read out
        sig[rowb + R[u]->out] = (uint8_t)q;
      }
    }
    __syncthreads();
  }
  // output rows back: the block's rows are one contiguous run of the output
  if ((a.n & 3) == 0 && (a.n_inputs & 3) == 0 && ((uintptr_t)a.out & 3) == 0)
    lds_to_rows<uint32_t>(sig + a.n_inputs, a.stride, ns, a.n / 4, a.out + s0 * a.n);
  else
    lds_to_rows<uint8_t>(sig + a.n_inputs, a.stride, ns, a.n, a.out + s0 * a.n);
}

long lutnet_fused_stride(int n_inputs, int n) {
  // the signals and the zero byte, rounded to an odd number of dwords
  long stride = ((long)n_inputs + n + 1 + 3) / 4 * 4;
  if ((stride / 4) % 2 == 0) stride += 4;
  return kNetSamples * stride <= kNetMaxLds ? stride : 0;
}

hipError_t launch_lutnet_fused(const NetArgs& a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  const long blocks = ((long)a.batch + kNetSamples - 1) / kNetSamples;
  const size_t lds = (size_t)kNetSamples * a.stride;
  const int fk = (a.fmax + 1) / 2;  // FMAX rounded up to even: 2, 4, 6, 8
#define TT_NET_LAUNCH(FM, OM)                                                                             \
  hipLaunchKernelGGL((lutnet_fused_kernel<FM, OM>), dim3((unsigned)blocks), dim3(kNetThreads), lds, s, a); \
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
