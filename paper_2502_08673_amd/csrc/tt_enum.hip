// tt_enum.hip -- truth-table enumeration kernels for gfx950.
//
// Factored enumeration.  Row r of a neuron splits into a word index h = r/64
// and a lane l = r%64.  Because the digits of r are bit fields, digit j of
// r = 64h + l is the sum of digit j of 64h and digit j of l, so the weighted
// sum splits exactly:
//
//     a(64h + l) = bias + P_hi[h] + P_lo[l],
//     P_hi[h] = sum_j w_j * x_j(64h),   P_lo[l] = sum_j w_j * x_j(l).
//
// P_hi over all words is the dense integer GEMM (digits of the rows 64h) x
// (weights): the main kernel computes it with v_mfma_i32_32x32x16_i8, digits
// generated from h in registers (the row matrix is never stored), exact int32
// accumulation.  P_lo takes only 64 values per neuron; the prep kernel turns
// it into a table of 64-bit row masks M[e] = { l : P_lo[l] - vmin >= e }.
// Row l of word h reaches threshold t iff P_lo[l] >= t - bias - P_hi[h], so
// the whole 64-row word of a threshold is M[clamp(t - bias - vmin - P_hi[h])]:
// one LDS lookup per threshold replaces 64 compares.  ReLU only matters for
// thresholds t <= 0, which every row reaches; the prep kernel folds that in.
// The masks of the 2^o - 1 thresholds are nested, so bit p of the code q is
// the XOR of the masks whose threshold index is a multiple of 2^p.
#include "tt_internal.h"

namespace tt {

typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// One wave per neuron: P_lo, its range, the mask table and the folded
// thresholds.  Block 0 also resets the persistent work counter.
__global__ __launch_bounds__(256) void prep_kernel(EnumArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.queue) a.queue[0] = 0u;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= a.prep_count) return;
  const int n = a.prep_list ? a.prep_list[i] : i;
  const tt_neuron* dp = a.desc + n;  // fields read from global memory, no private copy
  const int F = dp->F, b = dp->b, o = dp->o;
  const int Fb = F * b;
  const int R = Fb >= 6 ? 64 : (1 << Fb);
  const bool valid = lane < R;
  const int dmask = (1 << b) - 1;
  const uint64_t wv = *reinterpret_cast<const uint64_t*>(a.desc[n].w);
  int P = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < F) P += (int)(int8_t)(uint8_t)(wv >> (8 * j)) * ((lane >> (j * b)) & dmask);
  const int vmin = wave_min_i32(valid ? P : INT32_MAX);
  const int vmax = wave_max_i32(valid ? P : INT32_MIN);
  const int cap = a.lut_cap[n];
  const int r1 = min(vmax - vmin + 1, cap - 1);
  uint64_t* lut = a.lut + a.lut_off[n];
  for (int e0 = 0; e0 <= r1; e0 += 64) {
    const int lim = min(64, r1 + 1 - e0);
    uint64_t mine = 0;
    for (int e = 0; e < lim; ++e) {
      const uint64_t m = __ballot(valid && P - vmin >= e0 + e);
      if (lane == e) mine = m;
    }
    if (lane < lim) lut[e0 + lane] = mine;
  }
  if (lane < 8) {
    int32_t val = kPosBig;
    if (lane == 0) {
      val = r1;
    } else {
      const int k = lane - 1;
      if (k < (1 << o) - 1) {
        const int64_t t = dp->thr[k];
        if (dp->act == TT_ACT_RELU && t <= 0) {
          val = kNegBig;
        } else {
          int64_t te = t - (int64_t)dp->bias - (int64_t)vmin;
          te = te < kNegBig ? kNegBig : (te > kPosBig ? kPosBig : te);
          val = (int32_t)te;
        }
      }
    }
    reinterpret_cast<int32_t*>(&a.params[n])[lane] = val;
  }
}

struct LdsSlot {
  int32_t r1, te[7];
  int32_t base, W;
  uint64_t woff;
};

template <int O>
__device__ __forceinline__ void planes_from_masks(const uint64_t* mk, uint64_t* pl) {
  if constexpr (O == 1) {
    pl[0] = mk[0];
  } else if constexpr (O == 2) {
    pl[0] = mk[0] ^ mk[1] ^ mk[2];
    pl[1] = mk[1];
  } else {
    pl[0] = mk[0] ^ mk[1] ^ mk[2] ^ mk[3] ^ mk[4] ^ mk[5] ^ mk[6];
    pl[1] = mk[1] ^ mk[3] ^ mk[5];
    pl[2] = mk[3];
  }
}

// One work item's column tiles for output width O (uniform over the block).
// Each wave takes 32-word column tiles of the item: one MFMA gives P_hi for
// 32 neurons x 32 words; lane l then owns word (l % 32) of the neurons
// 8*(v/4) + 4*(l/32) + v%4 in accumulator register v, so every store writes
// two 256-byte runs of consecutive words.
template <int O, int NW, bool NT>
__device__ __forceinline__ void enum_item(const EnumArgs& a, const WorkItem& wi, const TileInfo& ti,
                                          const LdsSlot* s_slot, const uint64_t* s_lut, long A,
                                          int lane, int wave) {
  constexpr int K = (1 << O) - 1;
  const int F = ti.F, b = ti.b, W = ti.W;
  const uint32_t dmask = (1u << b) - 1u;
  const int hend = wi.h0 + wi.count;
  for (int ct = wave; ct * kTileN < wi.count; ct += NW) {
    const int hcol = wi.h0 + ct * kTileN + (lane & 31);
    // B operand: lanes 0..31 carry the digits of row 64*hcol (k = 0..7);
    // lanes 32..63 carry k = 8..15, which are zero.
    long B = 0;
    if (lane < 32) {
      const uint32_t r = (uint32_t)hcol << 6;
      uint64_t dg = 0;
      for (int j = 0; j < F; ++j) dg |= (uint64_t)((r >> (j * b)) & dmask) << (8 * j);
      B = (long)dg;
    }
    v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(A, B, acc, 0, 0, 0);
    const bool hok = hcol < hend;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      if (hok && m < ti.count) {
        const LdsSlot& sl = s_slot[m];
        const int P = acc[v];
        const int r1 = sl.r1;
        const int base = sl.base;
        uint64_t mk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          int c = sl.te[k] - P;
          c = min(max(c, 0), r1);
          mk[k] = s_lut[base + c];
        }
        uint64_t pl[O];
        planes_from_masks<O>(mk, pl);
        uint64_t* dst = a.tables + sl.woff + (uint64_t)hcol;
#pragma unroll
        for (int p = 0; p < O; ++p) {
          if constexpr (NT)
            __builtin_nontemporal_store(pl[p], dst + (uint64_t)p * (uint64_t)W);
          else
            dst[(uint64_t)p * (uint64_t)W] = pl[p];
        }
      }
    }
  }
}

// Work item = (tile of <= 32 neurons of one (F, b, o) group, range of words).
// Static mode: block i takes item item_base + i.  Persistent mode: blocks
// pull items from an atomic counter until the queue is empty.
template <int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void enum_kernel(EnumArgs a) {
  extern __shared__ uint64_t s_lut[];
  __shared__ LdsSlot s_slot[kTileM];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int cur_tile = -1;
  int iter = 0;
  for (;;) {
    // The first barrier retires every thread's previous item (including its
    // read of s_item and all LDS reads) before the slot and tables change.
    __syncthreads();
    if (threadIdx.x == 0) {
      int it;
      if (a.persistent)
        it = (int)atomicAdd(a.queue, 1u);
      else
        it = iter == 0 ? a.item_base + (int)blockIdx.x : a.n_items;
      s_item = it;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= a.n_items) break;
    ++iter;
    const WorkItem wi = a.items[item];
    const TileInfo ti = a.tiles[wi.tile];
    if (wi.tile != cur_tile) {
      for (int m = threadIdx.x; m < ti.count; m += blockDim.x) {
        const int idx = a.tile_neuron[ti.first + m];
        const NeuronParams pr = a.params[idx];
        LdsSlot sl;
        sl.r1 = pr.r1;
#pragma unroll
        for (int k = 0; k < 7; ++k) sl.te[k] = pr.te[k];
        sl.base = a.tile_lds[ti.first + m];
        sl.W = ti.W;
        sl.woff = a.desc[idx].word_off;
        s_slot[m] = sl;
      }
      for (int m = 0; m < ti.count; ++m) {
        const int idx = a.tile_neuron[ti.first + m];
        const uint64_t* src = a.lut + a.lut_off[idx];
        const int cnt = a.params[idx].r1 + 1;
        const int base = a.tile_lds[ti.first + m];
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) s_lut[base + e] = src[e];
      }
      __syncthreads();
      cur_tile = wi.tile;
    }
    // A operand: lanes 0..31 carry the weights of tile neuron `lane` (k = 0..7).
    long A = 0;
    if (lane < 32 && lane < ti.count) {
      const int idx = a.tile_neuron[ti.first + lane];
      uint64_t wv = *reinterpret_cast<const uint64_t*>(a.desc[idx].w);
      if (ti.F < 8) wv &= (1ull << (8 * ti.F)) - 1ull;
      A = (long)wv;
    }
    switch (ti.o) {
      case 1: enum_item<1, NW, NT>(a, wi, ti, s_slot, s_lut, A, lane, wave); break;
      case 2: enum_item<2, NW, NT>(a, wi, ti, s_slot, s_lut, A, lane, wave); break;
      default: enum_item<3, NW, NT>(a, wi, ti, s_slot, s_lut, A, lane, wave); break;
    }
  }
}

hipError_t launch_prep(const EnumArgs& a, hipStream_t s) {
  if (a.prep_count <= 0) return hipSuccess;
  const int waves_per_block = 4;
  const int grid = (a.prep_count + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(prep_kernel, dim3(grid), dim3(64 * waves_per_block), 0, s, a);
  return hipGetLastError();
}

template <int NW, bool NT>
static hipError_t launch_enum_t(const EnumArgs& a, int grid, hipStream_t s) {
  const size_t lds = sizeof(uint64_t) * kLutLdsEntries;
  hipLaunchKernelGGL((enum_kernel<NW, NT>), dim3(grid), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_enum(const EnumArgs& a, int grid, int waves, int nontemporal, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (waves == 8) return nontemporal ? launch_enum_t<8, true>(a, grid, s) : launch_enum_t<8, false>(a, grid, s);
  return nontemporal ? launch_enum_t<4, true>(a, grid, s) : launch_enum_t<4, false>(a, grid, s);
}

}  // namespace tt
