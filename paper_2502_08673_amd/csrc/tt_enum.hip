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
//
// Histogram, fused: the mask of threshold k holds the rows whose code is at
// least k, so c_k = sum over words of popcount(mask_k) counts them, and
// hist[v] = c_v - c_{v+1} (c_0 = all rows, c_{2^o} = 0).  Each lane keeps
// its c_k for its neurons in registers (two 16-bit counts per register),
// each wave sums them over its word-lanes at the end of a work item and adds
// them into LDS, and the block adds the item's share of the histogram,
// c_v - c_{v+1} with c_0 = the item's rows, into hist in global memory:
// modulo-2^32 adds whose sum over the items is the histogram itself (the
// prep kernel zeroes it first), so no conversion pass follows.
#include "tt_internal.h"

namespace tt {

typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// v_writelane_b32 of a 64-bit ballot: its low and high halves (wave-uniform
// SGPRs) into lane L of lo and hi.  Not a memory access.  The halves were
// just written by the compare (a VALU instruction), and a v_writelane that
// reads such an SGPR as data in the very next instruction gets the value
// before the write (measured on this hardware: the first of the two writes
// took the previous compare's half, the second, one instruction later, the
// right one).  The compiler does not see inside the asm, so the asm waits
// two cycles itself; the lane index is an inline constant.
template <int L>
__device__ __forceinline__ void write_lanes(int& lo, int& hi, uint64_t m) {
  asm("s_nop 1\n\tv_writelane_b32 %0, %2, %4\n\tv_writelane_b32 %1, %3, %4"
      : "+v"(lo), "+v"(hi)
      : "s"((int)(uint32_t)m), "s"((int)(uint32_t)(m >> 32)), "i"(L));
}

// Mask-table entries E .. E + 7 of a 64-entry chunk into lanes E .. E + 7 of
// (lo, hi): entry e holds the rows whose pe (P - vmin - chunk start; negative
// for rows past the table) is at least e.  Straight-line, lane indices as
// constants: one compare and two lane writes per entry, no scalar work.
template <int E>
__device__ __forceinline__ void mask_entries8(int& lo, int& hi, int pe) {
  write_lanes<E>(lo, hi, __ballot(pe >= E));
  if constexpr ((E & 7) != 7) mask_entries8<E + 1>(lo, hi, pe);
}

// entries 0 .. lim - 1 of a chunk in blocks of eight (the entries past lim
// of the last block land in lanes that are not stored)
template <int E>
__device__ __forceinline__ void mask_entries(int& lo, int& hi, int pe, int lim) {
  mask_entries8<E>(lo, hi, pe);
  if constexpr (E + 8 < 64) {
    if (E + 8 < lim) mask_entries<E + 8>(lo, hi, pe, lim);
  }
}

// prep_waves waves per neuron (role r = 0 .. prep_waves - 1): P_lo, its
// range, the mask table (64-entry chunks c, taken by role c mod prep_waves),
// the folded thresholds, the tile member's slot record and the zeroed
// histogram (role 0), and, when asked, the support of a small-range neuron
// (the last role).  Several waves per neuron shorten the chain each wave
// runs when the plan has few neurons.  Block 0 also resets the persistent
// work counter.
__global__ __launch_bounds__(256) void prep_kernel(EnumArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.queue) a.queue[0] = 0u;
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; said so, later branches on it are scalar
  const int gw = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int W = a.prep_waves;
  const int i = gw / W, role = gw - (gw / W) * W;
  if (i >= a.prep_count) return;
  const int n = a.prep_list ? __builtin_amdgcn_readfirstlane(a.prep_list[i]) : i;
  // every per-neuron input in one load instruction: lanes 0..15 the
  // descriptor, lanes 16..20 the plan's entries (a plan's arguments always
  // carry the tile arrays)
  const uint32_t* src = neuron_dword(a.desc + n, lane);
  if (lane == 16) src = reinterpret_cast<const uint32_t*>(a.lut_cap + n);
  if (lane == 17) src = reinterpret_cast<const uint32_t*>(a.lut_off + n);
  if (lane == 18) src = reinterpret_cast<const uint32_t*>(a.lut_off + n) + 1;
  if (lane == 19) src = reinterpret_cast<const uint32_t*>(a.tile_pos + n);
  if (lane == 20) src = reinterpret_cast<const uint32_t*>(a.tile_lds + n);
  const uint32_t x = lane < 21 ? *src : 0u;
  const NeuronRegs d = neuron_from_lanes(x);
  const int cap = __builtin_amdgcn_readlane((int)x, 16);
  const uint64_t loff = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)x, 18) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)x, 17);
  const int tp = __builtin_amdgcn_readlane((int)x, 19);
  const int tlds = __builtin_amdgcn_readlane((int)x, 20);
  uint64_t* lut = a.lut + loff;
  const int F = d.F, b = d.b, o = d.o;
  const int Fb = F * b;
  const int R = Fb >= 6 ? 64 : (1 << Fb);
  const bool valid = lane < R;
  const int dmask = (1 << b) - 1;
  // P of row `lane` (its low six bits) and the range of P over the rows, in
  // closed form: digit j contributes w_j times any value of its bits below
  // bit min(6, F b), independently of the others
  int P = 0, vmin = 0, vmax = 0;
  const int lowb = Fb < 6 ? Fb : 6;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j < F) {
      const int w = weight_at(d.wv, j);
      P += w * ((lane >> (j * b)) & dmask);
      const int nb = min(max(lowb - j * b, 0), b);
      const int top = w * ((1 << nb) - 1);
      vmin += min(top, 0);
      vmax += max(top, 0);
    }
  }
  const int r1 = min(vmax - vmin + 1, cap - 1);
  // entry e of the mask table: the rows with P - vmin >= e (one compare per
  // entry; writelane puts the mask into lane e)
  const int pv = valid ? P - vmin : -1;
  for (int e0 = 64 * role; e0 <= r1; e0 += 64 * W) {
    const int lim = __builtin_amdgcn_readfirstlane(min(64, r1 + 1 - e0));
    int lo = 0, hi = 0;
    mask_entries<0>(lo, hi, valid ? pv - e0 : -1, lim);
    if (lane < lim) lut[e0 + lane] = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  }
  if (role == 0) {
  // tile members: the LDS slot record at the neuron's tile position
  int32_t* slot = tp >= 0 ? reinterpret_cast<int32_t*>(a.slots + tp) : nullptr;
  const int32_t thr_mine = thr_lane(d, lane >= 1 && lane <= 7 ? lane - 1 : 0);  // lane k + 1: thr[k]
  if (lane < 8) {
    int32_t val = kPosBig;
    if (lane == 0) {
      val = r1;
    } else {
      const int k = lane - 1;
      if (k < (1 << o) - 1) {
        const int64_t t = thr_mine;
        if (d.act == TT_ACT_RELU && t <= 0) {
          val = kNegBig;
        } else {
          int64_t te = t - (int64_t)d.bias - (int64_t)vmin;
          te = te < kNegBig ? kNegBig : (te > kPosBig ? kPosBig : te);
          val = (int32_t)te;
        }
      }
    }
    reinterpret_cast<int32_t*>(&a.params[n])[lane] = val;
    if (slot) slot[lane] = val;
    if (a.hist) a.hist[(size_t)n * 8 + lane] = 0u;  // histogram accumulators
  } else if (slot && lane < 14) {
    const uint64_t wm = F < 8 ? d.wv & ((1ull << (8 * F)) - 1ull) : d.wv;
    const uint64_t woff = d.word_off;
    uint32_t v = 0;
    switch (lane) {
      case 8: v = (uint32_t)tlds; break;
      case 9: v = Fb >= 6 ? 1u << (Fb - 6) : 1u; break;
      case 10: v = (uint32_t)woff; break;
      case 11: v = (uint32_t)(woff >> 32); break;
      case 12: v = (uint32_t)wm; break;
      default: v = (uint32_t)(wm >> 32); break;
    }
    slot[lane] = (int32_t)v;
  }
  }
  // the support of a small-range neuron, decided from its parameters by this
  // wave (the step's support of the plan's own tables)
  const int range = neuron_sum_range(d);
  if (role == W - 1 && a.support && range < 512) {
    const uint32_t sup = small_support_wave(d, range);
    if (lane == 0) a.support[n] = (uint8_t)sup;
  }
}

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
// two 256-byte runs of consecutive words.  Tiles of at most 4*MV/2 neurons
// only use registers v < MV.  With a histogram, the wave's threshold counts
// are added into s_cnt[m * 8 + k] (k = 1..2^O - 1) at the end.
template <int O, int NW, bool NT, int MV>
__device__ __forceinline__ void enum_item(const EnumArgs& a, const WorkItem& wi, const TileInfo& ti,
                                          const LdsSlot* s_slot, const uint64_t* s_lut, uint32_t* s_cnt, long A,
                                          int lane, int wave) {
  constexpr int K = (1 << O) - 1;
  constexpr int NC = (K + 1) / 2;  // registers of packed counts per neuron
  const bool want_hist = a.hist != nullptr;
  const int F = ti.F, b = ti.b, W = ti.W;
  const uint32_t dmask = (1u << b) - 1u;
  const int hend = wi.h0 + wi.count;
  uint32_t cnt[MV][NC];
#pragma unroll
  for (int v = 0; v < MV; ++v)
#pragma unroll
    for (int c = 0; c < NC; ++c) cnt[v][c] = 0u;
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
    for (int v = 0; v < MV; ++v) {
      const int m = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      uint32_t inc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) inc[c] = 0u;
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
#pragma unroll
        for (int k = 0; k < K; ++k) inc[k >> 1] += (uint32_t)__popcll(mk[k]) << (16 * (k & 1));
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) cnt[v][c] += inc[c];
    }
  }
  if (want_hist) {  // uniform
#pragma unroll
    for (int v = 0; v < MV; ++v) {
      const int m = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        // sum over the 32 lanes that hold neuron m (xor masks < 32 stay in the half)
        uint32_t lo = cnt[v][c] & 0xFFFFu, hi = cnt[v][c] >> 16;
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) {
          lo += (uint32_t)__shfl_xor((int)lo, off, 64);
          hi += (uint32_t)__shfl_xor((int)hi, off, 64);
        }
        if ((lane & 31) == 0 && m < ti.count) {
          if (lo) atomicAdd(&s_cnt[m * 8 + 2 * c + 1], lo);
          if (2 * c + 1 < K && hi) atomicAdd(&s_cnt[m * 8 + 2 * c + 2], hi);
        }
      }
    }
  }
}

// Work item = (tile of <= 32 neurons of one (F, b, o) group, range of words).
// Static mode: block i takes item item_base + i.  Persistent mode: blocks
// pull items from an atomic counter until the queue is empty.  Tiles hold at
// most 2 * MV neurons.
template <int NW, bool NT, int MV>
__global__ __launch_bounds__(NW * 64) void enum_kernel(EnumArgs a) {
  extern __shared__ uint64_t s_lut[];
  __shared__ LdsSlot s_slot[kTileM];
  __shared__ uint32_t s_cnt[kTileM * 8];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < kTileM * 8; t += blockDim.x) s_cnt[t] = 0u;
  int cur_tile = -1;
  int iter = 0;
  int prev_first = 0, prev_count = 0, prev_K = 0;
  uint32_t prev_rows = 0;
  for (;;) {
    // The first barrier retires every thread's previous item (including its
    // read of s_item and all LDS reads) before the slot and tables change.
    __syncthreads();
    if (a.hist && (int)threadIdx.x < prev_count) {
      // The previous item's share of the member's histogram, from its
      // threshold counts c_k (rows with code >= k; c_0 = the item's rows):
      // hist[v] += c_v - c_{v+1}, in modulo-2^32 adds whose total is the
      // histogram itself (no later pass).
      const int m = threadIdx.x;
      uint32_t c[9];
      c[0] = prev_rows;
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        c[k] = k <= prev_K ? s_cnt[m * 8 + k] : 0u;
        s_cnt[m * 8 + k] = 0u;
      }
      c[8] = 0u;
      uint32_t* h = a.hist + (size_t)a.tile_neuron[prev_first + m] * 8;
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (v <= prev_K && c[v] != c[v + 1]) atomicAdd(h + v, c[v] - c[v + 1]);
    }
    if (threadIdx.x == 0) {
      // the first item is the block's own (the queue would hand out items
      // 0 .. grid - 1 first anyway); later ones come from the queue, which
      // counts from the grid size
      int it;
      if (a.persistent)
        it = iter == 0 ? (int)blockIdx.x
                       : ((int)gridDim.x >= a.n_items ? a.n_items : (int)gridDim.x + (int)atomicAdd(a.queue, 1u));
      else
        it = iter == 0 ? a.item_base + (int)blockIdx.x : a.n_items;
      s_item = it;
    }
    __syncthreads();
    const int item = s_item;
    if (item >= a.n_items) break;
    ++iter;
    const WorkItem wi = a.items[item];
    const TileInfo& ti = wi.t;
    if (wi.tile != cur_tile) {
      // the members' slot records and their mask tables: two contiguous
      // copies issued together (no dependent loads)
      const uint32_t* ssrc = reinterpret_cast<const uint32_t*>(a.slots + ti.first);
      uint32_t* sdst = reinterpret_cast<uint32_t*>(s_slot);
      constexpr int kSlotDw = (int)(sizeof(LdsSlot) / 4);
      for (int e = threadIdx.x; e < ti.count * kSlotDw; e += blockDim.x) sdst[e] = ssrc[e];
      const uint64_t* lsrc = a.lut + (((uint64_t)ti.lut_base_hi << 32) | ti.lut_base_lo);
      for (int e = threadIdx.x; e < ti.lut_total; e += blockDim.x) s_lut[e] = lsrc[e];
      __syncthreads();
      cur_tile = wi.tile;
    }
    prev_first = ti.first;
    prev_count = ti.count;
    prev_K = (1 << ti.o) - 1;
    {
      const int Fb = (int)ti.F * (int)ti.b;
      prev_rows = (uint32_t)wi.count * (Fb >= 6 ? 64u : (1u << Fb));
    }
    // A operand: lanes 0..31 carry the weights of tile neuron `lane` (k = 0..7).
    const long A = (lane < 32 && lane < ti.count) ? (long)s_slot[lane].wv : 0L;
    switch (ti.o) {
      case 1: enum_item<1, NW, NT, MV>(a, wi, ti, s_slot, s_lut, s_cnt, A, lane, wave); break;
      case 2: enum_item<2, NW, NT, MV>(a, wi, ti, s_slot, s_lut, s_cnt, A, lane, wave); break;
      default: enum_item<3, NW, NT, MV>(a, wi, ti, s_slot, s_lut, s_cnt, A, lane, wave); break;
    }
  }
}

// Wide tables (at least 2^kWideMinLog2 words per plane), one (F, b, o) group
// per launch.  A block of NW waves takes NW * upw consecutive 256-word
// units of one neuron (unit NW k + w for wave w in step k, so the block's
// stores at any time are adjacent), copies the neuron's mask table into LDS
// once, and then computes its units with no further global load: on this
// hardware a load issued after stores waits for those stores, so no load
// follows a store.  One v_mfma_i32_16x16x32_i8 gives P_hi of a unit's 256
// words.  Product row i = 4 q + v stands for word bits 0 (v % 2), 5-6 (q)
// and 7 (v / 2), column j for word bits 1-4; a digit of a row index is
// linear in the index's bits, so with
//     A[i][k] = x_k(row part of i),  B[k][j] = w_k            (k < 8),
//     A[i][8 + k] = w_k,             B[8 + k][j] = x_k(column part of j)
// the product is P_hi.  Lane l receives rows 4 (l / 16) + v (v = 0..3) of
// column l % 16: words 2 l + v (v < 2) and 128 + 2 l + v - 2 (v >= 2) of
// the unit, so each store instruction writes one contiguous 1 KiB run
// (16 bytes per lane) and a wave two per plane.  Threshold counts: packed per lane over the
// wave's units, summed over the wave, one atomic per threshold and wave.
template <int O, int NW, bool NT>
__global__ __launch_bounds__(NW * 64) void enum_wide_kernel(EnumArgs a) {
  constexpr int K = (1 << O) - 1;
  constexpr int NC = (K + 1) / 2;
  extern __shared__ uint64_t s_lut[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int upw = a.wide_upw;
  const int per_log2 = a.wide_wb - 8;  // units per neuron: W / 256, a multiple of NW * upw
  // XCD-aware order: blocks go round-robin to the eight XCDs, so block b
  // takes slot (b mod 8) * G/8 + b / 8 and each XCD writes one contiguous
  // eighth of the group's tables (a plain 2 GiB store stream measured 6.7
  // TB/s this way against 6.2 TB/s in launch order).  A tail of fewer than
  // eight blocks keeps its own slots.
  const uint32_t G8 = gridDim.x & ~7u;
  const uint32_t slot = blockIdx.x < G8 ? (blockIdx.x & 7u) * (G8 >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const long u0 = (long)slot * NW * upw;
  const int n = a.wide_list[u0 >> per_log2];
  const uint32_t hb = (uint32_t)(u0 & ((1L << per_log2) - 1)) << 8;  // the block's first word
  const tt_neuron* dp = a.desc + n;
  // bias, F and b share one aligned dword: a single scalar load
  static_assert(offsetof(tt_neuron, bias) % 4 == 0 && offsetof(tt_neuron, F) == offsetof(tt_neuron, bias) + 2 &&
                    offsetof(tt_neuron, b) == offsetof(tt_neuron, bias) + 3,
                "descriptor layout");
  const uint32_t fbw = *reinterpret_cast<const uint32_t*>(&dp->bias);
  const int F = (int)((fbw >> 16) & 0xFFu), b = (int)(fbw >> 24);
  const uint32_t dmask = (1u << b) - 1u;
  uint64_t wv = *reinterpret_cast<const uint64_t*>(dp->w);
  if (F < 8) wv &= (1ull << (8 * F)) - 1ull;
  const NeuronParams pr = a.params[n];
  const uint64_t* lut = a.lut + a.lut_off[n];
  for (int e = threadIdx.x; e <= pr.r1; e += blockDim.x) s_lut[e] = lut[e];
  __shared__ uint32_t s_cnt[8];
  if (threadIdx.x < 8) s_cnt[threadIdx.x] = 0u;
  const uint64_t W = 1ull << a.wide_wb;
  const uint64_t woff = dp->word_off;
  // digits of the column part (lanes 16-31), the same for every unit
  uint64_t dgc = 0;
  {
    const uint32_t r = (uint32_t)(lane & 15) << 7;  // word 2 j, row 64 * 2 j
    for (int j = 0; j < F; ++j) dgc |= (uint64_t)((r >> (j * b)) & dmask) << (8 * j);
  }
  __syncthreads();
  uint32_t cnt[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) cnt[c] = 0u;
  for (int k = 0; k < upw; ++k) {
    const uint32_t h0 = hb + ((uint32_t)(NW * k + wave) << 8);
    long A = 0, B = 0;
    if (lane < 16) {
      const uint32_t r = (h0 + (uint32_t)(lane & 1) + ((uint32_t)(lane >> 2) << 5) + ((uint32_t)((lane >> 1) & 1) << 7))
                         << 6;
      uint64_t dg = 0;
      for (int j = 0; j < F; ++j) dg |= (uint64_t)((r >> (j * b)) & dmask) << (8 * j);
      A = (long)dg;
      B = (long)wv;
    } else if (lane < 32) {
      A = (long)wv;
      B = (long)dgc;
    }
    v4i acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(A, B, acc, 0, 0, 0);
    uint64_t pl[4][O];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int P = acc[v];
      uint64_t mk[K];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        int c = pr.te[q] - P;
        c = min(max(c, 0), pr.r1);
        mk[q] = s_lut[c];
      }
      planes_from_masks<O>(mk, pl[v]);
#pragma unroll
      for (int q = 0; q < K; ++q) cnt[q >> 1] += (uint32_t)__popcll(mk[q]) << (16 * (q & 1));
    }
    uint64_t* dst = a.tables + woff + h0 + 2u * (uint32_t)lane;
    if ((woff & 1ull) == 0) {  // uniform: 16-byte aligned runs
#pragma unroll
      for (int p = 0; p < O; ++p) {
        u64x2* q = reinterpret_cast<u64x2*>(dst + (uint64_t)p * W);
        if constexpr (NT) {
          __builtin_nontemporal_store(u64x2{pl[0][p], pl[1][p]}, q);
          __builtin_nontemporal_store(u64x2{pl[2][p], pl[3][p]}, q + 64);
        } else {
          q[0] = u64x2{pl[0][p], pl[1][p]};
          q[64] = u64x2{pl[2][p], pl[3][p]};
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < O; ++p)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          uint64_t* d = dst + (uint64_t)p * W + (v >> 1) * 128 + (v & 1);
          if constexpr (NT)
            __builtin_nontemporal_store(pl[v][p], d);
          else
            *d = pl[v][p];
        }
    }
  }
  if (a.hist) {  // uniform
    // a lane counts at most 4 * 64 * upw <= 2^13 rows per threshold, so the
    // packed halves do not overflow; the wave sums run in 32 bits.  Lane q
    // of each wave adds the sum of threshold q + 1 into LDS; the block then
    // adds its share of the neuron's histogram, c_v - c_{v+1} with c_0 = its
    // rows, in at most 2^O global adds (modulo 2^32; the sum over the
    // neuron's blocks is the histogram).  About a hundred blocks share a
    // neuron's eight counters over the whole launch, so the adds do not
    // contend.  (The barrier does not wait for the block's table stores.)
    uint32_t mine = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uint32_t lo = cnt[c] & 0xFFFFu, hi = cnt[c] >> 16;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        lo += (uint32_t)__shfl_xor((int)lo, off, 64);
        hi += (uint32_t)__shfl_xor((int)hi, off, 64);
      }
      if (lane == 2 * c) mine = lo;
      if (lane == 2 * c + 1) mine = hi;
    }
    if (lane < K) atomicAdd(&s_cnt[lane], mine);
    __syncthreads();
    if ((int)threadIdx.x <= K) {
      const int v = threadIdx.x;
      const uint32_t cv = v == 0 ? (uint32_t)(NW * upw) << 14 : s_cnt[v - 1];
      const uint32_t cn = v < K ? s_cnt[v] : 0u;
      if (cv != cn) atomicAdd(&a.hist[(size_t)n * 8 + v], cv - cn);
    }
  }
}

// prep_waves waves per neuron of the list, four waves per block.
hipError_t launch_prep(const EnumArgs& a, hipStream_t s) {
  if (a.prep_count <= 0) return hipSuccess;
  if (a.prep_waves < 1 || a.prep_waves > 64) return hipErrorInvalidValue;
  const int waves_per_block = 4;
  const long waves = (long)a.prep_count * a.prep_waves;
  const int grid = (int)((waves + waves_per_block - 1) / waves_per_block);
  hipLaunchKernelGGL(prep_kernel, dim3(grid), dim3(64 * waves_per_block), 0, s, a);
  return hipGetLastError();
}

template <int NW, bool NT, int MV>
static hipError_t launch_enum_t(const EnumArgs& a, int grid, hipStream_t s) {
  // LDS for the largest tile's mask tables only: small tables leave room for
  // more resident blocks
  const int entries = a.tile_lut_max > 0 && a.tile_lut_max < kLutLdsEntries ? a.tile_lut_max : kLutLdsEntries;
  const size_t lds = sizeof(uint64_t) * (size_t)entries;
  hipLaunchKernelGGL((enum_kernel<NW, NT, MV>), dim3(grid), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

template <int MV>
static hipError_t launch_enum_mv(const EnumArgs& a, int grid, int waves, int nontemporal, hipStream_t s) {
  if (waves == 8)
    return nontemporal ? launch_enum_t<8, true, MV>(a, grid, s) : launch_enum_t<8, false, MV>(a, grid, s);
  return nontemporal ? launch_enum_t<4, true, MV>(a, grid, s) : launch_enum_t<4, false, MV>(a, grid, s);
}

hipError_t launch_enum(const EnumArgs& a, int grid, int waves, int nontemporal, int tile_neurons, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (tile_neurons <= 8) return launch_enum_mv<4>(a, grid, waves, nontemporal, s);
  if (tile_neurons <= 16) return launch_enum_mv<8>(a, grid, waves, nontemporal, s);
  return launch_enum_mv<16>(a, grid, waves, nontemporal, s);
}

template <int NW, bool NT>
static hipError_t launch_enum_wide_t(const EnumArgs& a, int o, hipStream_t s) {
  if (a.wide_count <= 0) return hipSuccess;
  if (a.wide_wb < kWideMinLog2 || a.wide_wb > 24) return hipErrorInvalidValue;
  const long units = (long)a.wide_count << (a.wide_wb - 8);
  const long per_block = (long)NW * a.wide_upw;
  if (a.wide_upw < 1 || a.wide_upw > kWideMaxUpw || (a.wide_upw & (a.wide_upw - 1)) ||
      per_block > (1L << (a.wide_wb - 8)) || a.wide_lds < 1 || a.wide_lds > kMaxLutCap)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(units / per_block));
  const size_t lds = sizeof(uint64_t) * (size_t)a.wide_lds;
  switch (o) {
    case 1: hipLaunchKernelGGL((enum_wide_kernel<1, NW, NT>), grid, dim3(NW * 64), lds, s, a); break;
    case 2: hipLaunchKernelGGL((enum_wide_kernel<2, NW, NT>), grid, dim3(NW * 64), lds, s, a); break;
    default: hipLaunchKernelGGL((enum_wide_kernel<3, NW, NT>), grid, dim3(NW * 64), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_enum_wide(const EnumArgs& a, int o, int waves, int nontemporal, hipStream_t s) {
  if (nontemporal)
    return waves == 8 ? launch_enum_wide_t<8, true>(a, o, s) : launch_enum_wide_t<4, true>(a, o, s);
  return waves == 8 ? launch_enum_wide_t<8, false>(a, o, s) : launch_enum_wide_t<4, false>(a, o, s);
}

}  // namespace tt
