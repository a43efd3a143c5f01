// tt_internal.h -- structures shared by the host planner and the HIP kernels
// of libtt.so (never installed; the public interface is include/tt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tt.h"

namespace tt {

// Enumeration tiles: 32 neurons (the M side of a 32x32x16 int8 MFMA) share a
// work item; the N side is 32 consecutive 64-row table words.
constexpr int kTileM = 32;
constexpr int kTileN = 32;
// Per-tile budget of LDS mask-table entries (uint64 each): 48 KiB.
constexpr int kLutLdsEntries = 6144;
// Largest mask table of one neuron: the low six row bits span at most
// 18 * 128 + 1 distinct sums (b = 4: 15*|w0| + 3*|w1|, int8 weights down to
// -128), plus the all-zero sentinel entry.
constexpr int kMaxLutCap = 18 * 128 + 2;
constexpr int32_t kNegBig = -(1 << 30);
constexpr int32_t kPosBig = (1 << 30);

// Per-neuron parameters written by the prep kernel (32 bytes).
// r1 = index of the all-zero mask entry (range + 1); te[k] = t_k - bias - vmin,
// so that row l of word h reaches threshold k iff
// P_lo[l] - vmin >= te[k] - P_hi[h], i.e. iff bit l of lut[clamp(te[k] - P_hi, 0, r1)].
struct NeuronParams {
  int32_t r1;
  int32_t te[7];
};

// A tile: neurons of one (F, b, o) group (host built).  Its members' mask
// tables lie back to back in the pool from lut_base, in member order, so the
// LDS copy of a tile is one contiguous read.
struct TileInfo {
  int32_t first;     // offset into the tile-neuron list (multiple of kTileM)
  int32_t count;     // neurons in the tile, 1..32
  int32_t W;         // words per plane
  int32_t lut_total; // LDS mask entries used by the tile
  uint8_t F, b, o, pad;
  uint32_t lut_base_lo, lut_base_hi;  // first pool entry of the tile's mask tables
  int32_t pad2;
};

// What the tile kernel keeps in LDS for each member of its current tile,
// written by the prep kernel at the member's tile position (56 bytes).
struct LdsSlot {
  int32_t r1, te[7];  // as NeuronParams
  int32_t base, W;    // LDS entry of the member's mask table; words per plane
  uint64_t woff;      // word_off of plane 0
  uint64_t wv;        // weights, entries j >= F zeroed
};

// A work item carries a copy of its tile's record, so a block fetches both
// with one load.
struct WorkItem {
  int32_t tile;
  int32_t h0;     // first word
  int32_t count;  // words
  int32_t pad;
  TileInfo t;     // == tiles[tile]
};

// Everything the enumeration kernels read, all in one plan workspace.
struct EnumArgs {
  const tt_neuron* desc;       // [n]
  const uint64_t* lut_off;     // [n] offset of each neuron's mask table in lut
  const int32_t* lut_cap;      // [n] entries reserved for it (range + 2)
  NeuronParams* params;        // [n]
  uint64_t* lut;               // mask-table pool
  const TileInfo* tiles;       // [n_tiles]
  const int32_t* tile_neuron;  // [n_tiles * 32], -1 padded
  const int32_t* tile_lds;     // [n] LDS entry base of each tile member's mask table
  const int32_t* tile_pos;     // [n] position of the neuron in the tile-neuron list, -1: none
  LdsSlot* slots;              // [n_tiles * 32] per tile position, written by the prep kernel
  int32_t tile_lut_max;        // largest lut_total of any tile (LDS entries the tile kernel needs)
  uint8_t* support;            // prep kernel: support of the small-range neurons (NULL: none)
  const WorkItem* items;       // [n_items]
  uint32_t* queue;             // persistent work counter
  const int32_t* prep_list;    // neurons to prepare (NULL: 0..prep_count-1)
  int32_t prep_count;
  int32_t prep_waves;          // waves per neuron in the prep kernel (>= 1; see prep_kernel)
  int32_t n_items;
  int32_t item_base;           // static mode: first item of this launch
  int32_t persistent;
  uint64_t* tables;
  uint32_t* hist;              // [n * 8] histogram, accumulated by the kernels (NULL: none)
  const int32_t* wide_list;    // launch_enum_wide: the neurons of one wide group
  int32_t wide_count;
  int32_t wide_wb;             // log2 of its words per plane (>= kWideMinLog2)
  int32_t wide_upw;            // 256-word units per wave (power of two, waves * upw <= W / 256)
  int32_t wide_lds;            // LDS mask entries: the group's largest table
};

// Groups with at least 2^kWideMinLog2 words per plane are enumerated by the
// wide kernel: blocks of 4 or 8 waves, 256 words of one neuron per wave and step.
constexpr int kWideMinLog2 = 12;
constexpr int kWideMaxUpw = 32;  // 2^15 words per block

// Support / histogram of packed tables (see tt_support.hip).
struct SupportArgs {
  const tt_neuron* desc;
  const uint64_t* tables;
  uint32_t* found;           // [n] row bits whose flip changes some code
  uint32_t* hist;            // [n * 8] or NULL
  uint8_t* support;          // [n] or NULL
  int32_t n;
  int32_t n_large;           // neurons of more than kSmallTableWords words:
  const int32_t* large;      // [n_large], handled wave by wave (the rest lane by lane)
};
constexpr int kSmallTableWords = 16;  // tables up to 2^10 rows: one lane each

struct PackArgs {
  const tt_neuron* desc;
  const uint8_t* codes;
  const uint64_t* code_off;  // [n]
  const int32_t* item_neuron;
  const int32_t* item_h0;    // first word of the item
  int32_t n_items;
  int32_t words_per_item;    // words per item (64 per wave)
  uint64_t* tables;
};

// Bits l of a 64-row word whose partner l + 2^i differs in row bit i only
// (row bit i of l clear), i < 6.
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

// Row bits of the digits that have no found bit yet.
__device__ __forceinline__ uint32_t unknown_row_bits(uint32_t found, int F, int b) {
  uint32_t need = 0;
  for (int j = 0; j < F; ++j) {
    const uint32_t D = ((1u << b) - 1u) << (j * b);
    if (!(found & D)) need |= D;
  }
  return need;
}

// a 64-bit value from lane src (an LDS permute per half)
__device__ __forceinline__ uint64_t shfl64_lane(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// v of lane l - 1 in lane l (a DPP row shift by one: no LDS round trip);
// the first lane of each 16-lane row gets 0.
__device__ __forceinline__ uint64_t prev_lane64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x111, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x111, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// A descriptor's fields in registers, read once by the wave, so later steps
// make no further memory round trips for them.
struct NeuronRegs {
  uint64_t wv;        // weights, byte j = w_j
  int32_t bias, F, b, o, act;
  uint64_t word_off;
  uint32_t raw;       // dword `lane` of the descriptor (lanes 0..15): thr[k] is dword 2 + k
};

static_assert(sizeof(tt_neuron) == 64 && offsetof(tt_neuron, thr) == 8 && offsetof(tt_neuron, bias) == 36 &&
                  offsetof(tt_neuron, F) == 38 && offsetof(tt_neuron, b) == 39 && offsetof(tt_neuron, o) == 40 &&
                  offsetof(tt_neuron, act) == 41 && offsetof(tt_neuron, word_off) == 48,
              "neuron_from_lanes reads the descriptor as 16 dwords");

// Dword `lane` of a descriptor (lanes 0..15): with the wave's other loads in
// the same instruction, the wave waits for memory once.
__device__ __forceinline__ const uint32_t* neuron_dword(const tt_neuron* dp, int lane) {
  return reinterpret_cast<const uint32_t*>(dp) + (lane & 15);
}

// The fields from the dwords held by lanes 0..15 (wave-uniform results).
__device__ __forceinline__ NeuronRegs neuron_from_lanes(uint32_t x) {
  auto at = [&](int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); };
  NeuronRegs r;
  r.raw = x;
  r.wv = ((uint64_t)at(1) << 32) | at(0);
  const uint32_t w9 = at(9), w10 = at(10);
  r.bias = (int32_t)(int16_t)(uint16_t)(w9 & 0xFFFFu);
  r.F = (int32_t)((w9 >> 16) & 0xFFu);
  r.b = (int32_t)(w9 >> 24);
  r.o = (int32_t)(w10 & 0xFFu);
  r.act = (int32_t)((w10 >> 8) & 0xFFu);
  r.word_off = ((uint64_t)at(13) << 32) | at(12);
  return r;
}

// One wave reads a descriptor (every lane gets the same fields).
__device__ __forceinline__ NeuronRegs load_neuron(const tt_neuron* dp) {
  const int lane = threadIdx.x & 63;
  const uint32_t x = lane < 16 ? *neuron_dword(dp, lane) : 0u;
  return neuron_from_lanes(x);
}

// thr[k] for a wave-uniform k, and for a k that differs by lane (k in 0..6)
__device__ __forceinline__ int32_t thr_uniform(const NeuronRegs& d, int k) {
  return __builtin_amdgcn_readlane((int)d.raw, 2 + k);
}
__device__ __forceinline__ int32_t thr_lane(const NeuronRegs& d, int k) {
  return __shfl((int)d.raw, 2 + k, 64);
}

__device__ __forceinline__ int weight_at(uint64_t wv, int j) { return (int)(int8_t)(uint8_t)(wv >> (8 * j)); }

__device__ __forceinline__ int neuron_sum_range(const NeuronRegs& d) {
  const int dmax = (1 << d.b) - 1;
  int R = 0;
  for (int k = 0; k < d.F; ++k) {
    const int w = weight_at(d.wv, k);
    R += (w < 0 ? -w : w) * dmax;
  }
  return R;
}

// Support of a neuron whose sums span fewer than 64 values: every set of
// reachable sums fits one 64-bit word, so lane 8j + k builds the set of digit
// j's complement in a register (no cross-lane traffic) and tests threshold k.
// All shifts stay below 64: each step adds |w_i| * 2^m <= |w_i| * (2^b - 1),
// which is at most the range.
__device__ __forceinline__ uint32_t tiny_support_wave(const NeuronRegs& d) {
  const int lane = threadIdx.x & 63, k = lane & 7, j = lane >> 3;
  const int F = d.F, b = d.b;
  const int K = (1 << d.o) - 1, dmax = (1 << b) - 1;
  const int wj = j < F ? weight_at(d.wv, j) : 0;
  uint64_t S = 1ull;
  int64_t base = d.bias;
  for (int i2 = 0; i2 < F; ++i2) {
    const int wi = weight_at(d.wv, i2);
    if (wi == 0) continue;
    const int aw = wi < 0 ? -wi : wi;
    const bool other = i2 != j;
    if (other && wi < 0) base += (int64_t)wi * dmax;
    for (int m = 0; m < b; ++m) {
      const uint64_t t = S | (S << (aw << m));
      S = other ? t : S;
    }
  }
  bool hit = false;
  const int64_t t = thr_lane(d, k < 7 ? k : 6);  // every lane takes part in the exchange
  if (wj != 0 && k < K) {
    if (!(d.act == TT_ACT_RELU && t < 1)) {
      const int64_t D = (int64_t)(wj < 0 ? -wj : wj) * dmax;
      int64_t lo = (wj > 0 ? t - D : t) - base, hi = (wj > 0 ? t - 1 : t + D - 1) - base;
      if (lo < 0) lo = 0;
      if (hi > 63) hi = 63;
      if (lo <= hi) {
        const uint64_t mask = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & ~((1ull << lo) - 1ull);
        hit = (S & mask) != 0ull;
      }
    }
  }
  const uint64_t bal = __ballot(hit);
  uint32_t sup = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g)
    if ((bal >> (8 * g)) & 0xFFull) sup |= 1u << g;
  return sup;
}

// Support of a neuron decided from its parameters (its tables being its own
// enumeration) by one wave, for neurons whose sums span fewer than 512
// values: sum_j |w_j| (2^b - 1) < 512.  q is non-decreasing in the
// pre-activation and jumps exactly at the thresholds (those >= 1 under
// ReLU); digit j matters iff some sum s of bias and the other digits puts a
// jump point t inside the range s + w_j x_j sweeps (lo < t <= hi).  Lane
// group g (8 lanes, 8 words = 512 bits) holds the set of those sums for
// digit g as offsets from its minimum, built by shift-ORs (x_i is the sum of
// its bits), every shift inside the group.  Returns the support bits
// (wave-uniform).
// range: neuron_sum_range(d), which must be below 512 (below 64: the
// one-register form above).
__device__ __forceinline__ uint32_t small_support_wave(const NeuronRegs& d, int range) {
  if (range < 64) return tiny_support_wave(d);
  const int lane = threadIdx.x & 63, li = lane & 7, j = lane >> 3;
  const int F = d.F, b = d.b;
  const int K = (1 << d.o) - 1, dmax = (1 << b) - 1;
  const int wj = j < F ? weight_at(d.wv, j) : 0;  // this group's digit weight
  const bool mine = wj != 0;  // the group has a digit to decide
  // all groups step through the digits together; the group of digit i
  // leaves its set unchanged
  uint64_t S = li == 0 ? 1ull : 0ull;
  int64_t base = d.bias;
  int R = 0;
  for (int i2 = 0; i2 < F; ++i2) {
    const int wi = weight_at(d.wv, i2);
    if (wi == 0) continue;
    const int aw = wi < 0 ? -wi : wi;
    if (i2 != j) {
      base += (int64_t)(wi < 0 ? wi : 0) * dmax;
      R += aw * dmax;
    }
    for (int m = 0; m < b; ++m) {
      const int a = aw << m, q = a >> 6, r = a & 63;
      uint64_t t1, t2;
      if (q == 0) {
        // a shift below 64 (every step when |w| 2^(b-1) < 64): the word
        // itself and the group's previous word, moved by DPP
        const uint64_t v2 = prev_lane64(S);
        t1 = S;
        t2 = li >= 1 ? v2 : 0ull;
      } else {
        const int g0 = lane & ~7;
        const uint64_t v1 = shfl64_lane(S, g0 + ((li - q) & 7)), v2 = shfl64_lane(S, g0 + ((li - q - 1) & 7));
        t1 = li >= q ? v1 : 0ull;
        t2 = li >= q + 1 ? v2 : 0ull;
      }
      const uint64_t out = S | (t1 << r) | (r ? (t2 >> (64 - r)) : 0ull);
      if (i2 != j) S = out;
    }
  }
  const int64_t D = (int64_t)(wj < 0 ? -wj : wj) * dmax;
  bool hit = false;
  for (int k = 0; k < K; ++k) {
    const int64_t t = thr_uniform(d, k);
    if (d.act == TT_ACT_RELU && t < 1) continue;
    // s with s < t <= s + D (w_j > 0) or s - D < t <= s (w_j < 0)
    int64_t lo = wj > 0 ? t - D : t, hi = wj > 0 ? t - 1 : t + D - 1;
    lo -= base;
    hi -= base;
    if (lo < 0) lo = 0;
    if (hi > R) hi = R;
    const int64_t k0 = (int64_t)li * 64;
    const int64_t a2 = lo > k0 ? lo : k0, e2 = hi < k0 + 63 ? hi : k0 + 63;
    if (mine && a2 <= e2) {
      const int sa = (int)(a2 - k0), se = (int)(e2 - k0);
      const uint64_t mask = (se == 63 ? ~0ull : ((1ull << (se + 1)) - 1ull)) & ~((1ull << sa) - 1ull);
      hit |= (S & mask) != 0ull;
    }
  }
  const uint64_t bal = __ballot(hit);
  uint32_t sup = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g)
    if ((bal >> (8 * g)) & 0xFFull) sup |= 1u << g;
  return sup;
}

// Launchers (tt_enum.hip / tt_support.hip); return hipError_t.
hipError_t launch_prep(const EnumArgs& a, hipStream_t s);
hipError_t launch_enum(const EnumArgs& a, int grid, int waves, int nontemporal, int tile_neurons, hipStream_t s);
hipError_t launch_enum_wide(const EnumArgs& a, int o, int waves, int nontemporal, hipStream_t s);
hipError_t launch_support_params(const tt_neuron* desc, const int32_t* list, int n, uint8_t* support,
                                 hipStream_t s);
hipError_t launch_support_params_small(const tt_neuron* desc, const int32_t* list, int count, uint8_t* support,
                                       hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_support_finish(const SupportArgs& a, hipStream_t s);
hipError_t launch_support_tasks(const SupportArgs& a, int units_per_neuron, int32_t* list, uint32_t* count,
                                hipStream_t s);
hipError_t launch_hist_tables(const SupportArgs& a, int units_per_neuron, hipStream_t s);
hipError_t launch_small_tables(const SupportArgs& a, hipStream_t s);
hipError_t launch_pack(const PackArgs& a, hipStream_t s);

// Networks evaluated through their tables (tt_lutnet.hip).
struct LutnetArgs {
  const tt_neuron* desc;     // [n]
  const int32_t* fanin;      // [n][8] signal indices
  const int32_t* level;      // the neurons of this launch's level
  int32_t count;             // how many
  int32_t n_inputs, n, batch;
  const uint64_t* tables;
  const uint8_t* inputs;     // [batch][n_inputs]
  uint8_t* out;              // [batch][n]
};
hipError_t launch_lutnet_level(const LutnetArgs& a, hipStream_t s);

// One neuron of a network evaluated in a single launch: 64 bytes, read with
// scalar loads, built on the host in level order.
struct NetRec {
  uint64_t tab;     // dword offset of the neuron's interleaved table
  uint32_t out;     // the neuron's byte in a signal row (n_inputs + i)
  uint32_t mask;    // 2^b - 1
  uint32_t b;
  uint32_t pad[3];
  uint32_t sig[8];  // fan-in bytes in a signal row; past F, the row's zero byte
};
static_assert(sizeof(NetRec) == 64, "NetRec is one 64-byte scalar load");
// The single-launch form reads a copy of the tables with the planes
// interleaved: dword g of every plane side by side, G = 1, 2 or 4 dwords per
// group for a network whose largest o is 1, 2 or 3 (planes past a neuron's o
// are zero), so that one load returns a row's bit of every plane.
struct RepackItem {
  uint64_t src_word;   // the neuron's word_off
  uint64_t dst_dword;  // its NetRec::tab
  uint32_t W, o, groups, pad;
};
struct NetArgs {
  const NetRec* rec;          // [n] in level order
  const int32_t* level_begin; // [depth + 1]
  int32_t depth, n_inputs, n, batch;
  int32_t stride;             // signal row in LDS, bytes
  int32_t fmax, omax;         // largest F and o of the network
  int32_t mask;               // readers mask codes to their digits (else every code already fits)
  const uint8_t* in_mask;     // [n_inputs] (8-byte aligned): input code masks applied when staging
  const uint32_t* tables;     // the interleaved copy
  const uint8_t* inputs;      // [batch][n_inputs]
  uint8_t* out;               // [batch][n]
  int32_t sample;             // draw the inputs and keep the draws that meet the targets (NetSample)
};
constexpr int kNetMaxTargets = 64;
// Sampling: draw d's input j is byte j % 8 of the SplitMix64 output number
// d * Q + j / 8 + 1 of the stream seeded with seed, Q = ceil(n_inputs / 8),
// reduced as the staging reduces input codes; a draw is kept when every
// target signal carries its value.
struct NetSample {
  uint64_t seed, first;    // draws first .. first + batch - 1
  uint8_t* found_inputs;   // [max_found][n_inputs]
  uint64_t* found_draw;    // [max_found]
  uint32_t* count;         // kept draws, added to
  int32_t max_found, n_targets;
  uint16_t tsig[kNetMaxTargets];
  uint8_t tval[kNetMaxTargets];
};
inline int net_group(int omax) { return omax <= 1 ? 1 : omax == 2 ? 2 : 4; }
// LDS row stride of the single-launch form, 0 when the network's signals do
// not fit (then one launch per level)
long lutnet_fused_stride(int n_inputs, int n);
hipError_t launch_lutnet_repack(const RepackItem* items, int n, int G, const uint64_t* tables, uint32_t* il,
                                hipStream_t s);
hipError_t launch_lutnet_fused(const NetArgs& a, const NetSample& smp, hipStream_t s);

// CNF transformation (tt_cnf.hip).
constexpr int kCnfMaxVars = TT_CNF_MAX_VARS;
struct CnfArgs {
  const int32_t* lits;
  const int32_t* clause_off;    // global clause index -> first literal
  const int32_t* inst_off;      // instance -> first global clause
  const int32_t* clause_reach;  // global clause -> last clause (instance-local) using any of its variables
  const int32_t* var_off;       // instance -> first class byte
  const int32_t* n_vars;
  const int32_t* order;         // block -> instance, by decreasing clause count (long walks start first)
  uint8_t* var_class;
  tt_cnf_expr* expr;
  int32_t* n_expr;
  int32_t* status;
  int32_t n_inst;
  int32_t stage_clauses, stage_lits;  // the largest instance's clause and literal counts
};
hipError_t launch_cnf_transform(const CnfArgs& a, int max_vars, hipStream_t s);

// Learned screen: BF16 MLP (tt_mlp.hip).
hipError_t mlp_forward(const uint16_t* x, int Bn, int in, const uint16_t* w, const float* bias, int out, int relu,
                       uint16_t* yb, float* yf, hipStream_t s);
hipError_t mlp_infer(const uint16_t* x, int n, const uint16_t* const* w, const float* const* b, float* logits,
                     hipStream_t s, const tt_neuron* desc = nullptr, int gated = 0);
hipError_t mlp_backward(const uint16_t* dy, int Bn, int out, const uint16_t* w, int in, const uint16_t* x,
                        int mask_relu, uint16_t* dx, float* dw, float* db, float* scratch, hipStream_t s);
size_t mlp_backward_scratch_floats(int Bn, int dim);
hipError_t mlp_loss(const float* z, int Bn, const float* y, const float* m, const float* h, uint16_t* dz,
                    float* loss, float* scratch, hipStream_t s);
constexpr int kAdamMaxTensors = 8;
hipError_t adam_step_multi(int count, float* const* p, const float* const* g, float* const* m, float* const* v,
                           uint16_t* const* pb, const size_t* n, float lr, float b1, float b2, float eps, float bc1,
                           float bc2, hipStream_t s);
hipError_t adam_step(float* p, const float* g, float* m, float* v, uint16_t* pb, size_t n, float lr, float b1,
                     float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t screen_features(const tt_neuron* d, int n, uint16_t* x, hipStream_t s);
hipError_t cast_bf16(const float* x, uint16_t* y, size_t n, hipStream_t s);
hipError_t screen_labels(const tt_neuron* d, int n, const uint8_t* sup, const uint32_t* hist, float* y, float* m,
                         float* h, hipStream_t s);

// Device-resident screening (tt_screen.hip).
hipError_t small_enumerate(const tt_neuron* d, int n, const uint8_t* active, uint64_t* tables, uint64_t total,
                           uint32_t* status, hipStream_t s);
hipError_t small_support(const tt_neuron* d, int n, const uint64_t* tables, uint64_t total, uint8_t* sup,
                         uint32_t* hist, uint32_t* status, hipStream_t s);
hipError_t screen_expand(const tt_neuron* d, int n, const uint8_t* mask, const uint8_t* mode, const uint8_t* accept,
                         const tt_neuron* res, const uint64_t* screened, uint64_t* full, hipStream_t s);
// One wave per candidate: predicted support, reduced tables with the exact
// check, fallback, support and histogram (plain: every candidate in full).
struct FusedArgs {
  const tt_neuron* desc;
  int n;
  int plain;
  const float* logits;
  float tau_logit;
  const uint8_t* force_mask;
  uint64_t* tables;
  uint64_t total_words;
  uint8_t* support;
  uint32_t* hist;
  tt_neuron* res;
  uint8_t* mask;
  uint8_t* mode;
  uint8_t* accept;
  uint32_t* status;
  uint8_t* mask_out;    // caller's copies of mask / accept, or NULL
  uint8_t* accept_out;
  int32_t* list;        // candidates left for the wave-per-candidate kernel
  uint32_t* list_count; // (zeroed before the lane kernel)
};
hipError_t screen_fused(const FusedArgs& a, hipStream_t s);

}  // namespace tt
