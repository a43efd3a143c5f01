// tt_screen.hip -- device-resident screening of candidate neurons (gfx950).
//
// The learned screen predicts, for each candidate, a set S of inputs that
// may matter.  Let T be the other inputs.  The code q is a non-decreasing
// function of the pre-activation a (ReLU and the threshold count are both
// monotone), and a = bias + a_S + a_T where a_T ranges over an interval
// whose ends, min_T = sum_{j in T} min(w_j, 0) * (2^b - 1) and the matching
// max_T, are both reached.  So the table does not depend on T iff, for every
// assignment of S, q(bias + a_S + min_T) = q(bias + a_S + max_T): the tables
// of two reduced neurons over S alone, with biases bias + min_T and
// bias + max_T, must be identical.  That costs 2 * 2^(|S| b) row-evaluations
// instead of 2^(F b), and it is exact: when it fails the candidate is
// enumerated in full.  An accepted candidate's full table is the reduced
// table broadcast over T, its histogram the reduced one times 2^(|T| b).
//
// Everything here reads descriptors from device memory, one block per
// neuron, for neurons with F*b <= 16 (at most 1024 words per plane), so the
// whole screening runs without a host round trip.
#include <map>
#include <mutex>

#include "tt_internal.h"

namespace tt {

constexpr int kSmallMaxFb = 16;

// Weight j of a packed little-endian int8 weight word (static-index friendly).
__device__ __forceinline__ int wt(uint64_t wv, int j) { return (int)(int8_t)(uint8_t)(wv >> (8 * j)); }

__device__ __forceinline__ uint64_t packed_weights(const tt_neuron* p) {
  return *reinterpret_cast<const uint64_t*>(p->w);
}


__device__ __forceinline__ int wmin_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wmax_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ bool small_valid(const tt_neuron* d, uint64_t total_words) {
  const int F = d->F, b = d->b, o = d->o;
  if (F < 1 || F > TT_MAX_F || b < 1 || b > TT_MAX_B || o < 1 || o > TT_MAX_O) return false;
  if (d->act > 1 || F * b > kSmallMaxFb) return false;
  const int K = (1 << o) - 1;
  for (int k = 1; k < K; ++k)
    if (d->thr[k] < d->thr[k - 1]) return false;
  const uint64_t fb = (uint64_t)(F * b);
  const uint64_t W = fb >= 6 ? (1ull << (fb - 6)) : 1ull;
  const uint64_t off = d->word_off;
  return off <= total_words && (uint64_t)o * W <= total_words - off;
}

// Full enumeration of one neuron per block (factored as in the batched
// kernel: low-six-bit mask table in LDS, high-digit partial sum per word).
__global__ __launch_bounds__(256) void small_enum_kernel(const tt_neuron* desc, int n, const uint8_t* active,
                                                         uint64_t* tables, uint64_t total_words, uint32_t* status) {
  __shared__ uint64_t s_lut[kMaxLutCap];
  __shared__ int32_t s_te[8];
  const int i = blockIdx.x;
  if (i >= n || (active && !active[i])) return;
  const tt_neuron* dp = desc + i;
  if (!small_valid(dp, total_words)) {
    if (threadIdx.x == 0 && status) atomicOr(status, 1u);
    return;
  }
  const int F = dp->F, b = dp->b, o = dp->o, Fb = F * b;
  const int W = Fb >= 6 ? (1 << (Fb - 6)) : 1;
  const int dmask = (1 << b) - 1;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    const int R = Fb >= 6 ? 64 : (1 << Fb);
    const bool valid = lane < R;
    const uint64_t wv0 = packed_weights(dp);
    int P = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < F) P += wt(wv0, j) * ((lane >> (j * b)) & dmask);
    const int vmin = wmin_i32(valid ? P : INT32_MAX);
    const int vmax = wmax_i32(valid ? P : INT32_MIN);
    const int r1 = vmax - vmin + 1;  // <= 18 * 128 + 1 < kMaxLutCap
    for (int e0 = 0; e0 <= r1; e0 += 64) {
      const int lim = min(64, r1 + 1 - e0);
      uint64_t mine = 0;
      for (int e = 0; e < lim; ++e) {
        const uint64_t m = __ballot(valid && P - vmin >= e0 + e);
        if (lane == e) mine = m;
      }
      if (lane < lim) s_lut[e0 + lane] = mine;
    }
    if (lane < 8) {
      int32_t val = kPosBig;
      if (lane == 0) {
        val = r1;
      } else if (lane - 1 < (1 << o) - 1) {
        const int64_t t = dp->thr[lane - 1];
        if (dp->act == TT_ACT_RELU && t <= 0) {
          val = kNegBig;
        } else {
          int64_t te = t - (int64_t)dp->bias - (int64_t)vmin;
          val = (int32_t)(te < kNegBig ? kNegBig : (te > kPosBig ? kPosBig : te));
        }
      }
      s_te[lane] = val;
    }
  }
  __syncthreads();
  const int r1 = s_te[0];
  const int K = (1 << o) - 1;
  const uint64_t wv = packed_weights(dp);
  uint64_t* dst = tables + dp->word_off;
  for (int h = tid; h < W; h += blockDim.x) {
    const uint32_t r = (uint32_t)h << 6;
    int P = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < F) P += wt(wv, j) * (int)((r >> (j * b)) & (uint32_t)dmask);
    uint64_t mk[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) mk[k] = k < K ? s_lut[min(max(s_te[1 + k] - P, 0), r1)] : 0ull;
    uint64_t p0, p1 = 0, p2 = 0;
    if (o == 1) {
      p0 = mk[0];
    } else if (o == 2) {
      p0 = mk[0] ^ mk[1] ^ mk[2];
      p1 = mk[1];
    } else {
      p0 = mk[0] ^ mk[1] ^ mk[2] ^ mk[3] ^ mk[4] ^ mk[5] ^ mk[6];
      p1 = mk[1] ^ mk[3] ^ mk[5];
      p2 = mk[3];
    }
    dst[h] = p0;
    if (o > 1) dst[W + h] = p1;
    if (o > 2) dst[2 * W + h] = p2;
  }
}

__device__ __forceinline__ uint64_t flip_select(int i) {
  switch (i) {
    case 0: return 0x5555555555555555ull;
    case 1: return 0x3333333333333333ull;
    case 2: return 0x0F0F0F0F0F0F0F0Full;
    case 3: return 0x00FF00FF00FF00FFull;
    case 4: return 0x0000FFFF0000FFFFull;
    default: return 0x00000000FFFFFFFFull;
  }
}

// Support and histogram of one small neuron per block, tables staged in LDS.
__global__ __launch_bounds__(256) void small_support_kernel(const tt_neuron* desc, int n, const uint64_t* tables,
                                                            uint64_t total_words, uint8_t* support, uint32_t* hist,
                                                            uint32_t* status) {
  __shared__ uint64_t s_pl[3 * 1024];
  __shared__ uint32_t s_found, s_hist[8];
  const int i = blockIdx.x;
  if (i >= n) return;
  const tt_neuron* dp = desc + i;
  if (!small_valid(dp, total_words)) {
    if (threadIdx.x == 0 && status) atomicOr(status, 1u);
    return;
  }
  const int F = dp->F, b = dp->b, o = dp->o, Fb = F * b;
  const uint64_t word_off = dp->word_off;
  const int W = Fb >= 6 ? (1 << (Fb - 6)) : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) s_found = 0;
  if (tid < 8) s_hist[tid] = 0;
  for (int p = 0; p < o; ++p)
    for (int h = tid; h < W; h += blockDim.x) s_pl[p * 1024 + h] = tables[word_off + (uint64_t)p * W + h];
  __syncthreads();
  const uint64_t valid = Fb >= 6 ? ~0ull : ((1ull << (1 << Fb)) - 1ull);
  const int lowbits = Fb < 6 ? Fb : 6;
  int wbits = 0;
  while ((1 << wbits) < W) ++wbits;
  uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t fl = 0;
  for (int h = tid; h < W; h += blockDim.x) {
    const uint64_t P0 = s_pl[h];
    const uint64_t P1 = o > 1 ? s_pl[1024 + h] : 0ull;
    const uint64_t P2 = o > 2 ? s_pl[2048 + h] : 0ull;
    if (hist) {
      for (int v = 0; v < (1 << o); ++v) {
        uint64_t m = valid & ((v & 1) ? P0 : ~P0);
        if (o > 1) m &= (v & 2) ? P1 : ~P1;
        if (o > 2) m &= (v & 4) ? P2 : ~P2;
        hv[v] += (uint32_t)__popcll(m);
      }
    }
    if (support) {
      for (int q = 0; q < lowbits; ++q) {
        if ((fl >> q) & 1) continue;
        const int sh = 1 << q;
        if (((P0 ^ (P0 >> sh)) | (P1 ^ (P1 >> sh)) | (P2 ^ (P2 >> sh))) & flip_select(q)) fl |= 1u << q;
      }
      for (int k = 0; k < wbits; ++k) {
        if (((h >> k) & 1) || ((fl >> (6 + k)) & 1)) continue;
        const int h2 = h | (1 << k);
        bool diff = s_pl[h] != s_pl[h2];
        if (o > 1) diff |= s_pl[1024 + h] != s_pl[1024 + h2];
        if (o > 2) diff |= s_pl[2048 + h] != s_pl[2048 + h2];
        if (diff) fl |= 1u << (6 + k);
      }
    }
  }
  if (hist)
    for (int v = 0; v < (1 << o); ++v) {
      uint32_t x = hv[v];
      for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0 && x) atomicAdd(&s_hist[v], x);
    }
  for (int off = 32; off >= 1; off >>= 1) fl |= __shfl_xor(fl, off, 64);
  if (lane == 0 && fl) atomicOr(&s_found, fl);
  __syncthreads();
  if (tid == 0) {
    if (support) {
      uint32_t s = 0;
      for (int j = 0; j < F; ++j)
        if (s_found & (((1u << b) - 1u) << (j * b))) s |= 1u << j;
      support[i] = (uint8_t)s;
    }
    if (hist)
      for (int v = 0; v < 8; ++v) hist[(size_t)i * 8 + v] = s_hist[v];
  }
}




// Full table of every candidate from the screened result: reduced tables
// are broadcast over the skipped inputs, full ones copied.  One thread per
// output word.
__global__ void screen_expand_kernel(const tt_neuron* desc, int n, const uint8_t* mask, const uint8_t* mode,
                                     const uint8_t* accept, const tt_neuron* res, const uint64_t* screened,
                                     uint64_t* full) {
  const int i = blockIdx.y * 65535 + blockIdx.x;
  if (i >= n) return;
  const tt_neuron d = desc[i];
  const int Fb = d.F * d.b;
  const int W = Fb >= 6 ? (1 << (Fb - 6)) : 1;
  const bool reduced = accept[i] && !mode[i];
  const tt_neuron L = res[i];
  const int Lfb = L.F * L.b;
  const int LW = Lfb >= 6 ? (1 << (Lfb - 6)) : 1;
  const uint32_t S = mask[i];
  const uint32_t dm = (1u << d.b) - 1u;
  for (int h = threadIdx.x; h < W; h += blockDim.x) {
    for (int p = 0; p < d.o; ++p) {
      uint64_t word;
      if (!reduced) {
        word = screened[d.word_off + (uint64_t)p * W + h];
      } else {
        word = 0;
        const int rows = Fb >= 6 ? 64 : (1 << Fb);
        for (int l = 0; l < rows; ++l) {
          const uint32_t r = ((uint32_t)h << 6) | (uint32_t)l;
          uint32_t rr = 0;
          int k = 0;
          for (int j = 0; j < d.F; ++j)
            if ((S >> j) & 1) {
              rr |= ((r >> (j * d.b)) & dm) << (k * d.b);
              ++k;
            }
          const uint64_t src = screened[L.word_off + (uint64_t)p * LW + (rr >> 6)];
          word |= ((src >> (rr & 63)) & 1ull) << l;
        }
      }
      full[d.word_off + (uint64_t)p * W + h] = word;
    }
  }
}

// ------------------------------------------------------------ fused screen
// One wave per candidate, candidates grid-strided over the waves.  The next
// candidate's descriptor (16 dwords, one per lane) and screen inputs are
// loaded while the current one is processed, so no global round trip sits on
// a candidate's path.  Per candidate: predicted support S, the two reduced
// tables compared word by word, fallback to the full table, then planes,
// histogram and support from the planes in registers.  Tables go in chunks of
// 512 words (8 per lane); a 1024-word table takes two, and its top word bit
// is tested against the first chunk, re-read by the lanes that stored it.
// Small tables are evaluated directly (one ballot per plane bit and word),
// larger ones through the wave's mask table.
constexpr int kWaveLut = 512;  // mask-table entries per wave (4 KiB of LDS)
constexpr int kFusedR = 8;     // words per lane per chunk
constexpr int kChunkWords = 64 * kFusedR;

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int fold_threshold(int64_t t, int bias, int vmin, int act) {
  if (act == TT_ACT_RELU && t <= 0) return kNegBig;
  int64_t te = t - (int64_t)bias - (int64_t)vmin;
  return (int)(te < kNegBig ? kNegBig : (te > kPosBig ? kPosBig : te));
}

// Weighted digit sum of row r (only digits j < F count).
__device__ __forceinline__ int digit_sum(uint64_t wv, int F, int b, uint32_t r) {
  const uint32_t dmask = (1u << b) - 1u;
  int P = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < F) P += wt(wv, j) * (int)((r >> (j * b)) & dmask);
  return P;
}

// Planes of words h0 + lane + 64k (k < kFusedR, local word < Wc) of the
// neuron (F, b, wv, act, th[]) with bias ba; with `two`, also compares them
// with bias bb and returns (wave-uniformly) whether any differ.  Lanes past
// the chunk's words keep zeros.  use_lut: the wave's mask table holds
// M[e] = {rows l : Plo(l) - vmin >= e}, e = 0..r1 (entry r1 is empty).
__device__ __forceinline__ bool eval_chunk(int F, int b, int act, uint64_t wv, const int (&th)[7], int Plo, bool valid,
                                           bool use_lut, uint64_t* lut, int vmin, int r1, int ba, bool two,
                                           int bb, int h0, int Wc, uint64_t (&P0)[kFusedR],
                                           uint64_t (&P1)[kFusedR], uint64_t (&P2)[kFusedR]) {
  const int lane = threadIdx.x & 63;
  bool diff = false;
#pragma unroll
  for (int k = 0; k < kFusedR; ++k) P0[k] = P1[k] = P2[k] = 0ull;
  if (use_lut) {
    int ta[7], tb[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      // thresholds past 2^o - 1 are INT32_MAX: they fold to the empty entry r1
      ta[k] = fold_threshold(th[k], ba, vmin, act);
      tb[k] = fold_threshold(th[k], bb, vmin, act);
    }
#pragma unroll
    for (int kk = 0; kk < kFusedR; ++kk) {
      if (kk * 64 < Wc) {  // uniform
        const int hl = lane + 64 * kk;
        const bool in = hl < Wc;
        const int P = digit_sum(wv, F, b, (uint32_t)(h0 + hl) << 6);
        uint64_t mk[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) mk[k] = lut[min(max(ta[k] - P, 0), r1)];
        const uint64_t p0 = mk[0] ^ mk[1] ^ mk[2] ^ mk[3] ^ mk[4] ^ mk[5] ^ mk[6];
        const uint64_t p1 = mk[1] ^ mk[3] ^ mk[5];
        P0[kk] = in ? p0 : 0ull;
        P1[kk] = in ? p1 : 0ull;
        P2[kk] = in ? mk[3] : 0ull;
        if (two) {
          bool d = false;
#pragma unroll
          for (int k = 0; k < 7; ++k) d |= lut[min(max(tb[k] - P, 0), r1)] != mk[k];
          diff |= in && d;
        }
      }
      // keep the scheduler from interleaving all eight words (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // Direct: lane = row inside the word, one ballot per plane bit.  The
    // words go through LDS in rounds of 128 (3 planes fit the table's space)
    // and each lane then picks up its own.
    constexpr int kSub = 2 * 64;
#pragma unroll
    for (int sb = 0; sb < kFusedR / 2; ++sb) {
      const int hs = sb * kSub;
      if (hs < Wc) {  // uniform
        const int cnt = min(kSub, Wc - hs);
        for (int h = 0; h < cnt; ++h) {  // uniform
          const int P = digit_sum(wv, F, b, (uint32_t)(h0 + hs + h) << 6);
          int x = ba + P + Plo;
          if (act == TT_ACT_RELU && x < 0) x = 0;
          int q = 0;
#pragma unroll
          for (int k = 0; k < 7; ++k) q += x >= th[k] ? 1 : 0;
          const uint64_t w0 = __ballot(valid && (q & 1)), w1 = __ballot(valid && (q & 2)),
                         w2 = __ballot(valid && (q & 4));
          if (two) {
            int x2 = bb + P + Plo;
            if (act == TT_ACT_RELU && x2 < 0) x2 = 0;
            int q2 = 0;
#pragma unroll
            for (int k = 0; k < 7; ++k) q2 += x2 >= th[k] ? 1 : 0;
            diff |= valid && q2 != q;
          }
          if (lane == 0) {
            lut[h] = w0;
            lut[kSub + h] = w1;
            lut[2 * kSub + h] = w2;
          }
        }
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int hl = lane + 64 * r;
          const bool in = hl < cnt;
          P0[2 * sb + r] = in ? lut[hl] : 0ull;
          P1[2 * sb + r] = in ? lut[kSub + hl] : 0ull;
          P2[2 * sb + r] = in ? lut[2 * kSub + hl] : 0ull;
        }
        wave_lds_sync();  // the next round overwrites the staging space
      }
    }
  }
  return __any(diff);
}

// Four lanes per candidate, for results of at most 64 rows (one word per
// plane): a reduced pair over S with |S| b <= 6 bits, or a full neuron with
// F b <= 6.  The group's lanes decode the same descriptor and evaluate every
// fourth row each; the plane words and the pair's disagreement are combined
// across the group (DPP quad permutes, a ballot) at points every lane
// reaches, and the group's first lane writes the outputs the wave kernel
// would write.  Four lanes per candidate give four times the waves of one
// lane each (the screen's candidates fill the chip about 1.5 waves deep
// otherwise) and a quarter of the serial row loop.  Every other candidate
// (larger tables, or a rejected pair whose full table is larger) goes to
// the list for the wave-per-candidate kernel.
constexpr int kLaneGroup = 4;
constexpr int kHeavyLfb = 12;  // a deferred table of 2^12 rows or more is heavy

// OR of v over the lane's group of four (quad_perm xor 1, then xor 2)
__device__ __forceinline__ uint64_t quad_or64(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0xB1, 0xF, 0xF, false);
  hi |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, 0xB1, 0xF, 0xF, false);
  lo |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, 0x4E, 0xF, 0xF, false);
  hi |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, 0x4E, 0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int kLaneBlock = 256;  // threads: 64 candidates (1024-thread blocks were slower)

__global__ __launch_bounds__(kLaneBlock) void screen_lane_kernel(FusedArgs a) {
  // candidate blockIdx.x * 64 + threadIdx.x / 4 (no overflow below 2^31 candidates)
  const int i = (int)blockIdx.x * (kLaneBlock / kLaneGroup) + (int)(threadIdx.x / kLaneGroup);
  const int sub = (int)(threadIdx.x % kLaneGroup);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool defer = false, live = false, done = false, accepted = true, full = false;
  int dlfb = 0;  // bits of the deferred table's row index
  int F = 0, b = 1, o = 1, act = 0, bias = 0, Fb = 0, LF = 1, Lbias = 0, bhi = 0, dmax = 1;
  uint32_t S = 0;
  uint64_t wv = 0, Lw = 0, word_off = 0;
  uint32_t d[16] = {};
  int th[7] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
  if (i < a.n) {
    const uint4* dp = reinterpret_cast<const uint4*>(a.desc + i);
    const uint4 q0 = dp[0], q1 = dp[1], q2 = dp[2], q3 = dp[3];
    const uint32_t dd[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                             q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k] = dd[k];
    F = (d[9] >> 16) & 0xFF;
    b = d[9] >> 24;
    o = d[10] & 0xFF;
    act = (d[10] >> 8) & 0xFF;
    bias = (int)(int16_t)(d[9] & 0xFFFFu);
    word_off = (uint64_t)d[12] | ((uint64_t)d[13] << 32);
    Fb = F * b;
    const int K = (1 << o) - 1;
    bool ok = F >= 1 && F <= TT_MAX_F && b >= 1 && b <= TT_MAX_B && o >= 1 && o <= TT_MAX_O && act <= 1 &&
              Fb <= kSmallMaxFb;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      th[k] = k < K ? (int)d[2 + k] : INT32_MAX;
      if (k >= 1 && k < K && th[k] < th[k - 1]) ok = false;
    }
    const int Wf = Fb >= 6 ? (1 << (Fb - 6)) : 1;
    if (ok) ok = word_off <= a.total_words && (uint64_t)o * (uint64_t)Wf <= a.total_words - word_off;
    if (!ok) {
      if (a.status && sub == 0) atomicOr(a.status, 1u);
    } else {
      live = true;
      wv = ((uint64_t)d[0] | ((uint64_t)d[1] << 32)) & (F < 8 ? (1ull << (8 * F)) - 1ull : ~0ull);
      const uint32_t fmask = (1u << F) - 1u;
      S = fmask;
      if (!a.plain) {
        if (a.force_mask) {
          S = a.force_mask[i] & fmask;
        } else {
          // The lane pass settles only candidates whose table reduced to the
          // inputs of nonzero weight has at most 64 rows (one word per
          // plane), where a prediction cannot save work, so their logits are
          // never read (the screen's network skips them).
          S = 0;
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (j < F && ((wv >> (8 * j)) & 0xFFu) != 0u) S |= 1u << j;
        }
      }
      dmax = (1 << b) - 1;
      uint64_t wl = 0;
      int kS = 0, mn = 0, mx = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j < F) {
          const int wj = wt(wv, j);
          if ((S >> j) & 1) {
            wl |= (uint64_t)(uint8_t)wj << (8 * kS);
            ++kS;
          } else {
            mn += min(wj, 0) * dmax;
            mx += max(wj, 0) * dmax;
          }
        }
      }
      const int blo = bias + mn;
      bhi = bias + mx;
      full = kS == F || blo < -32768 || blo > 32767 || bhi < -32768 || bhi > 32767;
      LF = full ? F : (kS > 0 ? kS : 1);
      Lw = full ? wv : wl;
      Lbias = full ? bias : blo;
    }
  }
  // two passes (the reduced pair, then the full neuron when the pair
  // disagrees), with the group's combines outside every branch
  uint64_t P0 = 0, P1 = 0, P2 = 0;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const bool run = live && !done && !defer && LF * b <= 6;
    if (live && !done && !defer && LF * b > 6) {
      defer = true;
      dlfb = LF * b;
    }
    const int rows = run ? 1 << (LF * b) : 0;
    uint64_t Q0 = 0, Q1 = 0, Q2 = 0;
    bool diff = false;
    for (int r = sub; r < rows; r += kLaneGroup) {
      int P = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < LF) P += wt(Lw, j) * ((r >> (j * b)) & dmax);
      int x = Lbias + P;
      if (act == TT_ACT_RELU && x < 0) x = 0;
      int q = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) q += x >= th[k] ? 1 : 0;
      Q0 |= (uint64_t)(q & 1) << r;
      Q1 |= (uint64_t)((q >> 1) & 1) << r;
      Q2 |= (uint64_t)((q >> 2) & 1) << r;
      if (!full) {
        int x2 = bhi + P;
        if (act == TT_ACT_RELU && x2 < 0) x2 = 0;
        int q2 = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) q2 += x2 >= th[k] ? 1 : 0;
        diff |= q2 != q;
      }
    }
    Q0 = quad_or64(Q0);
    Q1 = quad_or64(Q1);
    Q2 = quad_or64(Q2);
    diff = ((__ballot(diff) >> (lane & ~(kLaneGroup - 1))) & ((1ull << kLaneGroup) - 1ull)) != 0ull;
    if (run) {
      if (!full && diff) {
        // the pair disagrees: the full neuron
        accepted = false;
        full = true;
        LF = F;
        Lw = wv;
        Lbias = bias;
      } else {
        P0 = Q0;
        P1 = Q1;
        P2 = Q2;
        done = true;
      }
    }
  }
  if (done && sub == 0) {
    const int Lfb = LF * b;
    uint64_t* dst = a.tables + word_off;
    dst[0] = P0;
    if (o > 1) dst[1] = P1;
    if (o > 2) dst[2] = P2;
    const uint64_t validw = Lfb >= 6 ? ~0ull : ((1ull << (1 << Lfb)) - 1ull);
    uint32_t hv[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      uint64_t m = validw & ((v & 1) ? P0 : ~P0);
      m &= (v & 2) ? P1 : ~P1;
      m &= (v & 4) ? P2 : ~P2;
      hv[v] = (uint32_t)__popcll(m);
    }
    uint32_t fl = 0;
    for (int q = 0; q < Lfb; ++q) {
      const int sh = 1 << q;
      if (((P0 ^ (P0 >> sh)) | (P1 ^ (P1 >> sh)) | (P2 ^ (P2 >> sh))) & flip_select(q)) fl |= 1u << q;
    }
    uint32_t sres = 0;
    for (int j = 0; j < LF; ++j)
      if (fl & ((uint32_t)dmax << (j * b))) sres |= 1u << j;
    uint32_t sup = sres, scale = 0;
    const bool reduced = !full;
    if (reduced) {
      sup = 0;
      int k = 0;
      for (int j = 0; j < F; ++j)
        if ((S >> j) & 1) {
          if ((sres >> k) & 1) sup |= 1u << j;
          ++k;
        }
      scale = (uint32_t)(Fb - Lfb);
    }
    a.support[i] = (uint8_t)sup;
    uint4* hd = reinterpret_cast<uint4*>(a.hist + (size_t)i * 8);
    hd[0] = make_uint4(hv[0] << scale, hv[1] << scale, hv[2] << scale, hv[3] << scale);
    hd[1] = make_uint4(hv[4] << scale, hv[5] << scale, hv[6] << scale, hv[7] << scale);
    if (a.res) {
      uint4* rd = reinterpret_cast<uint4*>(a.res + i);
      const uint32_t d9 = ((uint32_t)(uint16_t)(int16_t)Lbias) | ((uint32_t)LF << 16) | ((uint32_t)b << 24);
      rd[0] = make_uint4((uint32_t)Lw, (uint32_t)(Lw >> 32), d[2], d[3]);
      rd[1] = make_uint4(d[4], d[5], d[6], d[7]);
      rd[2] = make_uint4(d[8], d9, d[10], d[11]);
      rd[3] = make_uint4(d[12], d[13], d[14], d[15]);
    }
    if (a.mask) a.mask[i] = (uint8_t)S;
    if (a.mode) a.mode[i] = reduced ? 0 : 1;
    if (a.accept) a.accept[i] = accepted ? 1 : 0;
    if (a.mask_out) a.mask_out[i] = (uint8_t)S;
    if (a.accept_out) a.accept_out[i] = accepted ? 1 : 0;
  }
  // append the deferred candidates (the group's first lane), the heavy ones
  // (tables of 2^kHeavyLfb rows or more) from the front of the list, the
  // others from the back, so that the wave kernel, which deals the list out
  // in order, starts every heavy one first (a wave holding two heavy
  // candidates set the kernel's tail otherwise); one add per class and
  // block (adds to one address from every wave of the grid serialise, about
  // 12 ns each)
  const bool app = defer && sub == 0, heavy = dlfb >= kHeavyLfb;
  __shared__ uint32_t s_cnt[2][kLaneBlock / 64];
  __shared__ uint32_t s_base[2];
  const uint64_t mh = __ballot(app && heavy), ml = __ballot(app && !heavy);
  if (lane == 0) {
    s_cnt[0][wave] = (uint32_t)__popcll(mh);
    s_cnt[1][wave] = (uint32_t)__popcll(ml);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t total = 0;
    for (int w = 0; w < kLaneBlock / 64; ++w) total += s_cnt[threadIdx.x][w];
    s_base[threadIdx.x] = total ? atomicAdd(a.list_count + threadIdx.x, total) : 0u;
  }
  __syncthreads();
  if (app) {
    const int c = heavy ? 0 : 1;
    uint32_t off = s_base[c];
    for (int w = 0; w < wave; ++w) off += s_cnt[c][w];
    off += (uint32_t)__popcll((heavy ? mh : ml) & ((1ull << lane) - 1ull));
    a.list[heavy ? (long)off : (long)a.n - 1 - off] = i;
  }
}

__global__ __launch_bounds__(256) void screen_fused_kernel(FusedArgs a) {
  __shared__ uint64_t s_lut[4][kWaveLut];
  const int lane = threadIdx.x & 63;
  uint64_t* lut = s_lut[threadIdx.x >> 6];
  const int gw = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  const uint32_t* dwords = reinterpret_cast<const uint32_t*>(a.desc);
  const bool use_logits = !a.plain && !a.force_mask;
  // prefetched inputs of the next candidate: descriptor dword `lane` (lanes
  // 0..15), logit `lane` (lanes 0..7), forced mask (lane 0)
  uint32_t nx_dw = 0, nx_fm = 0;
  float nx_lg = 0.f;
  auto fetch = [&](int c) {
    if (c < a.n) {
      if (lane < 16) nx_dw = dwords[(size_t)c * 16 + lane];
      if (use_logits && lane < 8) nx_lg = a.logits[(size_t)c * 12 + lane];
      if (a.force_mask && lane == 0) nx_fm = a.force_mask[c];
    }
  };
  // the candidates left by the lane kernel: lane l holds the list entry of
  // this wave's iteration 64 q + l (refilled every 64 iterations)
  // entry e: the heavy candidates (list_count[0], from the front of the
  // list) first, then the others (list_count[1], from the back)
  const int heavy = (int)__builtin_amdgcn_readfirstlane((int)a.list_count[0]);
  const int count = heavy + (int)__builtin_amdgcn_readfirstlane((int)a.list_count[1]);
  auto entries = [&](int e0) {
    const int e = e0 + lane * nw;
    return e < count ? a.list[e < heavy ? (long)e : (long)a.n - 1 - (e - heavy)] : 0;
  };
  int ent = entries(gw);
  fetch(count > gw ? __builtin_amdgcn_readfirstlane(ent) : a.n);
  for (int e = gw, it = 0; e < count; e += nw, ++it) {
    const int i = __builtin_amdgcn_readlane(ent, it & 63);
    const uint32_t dw = nx_dw, fm = nx_fm;
    const float lg = nx_lg;
    if (((it + 1) & 63) == 0) ent = entries(e + nw);  // next 64 entries
    fetch(e + nw < count ? __builtin_amdgcn_readlane(ent, (it + 1) & 63) : a.n);
    uint32_t d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k] = (uint32_t)__builtin_amdgcn_readlane((int)dw, k);
    const int F = (d[9] >> 16) & 0xFF, b = d[9] >> 24, o = d[10] & 0xFF, act = (d[10] >> 8) & 0xFF;
    const int bias = (int)(int16_t)(d[9] & 0xFFFFu);
    const uint64_t word_off = (uint64_t)d[12] | ((uint64_t)d[13] << 32);
    const int Fb = F * b, K = (1 << o) - 1;
    // the same checks as the host validation, for device-resident descriptors
    bool ok = F >= 1 && F <= TT_MAX_F && b >= 1 && b <= TT_MAX_B && o >= 1 && o <= TT_MAX_O && act <= 1 &&
              Fb <= kSmallMaxFb;
    int th[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      th[k] = k < K ? (int)d[2 + k] : INT32_MAX;
      if (k >= 1 && k < K && th[k] < th[k - 1]) ok = false;
    }
    const int Wf = Fb >= 6 ? (1 << (Fb - 6)) : 1;
    if (ok) ok = word_off <= a.total_words && (uint64_t)o * (uint64_t)Wf <= a.total_words - word_off;
    if (!ok) {
      if (lane == 0 && a.status) atomicOr(a.status, 1u);
      continue;
    }
    const uint64_t wv = ((uint64_t)d[0] | ((uint64_t)d[1] << 32)) & (F < 8 ? (1ull << (8 * F)) - 1ull : ~0ull);
    const uint32_t fmask = (1u << F) - 1u;
    uint32_t S = fmask;
    if (!a.plain) {
      if (a.force_mask)
        S = (uint32_t)__builtin_amdgcn_readfirstlane((int)fm) & fmask;
      else  // inputs with zero weight never matter: the prediction is kept to the others
        S = (uint32_t)__ballot(lane < F && lg > a.tau_logit && ((wv >> (8 * (lane & 7))) & 0xFFu) != 0u) & fmask;
    }
    // reduced neuron over S, biases at the two ends of the skipped inputs' range
    const int dmax = (1 << b) - 1;
    uint64_t wl = 0;
    int kS = 0, mn = 0, mx = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < F) {
        const int wj = wt(wv, j);
        if ((S >> j) & 1) {
          wl |= (uint64_t)(uint8_t)wj << (8 * kS);
          ++kS;
        } else {
          mn += min(wj, 0) * dmax;
          mx += max(wj, 0) * dmax;
        }
      }
    }
    const int blo = bias + mn, bhi = bias + mx;
    bool full = kS == F || blo < -32768 || blo > 32767 || bhi < -32768 || bhi > 32767;
    bool accepted = true;
    // current pass: the reduced pair (one chunk), else the full neuron
    int LF = full ? F : (kS > 0 ? kS : 1);
    uint64_t Lw = full ? wv : wl;
    int Lbias = full ? bias : blo;
    uint64_t P0[kFusedR], P1[kFusedR], P2[kFusedR];
    // per-lane code counts, two 16-bit counts per register (at most 64 rows
    // per word and 16 words per lane)
    uint32_t hp[4] = {0, 0, 0, 0};
    uint32_t fl = 0;  // row bits whose flip changes some code (wave-uniform)
    int W = 1, nch = 1, c = 0;
    int Plo = 0, vmin = 0, r1 = 0;
    bool valid = false, use_lut = false;
    for (;;) {
      if (c == 0) {
        // a new pass: this neuron's lane sums and, when it pays, its mask table
        const int Lfb = LF * b;
        W = Lfb >= 6 ? (1 << (Lfb - 6)) : 1;
        nch = (W + kChunkWords - 1) / kChunkWords;
        const int R0 = Lfb >= 6 ? 64 : (1 << Lfb);
        valid = lane < R0;
        Plo = digit_sum(Lw, LF, b, (uint32_t)lane);
        // range of Plo over the valid lanes: the lanes take every value of
        // the digits (or digit parts) below bit min(Lfb, 6) independently
        {
          const int lb = Lfb < 6 ? Lfb : 6;
          int lo = 0, hi = 0;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int sh = j * b;
            if (j < LF && sh < lb) {
              const int top = min(b, lb - sh);  // bits of digit j below bit lb
              const int wj = wt(Lw, j), dm = (1 << top) - 1;
              lo += min(wj, 0) * dm;
              hi += max(wj, 0) * dm;
            }
          }
          vmin = lo;
          r1 = hi - lo + 1;
        }
        // direct evaluation costs about one ballot round per word, the table
        // one per entry
        use_lut = r1 + 1 <= kWaveLut && W * 4 > r1;
        if (use_lut) {
          for (int e0 = 0; e0 <= r1; e0 += 64) {
            const int lim = min(64, r1 + 1 - e0);
            uint64_t mine = 0;
            for (int e = 0; e < lim; ++e) {
              const uint64_t m = __ballot(valid && Plo - vmin >= e0 + e);
              if (lane == e) mine = m;
            }
            if (lane < lim) lut[e0 + lane] = mine;
          }
          wave_lds_sync();
        }
      }
      const int h0 = c * kChunkWords;
      const int Wc = min(W - h0, kChunkWords);
      const bool two = !full;
      const bool diff = eval_chunk(LF, b, act, Lw, th, Plo, valid, use_lut, lut, vmin, r1, Lbias, two, bhi, h0, Wc,
                                   P0, P1, P2);
      wave_lds_sync();  // the table / staging space may be rewritten next
      if (two && diff) {
        // the pair disagrees: enumerate the full neuron
        accepted = false;
        full = true;
        LF = F;
        Lw = wv;
        Lbias = bias;
        c = 0;
        continue;
      }
      // store the chunk
      uint64_t* dst = a.tables + word_off + (uint64_t)h0;
#pragma unroll
      for (int kk = 0; kk < kFusedR; ++kk) {
        const int hl = lane + 64 * kk;
        if (hl < Wc) {
          dst[hl] = P0[kk];
          if (o > 1) dst[W + hl] = P1[kk];
          if (o > 2) dst[2 * W + hl] = P2[kk];
        }
      }
      // histogram of the chunk (lanes past the chunk hold zeros: masked out)
      const int Lfb = LF * b;
      const uint64_t validw = Lfb >= 6 ? ~0ull : ((1ull << (1 << Lfb)) - 1ull);
#pragma unroll
      for (int kk = 0; kk < kFusedR; ++kk) {
        if (kk * 64 < Wc) {  // uniform
          const uint64_t inw = lane + 64 * kk < Wc ? validw : 0ull;
#pragma unroll
          for (int v = 0; v < 8; ++v) {
            // planes at or above o are zero: codes >= 2^o get no rows
            uint64_t m = inw & ((v & 1) ? P0[kk] : ~P0[kk]);
            m &= (v & 2) ? P1[kk] : ~P1[kk];
            m &= (v & 4) ? P2[kk] : ~P2[kk];
            hp[v >> 1] += (uint32_t)__popcll(m) << (16 * (v & 1));
          }
        }
      }
      // support: row bits inside a word, then word bits inside the chunk,
      // skipping bits of digits already known to matter
      const uint32_t dgm = (uint32_t)dmax;
      const int lowbits = Lfb < 6 ? Lfb : 6;
      for (int q = 0; q < lowbits; ++q) {
        if ((fl >> (q - q % b)) & dgm) continue;
        const int sh = 1 << q;
        uint64_t x = 0;
#pragma unroll
        for (int kk = 0; kk < kFusedR; ++kk)
          if (kk * 64 < Wc)  // uniform
            x |= (P0[kk] ^ (P0[kk] >> sh)) | (P1[kk] ^ (P1[kk] >> sh)) | (P2[kk] ^ (P2[kk] >> sh));
        if (__any((x & flip_select(q)) != 0ull)) fl |= 1u << q;
      }
      int wbits = 0;
      while ((1 << wbits) < W) ++wbits;
      const int cbits = min(wbits, 9);  // word bits inside a chunk
      for (int t = 0; t < cbits; ++t) {
        const int q = 6 + t;
        if ((fl >> (q - q % b)) & dgm) continue;
        bool df = false;
        if (t < 6) {
#pragma unroll
          for (int kk = 0; kk < kFusedR; ++kk) {
            if (kk * 64 < Wc) {  // uniform
              df |= shfl_xor64(P0[kk], 1 << t) != P0[kk];
              df |= shfl_xor64(P1[kk], 1 << t) != P1[kk];
              df |= shfl_xor64(P2[kk], 1 << t) != P2[kk];
            }
          }
        } else {
          const int u = 1 << (t - 6);
#pragma unroll
          for (int kk = 0; kk < kFusedR; ++kk)
            if (!(kk & u) && (kk | u) * 64 < Wc)
              df |= P0[kk] != P0[kk | u] || P1[kk] != P1[kk | u] || P2[kk] != P2[kk | u];
        }
        if (__any(df)) fl |= 1u << q;
      }
      if (c == 1) {
        // word bit 9 (1024-word tables): this chunk against the first one,
        // which these same lanes stored above
        const int q = 6 + 9;
        if (!((fl >> (q - q % b)) & dgm)) {
          const uint64_t* first = a.tables + word_off;
          bool df = false;
#pragma unroll
          for (int kk = 0; kk < kFusedR; ++kk) {
            const int hl = lane + 64 * kk;
            df |= first[hl] != P0[kk];
            if (o > 1) df |= first[W + hl] != P1[kk];
            if (o > 2) df |= first[2 * W + hl] != P2[kk];
          }
          if (__any(df)) fl |= 1u << q;
        }
      }
      if (++c >= nch) break;
    }
    // histogram totals (a code may hold all 2^16 rows: sums are 32-bit)
    const int Lfb = LF * b;
    // only lanes below min(W, 64) hold words: sum over that many lanes
    const int span = W < 64 ? W : 64;
    uint32_t hv[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      hv[v] = (hp[v >> 1] >> (16 * (v & 1))) & 0xFFFFu;
      if (v < (1 << o)) {  // uniform
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
          if (off < span) hv[v] += (uint32_t)__shfl_xor((int)hv[v], off, 64);
      }
    }
    if (lane == 0) {
      uint32_t sres = 0;
      for (int j = 0; j < LF; ++j)
        if (fl & ((uint32_t)dmax << (j * b))) sres |= 1u << j;
      uint32_t sup = sres, scale = 0;
      const bool reduced = !full;
      if (reduced) {
        sup = 0;
        int k = 0;
        for (int j = 0; j < F; ++j)
          if ((S >> j) & 1) {
            if ((sres >> k) & 1) sup |= 1u << j;
            ++k;
          }
        scale = (uint32_t)(Fb - Lfb);
      }
      a.support[i] = (uint8_t)sup;
      uint4* hd = reinterpret_cast<uint4*>(a.hist + (size_t)i * 8);
      hd[0] = make_uint4(hv[0] << scale, hv[1] << scale, hv[2] << scale, hv[3] << scale);
      hd[1] = make_uint4(hv[4] << scale, hv[5] << scale, hv[6] << scale, hv[7] << scale);
      if (a.res) {
        // the result descriptor: the candidate's own, with the reduced weights
        uint4* rd = reinterpret_cast<uint4*>(a.res + i);
        const uint32_t d9 = ((uint32_t)(uint16_t)(int16_t)Lbias) | ((uint32_t)LF << 16) | ((uint32_t)b << 24);
        rd[0] = make_uint4((uint32_t)Lw, (uint32_t)(Lw >> 32), d[2], d[3]);
        rd[1] = make_uint4(d[4], d[5], d[6], d[7]);
        rd[2] = make_uint4(d[8], d9, d[10], d[11]);
        rd[3] = make_uint4(d[12], d[13], d[14], d[15]);
      }
      if (a.mask) a.mask[i] = (uint8_t)S;
      if (a.mode) a.mode[i] = reduced ? 0 : 1;
      if (a.accept) a.accept[i] = accepted ? 1 : 0;
      if (a.mask_out) a.mask_out[i] = (uint8_t)S;
      if (a.accept_out) a.accept_out[i] = accepted ? 1 : 0;
    }
  }
}

// Compute units and resident blocks per CU of the wave kernel, queried once
// per device.
hipError_t fused_fit(int* cus, int* per_cu) {
  static std::mutex mu;
  static std::map<int, std::pair<int, int>> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it == cache.end()) {
    int c = 0, p = 0;
    e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, screen_fused_kernel, 256, 0);
    if (e != hipSuccess) return e;
    it = cache.emplace(dev, std::make_pair(c, p)).first;
  }
  *cus = it->second.first;
  *per_cu = it->second.second;
  return hipSuccess;
}

hipError_t screen_fused(const FusedArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  int cus = 0, per_cu = 0;
  hipError_t e = fused_fit(&cus, &per_cu);
  if (e != hipSuccess) return e;
  // small results lane by lane; the rest, one wave per candidate, with as
  // many waves as fit at once (each takes every nw-th listed candidate)
  if ((e = launch_fill_u32(a.list_count, 2, 0u, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(screen_lane_kernel, dim3((unsigned)(((long)a.n * kLaneGroup + kLaneBlock - 1) / kLaneBlock)),
                     dim3(kLaneBlock), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long fit = (long)std::max(1, per_cu) * cus * 4;
  const long waves = std::min<long>(a.n, fit);
  hipLaunchKernelGGL(screen_fused_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
hipError_t small_enumerate(const tt_neuron* d, int n, const uint8_t* active, uint64_t* tables, uint64_t total,
                           uint32_t* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(small_enum_kernel, dim3(n), dim3(256), 0, s, d, n, active, tables, total, status);
  return hipGetLastError();
}

hipError_t small_support(const tt_neuron* d, int n, const uint64_t* tables, uint64_t total, uint8_t* sup,
                         uint32_t* hist, uint32_t* status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(small_support_kernel, dim3(n), dim3(256), 0, s, d, n, tables, total, sup, hist, status);
  return hipGetLastError();
}




hipError_t screen_expand(const tt_neuron* d, int n, const uint8_t* mask, const uint8_t* mode, const uint8_t* accept,
                         const tt_neuron* res, const uint64_t* screened, uint64_t* full, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(n < 65535 ? n : 65535, (n + 65534) / 65535);
  hipLaunchKernelGGL(screen_expand_kernel, grid, dim3(256), 0, s, d, n, mask, mode, accept, res, screened, full);
  return hipGetLastError();
}

}  // namespace tt
