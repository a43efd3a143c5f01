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
    const int r1 = vmax - vmin + 1;  // <= 18 * 127 + 1 < kMaxLutCap
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
// One wave per candidate (grid-stride): predicted support, the two reduced
// tables compared word by word, fallback to the full table, support and
// histogram from the planes held in registers, all without leaving the
// wave.  Plain mode enumerates every candidate in full.
constexpr int kWaveLut = 512;  // mask-table entries per wave (4 KiB of LDS)
// Words per lane: a candidate with W words per plane is handled by the
// instance with R = 8 (W <= 512) or R = 16 (W <= 1024).


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

// Planes of the neuron (F, b, o, act, packed weights wv, thr[]) with bias
// `ba`, word lane + 64k in register k.  With `two`, also evaluates bias `bb`
// and returns (wave-uniformly) whether any of its planes differ.  F, b, o,
// act and the biases are wave-uniform.  Every loop over thresholds, weights
// or registers has a compile-time trip count (no private-memory arrays),
// and a lane's plane words are written with selects, never under a branch
// on the lane's own word index.
template <int kSmallR>
__device__ __forceinline__ bool wave_planes(int F, int b, int o, int act, uint64_t wv, const int32_t* thr, int ba,
                                            bool two, int bb, uint64_t* lut, uint64_t (&P0)[kSmallR],
                                            uint64_t (&P1)[kSmallR], uint64_t (&P2)[kSmallR]) {
  const int lane = threadIdx.x & 63;
  const int Fb = F * b, K = (1 << o) - 1;
  const int W = Fb >= 6 ? (1 << (Fb - 6)) : 1;
  const int R0 = Fb >= 6 ? 64 : (1 << Fb);
  const int dmask = (1 << b) - 1;
  const bool valid = lane < R0;
  int Plo = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < F) Plo += wt(wv, j) * ((lane >> (j * b)) & dmask);
  const int vmin = wmin_i32(valid ? Plo : INT32_MAX);
  const int vmax = wmax_i32(valid ? Plo : INT32_MIN);
  const int r1 = vmax - vmin + 1;
  int th[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) th[k] = k < K ? thr[k] : INT32_MAX;
  bool diff = false;
#pragma unroll
  for (int k = 0; k < kSmallR; ++k) P0[k] = P1[k] = P2[k] = 0ull;
  const int Ruse = (W + 63) >> 6;
  if (r1 + 1 <= kWaveLut) {
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
    int ta[7], tb[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      ta[k] = k < K ? fold_threshold(th[k], ba, vmin, act) : kPosBig;
      tb[k] = k < K ? fold_threshold(th[k], bb, vmin, act) : kPosBig;
    }
#pragma unroll
    for (int kk = 0; kk < kSmallR; ++kk) {
      if (kk < Ruse) {  // uniform
        const int h = lane + 64 * kk;
        const bool in = h < W;
        // lanes past the last word evaluate a harmless row and keep zeros
        const uint32_t r = (uint32_t)h << 6;
        int P = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < F) P += wt(wv, j) * (int)((r >> (j * b)) & (uint32_t)dmask);
        // thresholds past K read entry r1, which is empty
        uint64_t mk[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) mk[k] = lut[min(max(ta[k] - P, 0), r1)];
        const uint64_t p0 = mk[0] ^ mk[1] ^ mk[2] ^ mk[3] ^ mk[4] ^ mk[5] ^ mk[6];
        const uint64_t p1 = mk[1] ^ mk[3] ^ mk[5];
        const uint64_t p2 = mk[3];
        P0[kk] = in ? p0 : 0ull;
        P1[kk] = in ? p1 : 0ull;
        P2[kk] = in ? p2 : 0ull;
        if (two) {
          bool d = false;
#pragma unroll
          for (int k = 0; k < 7; ++k) d |= lut[min(max(tb[k] - P, 0), r1)] != mk[k];
          diff |= in && d;
        }
      }
    }
    wave_lds_sync();  // the next candidate may overwrite the table
  } else {
    // Direct: lane = row inside the word, one ballot per plane bit.
    for (int h = 0; h < W; ++h) {
      const uint32_t r = (uint32_t)h << 6;
      int P = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < F) P += wt(wv, j) * (int)((r >> (j * b)) & (uint32_t)dmask);
      int a = ba + P + Plo;
      if (act == TT_ACT_RELU && a < 0) a = 0;
      int q = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) q += a >= th[k] ? 1 : 0;
      const uint64_t w0 = __ballot(valid && (q & 1)), w1 = __ballot(valid && (q & 2)), w2 = __ballot(valid && (q & 4));
      if (two) {
        int a2 = bb + P + Plo;
        if (act == TT_ACT_RELU && a2 < 0) a2 = 0;
        int q2 = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) q2 += a2 >= th[k] ? 1 : 0;
        diff |= valid && q2 != q;
      }
      const int kh = h >> 6;
      const bool mine = lane == (h & 63);
#pragma unroll
      for (int kk = 0; kk < kSmallR; ++kk)
        if (kk == kh) {  // uniform
          P0[kk] = mine ? w0 : P0[kk];
          P1[kk] = mine ? w1 : P1[kk];
          P2[kk] = mine ? w2 : P2[kk];
        }
    }
  }
  return __any(diff);
}

template <int kSmallR>
__global__ __launch_bounds__(256) void screen_fused_kernel(FusedArgs a) {
  __shared__ uint64_t s_lut[4][kWaveLut];
  const int lane = threadIdx.x & 63;
  const int wv_id = threadIdx.x >> 6;
  uint64_t* lut = s_lut[wv_id];
  // wave index made explicitly uniform so descriptor fields live in SGPRs
  const int gw = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  for (int i = gw; i < a.n; i += nw) {
    const tt_neuron* dp = a.desc + i;
    const int F = __builtin_amdgcn_readfirstlane(dp->F), b = __builtin_amdgcn_readfirstlane(dp->b);
    const int o = __builtin_amdgcn_readfirstlane(dp->o), Fb = F * b;
    // size class of this instance: words per plane in (64 * kSmallR / 2, 64 * kSmallR]
    const int Wc = Fb >= 6 ? (1 << (Fb - 6)) : 1;
    if (Fb <= kSmallMaxFb && (Wc > 64 * kSmallR || (kSmallR > 8 && Wc <= 512))) continue;
    if (!small_valid(dp, a.total_words)) {
      if (lane == 0 && a.status && kSmallR == 8) atomicOr(a.status, 1u);
      continue;
    }
    const int act = __builtin_amdgcn_readfirstlane(dp->act), bias = __builtin_amdgcn_readfirstlane(dp->bias);
    const int32_t* thr = dp->thr;
    const uint64_t word_off = dp->word_off;
    const int dmax = (1 << b) - 1;
    uint32_t S = (1u << F) - 1u;
    if (!a.plain) {
      if (a.force_mask) {
        S = a.force_mask[i] & ((1u << F) - 1u);
      } else {
        S = 0;
        for (int j = 0; j < F; ++j)
          if (a.logits[(size_t)i * 12 + j] > a.tau_logit) S |= 1u << j;
      }
    }
    // reduced neuron over S, biases at the two ends of the skipped inputs' range
    const uint64_t wv = packed_weights(dp);
    uint64_t wl = 0;
    int kS = 0, mn = 0, mx = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= F) continue;
      const int wj = wt(wv, j);
      if ((S >> j) & 1) {
        wl |= (uint64_t)(uint8_t)wj << (8 * kS);
        ++kS;
      } else {
        mn += min(wj, 0) * dmax;
        mx += max(wj, 0) * dmax;
      }
    }
    const int blo = bias + mn, bhi = bias + mx;
    bool full = kS == F || blo < -32768 || blo > 32767 || bhi < -32768 || bhi > 32767;
    int LF = kS > 0 ? kS : 1;
    int Lbias = blo;
    uint64_t P0[kSmallR], P1[kSmallR], P2[kSmallR];
    bool accepted = true;
    if (!full) {
      const bool diff = wave_planes<kSmallR>(LF, b, o, act, wl, thr, blo, true, bhi, lut, P0, P1, P2);
      if (diff) {
        accepted = false;
        full = true;
      }
    }
    if (full) {
      LF = F;
      Lbias = bias;
      wl = wv;
      wave_planes<kSmallR>(F, b, o, act, wv, thr, bias, false, 0, lut, P0, P1, P2);
    }
    // store the result table at the candidate's offset
    const int Lfb = LF * b;
    const int W = Lfb >= 6 ? (1 << (Lfb - 6)) : 1;
    uint64_t* dst = a.tables + word_off;
    const int Ruse = (W + 63) >> 6;
#pragma unroll
    for (int kk = 0; kk < kSmallR; ++kk) {
      if (kk >= Ruse) break;
      const int h = lane + 64 * kk;
      if (h < W) {
        dst[h] = P0[kk];
        if (o > 1) dst[W + h] = P1[kk];
        if (o > 2) dst[2 * W + h] = P2[kk];
      }
    }
    // histogram of the result table
    const uint64_t validw = Lfb >= 6 ? ~0ull : ((1ull << (1 << Lfb)) - 1ull);
    uint32_t hv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kSmallR; ++kk) {
      if (kk < Ruse) {  // uniform
        const uint64_t inw = lane + 64 * kk < W ? validw : 0ull;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          // planes at or above o are zero: codes >= 2^o get no rows
          uint64_t m = inw & ((v & 1) ? P0[kk] : ~P0[kk]);
          m &= (v & 2) ? P1[kk] : ~P1[kk];
          m &= (v & 4) ? P2[kk] : ~P2[kk];
          hv[v] += (uint32_t)__popcll(m);
        }
      }
    }
    for (int v = 0; v < 8; ++v)
      for (int off = 32; off >= 1; off >>= 1) hv[v] += __shfl_xor(hv[v], off, 64);
    // support of the result table: in-word row bits, then word bits
    uint32_t fl = 0;
    const int lowbits = Lfb < 6 ? Lfb : 6;
    for (int q = 0; q < lowbits; ++q) {
      const int sh = 1 << q;
      uint64_t x = 0;
#pragma unroll
      for (int kk = 0; kk < kSmallR; ++kk) {
        if (kk >= Ruse) break;
        x |= (P0[kk] ^ (P0[kk] >> sh)) | (P1[kk] ^ (P1[kk] >> sh)) | (P2[kk] ^ (P2[kk] >> sh));
      }
      if (__any((x & flip_select(q)) != 0ull)) fl |= 1u << q;
    }
    int wbits = 0;
    while ((1 << wbits) < W) ++wbits;
    for (int t = 0; t < wbits; ++t) {
      bool df = false;
      if (t < 6) {
#pragma unroll
        for (int kk = 0; kk < kSmallR; ++kk) {
          if (kk >= Ruse) break;
          df |= shfl_xor64(P0[kk], 1 << t) != P0[kk];
          if (o > 1) df |= shfl_xor64(P1[kk], 1 << t) != P1[kk];
          if (o > 2) df |= shfl_xor64(P2[kk], 1 << t) != P2[kk];
        }
      } else {
        const int u = 1 << (t - 6);
#pragma unroll
        for (int kk = 0; kk < kSmallR; ++kk)
          if (kk < Ruse && !(kk & u) && (kk | u) < kSmallR)
            df |= P0[kk] != P0[kk | u] || P1[kk] != P1[kk | u] || P2[kk] != P2[kk | u];
      }
      if (__any(df)) fl |= 1u << (6 + t);
    }
    if (lane == 0) {
      uint32_t sres = 0;
      for (int j = 0; j < LF; ++j)
        if (fl & (((1u << b) - 1u) << (j * b))) sres |= 1u << j;
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
      for (int v = 0; v < 8; ++v) a.hist[(size_t)i * 8 + v] = hv[v] << scale;
      if (a.res) {
        // the result descriptor: the candidate's own, with the reduced weights
        tt_neuron* L = a.res + i;
        const uint64_t* src = reinterpret_cast<const uint64_t*>(dp);
        uint64_t* out = reinterpret_cast<uint64_t*>(L);
        for (int q = 0; q < 8; ++q) out[q] = src[q];
        *reinterpret_cast<uint64_t*>(L->w) = wl;
        L->F = (uint8_t)LF;
        L->bias = (int16_t)Lbias;
      }
      if (a.mask) a.mask[i] = (uint8_t)S;
      if (a.mode) a.mode[i] = reduced ? 0 : 1;
      if (a.accept) a.accept[i] = accepted ? 1 : 0;
    }
  }
}

hipError_t screen_fused(const FusedArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int waves = a.n < 16 * cus ? a.n : 16 * cus;
  hipLaunchKernelGGL(screen_fused_kernel<8>, dim3((waves + 3) / 4), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(screen_fused_kernel<16>, dim3((waves / 8 + 3) / 4 + 1), dim3(256), 0, s, a);
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
