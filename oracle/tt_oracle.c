/*
 * tt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain, slow, obviously correct CPU oracle for truth-table enumeration
 * of quantised neurons.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header or table with
 * the HIP library: it has its own digit decode, its own plane layout
 * arithmetic, its own packing, histogram and support routines.
 *
 * What it computes (the plain definition, nothing blocked, fused or
 * reordered).  A neuron has F inputs of b unsigned bits, int8 weights w[j],
 * an int16 bias, an activation act (0 identity, 1 ReLU) and K = 2^o - 1
 * thresholds t[k].  For every row index r in [0, 2^(F*b)):
 *
 *   x_j = (r >> (j*b)) & (2^b - 1)          input j is digit j of r, input 0
 *                                            least significant; in a Karnaugh
 *                                            map the most significant bit of r
 *                                            is the first variable x1, as in
 *                                            the K-map templates of the
 *                                            paper's preamble (cell number =
 *                                            8*x1 + 4*x2 + 2*x3 + x4)
 *   a   = bias + sum_j w_j * x_j             exact, 64-bit
 *   a'  = act ? max(a, 0) : a
 *   q   = #{ k : a' >= t[k] }                ties go to the upper bin
 *   plane p, bit r  = (q >> p) & 1           word r/64, bit r%64 of plane p
 *   hist[v]         = #{ r : q(r) = v }
 *   support         = { j : some rows r, r' that differ only in digit j have
 *                       q(r) != q(r') }
 *
 * Plane layout: neuron i owns o_i planes of W_i = max(1, 2^(F_i*b_i) / 64)
 * little-endian uint64 words each, plane p at word_off[i] + p*W_i; the
 * canonical word_off is the prefix sum of o_i * W_i.  Bits for rows beyond
 * 2^(F*b) (only when F*b < 6) are zero.
 *
 * The paper itself contains no enumeration method: the neuron semantics above
 * follow the truth-table reading recorded with the design, and the only
 * passages of the paper used are the pruned-Gaussian weight density and the
 * Karnaugh-map numbering of its preamble.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_F 8
#define ORACLE_MAX_T 7

uint64_t oracle_rows(int F, int b) { return (uint64_t)1 << (F * b); }

uint64_t oracle_words_per_plane(int F, int b) {
  uint64_t r = oracle_rows(F, b);
  return r < 64 ? 1 : r / 64;
}

/* Canonical layout: prefix sum of o * W.  Returns 0. */
int oracle_offsets(int n, const uint8_t* F, const uint8_t* b, const uint8_t* o,
                   uint64_t* word_off, uint64_t* total_words) {
  uint64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    word_off[i] = acc;
    acc += (uint64_t)o[i] * oracle_words_per_plane(F[i], b[i]);
  }
  *total_words = acc;
  return 0;
}

/* The output code q of every row of one neuron, straight from the definition. */
void oracle_neuron_codes(int F, int b, int o, int act, const int8_t* w, int bias,
                         const int32_t* thr, uint8_t* codes) {
  const uint64_t rows = oracle_rows(F, b);
  const uint64_t digit_mask = ((uint64_t)1 << b) - 1;
  const int K = (1 << o) - 1;
  for (uint64_t r = 0; r < rows; ++r) {
    int64_t a = bias;
    for (int j = 0; j < F; ++j) {
      int64_t x = (int64_t)((r >> (j * b)) & digit_mask);
      a += (int64_t)w[j] * x;
    }
    if (act == 1 && a < 0) a = 0;
    int q = 0;
    for (int k = 0; k < K; ++k)
      if (a >= (int64_t)thr[k]) q++;
    codes[r] = (uint8_t)q;
  }
}

/* Scatter codes into o bit-planes of W words (planes must hold o*W words). */
void oracle_codes_to_planes(int F, int b, int o, const uint8_t* codes, uint64_t* planes) {
  const uint64_t rows = oracle_rows(F, b);
  const uint64_t W = oracle_words_per_plane(F, b);
  memset(planes, 0, sizeof(uint64_t) * W * (uint64_t)o);
  for (uint64_t r = 0; r < rows; ++r)
    for (int p = 0; p < o; ++p)
      if ((codes[r] >> p) & 1) planes[(uint64_t)p * W + r / 64] |= (uint64_t)1 << (r % 64);
}

/* Histogram of the o-bit codes: hist[v] for v in [0, 8); bins >= 2^o stay
 * zero.  Only the low o bits of a code are kept in the planes, so only they
 * are counted. */
void oracle_codes_hist(int F, int b, int o, const uint8_t* codes, uint32_t* hist8) {
  const uint64_t rows = oracle_rows(F, b);
  const int m = (1 << o) - 1;
  for (int v = 0; v < 8; ++v) hist8[v] = 0;
  for (uint64_t r = 0; r < rows; ++r) hist8[codes[r] & m]++;
}

/* Support bitmask (bit j = input j).  Input j is in the support iff two rows
 * that differ only in digit j carry different codes.  If rows with digit j
 * equal to u and v (u != v, everything else equal) differ, then the row with
 * digit j equal to 0 differs from at least one of them; so comparing every
 * row whose digit j is 0 with each of its 2^b - 1 siblings decides exactly
 * the same set. */
uint8_t oracle_codes_support(int F, int b, int o, const uint8_t* codes) {
  const uint64_t rows = oracle_rows(F, b);
  const uint64_t digit_mask = ((uint64_t)1 << b) - 1;
  const int m = (1 << o) - 1;
  uint8_t s = 0;
  for (int j = 0; j < F; ++j) {
    const int shift = j * b;
    int found = 0;
    for (uint64_t r = 0; r < rows && !found; ++r) {
      if ((r >> shift) & digit_mask) continue;
      for (uint64_t v = 1; v <= digit_mask; ++v) {
        if ((codes[r] & m) != (codes[r | (v << shift)] & m)) { found = 1; break; }
      }
    }
    if (found) s |= (uint8_t)(1u << j);
  }
  return s;
}

/* Enumerate n neurons (weights w[i*8 + j], thresholds thr[i*7 + k]).
 * Any of planes / hist (n*8) / support (n) may be NULL.  Neurons are
 * independent, so they are spread over nthreads host threads (<=0: all). */
int oracle_enumerate(int n, const uint8_t* F, const uint8_t* b, const uint8_t* o,
                     const uint8_t* act, const int8_t* w, const int16_t* bias,
                     const int32_t* thr, const uint64_t* word_off, uint64_t* planes,
                     uint32_t* hist, uint8_t* support, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n; ++i) {
    uint8_t* codes = (uint8_t*)malloc((size_t)oracle_rows(F[i], b[i]));
    if (!codes) { err = -4; continue; }
    oracle_neuron_codes(F[i], b[i], o[i], act[i], w + (size_t)i * ORACLE_MAX_F, bias[i],
                        thr + (size_t)i * ORACLE_MAX_T, codes);
    if (planes) oracle_codes_to_planes(F[i], b[i], o[i], codes, planes + word_off[i]);
    if (hist) oracle_codes_hist(F[i], b[i], o[i], codes, hist + (size_t)i * 8);
    if (support) support[i] = oracle_codes_support(F[i], b[i], o[i], codes);
    free(codes);
  }
  return err;
}

/* Codes of all neurons, concatenated (neuron i at the prefix sum of rows). */
int oracle_codes(int n, const uint8_t* F, const uint8_t* b, const uint8_t* o, const uint8_t* act,
                 const int8_t* w, const int16_t* bias, const int32_t* thr, uint8_t* codes_out) {
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    oracle_neuron_codes(F[i], b[i], o[i], act[i], w + (size_t)i * ORACLE_MAX_F, bias[i],
                        thr + (size_t)i * ORACLE_MAX_T, codes_out + off);
    off += oracle_rows(F[i], b[i]);
  }
  return 0;
}

/* Planes, histogram and support of arbitrary concatenated codes (the
 * counterpart of packing and support computed from given tables). */
int oracle_from_codes(int n, const uint8_t* F, const uint8_t* b, const uint8_t* o,
                      const uint8_t* codes, const uint64_t* word_off, uint64_t* planes,
                      uint32_t* hist, uint8_t* support) {
  uint64_t off = 0;
  for (int i = 0; i < n; ++i) {
    const uint8_t* c = codes + off;
    if (planes) oracle_codes_to_planes(F[i], b[i], o[i], c, planes + word_off[i]);
    if (hist) oracle_codes_hist(F[i], b[i], o[i], c, hist + (size_t)i * 8);
    if (support) support[i] = oracle_codes_support(F[i], b[i], o[i], c);
    off += oracle_rows(F[i], b[i]);
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
