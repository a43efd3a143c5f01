/*
 * tt.h -- C ABI of libtt.so: exhaustive truth-table enumeration of pruned,
 * quantised neurons on AMD Instinct MI355X (gfx950).
 *
 * A neuron (struct tt_neuron) has F inputs of b unsigned bits, int8 weights,
 * an int16 bias, an activation and 2^o - 1 thresholds.  For every row index
 * r in [0, 2^(F*b)) the library computes
 *
 *     x_j = (r >> (j*b)) & (2^b - 1)        input j = digit j of r (input 0
 *                                           least significant)
 *     a   = bias + sum_j w_j * x_j          exact integer arithmetic
 *     a'  = act == TT_ACT_RELU ? max(a, 0) : a
 *     q   = #{ k < 2^o - 1 : a' >= thr[k] } ties go to the upper bin
 *
 * and stores q as o bit-planes ("packed tables"): bit r of plane p is bit p
 * of q.  A plane is W = max(1, 2^(F*b) / 64) little-endian uint64 words; row
 * r is bit r % 64 of word r / 64.  Plane p of a neuron starts at word
 * word_off + p * W of the caller's table buffer.  Bits of rows beyond
 * 2^(F*b) (F*b < 6) are written as zero.  In a Karnaugh map of a table the
 * most significant bit of r is the first variable, as in the K-map templates
 * of the paper's preamble (cell number 8*x1 + 4*x2 + 2*x3 + x4).
 *
 * The paper provides the pruned-Gaussian weight density and the Karnaugh-map
 * numbering used here; the enumeration semantics themselves are the
 * truth-table reading of a quantised neuron stated above.
 *
 * Conventions for every entry point
 *  - Pointers prefixed d_ are device pointers (HIP device memory of the
 *    current device), h_ are host pointers.  The caller owns all of them; the
 *    library never frees them and keeps none after the call returns (plans
 *    excepted: a plan keeps its own copy of the descriptors and the device
 *    pointers it was last launched or captured with).
 *  - Descriptors are always passed from HOST memory; the library validates
 *    them and stages what the kernels need into its own device workspace.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously; the call returns after enqueue.  Outputs are valid once
 *    the stream has reached that point.  Library-owned workspace of a one-shot
 *    call is allocated and released in stream order.
 *  - Return value: TT_OK (0) or a negative status below; on error nothing has
 *    been enqueued (except for TT_EHIP, where a HIP call failed midway).
 */
#ifndef TT_H_
#define TT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_F 8    /* inputs per neuron */
#define TT_MAX_B 4    /* bits per input */
#define TT_MAX_O 3    /* output bits: up to 7 thresholds */
#define TT_MAX_FB 30  /* F*b: at most 2^30 rows per neuron */

#define TT_ACT_IDENTITY 0
#define TT_ACT_RELU 1

/* One neuron, 64 bytes, 8-byte aligned. */
typedef struct tt_neuron {
  int8_t w[8];       /* weights; entries j >= F are ignored */
  int32_t thr[7];    /* thresholds; the first 2^o - 1 must be non-decreasing,
                        the rest are ignored */
  int16_t bias;
  uint8_t F;         /* 1..8 */
  uint8_t b;         /* 1..4, F*b <= 30 */
  uint8_t o;         /* 1..3 */
  uint8_t act;       /* TT_ACT_IDENTITY or TT_ACT_RELU */
  uint8_t pad[6];    /* ignored */
  uint64_t word_off; /* word index of plane 0 in the table buffer */
  uint64_t reserved; /* ignored */
} tt_neuron;

/* Status codes. */
#define TT_OK 0
#define TT_EINVAL -1  /* null pointer, n < 0, F/b/o/act out of range,
                         decreasing thresholds, overlapping table ranges */
#define TT_ERANGE -2  /* F*b > 30, or a table range beyond total_words,
                         or a code buffer smaller than the rows */
#define TT_EHIP -3    /* a HIP runtime call failed; see tt_last_hip_error() */
#define TT_ENOMEM -4  /* device or host workspace allocation failed */
#define TT_ENOTSUP -5 /* the current device is not gfx950 */

/* Human-readable text of a status code (static storage). */
const char* tt_strerror(int status);

/* hipError_t of the last failing HIP call in this thread (0 if none). */
int tt_last_hip_error(void);

/* Library version, (major << 16) | minor. */
int tt_version(void);

/* TT_OK if the current HIP device is gfx950, TT_ENOTSUP otherwise,
 * TT_EHIP if no device can be queried. */
int tt_device_check(void);

/* ------------------------------------------------------------------ layout */

/* Host only.  Validates n descriptors (field ranges and threshold order; the
 * word_off fields are not inspected).  No device is needed. */
int tt_validate(const tt_neuron* h_desc, int n);

/* Host only.  Validates and fills word_off with the canonical layout: the
 * prefix sum over neurons of o * W.  *h_total_words receives the number of
 * uint64 words the table buffer needs.  No device is needed. */
int tt_layout(tt_neuron* h_desc, int n, uint64_t* h_total_words);

/* Host only.  Words per plane, W = max(1, 2^(F*b) / 64), or 0 if F*b is out
 * of range. */
uint64_t tt_words_per_plane(int F, int b);

/* ------------------------------------------------------------- enumeration */

/* Enumerate the full truth tables of n neurons into d_tables (a buffer of
 * total_words uint64 words; every neuron's o*W words at word_off must lie
 * inside it and ranges must not overlap).  If d_hist is not NULL it receives
 * hist[i*8 + v] = number of rows of neuron i with q = v (bins >= 2^o are 0).
 * One-shot ("plain") path: descriptors are grouped by (F, b, o) and each
 * group is enumerated by its own pair of kernel launches. */
int tt_enumerate(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                 uint32_t* d_hist, void* stream);

/* Pack per-row output codes into planes.  d_codes holds, for neuron i, its
 * 2^(F*b) codes (one byte per row, row order) starting at byte offset
 * sum_{k<i} 2^(F_k*b_k); total_codes is the size of d_codes in bytes.  Bit p
 * of code r goes to bit r of plane p for p < o; higher code bits are
 * ignored. */
int tt_pack(const tt_neuron* h_desc, int n, const uint8_t* d_codes, uint64_t total_codes,
            uint64_t* d_tables, uint64_t total_words, void* stream);

/* Input support and histogram of packed tables.  d_support[i] gets bit j set
 * iff two rows of neuron i that differ only in digit j carry different codes
 * (only the tables are read; the weights are not consulted).  d_hist, if not
 * NULL, receives the code histogram as in tt_enumerate.  d_support may be
 * NULL when only the histogram is wanted. */
int tt_support(const tt_neuron* h_desc, int n, const uint64_t* d_tables, uint64_t total_words,
               uint8_t* d_support, uint32_t* d_hist, void* stream);

/* ---------------------------------------------------------- batched plans */

typedef struct tt_plan tt_plan;

/* Launch configuration of the batched enumerator. */
typedef struct tt_tune {
  int chunk_words;   /* words per work item along a neuron's rows (multiple of 32) */
  int blocks_per_cu; /* persistent workgroups per compute unit */
  int waves;         /* waves per workgroup: 4 or 8 */
  int nontemporal;   /* 1: streaming (non-temporal) table stores */
  int tile_neurons;  /* neurons per work tile: 8, 16 or 32 (fewer neurons per
                        tile = fewer concurrent output streams, longer runs) */
} tt_tune;

#define TT_PLAN_PERSISTENT 1u /* one launch over an LPT-ordered work queue */
#define TT_PLAN_GRAPH 2u      /* replay the launches from a captured hipGraph */
#define TT_PLAN_TIMING 4u     /* record HIP events around the enumeration
                                 kernel of every launch (not with GRAPH) */

/* Create a plan for n host descriptors (copied; validated like
 * tt_enumerate, against total_words).  tune may be NULL for defaults.
 * Allocates device workspace.  Synchronous. */
int tt_plan_create(const tt_neuron* h_desc, int n, uint64_t total_words, const tt_tune* tune,
                   unsigned flags, tt_plan** plan);

/* Enqueue the enumeration of the plan's neurons into d_tables (and d_hist if
 * not NULL).  With TT_PLAN_GRAPH the first launch (and any launch with
 * different pointers) captures a graph; later launches replay it.  Calls on
 * one plan must not overlap in time (they share the plan's workspace). */
int tt_plan_launch(tt_plan* plan, uint64_t* d_tables, uint32_t* d_hist, void* stream);

/* Release the plan's workspace and graph (synchronises the device). */
int tt_plan_destroy(tt_plan* plan);

/* Support and/or histogram (as tt_support) of the plan's neurons over
 * d_tables, using work lists prepared when the plan was created.  Shares the
 * plan's workspace: must not overlap in time with other calls on the plan. */
int tt_plan_support(tt_plan* plan, const uint64_t* d_tables, uint8_t* d_support, uint32_t* d_hist,
                    void* stream);

/* With TT_PLAN_TIMING: waits for the recorded launches and returns the
 * duration in milliseconds of the enumeration kernel of each launch since
 * the previous call (oldest first, at most max_count; the plan keeps the
 * last 256).  *count receives how many were written. */
int tt_plan_kernel_times(tt_plan* plan, float* h_ms, int max_count, int* count);

/* Report the plan's configuration and size. */
int tt_plan_info(const tt_plan* plan, tt_tune* tune, int* n_items, int* n_groups, int* grid);

/* Time candidate tt_tune settings on the given descriptors and table buffer
 * (which it overwrites) and return the fastest in *best; if cache_path is
 * not NULL the result is read from / appended to that text file, keyed by
 * device and a signature of the workload.  Synchronous. */
int tt_autotune(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                const char* cache_path, tt_tune* best);

#ifdef __cplusplus
}
#endif

#endif /* TT_H_ */
