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
#define TT_ESCRATCH -6 /* tt_enumerate_noalloc: the input's workspace exceeds
                          TT_NOALLOC_SCRATCH_BYTES */

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
/* Source: no passage of the paper defines the enumeration, the packing or
 * the support; the semantics stated at the top of this file are this
 * library's reading.  Rows follow the digit order whose Karnaugh-map
 * numbering is the 4-variable map template of the paper's preamble. */

/* Enumerate the full truth tables of n neurons into d_tables (a buffer of
 * total_words uint64 words; every neuron's o*W words at word_off must lie
 * inside it and ranges must not overlap).  If d_hist is not NULL it receives
 * hist[i*8 + v] = number of rows of neuron i with q = v (bins >= 2^o are 0).
 * One-shot ("plain") path: descriptors are grouped by (F, b, o) and each
 * group is enumerated by its own pair of kernel launches. */
int tt_enumerate(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                 uint32_t* d_hist, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * enumeration, arguments, outputs and errors as tt_enumerate, but the
 * workspace (staged descriptors, mask tables, work lists, folded parameters)
 * lives in a fixed device array of TT_NOALLOC_SCRATCH_BYTES bytes inside the
 * library instead of a stream-ordered allocation.  The call makes no
 * hipMalloc/hipFree or other allocating device call; it copies the staged
 * descriptors from host memory with hipMemcpyAsync.
 *  - Limit: an input whose workspace exceeds the array returns TT_ESCRATCH
 *    before any device work.  The workspace is about 128 B per neuron, plus
 *    8 B per mask-table entry (per neuron: the sum over its low six row bits
 *    of |w_j| * 2^(bit within digit j), plus 2; at most 2306), plus about
 *    2 KiB per tile of up to 32 neurons of one (F, b, o).  For example, 8192
 *    neurons of up to 16 input bits with |w| <= 7 need about 3 MiB, and
 *    about 1800 neurons with the largest mask table fill the array.
 *  - Each device holds its own copy of the array from the first call on it
 *    until the process ends.  All calls on one device share it and it keeps
 *    the last call's contents (nothing in it needs to start at zero).  Calls
 *    on one stream are ordered; calls on one device that may overlap (other
 *    streams, other threads) race on the array and must not be issued. */
#define TT_NOALLOC_SCRATCH_BYTES (32u << 20)
int tt_enumerate_noalloc(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
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

/* One whole step on the plan's own tables: the results of tt_plan_launch
 * (enumeration, with the histogram when d_hist is not NULL) followed by
 * tt_plan_support_enumerated into d_support (skipped when NULL).  The
 * support of neurons whose sums span fewer than 512 values is decided by
 * the enumeration's own preparation pass; the others take one more kernel.
 * With TT_PLAN_GRAPH the whole step is captured once into one hipGraph and
 * replayed; it is captured again when a pointer changes.  With
 * TT_PLAN_TIMING (and no graph) the enumeration kernels are timed as in
 * tt_plan_launch.  Same sharing rules as tt_plan_launch. */
int tt_plan_step(tt_plan* plan, uint64_t* d_tables, uint32_t* d_hist, uint8_t* d_support, void* stream);

/* Release the plan's workspace and graph (synchronises the device). */
int tt_plan_destroy(tt_plan* plan);

/* Support and/or histogram (as tt_support) of the plan's neurons over
 * d_tables, using work lists prepared when the plan was created.  Shares the
 * plan's workspace: must not overlap in time with other calls on the plan. */
int tt_plan_support(tt_plan* plan, const uint64_t* d_tables, uint8_t* d_support, uint32_t* d_hist,
                    void* stream);

/* As tt_plan_support, for tables that hold this plan's own enumeration of
 * its neurons (written by tt_plan_launch, or any exact enumeration of the
 * same descriptors, and unchanged since).  The support is then decided from
 * the neurons' parameters, with no table read: q is non-decreasing in the
 * pre-activation a and jumps exactly at the thresholds (at those >= 1 under
 * ReLU), so input j matters iff for some value s of bias + the other inputs'
 * weighted sum, the range of s + w_j x_j over x_j = 0 .. 2^b - 1 contains a
 * jump point t (lo < t <= hi); the set of such s is a subset sum, computed
 * as a bitset.  d_hist, if given, is still counted from the tables.  Results
 * equal tt_plan_support's on such tables; on other tables they are
 * unspecified.  Same errors and sharing rules as tt_plan_support. */
int tt_plan_support_enumerated(tt_plan* plan, const uint64_t* d_tables, uint8_t* d_support, uint32_t* d_hist,
                               void* stream);

/* With TT_PLAN_TIMING: waits for the recorded launches and returns the
 * duration in milliseconds of the enumeration kernel of each launch since
 * the previous call (oldest first, at most max_count; the plan keeps the
 * last 256).  *count receives how many were written. */
int tt_plan_kernel_times(tt_plan* plan, float* h_ms, int max_count, int* count);

/* Report the plan's configuration and size. */
int tt_plan_info(const tt_plan* plan, tt_tune* tune, int* n_items, int* n_groups, int* grid);

/* Number of the plan's neurons with at least 2^12 words per plane
 * (F*b >= 18).  Their tables are written by the wide kernel, one wave per
 * 256 words of one neuron with no work queue; the tune settings apply to the
 * other neurons.  TT_EINVAL for a NULL argument. */
int tt_plan_wide_neurons(const tt_plan* plan, int* n_wide);

/* Time candidate tt_tune settings on the given descriptors and table buffer
 * (which it overwrites) and return the fastest in *best; if cache_path is
 * not NULL the result is read from / appended to that text file, keyed by
 * device and a signature of the workload.  Synchronous. */
int tt_autotune(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                const char* cache_path, tt_tune* best);

/* ------------------------------------------------------------------------
 * Networks of enumerated neurons evaluated through their packed tables
 * (lookups only).  Signals 0 .. n_inputs - 1 are primary input codes and
 * signal n_inputs + i is the output code of neuron i.  Neuron i reads its
 * input j < F from signal h_fanin[8 i + j] (entries j >= F are ignored),
 * which must lie below n_inputs + i, and takes that code modulo 2^b; its
 * output is q at the row r those digits form: bit r % 64 of word r / 64 of
 * each plane p (the tables at word_off, e.g. from tt_enumerate).  Inputs
 * are uint8 [batch][n_inputs] and outputs uint8 [batch][n] (codes < 2^o),
 * both device memory.  Evaluated level by level (a level reads only the
 * inputs and earlier levels): one launch for the whole network, with each
 * block's 64 samples' codes in LDS, when n_inputs + n is at most 1019; else
 * one launch per level.
 * --------------------------------------------------------------------- */
typedef struct tt_lutnet tt_lutnet;

/* Build a reusable handle for a network: validates the descriptors and the
 * fan-in, groups the neurons by level and stages everything the kernels read
 * into a device workspace owned by the handle (in the single-launch form
 * this includes a copy of the tables with the planes interleaved, made on
 * stream).  d_tables must hold the tables when stream reaches this call and
 * must not change while the handle exists.  TT_EINVAL for bad descriptors,
 * fan-in out of range or NULL pointers; TT_ERANGE for tables beyond
 * total_words; TT_ENOMEM when the workspace cannot be allocated. */
int tt_lutnet_create(const tt_neuron* h_desc, int n, const int32_t* h_fanin, int n_inputs, const uint64_t* d_tables,
                     uint64_t total_words, void* stream, tt_lutnet** net);

/* Evaluate batch samples: d_inputs [batch][n_inputs], d_out [batch][n];
 * asynchronous on stream, no allocation.  Calls on different streams may
 * overlap (the handle is only read).  TT_EINVAL for a NULL handle or
 * buffer, or batch < 0. */
int tt_lutnet_run(const tt_lutnet* net, const uint8_t* d_inputs, int batch, uint8_t* d_out, void* stream);

/* Sample inputs that meet output constraints (rejection sampling, single-
 * launch form only).  Draws first_draw .. first_draw + n_draws - 1 are
 * evaluated; draw d's input j is byte j % 8 of output number d Q + j / 8 + 1
 * (Q = ceil(n_inputs / 8)) of a SplitMix64 stream seeded with seed (Steele,
 * Lea and Flood, OOPSLA 2014), reduced modulo 2^b when every reader of input
 * j takes b digits (else the whole byte).  A draw is kept when signal
 * h_target_signal[t] carries h_target_value[t] for every t < n_targets (up
 * to 64 targets; no targets keep every draw).  *d_count (device, uint32) is
 * increased by the number of kept draws; the k-th draw kept by this call is
 * stored at place c + k, c = *d_count before the call, if that is below
 * max_found: its inputs in d_found_inputs [max_found][n_inputs] and its
 * draw number in d_found_draw [max_found].  Which draws are kept is exact;
 * the order of the places is not (concurrent blocks).  Asynchronous on
 * stream, no allocation.  TT_EINVAL for a NULL or empty network, targets
 * out of range or NULL buffers; TT_ERANGE when the network only takes the
 * per-level form. */
int tt_lutnet_sample(const tt_lutnet* net, const int32_t* h_target_signal, const uint8_t* h_target_value,
                     int n_targets, uint64_t seed, uint64_t first_draw, int n_draws, uint8_t* d_found_inputs,
                     uint64_t* d_found_draw, int max_found, uint32_t* d_count, void* stream);

/* Wait for the device and free the handle (NULL is a no-op). */
int tt_lutnet_destroy(tt_lutnet* net);

/* One-shot form: create, run and free in stream order (the workspace is
 * allocated and freed with the stream-ordered allocator).  Errors as
 * tt_lutnet_create and tt_lutnet_run; with batch 0 only the arguments are
 * checked. */
int tt_lutnet_eval(const tt_neuron* h_desc, int n, const int32_t* h_fanin, int n_inputs, const uint64_t* d_tables,
                   uint64_t total_words, const uint8_t* d_inputs, int batch, uint8_t* d_out, void* stream);

/* ------------------------------------------------------------------------
 * CNF to multi-level circuit (the transformation algorithm of the paper's
 * Section "Transformation Algorithm", Algorithm 1), with every candidate
 * expression evaluated as a packed truth table.  Clauses are appended in
 * order to a sub-clause list SC; after each append the variables of SC that
 * are neither primary inputs nor intermediate are tried in decreasing index
 * as its output v: f is the conjunction of the clauses of SC holding -v
 * (that literal removed), g the same for +v, over the other variables of SC;
 * v is accepted when f is the complement of g.  Then v becomes a primary
 * output (f constant) or intermediate, the other variables of SC that are
 * not intermediate become primary inputs, and SC is emptied.  An SC with no
 * output whose variables occur in no later clause becomes an auxiliary
 * output constrained to 1 (the conjunction of SC).
 * --------------------------------------------------------------------- */
#define TT_CNF_MAX_VARS 12 /* variables in one SC */
#define TT_CNF_IV 1        /* expression kinds */
#define TT_CNF_PO 2
#define TT_CNF_AUX 3
#define TT_CNF_CLS_PI 1    /* variable class bits */
#define TT_CNF_CLS_IV 2
#define TT_CNF_CLS_PO 4

/* One found expression, 640 bytes. */
typedef struct tt_cnf_expr {
  int32_t out;       /* output variable; 0 for an auxiliary output */
  int32_t kind;      /* TT_CNF_IV, TT_CNF_PO (f constant) or TT_CNF_AUX */
  int32_t first;     /* SC = the instance's clauses first .. last (0-based) */
  int32_t last;
  int32_t n_vars;    /* table variables */
  uint32_t support;  /* bit j: the table depends on vars[j] */
  int32_t vars[TT_CNF_MAX_VARS]; /* ascending; vars[j] is digit j of the row */
  int32_t pad[14];
  uint64_t table[64]; /* bit r of the 2^n_vars-row table: bit r % 64 of word r / 64 */
} tt_cnf_expr;

typedef struct tt_cnf tt_cnf;

/* Stage n_inst CNF instances for transformation.  Host CSR input: instance
 * t owns clauses h_inst_off[t] .. h_inst_off[t + 1] - 1, clause c owns
 * literals h_lits[h_clause_off[c] .. h_clause_off[c + 1] - 1] (DIMACS: +x or
 * -x, 1 <= x <= h_n_vars[t] <= 32767; no empty clause, no clause holding x
 * and -x; a literal repeated in a clause counts once, as a clause is a set
 * of literals).  The handle owns a device copy (uploaded on stream) and the
 * last use of every clause's variables.  TT_EINVAL for malformed input. */
int tt_cnf_create(const int32_t* h_lits, const int32_t* h_clause_off, const int32_t* h_inst_off, int n_inst,
                  const int32_t* h_n_vars, void* stream, tt_cnf** cnf);

/* Transform the staged instances, one wave each; asynchronous on stream, no
 * allocation.  Device outputs: d_var_class, for instance t at offset
 * sum_{u<t} (h_n_vars[u] + 1), one byte per variable 0 .. n_vars of
 * TT_CNF_CLS_* bits; d_expr, instance t's expressions at d_expr[h_inst_off[t]
 * ...] in the order found (capacity: one per clause); d_n_expr[t] their
 * count; d_status[t] 0, or 1 when an SC grew past TT_CNF_MAX_VARS variables
 * (the instance stops there; what it found before is kept). */
int tt_cnf_run(const tt_cnf* cnf, uint8_t* d_var_class, tt_cnf_expr* d_expr, int32_t* d_n_expr, int32_t* d_status,
               void* stream);

/* Wait for the device and free the handle (NULL is a no-op). */
int tt_cnf_destroy(tt_cnf* cnf);

/* One-shot form: create, run, and free the staged copy once the stream has
 * passed the kernel (synchronises the stream).  Errors as above. */
int tt_cnf_transform(const int32_t* h_lits, const int32_t* h_clause_off, const int32_t* h_inst_off, int n_inst,
                     const int32_t* h_n_vars, uint8_t* d_var_class, tt_cnf_expr* d_expr, int32_t* d_n_expr,
                     int32_t* d_status, void* stream);

/* ------------------------------------------------------------------------
 * Gradient-descent sampling of a transformed CNF (the paper's Methodology:
 * the circuit's logical operators replaced by Table 1's probabilistic ones,
 * the sigmoid embedding P = sigmoid(V), the L2 loss on the constrained
 * outputs, GD, then hardening and the satisfiable / non-redundant filter),
 * one sample per lane.  Each expression is taken in its simplified form
 * (tt_simplify) and valued by composing Table 1's operators over it;
 * derivatives follow the chain rule through those operators.  Primary
 * inputs carry the logits; intermediate variables their expression's value;
 * a constant expression (TT_CNF_PO) fixes its variable unless that variable
 * is also a primary input, in which case it adds (P - c)^2 to the loss; an
 * auxiliary output adds (P - 1)^2.
 * --------------------------------------------------------------------- */
typedef struct tt_gd tt_gd;

/* Build the sampler of one transformed instance: its clauses (host CSR as
 * for tt_cnf_create, one instance), its expressions and class bytes as
 * tt_cnf_run wrote them (copied to the host; the transformation must have
 * ended with status 0).  Simplifies every expression on the host and
 * compiles the circuit's own kernel (see tt_gd_kernel; host time grows with
 * the circuit, about 0.1 to 1 s).
 * TT_EINVAL for malformed input; TT_ERANGE when a form cannot be found
 * within tt_simplify's search budget. */
int tt_gd_create(const int32_t* h_lits, const int32_t* h_clause_off, int n_clauses, int n_vars,
                 const tt_cnf_expr* h_expr, int n_expr, const uint8_t* h_var_class, void* stream, tt_gd** gd);

/* Number of primary inputs (logit columns). */
int tt_gd_inputs(const tt_gd* gd, int* n_pi);

/* The variable of each logit column, h_vars[n_pi] (host): the primary inputs
 * in the order the transformation appended them (an expression's variables
 * in ascending index, expressions in the order found). */
int tt_gd_input_vars(const tt_gd* gd, int32_t* h_vars);

/* Run iters GD steps of rate lr on batch samples: d_V [batch][n_pi] fp32
 * holds the initial logits and receives the final ones; d_valid[batch] gets
 * 1 where the hardened assignment (primary input = V > 0, the rest through the
 * forms) satisfies every clause; d_solution [batch][ceil(n_pi / 64)] the
 * hardened primary inputs as bits (column q = bit q % 64 of word q / 64).
 * Asynchronous on stream.  With at most 20 slots (variables in use plus the
 * largest form's temporaries) the state of a wave's samples lives in LDS
 * and nothing is allocated; larger circuits use a stream-ordered workspace
 * of 8 bytes per variable plus 4 per primary input per sample (more waves
 * per CU than LDS-resident state would allow), the forms' temporaries
 * staying in LDS (in the workspace too, 8 bytes each per sample, when they
 * exceed 32 KiB per wave). */
int tt_gd_run(const tt_gd* gd, float* d_V, int batch, float lr, int iters, uint8_t* d_valid, uint64_t* d_solution,
              void* stream);

/* tt_gd_run with the initial and final logits apart: d_V0 [batch][n_pi]
 * fp32 holds the initial logits and is only read; d_V receives the final
 * logits, and may be NULL (not kept) or d_V0 itself (tt_gd_run); otherwise
 * it must not overlap d_V0.  d_valid and d_solution as in tt_gd_run.  The
 * compiled kernel keeps a sample's logits in registers, so it reads d_V0
 * and writes d_V directly; the interpreter works in place, on d_V (a
 * device copy of d_V0 first) or, with d_V NULL, on a stream-ordered copy
 * freed after the run.  Asynchronous on stream.  TT_EINVAL for missing
 * arguments. */
int tt_gd_run_from(const tt_gd* gd, const float* d_V0, float* d_V, int batch, float lr, int iters,
                   uint8_t* d_valid, uint64_t* d_solution, void* stream);

/* Distinct valid solutions: d_first[i] = 1 for exactly one sample of every
 * distinct valid solution (which one is not fixed), 0 otherwise; *d_count is
 * increased by their number.  Uses a stream-ordered workspace of 4 bytes per
 * place of two tables: a power of two of about 16 batch places (between 2^10
 * and 2^24; 64 MiB at 2^20 samples) that each valid sample writes and reads
 * back, and a power of two of at least 2 batch places for the samples whose
 * place another solution took.  TT_ERANGE for a batch above 2^30. */
int tt_gd_unique(const tt_gd* gd, const uint8_t* d_valid, const uint64_t* d_solution, int batch, uint8_t* d_first,
                 uint32_t* d_count, void* stream);

/* tt_gd_run_from followed by tt_gd_unique, with the same arguments and
 * results (the sample marked first for a solution may differ between runs),
 * in fewer passes: with the compiled kernel selected, that kernel also does
 * the filter's first pass (each valid sample stores its index at its
 * solution's place) and clears the filter's second table, so one filter
 * launch follows instead of three.  The same stream-ordered workspace as
 * tt_gd_unique.  With the interpreter selected it makes the two calls.
 * TT_EINVAL for missing arguments, TT_ERANGE for a batch above 2^30. */
int tt_gd_sample_unique(const tt_gd* gd, const float* d_V0, float* d_V, int batch, float lr, int iters,
                        uint8_t* d_valid, uint64_t* d_solution, uint8_t* d_first, uint32_t* d_count, void* stream);

/* Which kernel tt_gd_run launches.  tt_gd_create also compiles the circuit
 * with the HIP run-time compiler into a kernel of its own: the same
 * computation written out as straight-line code, a sample's probabilities,
 * adjoints and logits held in registers, one sample per thread (no memory
 * traffic beyond its logits and results).  That kernel is the default.
 * Circuits above 8192 gates, 512 variables or 32768 clause literals, or a
 * failed compilation, leave the interpreted kernel only (one kernel for
 * every circuit, walking the gate program with the state in LDS or a
 * workspace).  Both give the same results up to float rounding order.
 * tt_gd_kernel reports the current choice; tt_gd_set_kernel selects one
 * (TT_ENOTSUP for TT_GD_COMPILED without a compiled kernel).  The compiled
 * kernel is loaded on the device current at tt_gd_create. */
#define TT_GD_INTERPRETED 0
#define TT_GD_COMPILED 1
int tt_gd_kernel(const tt_gd* gd, int* kernel);
int tt_gd_set_kernel(tt_gd* gd, int kernel);

/* Wait for the device and free the sampler (NULL is a no-op). */
int tt_gd_destroy(tt_gd* gd);

/* ------------------------------------------------------------------------
 * Two-level minimisation of one plane, on the host (the step after
 * enumeration; runs on the CPU, reading a plane copied back from the
 * device or from tt_pack).
 * --------------------------------------------------------------------- */

/* Minimal sum of products of one plane over n_vars <= 12 digits (row r =
 * bit r % 64 of word r / 64, digit j of r = variable j): Quine-McCluskey
 * prime implicants, essential primes, then a branch-and-bound search for a
 * cover of fewest terms and, among those, fewest literals; among covers of
 * equal cost the one whose sorted list of term keys is smallest (the key of
 * a term lists its literals in ascending variable order, x_j as 2j and
 * NOT x_j as 2j + 1; lists compare lexicographically, a prefix first).
 * Terms are written in ascending key order.  Term t covers
 * the rows r with (r & h_care[t]) == h_value[t] (variable j appears when
 * bit j of care is set, positive when bit j of value is set); up to
 * max_terms terms are written.  *exact is 1 when the search finished within
 * node_budget nodes (<= 0: one million), else 0 (the best cover found is
 * returned).  The constant 0 has no terms; the constant 1 one term with no
 * literals.  TT_EINVAL for NULL arguments or n_vars out of range. */
int tt_sop_minimize(const uint64_t* h_plane, int n_vars, long node_budget, int max_terms, uint32_t* h_care,
                    uint32_t* h_value, int* n_terms, int* n_literals, int* exact);

/* Simplify (Algorithm 1 appends the simplified form of each found
 * expression; the Methodology then replaces the form's logical operators by
 * Table 1's probabilistic ones).  The form of a table over n_vars <= 12
 * digits, as a program of gates:
 *   - the table is restricted to its support (the digits it depends on);
 *   - no support: the constant;
 *   - the parity of two or more support digits: XOR chained over them in
 *     ascending digit, XNOR as the last link for the complement of parity;
 *   - otherwise the minimal sum of products of tt_sop_minimize (its tie
 *     rule; terms in ascending key order) as an OR chain of the terms, each
 *     an AND chain of its literals in ascending digit, NOT x as a negated
 *     operand.
 * A chain op(op(x0, x1), x2) ... is written left to right.  Gate i computes
 * op over its operands a (and b) and writes temporary i (dst = i), except
 * the last gate, which writes the form's value (dst = -1).  An operand is a
 * digit index, or with TT_OPD_TEMP set a temporary's index, and with
 * TT_OPD_NEG set the operand is NOT of that value.  TT_GATE_CONST outputs a
 * (0 or 1); TT_GATE_COPY outputs operand a (a lone literal).  Writes up to
 * max_gates gates, *n_gates their number (TT_ERANGE and the number needed
 * when max_gates is smaller); *exact as for tt_sop_minimize.  Host only.
 * TT_EINVAL for NULL arguments or n_vars out of range. */
#define TT_GATE_CONST 0
#define TT_GATE_COPY 1
#define TT_GATE_AND 2
#define TT_GATE_OR 3
#define TT_GATE_XOR 4
#define TT_GATE_XNOR 5
#define TT_OPD_TEMP (1 << 16)
#define TT_OPD_NEG (1 << 17)
typedef struct tt_gate {
  int32_t op, a, b, dst;
} tt_gate;
int tt_simplify(const uint64_t* h_table, int n_vars, int max_gates, tt_gate* h_gates, int* n_gates, int* exact);

/* Text of the four-variable Karnaugh map of a one-word plane (rows x1 x2,
 * columns x3 x4 in Gray order; the cell holds row 8 x1 + 4 x2 + 2 x3 + x4,
 * x1 the most significant digit of r).  buf needs at least 128 bytes. */
int tt_kmap_text(const uint64_t* h_plane, char* buf, int size);

/* ------------------------------------------------------------------------
 * Learned screen.  These entry points take DEVICE descriptors (d_desc: a
 * device copy of tt_neuron[n], word_off already laid out), so that a whole
 * screening pass runs on the device without a host round trip.  Device
 * descriptors are checked by the kernels: a neuron with fields out of range,
 * F*b > 16, or tables beyond total_words is skipped and bit 0 of *d_status
 * (if not NULL) is set.  All matrices are row-major; bf16 values are passed
 * as uint16_t bit patterns; products accumulate in fp32.
 * --------------------------------------------------------------------- */

/* Enumerate small neurons (F*b <= 16), one workgroup per neuron, from device
 * descriptors; neurons with d_active[i] == 0 are skipped (d_active may be
 * NULL). */
int tt_enumerate_device(const tt_neuron* d_desc, int n, const uint8_t* d_active, uint64_t* d_tables,
                        uint64_t total_words, uint32_t* d_status, void* stream);

/* Support and histogram (as tt_support) of small neurons from device
 * descriptors; either output may be NULL. */
int tt_support_device(const tt_neuron* d_desc, int n, const uint64_t* d_tables, uint64_t total_words,
                      uint8_t* d_support, uint32_t* d_hist, uint32_t* d_status, void* stream);

/* Screen input features, d_x[n][32] in bf16: w_j/8, w_j(2^b-1)/32, bias/16,
 * thresholds/32 (the last used one repeated), largest and smallest
 * pre-activation /32, b/4, one-hot o, F/8, act. */
int tt_screen_features(const tt_neuron* d_desc, int n, uint16_t* d_x, void* stream);

/* Training targets from exact support and histogram: d_y[n][8] support bits,
 * d_m[n][8] valid-input mask (j < F), d_h[n][4] histogram fractions (o = 1:
 * bins {0, 1}; o = 2: the codes; o = 3: bin v holds codes 2v and 2v+1). */
int tt_screen_labels(const tt_neuron* d_desc, int n, const uint8_t* d_support, const uint32_t* d_hist, float* d_y,
                     float* d_m, float* d_h, void* stream);

/* One dense layer: y = x W^T + bias (then max(y, 0) if relu), x[batch][in]
 * bf16, W[out][in] bf16, bias[out] fp32 (may be NULL); the result goes to
 * y_bf16 and/or y_f32 (either may be NULL). */
int tt_mlp_forward(const uint16_t* d_x, int batch, int in, const uint16_t* d_w, const float* d_bias, int out,
                   int relu, uint16_t* d_y_bf16, float* d_y_f32, void* stream);

/* Inference of the whole screening network 32 -> 256 -> 256 -> 256 -> 12 in
 * one launch: logits[n][12] (fp32) for features x[n][32] (bf16), weights
 * W1[256][32], W2[256][256], W3[256][256], W4[12][256] (bf16, [out][in]),
 * biases fp32 (any may be NULL), ReLU after the hidden layers.  The same
 * arithmetic as four tt_mlp_forward calls (fp32 accumulation, hidden
 * activations rounded to bf16), with the activations kept on chip; sums may
 * be ordered differently, so results agree to fp32 rounding.  x, the
 * weights and the biases must be 16-byte aligned (TT_EINVAL otherwise, or
 * for n < 0 or a NULL x, weight or logits pointer). */
int tt_mlp_infer(const uint16_t* d_x, int n, const uint16_t* d_w1, const float* d_b1, const uint16_t* d_w2,
                 const float* d_b2, const uint16_t* d_w3, const float* d_b3, const uint16_t* d_w4, const float* d_b4,
                 float* d_logits, void* stream);

/* Backward of one layer given dL/dy[batch][out] (bf16): dx = dy W (times the
 * ReLU derivative x > 0 of the layer input when relu_mask, bf16, may be
 * NULL), dW = dy^T x (fp32 [out][in], may be NULL), db = column sums of dy
 * (fp32 [out], may be NULL).  dW and db need x and d_scratch; a d_scratch,
 * when given, must hold scratch_floats >= tt_mlp_scratch_floats(batch,
 * max(in, out)) floats (TT_ERANGE if smaller), and dx then uses it for a
 * transposed copy of W.  dW and db are summed over batch slices whose
 * partial products are reduced in a fixed order, so results do not depend
 * on scheduling. */
int tt_mlp_backward(const uint16_t* d_dy, int batch, int out, const uint16_t* d_w, int in, const uint16_t* d_x,
                    int relu_mask, uint16_t* d_dx, float* d_dw, float* d_db, float* d_scratch, size_t scratch_floats,
                    void* stream);

/* Scratch floats needed by tt_mlp_backward / tt_mlp_loss for this batch and
 * layers whose in and out are at most dim. */
size_t tt_mlp_scratch_floats(int batch, int dim);

/* Loss (averaged over the batch, into d_loss[0]) and dL/dz (bf16 [batch][12])
 * for logits z[batch][12]: binary cross-entropy of the 8 support logits
 * masked by m, plus the squared error of the 4 histogram outputs (a
 * squared-difference regression loss of the kind the paper's Methodology
 * section minimises by gradient descent; the rest of the screen is not in
 * the paper). */
int tt_mlp_loss(const float* d_z, int batch, const float* d_y, const float* d_m, const float* d_h, uint16_t* d_dz,
                float* d_loss, float* d_scratch, void* stream);

/* Adam with bias correction on n fp32 master parameters (step >= 1 counts
 * updates); writes the bf16 copy used by the layers if d_p_bf16 is not NULL. */
int tt_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, uint16_t* d_p_bf16, size_t n, float lr,
                 float beta1, float beta2, float eps, int step, void* stream);

/* tt_adam_step on count (<= 8) tensors in one launch: h_d_p[t] ... are HOST
 * arrays of device pointers (h_d_p_bf16 may be NULL, or hold NULL entries),
 * h_n[t] the element counts; every tensor takes the same lr, betas, eps and
 * step.  Identical results to count separate tt_adam_step calls. */
int tt_adam_step_multi(int count, float* const* h_d_p, const float* const* h_d_g, float* const* h_d_m,
                       float* const* h_d_v, uint16_t* const* h_d_p_bf16, const size_t* h_n, float lr, float beta1,
                       float beta2, float eps, int step, void* stream);

/* y = x rounded to bf16 (nearest, ties to even), n elements. */
int tt_cast_bf16(const float* d_x, uint16_t* d_y, size_t n, void* stream);

/* Device workspace tt_screen_run needs for n candidates. */
size_t tt_screen_work_bytes(int n);

/* Screen n candidates (F*b <= 16) after the screen's forward pass.  A lane
 * pass settles every candidate whose table, reduced to the inputs of nonzero
 * weight (or full, when every weight is nonzero), has at most 64 rows: there
 * S = the inputs of nonzero weight (an input with zero weight never
 * matters; a prediction cannot save work on one word per plane).  A wave
 * pass, one wavefront per candidate, takes the others: their predicted
 * support is S = { j < F : w_j != 0 and logits[i][j] > logit(tau) }, so only
 * their rows of d_logits are read.  d_force_mask[i], if not NULL, replaces S
 * for every candidate; with d_logits and d_force_mask both NULL every
 * candidate is enumerated in full, the method without the screen.  The two
 * reduced neurons over S alone, with the skipped inputs at the two ends of
 * their range, are evaluated word by word; the candidate is accepted iff
 * their tables agree, which holds exactly when no skipped input matters;
 * otherwise (or when nothing can be skipped) it is enumerated in full.
 * Outputs: d_support and d_hist of the FULL table of every candidate (exact
 * either way); d_tables: the reduced table of an accepted candidate / the
 * full table of the others, at its word_off; d_mask / d_accept (may be
 * NULL): S and the acceptance.  d_work: tt_screen_work_bytes(n) bytes, kept
 * for tt_screen_expand. */
int tt_screen_run(const tt_neuron* d_desc, int n, const float* d_logits, float tau, const uint8_t* d_force_mask,
                  uint64_t* d_tables, uint64_t total_words, uint8_t* d_support, uint32_t* d_hist, uint8_t* d_mask,
                  uint8_t* d_accept, void* d_work, uint32_t* d_status, void* stream);

/* The screen's network on device descriptors in one launch: the features of
 * tt_screen_features computed in the kernel (no feature buffer), then the
 * layers of tt_mlp_infer.  gated = 0: logits[i][0..12) for every candidate.
 * gated = 1: only for the candidates tt_screen_run's wave pass takes (table
 * reduced to the inputs of nonzero weight, or full, above 64 rows); the
 * other rows of d_logits are not written.  Up to 2^21 candidates a first
 * pass compacts them into a list in d_work (tt_screen_infer_work_bytes(n)
 * bytes, 4-byte aligned; NULL: a stream-ordered allocation made and freed
 * in the call) that one block per CU then takes in even chunks; above,
 * each block finds and compacts the ones among its own 256 candidates and
 * d_work is not used.  Weights and biases as in tt_mlp_infer.  TT_EINVAL
 * for missing or misaligned arguments. */
int tt_screen_infer(const tt_neuron* d_desc, int n, int gated, const uint16_t* d_w1, const float* d_b1,
                    const uint16_t* d_w2, const float* d_b2, const uint16_t* d_w3, const float* d_b3,
                    const uint16_t* d_w4, const float* d_b4, float* d_logits, void* d_work, void* stream);

/* Bytes of the gated tt_screen_infer's list for n candidates (0 when n is
 * not positive or above 2^21, where no list is used). */
size_t tt_screen_infer_work_bytes(int n);

/* Full tables of the candidates of the last tt_screen_run on d_work: reduced
 * tables broadcast over the skipped inputs, full tables copied. */
int tt_screen_expand(const tt_neuron* d_desc, int n, const void* d_work, const uint64_t* d_screened,
                     uint64_t* d_full, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TT_H_ */
