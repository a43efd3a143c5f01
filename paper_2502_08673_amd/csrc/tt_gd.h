// tt_gd.h -- GD sampling of a transformed CNF: the interpreted kernel
// (tt_gd.hip), the circuit's compiled kernel (tt_gd_compile.hip) and the
// distinct-solution filter.
#pragma once

#include <string>
#include <vector>

#include "tt_internal.h"

namespace tt {

// GD sampling of a transformed CNF (tt_gd.hip).  Slots: primary inputs
// first (in the transformation's order of entry), then every other variable
// in use, then a temporaries region shared by all expressions.
struct GdGate {
  int32_t op, a, b, dst;  // op: TT_GATE_*; a, b: slot | kGdTemp | kGdNeg; dst: slot
};
constexpr int32_t kGdSlot = 0x00FFFFFF, kGdTemp = 1 << 29, kGdNeg = 1 << 30;
struct GdArgs {
  const GdGate* gate;         // intermediate expressions' gates, then the auxiliary outputs'
  const int32_t* iv_rng;      // [n_iv + 1]: intermediate expression x owns gates iv_rng[x] .. iv_rng[x + 1] - 1
  const int32_t* aux_rng;     // [n_aux + 1]: the same for the auxiliary outputs (last gate: a temporary)
  const int32_t* po;          // [n_po][2]: slot of a primary input fixed by a constant expression, the constant
  const int32_t* clause_off;  // [n_clauses + 1]
  const int32_t* lits;        // slot * 2 + (1 if negated)
  const float* slot_const;    // [n_vslots]: the value of a constant slot (0 for the others)
  int32_t n_iv, n_aux, n_po, n_clauses, n_pi;
  int32_t n_vslots;           // variable slots
  int32_t n_slots;            // variable slots and temporaries
  int32_t words;
  float* V;                   // [batch][n_pi] logits, updated in place
  int32_t batch, iters;
  float lr;
  uint8_t* valid;             // [batch]
  uint64_t* sol;              // [batch][words]
  float* state;               // NULL: state in LDS; else [blocks][2 n_vslots + n_pi (+ 2 temporaries)][64] in global memory
  int32_t temps_lds;          // global state: the temporaries in LDS (else after the logits in the global block)
};
constexpr size_t kGdLdsLimit = 10 * 1024;      // bytes of LDS state per wave (above: global state, more waves per CU)
constexpr size_t kGdTempLdsLimit = 32 * 1024;  // bytes of LDS for the temporaries of the global form
hipError_t launch_gd_sample(const GdArgs& a, hipStream_t s);

// Distinct valid solutions (tt_gd.hip): each valid sample stores its index
// at its solution's place in a table of primary_places (a power of two, no
// clearing needed) and reads it back; the samples whose place another
// solution took go to an open-addressing table of cap places (a power of
// two of at least 2 batch, cleared here) claimed by compare-and-swap.
uint32_t gd_unique_primary_places(int batch);
// The solution hash (both tables): h = seed; per word h ^= word, h *= mul,
// h ^= h >> 31 (a SplitMix64-style mix); the low 32 bits pick the place in
// the first table, the high 32 bits in the second.
constexpr uint64_t kGdHashSeed = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kGdHashMul = 0xBF58476D1CE4E5B9ull;
hipError_t launch_gd_unique(const uint8_t* valid, const uint64_t* sol, int words, int batch, int32_t* primary,
                            int32_t* table, uint32_t cap, uint8_t* first, uint32_t* count, hipStream_t s);
// The last pass alone, for a producer that placed every valid sample in
// primary (primary_places places) and cleared table (cap places) itself.
hipError_t launch_gd_unique_placed(const uint8_t* valid, const uint64_t* sol, int words, int batch,
                                   const int32_t* primary, uint32_t primary_places, int32_t* table, uint32_t cap,
                                   uint8_t* first, uint32_t* count, hipStream_t s);


// Host copy of a sampler's program: the input of its compiled form.
struct GdProgram {
  std::vector<GdGate> gate;  // intermediate expressions' gates, then the auxiliary outputs'
  std::vector<int32_t> iv_rng, aux_rng, po, coff, lits;
  std::vector<float> cst;    // [n_vslots]
  int n_pi = 0, n_vslots = 0, words = 0;
};

// Device source of the compiled sampler (empty: the circuit is too large).
std::string gd_compiled_source(const GdProgram& p);

// Compile it and load it on the current device: 0 on success (else nothing
// is loaded and the interpreter serves the sampler).
int gd_compile(const GdProgram& p, hipModule_t* mod, hipFunction_t* fn);

// One sample per thread, 256 threads per block.
// primary (may be null): every valid sample also stores its index at its
// solution's place (primary_places places, the first pass of the distinct
// filter), and the threads clear table (cap places; may be null) for the
// filter's second table.
hipError_t launch_gd_compiled(hipFunction_t fn, const float* V0, float* V, int batch, float lr, int iters, uint8_t* valid,
                              uint64_t* sol, int32_t* primary, uint32_t primary_places, int32_t* table, uint32_t cap,
                              hipStream_t s);

}  // namespace tt
