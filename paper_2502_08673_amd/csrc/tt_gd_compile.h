// tt_gd_compile.h -- the GD sampler compiled for one circuit (host side).
#pragma once

#include <string>
#include <vector>

#include "tt_internal.h"

namespace tt {

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
hipError_t launch_gd_compiled(hipFunction_t fn, float* V, int batch, float lr, int iters, uint8_t* valid,
                              uint64_t* sol, hipStream_t s);

}  // namespace tt
