// tt_mlp.h -- the screen network's inference over the wave pass's
// candidates compacted first (tt_mlp.hip), for tt_screen_infer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tt.h"

namespace tt {

// Candidates per span of the compaction pass (one block each), and the most
// spans the inference blocks' prefix sums hold (n up to 2^21).
constexpr int kGateSpan = 512;
constexpr int kGateMaxSpans = 4096;

// int32 elements of the work buffer for n candidates: the compacted list
// (kGateSpan per span) and one count per span.
inline size_t gate_work_ints(int n) {
  const size_t spans = ((size_t)n + kGateSpan - 1) / kGateSpan;
  return spans * kGateSpan + spans;
}

// Gated inference in two launches: a pass that compacts the candidates the
// screen's wave pass takes, span by span, into work; then the network over
// that list in chunks of 128 rows by a persistent grid of `blocks` blocks
// (one per CU: every block but the last gets a full chunk).  Requires
// n <= kGateSpan * kGateMaxSpans.  Weights and biases as mlp_infer; logits
// rows of the other candidates are not written.
hipError_t mlp_infer_gated_list(const tt_neuron* desc, int n, const uint16_t* const* w, const float* const* b,
                                float* logits, int32_t* work, int blocks, hipStream_t s);

}  // namespace tt
