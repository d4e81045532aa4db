// Host-side launch interface of the candidate construction kernels (internal; the public ABI is
// mlpf_candidates in mlpf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlpf {

struct CandArgs {
  const int32_t* row_start = nullptr;  // [n_events + 1]
  const int32_t* n_valid = nullptr;    // [n_events] or NULL
  int n_events = 0, total_rows = 0, max_seqlen = 0;
  const int32_t* cls = nullptr;        // [total_rows]
  const float* decoded = nullptr;      // [total_rows][4] or NULL
  int32_t* offsets = nullptr;          // [n_events + 1]
  int32_t* cand_row = nullptr;         // [cap]
  int32_t* cand_cls = nullptr;         // [cap]
  float* cand_kin = nullptr;           // [cap][4] or NULL
  int cap = 0;
};

// Counts, scans and writes the candidates (three launches on `stream`).
hipError_t launch_candidates(const CandArgs& args, hipStream_t stream);

}  // namespace mlpf
