// Kernel argument blocks and host-side launchers shared by the engine's
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace nufold {

struct FoldArgs {
  const void* u;        // double (M64) or float (M32), padded, sorted
  const float* w;       // f32 weights (0 for padding)
  const WorkItem* items;
  int nitems;
  const double* theta;  // device parameter vector
  OscPlan osc;
  double* part;         // [num_moments][nitems]
};

struct TailArgs {
  DevPlan plan;
  const double* theta;  // P
  const double* part;   // [NM][nitems] fold partials
  const double* data;   // observed counts (concatenated bins)
  double* out;          // 1 + P: NLL, gradient
  int32_t* status;      // 1 int (may be null)
  double* mu_out;       // concatenated expectations (may be null)
  double* scratch;      // max_S * max_K doubles (per-source fine spectra)
  int want_grad;
  int want_nll;         // 0: only mu_out (no data needed)
};

constexpr int ST_DOMAIN = 1;

// Dynamic LDS bytes used by the bin-stage kernel for a plan.
__host__ __device__ inline size_t tail_lds_bytes(const DevPlan& p, int nt) {
  const size_t K = p.max_K, E = p.max_Nb + 1;
  const size_t nd = 2 * (size_t)p.P + 40 + p.max_S + K * 7 + (K + 1) * 4 + E * 4 + p.max_Nb +
                    8 * (nt / 64) + 8;
  return nd * sizeof(double) + (E + 2) * sizeof(int);
}

hipError_t launch_fold(int mode, const FoldArgs& a, int block, hipStream_t stream);
hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream);
hipError_t tail_set_lds_limit(size_t bytes);

}  // namespace nufold
