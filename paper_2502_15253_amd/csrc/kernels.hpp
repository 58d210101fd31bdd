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
  double* Sseg;         // G: oscillated fine spectrum S per segment (before A_s)
  double* bin;          // 6 KT: per dataset [Hs | dHs/dslot_0..3 | 1 + F] over its K fine bins, at 6 kt0
  double* prior;        // 2 NR: per prior row v (gradient contribution) and NLL contribution
  int* counter;         // workgroup completion counter (0 between launches)
  int want_grad;
  int want_nll;         // 0: only mu_out (no data needed)
};

constexpr int ST_DOMAIN = 1;
constexpr int MAX_BKG = 8;  // backgrounds per dataset

// Dynamic LDS bytes used by the bin-stage kernel for a plan (matches carve()).
__host__ __device__ inline size_t tail_lds_bytes(const DevPlan& p, int nt) {
  const size_t K = p.max_K, E = p.max_Nb + 1, Nb = p.max_Nb;
  const size_t nd = 2 * (size_t)p.P + 40 + 16 * (nt / 64) + 16 + 6 * K + (size_t)p.max_S * K + Nb +
                    4 * (K + 1) + K + 3 * E + Nb + p.max_blob;
  const size_t ni = E + 2;
  return nd * sizeof(double) + ni * sizeof(int);
}

int tail_blocks(const DevPlan& p, int nt);
hipError_t launch_fold(int mode, const FoldArgs& a, int block, hipStream_t stream);
hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream);
hipError_t tail_set_lds_limit(size_t bytes);

}  // namespace nufold
