// Kernel argument blocks and host-side launchers shared by the engine's
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace nufold {

// Minimiser state of one fit (device memory).
constexpr int FIT_RUNNING = 0, FIT_CONVERGED = 1, FIT_MAXITER = 2, FIT_LSFAIL = 3, FIT_DOMAIN = 4;
struct FitHeader {
  int status, phase, iter, nevals, ls_steps, hist_n, hist_head, resets, max_iter, checks;
  double f, edm, alpha, dphi0;
  double a_prev, f_prev, d_prev;
  double a_lo, f_lo, d_lo, a_hi, f_hi, d_hi;
  double edm_tol;
  double df;        // decrease of f in the last accepted step
};
struct FitArgs {
  FitHeader* hdr;
  double* x;           // accepted point [P]
  double* g;           // masked gradient at x [P]
  double* p;           // search direction [P]
  const double* d2;    // diagonal preconditioner D [P]
  const double* freem; // 1 free, 0 fixed [P]
  double* S;           // history s [m][P]
  double* Y;           // history y [m][P]
  double* rho;         // 1 / s^T y [m]
  double* gam;         // s^T y / y^T D y [m]
  double* theta_next;  // the evaluation input buffer, written with the next trial point
  int m;
};
// LDS doubles used by the minimiser step (matches lbfgs_step's carve).
__host__ __device__ inline size_t fit_lds_doubles(int P, int m) {
  return 2 * (size_t)m * P + 7 * (size_t)P + 3 * (size_t)m + 16;
}

// Reduction of the single evaluation's fold results to fine bins, done by the
// fold kernel itself: the last wavefront to finish a segment sums the
// segment's item partials (fixed item order) and applies the oscillation
// coefficients. The segment's rows, scaled by its source norm, then reach the
// fine bin either by device-scope atomic adds (atomic_rows = 1: no waiting,
// the order of the additions of a bin's sources varies) or through the last
// segment of the fine bin to finish, which sums them in source order and
// stores the rows (atomic_rows = 0: reproducible bit for bit). Counters
// return to zero.
struct FoldFuse {
  const ItemEpi* epi;   // [nitems] per-item epilogue record
  const int* seg_item;  // [G+1] work-item range of each segment
  const int* seg_kt;    // [G] global fine bin of each segment
  const int* kt_need;   // [KT] segments with at least one work item, per fine bin
  const int* kt_info;   // [5 KT] g0, K, S, fs0, kt0 of each fine bin
  const int* fs_nl;     // [NLMAX per (dataset, source)] norm parameter indices (-1: none)
  int* seg_cnt;         // [G] arrival counters
  int* kt_cnt;          // [KT] arrival counters
  double* segm;         // [MAX_MOM + 1][G] segment moments (W, M_1..M_NM), write-through
  double* Sseg;         // [G] oscillated fine spectrum S per segment (before the source norm)
  double* bin;          // per dataset at 6 kt0: rows Hs, dHs/dslot_0..3 over its K fine bins
  int G;
  int atomic_rows;      // 1: every segment adds its rows with device-scope atomics (the bin
                        // stages read and clear them); 0: the last segment of a fine bin
                        // sums the segments in source order and stores the rows
};

struct FoldArgs {
  const void* u;        // double (M64) or float (M32), padded, sorted
  const float* w;       // f32 weights (0 for padding)
  const WorkItem* items;
  int nitems;
  int64_t zpad;         // index of 4 trailing zero-weight events (loads past an item's end read these)
  const double* theta;  // device parameter vector
  OscPlan osc;
  double* part;         // [num_moments][nitems]
  const int* skip;      // nullable: skip the launch unless *skip == FIT_RUNNING
  FoldFuse fuse;        // used when fuse.seg_cnt != nullptr
  // parameter pass of the single evaluation, run by the launch's first npre
  // workgroups (three per dataset, then one for the prior rows) alongside
  // the event stream, into pre (see DevPlan.pre_*); npre = 0: none
  DevPlan plan;
  double* pre;
  int npre;
  const double* Lseg;   // G: baseline of each segment's source (m; the matter form)
};

// Batched fold: a tile of FT fits per wavefront (FT = 1, 2, 4 or 8, a launch
// choice), each event read once per tile.
constexpr int FOLD_FT = 4;  // default tile
struct BatchFoldArgs {
  const void* u;
  const float* w;
  const WorkItem* items;
  int nitems;
  int P, B;
  const double* theta;     // [B][P] trial points
  OscPlan osc;
  const double* Lseg;      // G: baseline of each segment's source (m; the matter form)
  double* part;            // [B][NM][nitems]
  const FitHeader* hdr;    // [B] nullable: fits that are not RUNNING are skipped
  const double* osc_last;  // [B][4] nullable: fits whose slot values equal these are skipped
};

// Pointers of one evaluation (the single evaluation, or one fit of a batch).
struct EvalIO {
  const double* theta;  // P trial point
  const double* part;   // [NM][nitems] fold partials of this evaluation
  const double* data;   // concatenated observed counts
  double* out;          // 1 + P: NLL, gradient (nullable)
  int32_t* status;      // nullable
  double* mu_out;       // nullable
  double* Sseg;         // G
  double* bin;          // 6 KT
  int fused;            // bin rows 0..4 and Sseg come from the fold kernel; row 5 (1 + F) is formed here
  int keep_rows;        // fused: leave rows 0..4 in place for a later evaluation that reuses the fold
  const double* pre;    // nullable: the parameter pass done by the fold launch (DevPlan.pre_*)
};

// Single evaluation: one workgroup, after the fold kernel has written Sseg and
// bin rows 0..4.
struct TailArgs {
  DevPlan plan;
  const double* theta;  // P
  const double* data;   // observed counts (concatenated bins)
  double* out;          // 1 + P: NLL, gradient
  int32_t* status;      // 1 int (may be null)
  double* mu_out;       // concatenated expectations (may be null)
  const double* Sseg;   // G: oscillated fine spectrum S per segment (before A_s)
  const double* bin;    // 6 KT: per dataset [Hs | dHs/dslot_0..3 | unused] over its K fine bins, at 6 kt0
  int want_grad;
  int want_nll;         // 0: only mu_out (no data needed)
  int has_fit;          // run the minimiser step after the evaluation
  int keep_rows;        // leave bin rows 0..4 in place (stage cache: a later evaluation
                        // with the same fold parameters reuses them without a fold)
  FitArgs fit;
  const int* skip;      // nullable: skip the launch unless *skip == FIT_RUNNING
  const double* pre;    // the parameter pass written by the fold launch (DevPlan.pre_*)
};

struct BatchTailArgs {
  DevPlan plan;
  int B;
  const double* theta;    // [B][P] trial points
  const double* part;     // [B][NM][nitems]
  const int* part_idx;    // [B] fold partials row of each fit (nullable: row f)
  const double* data;     // [nsets][nbins_total] (unused when want_nll == 0)
  const int* data_idx;    // [B] data row of each fit (nullable: row f)
  double* mu_out;         // [B][nbins_total] expectations (nullable)
  double* out;            // [B][1+P] (nullable)
  int32_t* status;        // [B] (nullable)
  double* Sseg;           // [B][G]
  double* bin;            // [B][6 KT]
  double* segtmp;         // [B][5 G] in-block phase A scratch
  double* osc_last;       // [B][4] (nullable): slot values of each fit's last fold
  int want_grad;
  int want_nll;
  int has_fit;
  FitArgs fit;            // base pointers; fit f uses hdr + f, vectors + f P, history + f m P
};

constexpr int ST_DOMAIN = 1;
constexpr int MAX_BKG = 8;  // backgrounds per dataset

// Reduction scratch of the bin stages' block sums (32 values x 4 rows per
// wavefront, then the totals).
__host__ __device__ constexpr int red_doubles(int nt) { return 32 * 4 * (nt / 64) + 32; }

// Dynamic LDS bytes used by the bin-stage kernel for a plan (matches carve()).
__host__ __device__ inline size_t tail_lds_bytes(const DevPlan& p, int nt) {
  const size_t K = p.max_K, E = p.max_Nb + 1, Nb = p.max_Nb;
  // six alignment pads, the regions with a slack double, then the rest
  const size_t nd = 6 + (size_t)p.max_pre + p.max_blob + p.NR + (p.NR + 1) / 2 + 2 + p.D +
                    (size_t)p.D * DSPLAN_DOUBLES + (p.P + 1) + ((size_t)p.max_S * K + 1) + (Nb + 1) + K + p.P +
                    CF_SIZE + red_doubles(nt) + 4 * K + 2 * E;
  const size_t ni = K + 2 + 2;
  return (nd + fit_lds_doubles(p.P, p.fit_m)) * sizeof(double) + ni * sizeof(int);
}

hipError_t launch_fold(int mode, const FoldArgs& a, int block, hipStream_t stream, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr);
hipError_t launch_fold_batch(int mode, const BatchFoldArgs& a, hipStream_t stream, int ft = FOLD_FT);
hipError_t launch_tail(const TailArgs& a, int nt, hipStream_t stream, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr);
hipError_t tail_set_lds_limit(size_t bytes);
hipError_t launch_batch_tail(const BatchTailArgs& a, int nt, hipStream_t stream);
// n doubles set to zero by a plain fill kernel (usable inside captured graphs).
hipError_t launch_zero(double* p, int64_t n, hipStream_t stream);

}  // namespace nufold
