// Event fold: step 1 of the signal calculation (paper, "Structure of the
// framework"; offload of the oscillation weighting, "GPU accelerated
// computation"), re-designed for gfx950.
//
// The survival probability is a fixed linear combination of cos(x_ab) terms,
// x_ab = 2 k dm2_ab L/E (sin^2(x/2) = (1 - cos x)/2), with coefficients that
// depend only on the mixing angles. So, per (dataset, source, fine bin)
// segment, the fold streams the sorted events once and accumulates
//   eq1 (Eq. 1):   C_ee, C_21, Q_ee, Q_21
//   3nu (exact):   C_21, C_31, C_32, Q_21, Q_31, Q_32
//   4nu (3+1):     C and Q of 21, 31, 32, 41, 42, 43
// with C_ab = sum_e w_e cos x_ab,e and Q_ab = sum_e w_e u_e sin x_ab,e,
// u_e = L/E. The bin-stage kernel turns these moments into the oscillated
// spectrum sum_e w_e P_e and its derivatives with respect to every
// oscillation parameter (forward-mode Jacobian, exact), so mixing-angle
// changes never re-read events. Only the phases 21, 31 (and 41) are
// computed; the others come from their sin/cos pairs by angle subtraction.
//
// Layout: u[] and w[] are SoA, sorted by segment, every segment padded with
// zero-weight events to a multiple of 4, so each lane reads 4 consecutive
// events with 16-byte loads. One wavefront (64 lanes) reduces one work item
// (<= chunk events of one segment) to one partial per moment.
//
// Single evaluation: the fold also finishes the reduction to fine bins. The
// last wavefront to complete a segment sums the segment's partials (item
// order) and applies the oscillation coefficients (computed by each
// wavefront into its own LDS rows) and the source norm; the segment's rows
// reach the fine bin by device-scope atomic adds or, in the deterministic
// mode, through the last segment of the fine bin to complete, which sums
// them in source order. Hand-offs use write-through stores and device-scope
// counters that the last arrival resets: no extra launch or cache write-back.
// Batched evaluations keep the raw partials; their bin stages reduce them.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <type_traits>

#include "fastmath.hpp"
#include "kernels.hpp"
#include "matter.hpp"
#include "osc.hpp"
#include "stages.hpp"

namespace nufold {


__device__ __forceinline__ double slot_val(const OscPlan& o, const double* th, int j) {
  const int p = o.slot_param[j];
  return p >= 0 ? th[p] : o.slot_value[j];
}

// Streaming loads of the event arrays in the single evaluation: each event is
// read once per evaluation, so the loads carry the non-temporal hint and do
// not displace the bin-stage kernel's inputs and code from the caches. (The
// batched fold re-reads events for every tile of fits and keeps plain loads.)
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 load_stream2(const double* p) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return double2{v.x, v.y};
}
__device__ __forceinline__ float4 load_stream4(const float* p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return float4{v.x, v.y, v.z, v.w};
}

template <int FORM>
constexpr int form_moments() { return FORM == FORM_EQ1 ? 4 : FORM == FORM_3NU ? 6 : 12; }
template <int FORM>
constexpr int form_phases() { return FORM == FORM_4NU ? 3 : 2; }

// Moments of one event from the sin/cos of its computed phases (s[q], c[q]):
//   eq1: C_ee, C_21, Q_ee, Q_21
//   3nu: C_21, C_31, C_32, Q_21, Q_31, Q_32           (32 = 31 - 21)
//   4nu: C of 21, 31, 32, 41, 42, 43, then their Q    (4j = 41 - j1)
template <int FORM, typename T>
__device__ __forceinline__ void accum_moments(T w, T wu, const T* s, const T* c, T* m) {
  if constexpr (FORM == FORM_EQ1) {
    m[0] = fma(w, c[0], m[0]);
    m[1] = fma(w, c[1], m[1]);
    m[2] = fma(wu, s[0], m[2]);
    m[3] = fma(wu, s[1], m[3]);
  } else if constexpr (FORM == FORM_3NU) {
    const T c3 = fma(c[1], c[0], s[1] * s[0]);
    const T s3 = fma(s[1], c[0], -(c[1] * s[0]));
    m[0] = fma(w, c[0], m[0]);
    m[1] = fma(w, c[1], m[1]);
    m[2] = fma(w, c3, m[2]);
    m[3] = fma(wu, s[0], m[3]);
    m[4] = fma(wu, s[1], m[4]);
    m[5] = fma(wu, s3, m[5]);
  } else {
    const T c32 = fma(c[1], c[0], s[1] * s[0]), s32 = fma(s[1], c[0], -(c[1] * s[0]));
    const T c42 = fma(c[2], c[0], s[2] * s[0]), s42 = fma(s[2], c[0], -(c[2] * s[0]));
    const T c43 = fma(c[2], c[1], s[2] * s[1]), s43 = fma(s[2], c[1], -(c[2] * s[1]));
    m[0] = fma(w, c[0], m[0]);
    m[1] = fma(w, c[1], m[1]);
    m[2] = fma(w, c32, m[2]);
    m[3] = fma(w, c[2], m[3]);
    m[4] = fma(w, c42, m[4]);
    m[5] = fma(w, c43, m[5]);
    m[6] = fma(wu, s[0], m[6]);
    m[7] = fma(wu, s[1], m[7]);
    m[8] = fma(wu, s32, m[8]);
    m[9] = fma(wu, s[2], m[9]);
    m[10] = fma(wu, s42, m[10]);
    m[11] = fma(wu, s43, m[11]);
  }
}

// FP64 path: ak = a TAB_PER_RAD, the angular frequencies in sin/cos table
// units per (m/MeV); tab: the table in LDS (see load_sincos_table).
template <int FORM>
__device__ __forceinline__ void accum64(double u, float wf, const double* ak, const double* tab, double* m) {
  constexpr int NPH = form_phases<FORM>();
  const double w = (double)wf;
  const double wu = w * u;
  double s[NPH], c[NPH];
#pragma unroll
  for (int q = 0; q < NPH; ++q) sincos_tab(ak[q] * u, tab, s[q], c[q]);
  accum_moments<FORM, double>(w, wu, s, c, m);
}

// The FP64 folds' sin/cos table (TAB_N (sin, cos) pairs, 4 KiB) goes to LDS
// in two halves: thread i's global load of entry i first, the LDS stores
// later, so that a kernel can issue its first event loads in between and the
// table's latency overlaps theirs. One entry per thread keeps the registers
// held across those loads to one pair; entries past the block size (blocks
// of fewer than TAB_N threads) are loaded and stored by the second half. A
// block barrier must follow the stores.
struct TabRegs {
  double2 v;
};
__device__ __forceinline__ void load_sincos_table(TabRegs& r) {
  const double2* T = reinterpret_cast<const double2*>(SINCOS_TAB);
  if (threadIdx.x < TAB_N) r.v = T[threadIdx.x];
}
__device__ __forceinline__ void store_sincos_table(const TabRegs& r, double* tab) {
  const double2* T = reinterpret_cast<const double2*>(SINCOS_TAB);
  double2* D = reinterpret_cast<double2*>(tab);
  if (threadIdx.x < TAB_N) D[threadIdx.x] = r.v;
  for (int e = threadIdx.x + blockDim.x; e < TAB_N; e += blockDim.x) D[e] = T[e];
}

// FP32 path: phases in revolutions, t = fract(f u) with the FP32 frequency
// f = fp32_rev(a) (the product rounded once); hardware sin/cos take
// revolutions. The moments are those of the frequency 2 pi f; the coefficient
// rows correct them to a at first order (fp32_frequency_correction), which
// removes the systematic phase error an FP32 frequency would leave. (Adding
// the remainder of the frequency per event instead would be lost whenever it
// is below half an ulp of the phase, as at short baselines.)
template <int FORM>
__device__ __forceinline__ void accum32(float u, float w, const float* f, float* m) {
  constexpr int NPH = form_phases<FORM>();
  const float wu = w * u;
  float s[NPH], c[NPH];
#pragma unroll
  for (int q = 0; q < NPH; ++q) {
    const float t = __builtin_amdgcn_fractf(f[q] * u);  // p - floor(p) in one instruction
    s[q] = __builtin_amdgcn_sinf(t);
    c[q] = __builtin_amdgcn_cosf(t);
  }
  accum_moments<FORM, float>(w, wu, s, c, m);
}

template <int NM>
__device__ __forceinline__ void wave_sum_store(double* m, double* part, int nitems, int item, int lane) {
#pragma unroll
  for (int c = 0; c < NM; ++c) {
    double v = m[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    m[c] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NM; ++c) part[(int64_t)c * nitems + item] = m[c];
  }
}

// One wavefront folds one work item. Each lane takes 4 consecutive events
// per step (16-byte loads) and the loop is software-pipelined: a step's loads
// are issued three steps (M32) or two steps (M64, whose registers are the
// tighter budget) ahead of its folding, held there by scheduling barriers
// (left alone, the compiler sinks them below the first arithmetic on the step
// before, and a wave then has a single step in flight). With every wave of the
// launch resident at once, the bytes a wave keeps in flight bound the stream.
// Steps past the item's end are loaded (from zpad) but not folded. Positions past the item's end load the 4
// zero-weight events at zpad, which add nothing (so the second half of the
// last step may fold zeros); the loop is uniform over the wave and no load
// sits under a branch.
// Fine-bin reduction by the last arrivals (see FoldFuse). m: this item's NM
// moment sums, identical in every lane; cf: the coefficient rows (LDS).
// ep: the item's epilogue record; A: its source norm (both read before the
// event loop).
template <int NM>
__device__ void fold_bin_epilogue(const FoldArgs& a, const double* cf, const double* m, int item, int seg,
                                  int lane, const ItemEpi& ep, double A) {
  const FoldFuse& F = a.fuse;
  const int ib = ep.first, ie = ep.first + ep.nseg;
  double M[NM + 1];
  M[0] = ep.W;
  if (ie - ib == 1) {
#pragma unroll
    for (int c = 0; c < NM; ++c) M[1 + c] = m[c];
  } else {
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < NM; ++c) store_agent(&a.part[(int64_t)c * a.nitems + item], m[c]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    int last = 0;
    if (lane == 0) {
      const int done = __hip_atomic_fetch_add(&F.seg_cnt[seg], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = done == ie - ib - 1;
      if (last) __hip_atomic_store(&F.seg_cnt[seg], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!__builtin_amdgcn_readlane(last, 0)) return;
#pragma unroll
    for (int c = 0; c < NM; ++c) M[1 + c] = 0.0;
#pragma unroll 1
    for (int it = ib; it < ie; ++it) {
#pragma unroll
      for (int c = 0; c < NM; ++c) M[1 + c] += load_agent(&a.part[(int64_t)c * a.nitems + it]);
    }
  }
  if (F.atomic_rows) {
    // this segment's rows: lane r < 5 forms row r from the coefficients and
    // adds A_s times it to the fine bin (fire-and-forget device-scope adds;
    // the rows start at zero and the bin stages clear them after reading)
    if (lane < 5) {
      int z = 0;  // opaque zero: keeps the coefficient loads here (see below)
      asm volatile("" : "+v"(z));
      const double* c0 = cf + CF_STRIDE * lane + z;
      double r = 0.0;
#pragma unroll
      for (int c = 0; c <= NM; ++c) r += c0[c] * M[c];
      if (lane == 0) F.Sseg[seg] = r;
      __hip_atomic_fetch_add(F.bin + ep.row + (int64_t)lane * ep.K, A * r, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const int kt = F.seg_kt[seg];
  if (F.kt_need[kt] > 1) {
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c <= NM; ++c) store_agent(&F.segm[(int64_t)c * F.G + seg], M[c]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    int last = 0;
    if (lane == 0) {
      const int done = __hip_atomic_fetch_add(&F.kt_cnt[kt], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = done == F.kt_need[kt] - 1;
      if (last) __hip_atomic_store(&F.kt_cnt[kt], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!__builtin_amdgcn_readlane(last, 0)) return;
  }
  // this wavefront holds the fine bin's last segment: lane s takes source s
  const int* info = F.kt_info + 5 * kt;
  const int g0 = info[0], K = info[1], S = info[2], fs0 = info[3], kt0 = info[4];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int s = lane; s < S; s += 64) {
    const int g = g0 + s * K;
    const int src = g == seg ? 0 : (F.seg_item[g + 1] > F.seg_item[g] ? 1 : 2);  // registers, stored, empty
    double Sv = 0.0, gj[4] = {0.0, 0.0, 0.0, 0.0};
    if (src != 2) {
      // an opaque zero offset keeps the coefficient loads inside this loop:
      // hoisted, the 35 values would hold registers for the whole kernel
      int z = 0;
      asm volatile("" : "+v"(z));
      const double* c0 = cf + z;
#pragma unroll
      for (int c = 0; c <= NM; ++c) {
        const double Mc = src == 0 ? M[c] : load_agent(&F.segm[(int64_t)c * F.G + g]);
        Sv += c0[c] * Mc;
#pragma unroll
        for (int j = 0; j < 4; ++j) gj[j] += c0[CF_STRIDE * (j + 1) + c] * Mc;
      }
    }
    const int* nl = F.fs_nl + NLMAX * (fs0 + s);
    double A = 1.0;
#pragma unroll
    for (int q = 0; q < NLMAX; ++q)
      if (nl[q] >= 0) A *= a.theta[nl[q]];
    F.Sseg[g] = Sv;
    v[0] += A * Sv;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[1 + j] += A * gj[j];
  }
#pragma unroll
  for (int r = 0; r < 5; ++r) v[r] = wave_sum_fixed(v[r]);
  if (lane == 0) {
    double* b = F.bin + 6 * (int64_t)kt0;
    const int k = kt - kt0;
#pragma unroll
    for (int r = 0; r < 5; ++r) b[r * K + k] = v[r];
  }
}

// The item's epilogue record and the values of its source's norm parameters
// (fused launches only), issued right after the first event loads: the loads
// are independent of each other and are only waited for in the epilogue.
__device__ __forceinline__ void item_prefetch(const FoldArgs& a, int item, ItemEpi& ep, double* thv) {
  if (!a.fuse.seg_cnt) return;
  ep = a.fuse.epi[item];
#pragma unroll
  for (int q = 0; q < NLMAX; ++q) thv[q] = a.theta[ep.nl[q] >= 0 ? ep.nl[q] : 0];
}
// Source norm A_s: the product of the source's norm parameters.
__device__ __forceinline__ double item_norm(const ItemEpi& ep, const double* thv) {
  double A = 1.0;
#pragma unroll
  for (int q = 0; q < NLMAX; ++q)
    if (ep.nl[q] >= 0) A *= thv[q];
  return A;
}

// Oscillation coefficients of this launch's parameters into the wavefront's
// own LDS rows (fused launches only), by lane 0 with no barrier. Called after
// the first event loads are issued, so its parameter loads and FP64 work
// overlap their latency instead of delaying the stream.
__device__ __forceinline__ void wave_coefficients(const FoldArgs& a, double* cf) {
  if (a.fuse.seg_cnt && (threadIdx.x & 63) == 0) (void)osc_coefficients(a.osc, a.theta, cf);
}

template <int NM>
__device__ __forceinline__ void fold_finish(const FoldArgs& a, const double* cf, double* m, int item, int seg,
                                            const ItemEpi& ep, double A) {
  // the lane id is recomputed here rather than kept live across the event
  // loop (the register allocator would park it above the loop's registers)
  const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
  for (int c = 0; c < NM; ++c) m[c] = wave_sum_fixed(m[c]);
  if (a.fuse.seg_cnt) {
    fold_bin_epilogue<NM>(a, cf, m, item, seg, lane, ep, A);
  } else if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NM; ++c) a.part[(int64_t)c * a.nitems + item] = m[c];
  }
}

// Parameter pass of the single evaluation, in the first npre = 3 D + 1
// workgroups of the fold launch (they run alongside the event stream):
// workgroups 3d, 3d + 1 and 3d + 2 form dataset d's flux factors, its mapped
// edges (and the energy map's domain flag) and its background terms; the
// last one evaluates the prior rows, sums their NLL in a fixed order and
// checks the parameters' domain. (One workgroup per dataset took about
// 13 us, longer than the whole event stream below a few million events.) The parameters are read from global memory
// (a few hundred values, cached). red: this workgroup's LDS rows (at least
// 2 x (blockDim / 64) doubles).
__device__ void parameter_pass(const FoldArgs& a, int b, double* red) {
  const DevPlan& p = a.plan;
  const double* th = a.theta;
  double* pre = a.pre;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (b < 3 * p.D) {
    const int part = b % 3;
    b /= 3;
    const DsPlan& ds = b == 0 ? p.ds0 : p.ds[b];
    const int K = ds.K, Nb = ds.Nb, E = Nb + 1, NB = ds.nbkg;
    const double wf = ds.wf, iwf = 1.0 / wf, y0 = ds.y0, yK = ds.y0 + ds.wf * K;
    const BlobLayout BL = blob_layout(E, NB, Nb, ds.nnz, ds.M, ds.S, ds.nl, K, ds.fw);
    const double* blob = p.dpool + ds.blob;
    const double c0 = pval(th, ds.cidx[0], 0.0);
    const double c2 = pval(th, ds.cidx[2], 0.0);
    const double bb = 1.0 + pval(th, ds.cidx[1], 0.0);
    const PreLayout PL = pre_layout(K, Nb, NB);
    double* q = pre + ds.pre0;
    if (part == 0) {
      for (int k = tid; k < K; k += nt) q[PL.F1 + k] = flux_factor(th, blob, BL, ds.fw, k);
    } else if (part == 1) {
      if (tid == 0) pre[p.pre_misc + 2 + b] = map_ok(bb, c2, y0, yK) ? 0.0 : 1.0;
      for (int e = tid; e < E; e += nt) {
        const MappedEdge m = map_edge(blob[BL.edges + e], c0, bb, c2, y0, yK, wf, iwf, K);
        reinterpret_cast<int*>(q + PL.ek)[e] = m.k;
        q[PL.et + e] = m.t;
        q[PL.ey + e] = m.y;
        q[PL.eq + e] = m.ifp;
      }
    } else {
      for (int i = tid; i < Nb; i += nt)
        q[PL.B + i] = background(th, blob, BL, NB, Nb, i, q + PL.bkr + i, q + PL.bks + i);
    }
    return;
  }
  double e_sum = 0.0, bad = 0.0;
  for (int r = tid; r < p.NR; r += nt) {
    int idx;
    double v, e;
    prior_row(p, th, r, idx, v, e);
    pre[p.pre_prv + r] = v;
    reinterpret_cast<int*>(pre + p.pre_pri)[r] = idx;
    e_sum += e;
  }
  for (int i = tid; i < p.P; i += nt)
    if (!isfinite(th[i])) bad = 1.0;
  if (tid == 0 && !osc_domain_ok(p.osc, th)) bad = 1.0;
  e_sum = wave_sum_fixed(e_sum);
  bad = wave_sum_fixed(bad);
  const int nw = nt >> 6, w = tid >> 6;
  if ((tid & 63) == 0) {
    red[w] = e_sum;
    red[nw + w] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0, f = 0.0;
    for (int j = 0; j < nw; ++j) {
      s += red[j];
      f += red[nw + j];
    }
    pre[p.pre_misc] = s;
    pre[p.pre_misc + 1] = f > 0.0 ? 1.0 : 0.0;
  }
}

template <int FORM>
__global__ __launch_bounds__(256) void fold_m64_kernel(FoldArgs a) {
  constexpr int NM = form_moments<FORM>();
  __shared__ double cfw[4][CF_SIZE];  // coefficient rows per wavefront (blocks of at most 256 threads)
  __shared__ __attribute__((aligned(16))) double tab[2 * TAB_N];
  if (a.skip && *a.skip != FIT_RUNNING) return;  // uniform over the launch
  if ((int)blockIdx.x < a.npre) {
    parameter_pass(a, blockIdx.x, &cfw[0][0]);
    return;
  }
  if (a.nitems == 0) return;
  TabRegs tr;
  load_sincos_table(tr);
  __builtin_amdgcn_sched_barrier(0);
  const int lane = threadIdx.x & 63;
  const int item = __builtin_amdgcn_readfirstlane(
      (int)(((blockIdx.x - (unsigned)a.npre) * (unsigned)blockDim.x + threadIdx.x) >> 6));
  // wavefronts past the last item take part in the table's barrier, with
  // no events (every position loads from zpad), then leave
  const bool live = item < a.nitems;
  const int ic = live ? item : 0;
  double* cf = cfw[threadIdx.x >> 6];
  ItemEpi ep{};
  double thv[NLMAX];
  double af[3];
  osc_freqs_form<FORM>(a.osc, a.theta, af);
#pragma unroll
  for (int q = 0; q < 3; ++q) af[q] *= TAB_PER_RAD;
  const WorkItem it = a.items[ic];
  const double* __restrict__ u = static_cast<const double*>(a.u);
  const float* __restrict__ w = a.w;
  const int cnt = live ? it.count : 0;
  const int niter = (cnt + 255) >> 8;
  double m[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c) m[c] = 0.0;
  int j = lane * 4;
  auto at = [&](int off) { return j + off < cnt ? it.begin + j + off : a.zpad; };
  int64_t o = at(0);
  double2 pa = load_stream2(u + o);
  double2 qa = load_stream2(u + o + 2);
  float4 wa = load_stream4(w + o);
  o = at(256);
  double2 pb = load_stream2(u + o);
  double2 qb = load_stream2(u + o + 2);
  float4 wb = load_stream4(w + o);
  item_prefetch(a, ic, ep, thv);
  wave_coefficients(a, cf);
  store_sincos_table(tr, tab);
  __syncthreads();
  if (!live) return;  // whole wavefronts leave together
  auto fold4 = [&](const double2& pp, const double2& qq, const float4& ww) {
    accum64<FORM>(pp.x, ww.x, af, tab, m);
    accum64<FORM>(pp.y, ww.y, af, tab, m);
    accum64<FORM>(qq.x, ww.z, af, tab, m);
    accum64<FORM>(qq.y, ww.w, af, tab, m);
  };
  // three register sets rotate: each step's loads are issued two steps ahead
  // of its folding (the scheduling barriers keep them ahead of the
  // arithmetic); steps past the item's end are loaded but not folded
  for (int t = 0; t < niter; t += 3) {
    o = at(512);
    const double2 pc = load_stream2(u + o);
    const double2 qc = load_stream2(u + o + 2);
    const float4 wc = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    fold4(pa, qa, wa);
    o = at(768);
    pa = load_stream2(u + o);
    qa = load_stream2(u + o + 2);
    wa = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < niter) fold4(pb, qb, wb);
    o = at(1024);
    pb = load_stream2(u + o);
    qb = load_stream2(u + o + 2);
    wb = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 2 < niter) fold4(pc, qc, wc);
    j += 768;
  }
  fold_finish<NM>(a, cf, m, item, it.seg, ep, a.fuse.seg_cnt ? item_norm(ep, thv) : 1.0);
}

template <int FORM>
__global__ __launch_bounds__(256) void fold_m32_kernel(FoldArgs a) {
  constexpr int NM = form_moments<FORM>();
  constexpr int NPH = form_phases<FORM>();
  __shared__ double cfw[4][CF_SIZE];  // coefficient rows per wavefront (blocks of at most 256 threads)
  if (a.skip && *a.skip != FIT_RUNNING) return;  // uniform over the launch
  if ((int)blockIdx.x < a.npre) {
    parameter_pass(a, blockIdx.x, &cfw[0][0]);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int item = __builtin_amdgcn_readfirstlane(
      (int)(((blockIdx.x - (unsigned)a.npre) * (unsigned)blockDim.x + threadIdx.x) >> 6));
  if (item >= a.nitems) return;
  double* cf = cfw[threadIdx.x >> 6];
  ItemEpi ep{};
  double thv[NLMAX];
  double af[3];
  osc_freqs_form<FORM>(a.osc, a.theta, af);
  float fr[NPH];
#pragma unroll
  for (int q = 0; q < NPH; ++q) fr[q] = fp32_rev(af[q]);
  const WorkItem it = a.items[item];
  const float* __restrict__ u = static_cast<const float*>(a.u);
  const float* __restrict__ w = a.w;
  const int cnt = it.count;
  const int niter = (cnt + 255) >> 8;
  float mf[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c) mf[c] = 0.0f;
  int j = lane * 4;
  auto at = [&](int off) { return j + off < cnt ? it.begin + j + off : a.zpad; };
  int64_t o = at(0);
  float4 ua = load_stream4(u + o);
  float4 wa = load_stream4(w + o);
  o = at(256);
  float4 ub = load_stream4(u + o);
  float4 wb = load_stream4(w + o);
  o = at(512);
  float4 uc = load_stream4(u + o);
  float4 wc = load_stream4(w + o);
  item_prefetch(a, item, ep, thv);
  wave_coefficients(a, cf);
  auto fold4 = [&](const float4& uu, const float4& ww) {
    accum32<FORM>(uu.x, ww.x, fr, mf);
    accum32<FORM>(uu.y, ww.y, fr, mf);
    accum32<FORM>(uu.z, ww.z, fr, mf);
    accum32<FORM>(uu.w, ww.w, fr, mf);
  };
  // four register sets rotate: each step's loads are issued three steps
  // ahead of its folding (the scheduling barriers keep them ahead of the
  // arithmetic). While every load of an iteration lies inside the item, the
  // addresses are plain pointer offsets; the last iterations go through at()
  // (loads past the end read zpad, those steps are not folded).
  int t = 0;
  const float* pu = u + it.begin + j;
  const float* pw = w + it.begin + j;
  for (; (t << 8) + 1792 <= cnt; t += 4) {
    const float4 ud = load_stream4(pu + 768);
    const float4 wd = load_stream4(pw + 768);
    __builtin_amdgcn_sched_barrier(0);
    fold4(ua, wa);
    ua = load_stream4(pu + 1024);
    wa = load_stream4(pw + 1024);
    __builtin_amdgcn_sched_barrier(0);
    fold4(ub, wb);
    ub = load_stream4(pu + 1280);
    wb = load_stream4(pw + 1280);
    __builtin_amdgcn_sched_barrier(0);
    fold4(uc, wc);
    uc = load_stream4(pu + 1536);
    wc = load_stream4(pw + 1536);
    __builtin_amdgcn_sched_barrier(0);
    fold4(ud, wd);
    pu += 1024;
    pw += 1024;
    j += 1024;
  }
  for (; t < niter; t += 4) {
    o = at(768);
    const float4 ud = load_stream4(u + o);
    const float4 wd = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    fold4(ua, wa);
    o = at(1024);
    ua = load_stream4(u + o);
    wa = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < niter) fold4(ub, wb);  // steps past the item's end are not folded
    o = at(1280);
    ub = load_stream4(u + o);
    wb = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 2 < niter) fold4(uc, wc);
    o = at(1536);
    uc = load_stream4(u + o);
    wc = load_stream4(w + o);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 3 < niter) fold4(ud, wd);
    j += 1024;
  }
  double m[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c) m[c] = (double)mf[c];
  fold_finish<NM>(a, cf, m, item, it.seg, ep, a.fuse.seg_cnt ? item_norm(ep, thv) : 1.0);
}

// Matter form (both event formats, FP64 arithmetic): no moments; per event P
// and its four slot derivatives (matter_event), summed per item as five
// values, with the item records, parameter-pass workgroups and fine-bin
// epilogue of the vacuum forms (identity coefficient rows). Zero-weight
// padding events are evaluated at u = 1 and contribute nothing.
template <typename T>
__device__ __forceinline__ void matter_accum(T ut, float wf, double aL, const double* v, double* m) {
  const double w = (double)wf;
  const double u = wf != 0.0f ? (double)ut : 1.0;
  double P, dP[NSLOT];
  matter_event(u, aL, v[0], v[1], v[2], v[3], P, dP);
  m[0] = fma(w, P, m[0]);
#pragma unroll
  for (int j = 0; j < NSLOT; ++j) m[1 + j] = fma(w, dP[j], m[1 + j]);
}
// slot values of the matter form: sin^2 th12, sin^2 th13, dm2_21 and dm2_31 in eV^2
__device__ __forceinline__ void matter_slots(const OscPlan& o, const double* th, double* v) {
  v[0] = slot_val(o, th, 0);
  v[1] = slot_val(o, th, 1);
  v[2] = slot_val(o, th, 2) * UNIT_1EM5;
  v[3] = slot_val(o, th, 3) * UNIT_1EM3;
}

template <typename T>
__global__ __launch_bounds__(256) void fold_matter_kernel(FoldArgs a) {
  constexpr int NM = 5;
  __shared__ double cfw[4][CF_SIZE];  // coefficient rows per wavefront (blocks of at most 256 threads)
  if (a.skip && *a.skip != FIT_RUNNING) return;  // uniform over the launch
  if ((int)blockIdx.x < a.npre) {
    parameter_pass(a, blockIdx.x, &cfw[0][0]);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int item = __builtin_amdgcn_readfirstlane(
      (int)(((blockIdx.x - (unsigned)a.npre) * (unsigned)blockDim.x + threadIdx.x) >> 6));
  if (item >= a.nitems) return;  // whole wavefronts leave together
  double* cf = cfw[threadIdx.x >> 6];
  ItemEpi ep{};
  double thv[NLMAX];
  const WorkItem it = a.items[item];
  double v[NSLOT];
  matter_slots(a.osc, a.theta, v);
  const double aL = a.osc.cst[0] * a.Lseg[it.seg];
  item_prefetch(a, item, ep, thv);
  wave_coefficients(a, cf);
  const T* __restrict__ u = static_cast<const T*>(a.u) + it.begin;
  const float* __restrict__ w = a.w + it.begin;
  double m[NM];
#pragma unroll
  for (int c = 0; c < NM; ++c) m[c] = 0.0;
  for (int e = lane * 4; e < it.count; e += 256) {
    const float4 w4 = *reinterpret_cast<const float4*>(w + e);
    T u4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u4[q] = u[e + q];
    matter_accum<T>(u4[0], w4.x, aL, v, m);
    matter_accum<T>(u4[1], w4.y, aL, v, m);
    matter_accum<T>(u4[2], w4.z, aL, v, m);
    matter_accum<T>(u4[3], w4.w, aL, v, m);
  }
  fold_finish<NM>(a, cf, m, item, it.seg, ep, a.fuse.seg_cnt ? item_norm(ep, thv) : 1.0);
}

// ---------------------------------------------------------------- batched
// One wavefront per (work item, tile of FOLD_FT fits): the events are read
// once and folded for every active fit of the tile. A fit is skipped when its
// minimiser has stopped or when its oscillation slot values equal those of
// its previous fold (its partials are still valid).
template <int FORM>
__device__ __forceinline__ bool batch_fit_active(const BatchFoldArgs& a, int f, double* af) {
  if (f >= a.B) return false;
  if (a.hdr && a.hdr[f].status != FIT_RUNNING) return false;
  const double* th = a.theta + (int64_t)f * a.P;
  if (a.osc_last) {
    bool same = true;
    for (int j = 0; j < NSLOT; ++j) same = same && (slot_val(a.osc, th, j) == a.osc_last[4 * f + j]);
    if (same) return false;
  }
  osc_freqs_form<FORM>(a.osc, th, af);
  return true;
}

template <int FORM, int FT>
__global__ __launch_bounds__(256) void fold_batch_m64_kernel(BatchFoldArgs a) {
  constexpr int NM = form_moments<FORM>();
  __shared__ __attribute__((aligned(16))) double tab[2 * TAB_N];
  {
    TabRegs tr;
    load_sincos_table(tr);
    store_sincos_table(tr, tab);
  }
  __syncthreads();  // before any wavefront leaves
  const int lane = threadIdx.x & 63;
  const int item = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) >> 6);
  if (item >= a.nitems) return;
  const int f0 = blockIdx.y * FT;
  double af[FT][3];
  bool act[FT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < FT; ++j) {
    af[j][0] = af[j][1] = af[j][2] = 0.0;
    act[j] = batch_fit_active<FORM>(a, f0 + j, af[j]);
    any = any || act[j];
#pragma unroll
    for (int q = 0; q < 3; ++q) af[j][q] *= TAB_PER_RAD;
  }
  if (!any) return;
  const WorkItem it = a.items[item];
  const double* __restrict__ u = static_cast<const double*>(a.u) + it.begin;
  const float* __restrict__ w = a.w + it.begin;
  double m[FT][NM];
#pragma unroll
  for (int j = 0; j < FT; ++j)
#pragma unroll
    for (int c = 0; c < NM; ++c) m[j][c] = 0.0;
  for (int e = lane * 4; e < it.count; e += 256) {
    const double2 u01 = *reinterpret_cast<const double2*>(u + e);
    const double2 u23 = *reinterpret_cast<const double2*>(u + e + 2);
    const float4 w4 = *reinterpret_cast<const float4*>(w + e);
#pragma unroll
    for (int j = 0; j < FT; ++j) {
      if (!act[j]) continue;
      accum64<FORM>(u01.x, w4.x, af[j], tab, m[j]);
      accum64<FORM>(u01.y, w4.y, af[j], tab, m[j]);
      accum64<FORM>(u23.x, w4.z, af[j], tab, m[j]);
      accum64<FORM>(u23.y, w4.w, af[j], tab, m[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < FT; ++j)
    if (act[j]) wave_sum_store<NM>(m[j], a.part + (int64_t)(f0 + j) * NM * a.nitems, a.nitems, item, lane);
}

template <int FORM, int FT>
__global__ __launch_bounds__(256) void fold_batch_m32_kernel(BatchFoldArgs a) {
  constexpr int NM = form_moments<FORM>();
  constexpr int NPH = form_phases<FORM>();
  const int lane = threadIdx.x & 63;
  const int item = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) >> 6);
  if (item >= a.nitems) return;
  const int f0 = blockIdx.y * FT;
  float fr[FT][NPH];
  bool act[FT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < FT; ++j) {
    double af[3] = {0.0, 0.0, 0.0};
    act[j] = batch_fit_active<FORM>(a, f0 + j, af);
    any = any || act[j];
#pragma unroll
    for (int q = 0; q < NPH; ++q) fr[j][q] = fp32_rev(af[q]);
  }
  if (!any) return;
  const WorkItem it = a.items[item];
  const float* __restrict__ u = static_cast<const float*>(a.u) + it.begin;
  const float* __restrict__ w = a.w + it.begin;
  float mf[FT][NM];
#pragma unroll
  for (int j = 0; j < FT; ++j)
#pragma unroll
    for (int c = 0; c < NM; ++c) mf[j][c] = 0.0f;
  for (int e = lane * 4; e < it.count; e += 256) {
    const float4 u4 = *reinterpret_cast<const float4*>(u + e);
    const float4 w4 = *reinterpret_cast<const float4*>(w + e);
#pragma unroll
    for (int j = 0; j < FT; ++j) {
      if (!act[j]) continue;
      accum32<FORM>(u4.x, w4.x, fr[j], mf[j]);
      accum32<FORM>(u4.y, w4.y, fr[j], mf[j]);
      accum32<FORM>(u4.z, w4.z, fr[j], mf[j]);
      accum32<FORM>(u4.w, w4.w, fr[j], mf[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < FT; ++j) {
    if (!act[j]) continue;
    double m[NM];
#pragma unroll
    for (int c = 0; c < NM; ++c) m[c] = (double)mf[j][c];
    wave_sum_store<NM>(m, a.part + (int64_t)(f0 + j) * NM * a.nitems, a.nitems, item, lane);
  }
}

// Matter form, batched: per event and active fit of the tile, P and its slot
// derivatives (five values per fit).
template <typename T, int FT>
__global__ __launch_bounds__(256) void fold_batch_matter_kernel(BatchFoldArgs a) {
  constexpr int NM = 5;
  const int lane = threadIdx.x & 63;
  const int item = (int)((blockIdx.x * (unsigned)blockDim.x + threadIdx.x) >> 6);
  if (item >= a.nitems) return;
  const int f0 = blockIdx.y * FT;
  double v[FT][NSLOT];
  bool act[FT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < FT; ++j) {
    double af[3];
    act[j] = batch_fit_active<FORM_MATTER>(a, f0 + j, af);
    if (act[j]) matter_slots(a.osc, a.theta + (int64_t)(f0 + j) * a.P, v[j]);
    any = any || act[j];
  }
  if (!any) return;
  const WorkItem it = a.items[item];
  const double aL = a.osc.cst[0] * a.Lseg[it.seg];
  const T* __restrict__ u = static_cast<const T*>(a.u) + it.begin;
  const float* __restrict__ w = a.w + it.begin;
  double m[FT][NM];
#pragma unroll
  for (int j = 0; j < FT; ++j)
#pragma unroll
    for (int c = 0; c < NM; ++c) m[j][c] = 0.0;
  for (int e = lane * 4; e < it.count; e += 256) {
    const float4 w4 = *reinterpret_cast<const float4*>(w + e);
    T u4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u4[q] = u[e + q];
#pragma unroll
    for (int j = 0; j < FT; ++j) {
      if (!act[j]) continue;
      matter_accum<T>(u4[0], w4.x, aL, v[j], m[j]);
      matter_accum<T>(u4[1], w4.y, aL, v[j], m[j]);
      matter_accum<T>(u4[2], w4.z, aL, v[j], m[j]);
      matter_accum<T>(u4[3], w4.w, aL, v[j], m[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < FT; ++j)
    if (act[j]) wave_sum_store<NM>(m[j], a.part + (int64_t)(f0 + j) * NM * a.nitems, a.nitems, item, lane);
}

// ft: fits per wavefront tile (1, 2, 4 or 8); each tile reads the events once.
hipError_t launch_fold_batch(int mode, const BatchFoldArgs& a, hipStream_t stream, int ft) {
  if (a.nitems <= 0 || a.B <= 0) return hipSuccess;
  const dim3 grid((a.nitems + 3) / 4, (a.B + ft - 1) / ft);
  const dim3 block(256);
  auto go = [&](auto tile) {
    constexpr int T = decltype(tile)::value;
    if (a.osc.formula == FORM_MATTER) {
      // at most two fits per wavefront: the per-event work is large and
      // each fit's registers are many
      constexpr int TM = T < 2 ? T : 2;
      const dim3 gm((a.nitems + 3) / 4, (a.B + TM - 1) / TM);
      if (mode == 0) hipLaunchKernelGGL((fold_batch_matter_kernel<double, TM>), gm, block, 0, stream, a);
      else hipLaunchKernelGGL((fold_batch_matter_kernel<float, TM>), gm, block, 0, stream, a);
    } else if (mode == 0) {
      if (a.osc.formula == FORM_EQ1) hipLaunchKernelGGL((fold_batch_m64_kernel<FORM_EQ1, T>), grid, block, 0, stream, a);
      else if (a.osc.formula == FORM_3NU) hipLaunchKernelGGL((fold_batch_m64_kernel<FORM_3NU, T>), grid, block, 0, stream, a);
      else hipLaunchKernelGGL((fold_batch_m64_kernel<FORM_4NU, T>), grid, block, 0, stream, a);
    } else {
      if (a.osc.formula == FORM_EQ1) hipLaunchKernelGGL((fold_batch_m32_kernel<FORM_EQ1, T>), grid, block, 0, stream, a);
      else if (a.osc.formula == FORM_3NU) hipLaunchKernelGGL((fold_batch_m32_kernel<FORM_3NU, T>), grid, block, 0, stream, a);
      else hipLaunchKernelGGL((fold_batch_m32_kernel<FORM_4NU, T>), grid, block, 0, stream, a);
    }
  };
  switch (ft) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 8: go(std::integral_constant<int, 8>{}); break;
    default: go(std::integral_constant<int, 4>{}); break;
  }
  return hipGetLastError();
}

// Host-side launcher (same translation unit as the kernels). With events, the
// launch carries them in its dispatch (hipExtLaunchKernel), so they take the
// kernel's own start and end times.
hipError_t launch_fold(int mode, const FoldArgs& a, int block, hipStream_t stream, hipEvent_t start,
                       hipEvent_t stop) {
  if (a.nitems <= 0 && a.npre <= 0) return hipSuccess;
  const int waves_per_block = block / 64;
  const dim3 grid(a.npre + (a.nitems + waves_per_block - 1) / waves_per_block);
  auto go = [&](auto kernel) {
    if (start || stop) hipExtLaunchKernelGGL(kernel, grid, dim3(block), 0, stream, start, stop, 0, a);
    else hipLaunchKernelGGL(kernel, grid, dim3(block), 0, stream, a);
  };
  if (a.osc.formula == FORM_MATTER) {
    if (mode == 0) go(fold_matter_kernel<double>);
    else go(fold_matter_kernel<float>);
  } else if (mode == 0) {
    if (a.osc.formula == FORM_EQ1) go(fold_m64_kernel<FORM_EQ1>);
    else if (a.osc.formula == FORM_3NU) go(fold_m64_kernel<FORM_3NU>);
    else go(fold_m64_kernel<FORM_4NU>);
  } else {
    if (a.osc.formula == FORM_EQ1) go(fold_m32_kernel<FORM_EQ1>);
    else if (a.osc.formula == FORM_3NU) go(fold_m32_kernel<FORM_3NU>);
    else go(fold_m32_kernel<FORM_4NU>);
  }
  return hipGetLastError();
}

}  // namespace nufold
