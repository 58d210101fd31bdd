// Host runtime and C-ABI of the engine: model parsing into a flat device plan,
// the device-resident event store (sorted by dataset, source and fine bin,
// padded, split into work items), and the evaluation entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nufold.h"
#include "json.hpp"
#include "kernels.hpp"

using namespace nufold;

namespace nufold {
int mlp_shape(const nf_mlp* n, int* n_in, int* n_out, int* max_batch);  // mlp.hip
}

// Scratch of the allocation-free evaluation (nf_eval_device_noalloc): one
// array per GPU, part of the loaded code object, held until the process
// ends. Host code never uses the array's name as an address: each device's
// address comes from hipGetSymbolAddress (scratch_address below).
static __device__ __align__(256) unsigned char scratch[NF_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; nullptr if the lookup fails.
void* scratch_address() {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) ptr = nullptr;
  addr[dev] = ptr;
  return ptr;
}

struct ApiError : std::runtime_error {
  int code;
  ApiError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& m) { throw ApiError(code, m); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? NF_ENOMEM : NF_EDEVICE,
                            std::string(what) + ": " + hipGetErrorString(e));
}

struct HostBkg {
  int rate = -1;
  double scale = 0.0;
  std::vector<double> tmpl;
  std::vector<int> shape;  // empty: no shape parameters
};

struct HostDataset {
  std::string name;
  double y0 = 0, wf = 0;
  int K = 0, Nb = 0, S = 0, M = 0;
  std::vector<double> edges;
  std::vector<double> baselines;
  std::vector<std::vector<int>> srcnorm;  // dataset norms followed by source norms
  std::vector<int> flux_param;
  std::vector<double> basis;  // M x K
  int cidx[3] = {-1, -1, -1};
  std::vector<HostBkg> bkgs;
  // events, sorted by (source, fine bin), each segment padded to a multiple of 4
  bool has_events = false;
  bool has_data = false;
  std::vector<double> u64;
  std::vector<float> u32;
  std::vector<float> w;
  std::vector<int64_t> seg_count;  // padded events per segment, S*K
  std::vector<double> Wseg;        // weight sum per segment
  int64_t dropped = 0;
  std::vector<double> data;
  int seg0 = 0, bins0 = 0;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    hip_check(hipMalloc(&p, count * sizeof(T)), "hipMalloc");
    n = count;
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    if (v.size() != n) alloc(v.size());
    if (!v.empty()) hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s),
                              "hipMemcpyAsync H2D");
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Inverse of a symmetric positive-definite matrix by Cholesky (host, FP64).
bool spd_inverse(const std::vector<double>& A, int n, std::vector<double>& inv) {
  std::vector<double> L(A.size(), 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  inv.assign((size_t)n * n, 0.0);
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    // solve L y = e_c, then L^T x = y
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * col[k];
      col[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = col[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * inv[(size_t)k * n + c];
      inv[(size_t)i * n + c] = t / L[(size_t)i * n + i];
    }
  }
  return true;
}

}  // namespace

struct nf_ctx {
  std::string err;
  int mode = NF_M64;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  int P = 0;
  std::vector<std::string> names;
  std::vector<char> fixed_default;
  std::map<std::string, int> index;
  OscPlan osc{};
  std::vector<HostDataset> ds;
  int nbins_total = 0;

  // flat plan
  std::vector<double> dpool;
  std::vector<int> ipool;
  std::vector<DsPlan> dsplan;
  std::vector<BkgPlan> bkgplan;
  DevPlan plan{};

  DevBuf<double> d_dpool;
  DevBuf<int> d_ipool;
  DevBuf<DsPlan> d_ds;
  DevBuf<BkgPlan> d_bkg;
  DevBuf<double> d_u64;
  DevBuf<float> d_u32;
  DevBuf<float> d_w;
  DevBuf<WorkItem> d_items;
  DevBuf<int> d_seg_item;
  DevBuf<double> d_Wseg;
  DevBuf<double> d_Lseg;           // baseline of each segment's source (the matter form)
  DevBuf<double> d_part;
  DevBuf<double> d_theta;
  DevBuf<double> d_out;
  DevBuf<int32_t> d_status;
  DevBuf<double> d_data;
  DevBuf<double> d_mu;
  DevBuf<double> d_Sseg;
  DevBuf<double> d_bin;
  DevBuf<int> d_seg_cnt, d_kt_cnt, d_seg_kt, d_kt_need;  // fused fine-bin reduction in the fold
  DevBuf<ItemEpi> d_epi;                                   // per work item epilogue records
  DevBuf<double> d_segm;
  DevBuf<double> d_pre;  // parameter-pass buffer of the single evaluation
  double* h_stage = nullptr;  // pinned: theta, out, mu
  int32_t* h_status = nullptr;
  int nitems = 0;
  int64_t zpad = 0;  // first of the 4 zero-weight events after all datasets' events
  int batch_threads_opt = 0;  // bin-stage threads per fit in batched launches (0: by model size)

  int64_t chunk = 4096;
  int fold_block = 256;
  int tail_threads = 512;
  int timing = 0;
  int deterministic = 0;  // fine-bin rows by ordered hand-off (1) or atomic adds (0)
  int batch_tile = FOLD_FT;  // fits per wavefront tile of the batched fold
  int max_lds = 65536;       // LDS bytes one workgroup may use on this device
  // stage cache of the host evaluation path (option "stage_cache"): the fold
  // depends only on the oscillation parameters and the source norms, so an
  // evaluation whose values of those equal the last fold's reuses its rows
  int stage_cache = 0;
  bool rows_kept = false;            // bin rows 0..4 hold the fold of cache_key (not cleared)
  std::vector<double> cache_key;
  // minimiser buffers (allocated at the first fit) and the captured iteration graph
  int fit_m = 8;
  DevBuf<FitHeader> f_hdr;
  DevBuf<double> f_x, f_g, f_p, f_d2, f_fr, f_S, f_Y, f_rho, f_gam;
  FitHeader* h_hdr = nullptr;  // pinned
  hipGraphExec_t fit_graph = nullptr;
  // batched evaluations and fits (capacity bt_cap fits)
  int bt_cap = 0, bt_nsets = 0;
  DevBuf<double> bt_theta, bt_part, bt_out, bt_Sseg, bt_bin, bt_segtmp, bt_osc_last, bt_data;
  DevBuf<double> bt_fold_theta, bt_mu;  // distinct oscillation points; expectations (nf_expected_batch)
  DevBuf<int32_t> bt_status;
  DevBuf<int> bt_didx, bt_pidx;
  DevBuf<FitHeader> bf_hdr;
  DevBuf<double> bf_x, bf_g, bf_p, bf_d2, bf_fr, bf_S, bf_Y, bf_rho, bf_gam;
  std::vector<FitHeader> bh_hdr;
  hipGraphExec_t bf_graph = nullptr;
  int bf_graph_B = 0;
  // graph of n consecutive device evaluations (nf_eval_device_many), keyed by
  // its arguments
  hipGraphExec_t ev_graph = nullptr;
  int ev_n = 0, ev_grad = -1;
  const double* ev_theta = nullptr;
  double* ev_out = nullptr;
  int32_t* ev_status = nullptr;
  // surrogate for warm starts (nf_set_surrogate; the network is the caller's)
  struct Surrogate {
    nf_mlp* net = nullptr;
    int n_in = 0, n_out = 0, max_batch = 0, n_starts = 0, iters = 0;
    float lr = 0.f;
    std::vector<int> idx;
    std::vector<double> center, half;
    std::vector<float> out_mean, out_std, x_prior, x_weight, starts;
  } sur;
  void* scratch_dev = nullptr;  // this device's `scratch` array (nf_eval_device_noalloc)
  std::vector<std::array<hipEvent_t, 4>> tev;  // per-evaluation kernel start/stop events (fold, bin stages)
  size_t tcount = 0;

  ~nf_ctx() {
    d_dpool.release(); d_ipool.release(); d_ds.release(); d_bkg.release();
    d_u64.release(); d_u32.release(); d_w.release(); d_items.release(); d_seg_item.release();
    d_Wseg.release(); d_Lseg.release(); d_part.release(); d_theta.release(); d_out.release(); d_status.release();
    d_data.release(); d_mu.release(); d_Sseg.release(); d_bin.release();
    d_seg_cnt.release(); d_kt_cnt.release(); d_seg_kt.release(); d_kt_need.release(); d_segm.release();
    d_epi.release();
    d_pre.release();
    if (h_stage) (void)hipHostFree(h_stage);
    if (h_status) (void)hipHostFree(h_status);
    if (h_hdr) (void)hipHostFree(h_hdr);
    if (fit_graph) (void)hipGraphExecDestroy(fit_graph);
    f_hdr.release(); f_x.release(); f_g.release(); f_p.release(); f_d2.release(); f_fr.release();
    f_S.release(); f_Y.release(); f_rho.release(); f_gam.release();
    if (bf_graph) (void)hipGraphExecDestroy(bf_graph);
    if (ev_graph) (void)hipGraphExecDestroy(ev_graph);
    for (auto* b : {&bt_theta, &bt_part, &bt_out, &bt_Sseg, &bt_bin, &bt_segtmp, &bt_osc_last, &bt_data,
                    &bt_fold_theta, &bt_mu, &bf_x, &bf_g, &bf_p, &bf_d2, &bf_fr, &bf_S, &bf_Y, &bf_rho, &bf_gam})
      b->release();
    bt_status.release(); bt_didx.release(); bt_pidx.release(); bf_hdr.release();
    for (auto& t : tev)
      for (auto& e : t)
        if (e) (void)hipEventDestroy(e);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

thread_local std::string g_create_error;

int param_ref(nf_ctx* c, const Json& v, bool allow_null, const std::string& where) {
  if (v.is_null()) {
    if (allow_null) return -1;
    fail(NF_EPARSE, where + ": parameter name required");
  }
  auto it = c->index.find(v.string());
  if (it == c->index.end()) fail(NF_EPARSE, where + ": unknown parameter '" + v.string() + "'");
  return it->second;
}

std::vector<double> num_array(const Json& v, const std::string& where) {
  std::vector<double> out;
  for (const auto& e : v.array()) {
    if (e.kind != Json::Number) fail(NF_EPARSE, where + ": expected numbers");
    out.push_back(e.num);
  }
  return out;
}

void parse_model(nf_ctx* c, const char* text) {
  Json root;
  try {
    root = parse_json(text);
  } catch (const JsonError& e) {
    fail(NF_EPARSE, e.what());
  }
  try {
    // parameters
    const auto& params = root.at("params").array();
    if (params.empty()) fail(NF_EPARSE, "params: empty");
    for (const auto& p : params) {
      const std::string& n = p.at("name").string();
      if (c->index.count(n)) fail(NF_EPARSE, "duplicate parameter '" + n + "'");
      c->index[n] = (int)c->names.size();
      c->names.push_back(n);
    }
    c->P = (int)c->names.size();
    for (const auto& p : params) {
      const Json& fx = p.get("fixed");
      c->fixed_default.push_back(fx.kind == Json::Bool && fx.b ? 1 : 0);
    }
    std::vector<int> gidx;
    std::vector<double> gmean, ginv;
    for (int i = 0; i < c->P; ++i) {
      const Json& pr = params[i].get("prior");
      if (pr.is_null()) continue;
      const auto& a = pr.array();
      if (a.size() != 2 || !(a[1].number() > 0.0)) fail(NF_EPARSE, "prior of '" + c->names[i] + "' must be [mean, sigma>0]");
      gidx.push_back(i);
      gmean.push_back(a[0].number());
      ginv.push_back(1.0 / (a[1].number() * a[1].number()));
    }
    // oscillation
    const Json& o = root.at("osc");
    const std::string& f = o.at("formula").string();
    static const char* eq1[NSLOT] = {"sin2_2t13", "dm2_ee", "sin2_t12", "dm2_21"};
    static const char* nu3[NSLOT] = {"sin2_t12", "sin2_t13", "dm2_21", "dm2_31"};
    static const char* nu4[NSLOT] = {"sin2_t13", "dm2_31", "sin2_2t14", "dm2_41"};
    const char** slots;
    if (f == "eq1") { c->osc.formula = FORM_EQ1; slots = eq1; }
    else if (f == "3nu") { c->osc.formula = FORM_3NU; slots = nu3; }
    else if (f == "4nu") {
      // 3+1: the solar pair is a pair of constants
      c->osc.formula = FORM_4NU;
      slots = nu4;
      c->osc.cst[0] = o.at("sin2_t12").at("value").number();
      c->osc.cst[1] = o.at("dm2_21").at("value").number();
    }
    else if (f == "3nu_matter") {
      // exact three flavours in matter of constant density rho Y_e (g/cm^3)
      c->osc.formula = FORM_MATTER;
      slots = nu3;
      const double rho_ye = o.at("rho_ye").number();
      if (!(rho_ye >= 0.0) || !std::isfinite(rho_ye)) fail(NF_EPARSE, "osc.rho_ye must be a finite number >= 0");
      c->osc.cst[0] = MATTER_A_PER_MEV * rho_ye;
    }
    else fail(NF_EPARSE, "osc.formula must be eq1, 3nu, 4nu or 3nu_matter");
    // FP32 phases and their frequency correction: vacuum forms only (the
    // matter form evaluates every event in FP64 in both modes)
    c->osc.fp32_phase = (c->mode == NF_M32 && c->osc.formula != FORM_MATTER) ? 1 : 0;
    for (int j = 0; j < NSLOT; ++j) {
      const Json& s = o.at(slots[j]);
      if (s.has("param")) {
        c->osc.slot_param[j] = param_ref(c, s.at("param"), false, std::string("osc.") + slots[j]);
        c->osc.slot_value[j] = 0.0;
      } else {
        c->osc.slot_param[j] = -1;
        c->osc.slot_value[j] = s.at("value").number();
      }
    }
    // datasets
    const auto& dsj = root.at("datasets").array();
    if (dsj.empty()) fail(NF_EPARSE, "datasets: empty");
    int seg0 = 0, bins0 = 0;
    for (const auto& dj : dsj) {
      if (!dj.get("backgrounds").is_null() && (int)dj.at("backgrounds").array().size() > MAX_BKG)
        fail(NF_EPARSE, "at most 8 backgrounds per dataset");
      HostDataset d;
      d.name = dj.get("name").kind == Json::String ? dj.get("name").string() : "";
      const Json& fine = dj.at("fine");
      d.y0 = fine.at("y0").number();
      d.wf = fine.at("width").number();
      d.K = (int)fine.at("n").number();
      if (!(d.wf > 0.0) || d.K < 1 || d.K > 8192) fail(NF_EPARSE, "fine binning invalid in dataset " + d.name);
      d.edges = num_array(dj.at("edges"), "edges");
      d.Nb = (int)d.edges.size() - 1;
      if (d.Nb < 1 || d.Nb > 8192) fail(NF_EPARSE, "edges: need 2..8193 values");
      for (int i = 0; i < d.Nb; ++i)
        if (!(d.edges[i + 1] > d.edges[i])) fail(NF_EPARSE, "edges must increase");
      std::vector<int> dnorm;
      if (!dj.get("norm").is_null())
        for (const auto& n : dj.at("norm").array()) dnorm.push_back(param_ref(c, n, false, "norm"));
      const auto& srcs = dj.at("sources").array();
      d.S = (int)srcs.size();
      if (d.S < 1 || d.S > MAX_SOURCES) fail(NF_EPARSE, "sources: need 1..64");
      for (const auto& s : srcs) {
        const double L = s.at("baseline_m").number();
        if (!(L > 0.0)) fail(NF_EPARSE, "baseline_m must be > 0");
        d.baselines.push_back(L);
        std::vector<int> lst = dnorm;
        if (!s.get("norm").is_null())
          for (const auto& n : s.at("norm").array()) lst.push_back(param_ref(c, n, false, "source norm"));
        if ((int)lst.size() > NLMAX) fail(NF_EPARSE, "at most 8 norm parameters per source");
        d.srcnorm.push_back(lst);
      }
      const Json& fl = dj.get("flux");
      if (!fl.is_null()) {
        for (const auto& n : fl.at("params").array()) d.flux_param.push_back(param_ref(c, n, false, "flux"));
        d.M = (int)d.flux_param.size();
        const auto& basis = fl.at("basis").array();
        if ((int)basis.size() != d.M) fail(NF_EPARSE, "flux.basis must have one row per mode");
        for (const auto& row : basis) {
          auto r = num_array(row, "flux.basis");
          if ((int)r.size() != d.K) fail(NF_EPARSE, "flux.basis rows must have fine.n entries");
          d.basis.insert(d.basis.end(), r.begin(), r.end());
        }
      }
      const Json& es = dj.get("escale");
      if (!es.is_null()) {
        d.cidx[0] = param_ref(c, es.get("c0"), true, "escale.c0");
        d.cidx[1] = param_ref(c, es.get("c1"), true, "escale.c1");
        d.cidx[2] = param_ref(c, es.get("c2"), true, "escale.c2");
      }
      if (!dj.get("backgrounds").is_null()) {
        for (const auto& bj : dj.at("backgrounds").array()) {
          HostBkg b;
          b.rate = param_ref(c, bj.get("rate"), true, "background rate");
          b.scale = bj.at("scale").number();
          b.tmpl = num_array(bj.at("template"), "template");
          if ((int)b.tmpl.size() != d.Nb) fail(NF_EPARSE, "template must have Nb entries");
          const Json& sh = bj.get("shape");
          if (!sh.is_null()) {
            if ((int)sh.array().size() != d.Nb) fail(NF_EPARSE, "shape must have Nb entries");
            for (const auto& n : sh.array()) b.shape.push_back(param_ref(c, n, true, "background shape"));
          }
          d.bkgs.push_back(b);
        }
      }
      d.seg0 = seg0;
      d.bins0 = bins0;
      seg0 += d.S * d.K;
      bins0 += d.Nb;
      c->ds.push_back(std::move(d));
    }
    c->nbins_total = bins0;

    // ---- flat pools
    auto& dp = c->dpool;
    auto& ip = c->ipool;
    DevPlan& pl = c->plan;
    pl.P = c->P;
    pl.D = (int)c->ds.size();
    pl.G = seg0;
    pl.nbins_total = bins0;
    pl.osc = c->osc;
    pl.max_K = pl.max_Nb = pl.max_S = pl.max_B = pl.max_M = pl.max_nnz = pl.max_nl = 0;
    int kt = 0, fs = 0;
    for (auto& d : c->ds) {
      DsPlan q{};
      q.kt0 = kt;
      q.fs0 = fs;
      kt += d.K;
      fs += d.S;
      q.y0 = d.y0; q.wf = d.wf; q.K = d.K; q.Nb = d.Nb; q.S = d.S; q.M = d.M;
      q.nbkg = (int)d.bkgs.size();
      q.seg0 = d.seg0;
      q.data = d.bins0;
      q.bins0 = d.bins0;
      q.edges = (int)dp.size();
      dp.insert(dp.end(), d.edges.begin(), d.edges.end());
      // source norm lists: S+1 absolute offsets, then indices
      q.srcnorm_ptr = (int)ip.size();
      ip.resize(ip.size() + d.S + 1);
      for (int s = 0; s < d.S; ++s) {
        ip[q.srcnorm_ptr + s] = (int)ip.size();
        ip.insert(ip.end(), d.srcnorm[s].begin(), d.srcnorm[s].end());
      }
      ip[q.srcnorm_ptr + d.S] = (int)ip.size();
      q.nl0 = ip[q.srcnorm_ptr];
      q.nl = ip[q.srcnorm_ptr + d.S] - q.nl0;
      // flux basis: CSR over fine bins, CSC over modes (exact zeros dropped)
      q.md_param = (int)ip.size();
      ip.insert(ip.end(), d.flux_param.begin(), d.flux_param.end());
      std::vector<int> rmode, rptr(d.K + 1, 0), ck, cptr(d.M + 1, 0);
      std::vector<double> rcoef, ccoef;
      for (int k = 0; k < d.K; ++k) {
        rptr[k] = (int)rmode.size();
        for (int m = 0; m < d.M; ++m) {
          const double v = d.basis[(size_t)m * d.K + k];
          if (v != 0.0) { rmode.push_back(m); rcoef.push_back(v); }
        }
      }
      rptr[d.K] = (int)rmode.size();
      for (int m = 0; m < d.M; ++m) {
        cptr[m] = (int)ck.size();
        for (int k = 0; k < d.K; ++k) {
          const double v = d.basis[(size_t)m * d.K + k];
          if (v != 0.0) { ck.push_back(k); ccoef.push_back(v); }
        }
      }
      cptr[d.M] = (int)ck.size();
      q.nnz = (int)ck.size();
      q.fx_coef = (int)dp.size();
      dp.insert(dp.end(), rcoef.begin(), rcoef.end());
      q.fx_mode = (int)ip.size();
      ip.insert(ip.end(), rmode.begin(), rmode.end());
      // row pointers and column pointers are entry numbers relative to the
      // dataset's entry arrays (fx_mode/fx_coef and md_k/md_coef bases)
      q.fx_row = (int)ip.size();
      ip.insert(ip.end(), rptr.begin(), rptr.end());
      q.md_coef = (int)dp.size();
      dp.insert(dp.end(), ccoef.begin(), ccoef.end());
      q.md_k = (int)ip.size();
      ip.insert(ip.end(), ck.begin(), ck.end());
      q.md_col = (int)ip.size();
      for (int m = 0; m <= d.M; ++m) ip.push_back(cptr[m]);
      for (int j = 0; j < 3; ++j) q.cidx[j] = d.cidx[j];
      q.bkg0 = (int)c->bkgplan.size();
      for (auto& b : d.bkgs) {
        BkgPlan bp{};
        bp.scale = b.scale;
        bp.rate = b.rate;
        bp.tmpl = (int)dp.size();
        dp.insert(dp.end(), b.tmpl.begin(), b.tmpl.end());
        if (b.shape.empty()) bp.shape = -1;
        else {
          bp.shape = (int)ip.size();
          ip.insert(ip.end(), b.shape.begin(), b.shape.end());
        }
        c->bkgplan.push_back(bp);
      }
      c->dsplan.push_back(q);
      pl.max_K = std::max(pl.max_K, d.K);
      pl.max_Nb = std::max(pl.max_Nb, d.Nb);
      pl.max_S = std::max(pl.max_S, d.S);
      pl.max_B = std::max(pl.max_B, q.nbkg);
      pl.max_M = std::max(pl.max_M, q.M);
      pl.max_nnz = std::max(pl.max_nnz, q.nnz);
      pl.max_nl = std::max(pl.max_nl, q.nl);
    }
    pl.KT = kt;
    pl.FS = fs;
    // parameter-pass buffer of the single evaluation
    {
      int o = 0;
      pl.max_pre = 0;
      for (size_t di = 0; di < c->dsplan.size(); ++di) {
        DsPlan& q = c->dsplan[di];
        const PreLayout L = pre_layout(q.K, q.Nb, q.nbkg);
        q.pre0 = o;
        o += L.total;
        pl.max_pre = std::max(pl.max_pre, L.total);
      }
      pl.pre_prv = o;  // NR is known after the priors below
      pl.pre_total = o;
    }
    c->fit_m = std::min(std::max(c->P, 8), 24);  // L-BFGS history; reduced below if LDS is short
    pl.fit_m = c->fit_m;
    // static blobs (one per dataset) for the serial bin stages
    pl.max_blob = 0;
    for (size_t di = 0; di < c->dsplan.size(); ++di) {
      DsPlan& q = c->dsplan[di];
      const HostDataset& d = c->ds[di];
      int fw = 1;
      for (int k = 0; k < q.K; ++k) fw = std::max(fw, ip[q.fx_row + k + 1] - ip[q.fx_row + k]);
      if (fw > FLUX_FW_MAX)
        fail(NF_EPARSE, "at most " + std::to_string(FLUX_FW_MAX) + " flux modes may be non-zero in one fine bin");
      q.fw = fw;
      const BlobLayout B = blob_layout(q.Nb + 1, q.nbkg, q.Nb, q.nnz, q.M, q.S, q.nl, q.K, fw);
      std::vector<double> blob(B.total, 0.0);
      // 32-bit integer j of the int array at double offset off
      auto put = [&](int off, int j, int v) { std::memcpy(reinterpret_cast<char*>(&blob[off]) + 4 * (size_t)j, &v, 4); };
      for (int i = 0; i <= q.Nb; ++i) blob[B.edges + i] = d.edges[i];
      for (int b = 0; b < q.nbkg; ++b) {
        const HostBkg& hb = d.bkgs[b];
        blob[B.bsc + b] = hb.scale;
        put(B.brt, b, hb.rate);
        for (int i = 0; i < q.Nb; ++i) {
          blob[B.tmpl + b * q.Nb + i] = hb.tmpl[i];
          put(B.shp, b * q.Nb + i, hb.shape.empty() ? -1 : hb.shape[i]);
        }
      }
      for (int e = 0; e < q.nnz; ++e) {
        blob[B.mdc + e] = dp[q.md_coef + e];
        put(B.mdk, e, ip[q.md_k + e]);
      }
      for (int m = 0; m <= q.M; ++m) put(B.mdcol, m, ip[q.md_col + m]);
      for (int m = 0; m < q.M; ++m) put(B.mdp, m, ip[q.md_param + m]);
      for (int s = 0; s <= q.S; ++s) put(B.nlp, s, ip[q.srcnorm_ptr + s] - q.nl0);
      for (int j = 0; j < q.nl; ++j) put(B.nli, j, ip[q.nl0 + j]);
      for (int k = 0; k < q.K; ++k) {
        const int e0 = ip[q.fx_row + k], e1 = ip[q.fx_row + k + 1];
        for (int j = 0; j < fw; ++j) {
          const int e = e0 + j;
          put(B.fpar, k * fw + j, e < e1 ? d.flux_param[ip[q.fx_mode + e]] : -1);
          blob[B.fcf + k * fw + j] = e < e1 ? dp[q.fx_coef + e] : 0.0;
        }
      }
      if (dp.size() % 2) dp.push_back(0.0);  // 16-byte aligned blobs (direct LDS copies in 16-byte units)
      q.blob = (int)dp.size();
      q.blob_n = B.total;
      dp.insert(dp.end(), blob.begin(), blob.end());
      pl.max_blob = std::max(pl.max_blob, B.hpart);
    }
    // per global fine bin: first segment, stride, sources, first flat source
    pl.kt_info = (int)ip.size();
    for (const auto& q : c->dsplan)
      for (int k = 0; k < q.K; ++k) {
        ip.push_back(q.seg0 + k);
        ip.push_back(q.K);
        ip.push_back(q.S);
        ip.push_back(q.fs0);
        ip.push_back(q.kt0);
      }
    // per flat source: fixed-width norm list
    pl.fs_nl = (int)ip.size();
    for (size_t di = 0; di < c->ds.size(); ++di)
      for (int s = 0; s < c->ds[di].S; ++s)
        for (int j = 0; j < NLMAX; ++j)
          ip.push_back(j < (int)c->ds[di].srcnorm[s].size() ? c->ds[di].srcnorm[s][j] : -1);
    // per-segment flat source, per-fine-bin dataset, per-flat-source norm-list range
    pl.seg_fs = (int)ip.size();
    for (size_t di = 0; di < c->dsplan.size(); ++di) {
      const DsPlan& q = c->dsplan[di];
      for (int s = 0; s < q.S; ++s)
        for (int k = 0; k < q.K; ++k) ip.push_back(q.fs0 + s);
    }
    pl.kt_ds = (int)ip.size();
    for (size_t di = 0; di < c->dsplan.size(); ++di)
      for (int k = 0; k < c->dsplan[di].K; ++k) ip.push_back((int)di);
    // flux basis rows per global fine bin with parameter indices (for phase A)
    {
      std::vector<int> rows(1, 0), par;
      std::vector<double> cf;
      for (const auto& d : c->ds)
        for (int k = 0; k < d.K; ++k) {
          for (int m = 0; m < d.M; ++m) {
            const double v = d.basis[(size_t)m * d.K + k];
            if (v != 0.0) {
              par.push_back(d.flux_param[m]);
              cf.push_back(v);
            }
          }
          rows.push_back((int)par.size());
        }
      pl.kt_row = (int)ip.size();
      ip.insert(ip.end(), rows.begin(), rows.end());
      pl.kt_par = (int)ip.size();
      ip.insert(ip.end(), par.begin(), par.end());
      pl.kt_coef = (int)dp.size();
      dp.insert(dp.end(), cf.begin(), cf.end());
    }
    pl.fs_ptr = (int)ip.size();
    for (size_t di = 0; di < c->dsplan.size(); ++di) {
      const DsPlan& q = c->dsplan[di];
      for (int s = 0; s < q.S; ++s) {
        ip.push_back(ip[q.srcnorm_ptr + s]);
        ip.push_back(ip[q.srcnorm_ptr + s + 1]);
      }
    }
    // priors
    pl.ngauss = (int)gidx.size();
    pl.gidx = (int)ip.size();
    ip.insert(ip.end(), gidx.begin(), gidx.end());
    pl.gmean = (int)dp.size();
    dp.insert(dp.end(), gmean.begin(), gmean.end());
    pl.ginv = (int)dp.size();
    dp.insert(dp.end(), ginv.begin(), ginv.end());
    const Json& cp = root.get("cov_priors");
    std::vector<int> bptr, bidx, binv;
    std::vector<double> bmean;
    if (!cp.is_null()) {
      for (const auto& bj : cp.array()) {
        std::vector<int> idx;
        for (const auto& n : bj.at("params").array()) idx.push_back(param_ref(c, n, false, "cov_priors"));
        auto mean = num_array(bj.at("mean"), "cov_priors.mean");
        const int n = (int)idx.size();
        if (n < 1 || (int)mean.size() != n) fail(NF_EPARSE, "cov_priors: params/mean size mismatch");
        std::vector<double> cov;
        const auto& rows = bj.at("cov").array();
        if ((int)rows.size() != n) fail(NF_EPARSE, "cov_priors: cov must be n x n");
        for (const auto& r : rows) {
          auto v = num_array(r, "cov_priors.cov");
          if ((int)v.size() != n) fail(NF_EPARSE, "cov_priors: cov must be n x n");
          cov.insert(cov.end(), v.begin(), v.end());
        }
        std::vector<double> inv;
        if (!spd_inverse(cov, n, inv)) fail(NF_EPARSE, "cov_priors: covariance not positive definite");
        bptr.push_back((int)bidx.size());
        bidx.insert(bidx.end(), idx.begin(), idx.end());
        bmean.insert(bmean.end(), mean.begin(), mean.end());
        binv.push_back((int)dp.size());
        dp.insert(dp.end(), inv.begin(), inv.end());
      }
    }
    pl.nblk = (int)binv.size();
    bptr.push_back((int)bidx.size());
    pl.blk_ptr = (int)ip.size();
    ip.insert(ip.end(), bptr.begin(), bptr.end());
    pl.blk_idx = (int)ip.size();
    ip.insert(ip.end(), bidx.begin(), bidx.end());
    pl.blk_mean = (int)dp.size();
    dp.insert(dp.end(), bmean.begin(), bmean.end());
    pl.blk_inv = (int)ip.size();
    ip.insert(ip.end(), binv.begin(), binv.end());
    pl.NR = pl.ngauss + (int)bidx.size();
    pl.prow_blk = (int)ip.size();
    for (int b = 0; b < pl.nblk; ++b)
      for (int r = bptr[b]; r < bptr[b + 1]; ++r) ip.push_back(b);
    pl.pre_pri = pl.pre_prv + pl.NR;
    pl.pre_misc = pl.pre_pri + (pl.NR + 1) / 2;
    pl.pre_glob = pl.pre_misc + 2 + pl.D - pl.pre_prv;
    pl.pre_total = pl.pre_misc + 2 + pl.D;
  } catch (const JsonError& e) {
    fail(NF_EPARSE, e.what());
  }
}

void upload_plan(nf_ctx* c) {
  c->d_dpool.upload(c->dpool.empty() ? std::vector<double>{0.0} : c->dpool, c->stream);
  c->d_ipool.upload(c->ipool.empty() ? std::vector<int>{0} : c->ipool, c->stream);
  c->d_ds.upload(c->dsplan, c->stream);
  std::vector<BkgPlan> b = c->bkgplan;
  if (b.empty()) b.push_back(BkgPlan{});
  c->d_bkg.upload(b, c->stream);
  c->plan.ds = c->d_ds.p;
  c->plan.ds0 = c->dsplan.empty() ? DsPlan{} : c->dsplan[0];
  c->plan.bkg = c->d_bkg.p;
  c->plan.dpool = c->d_dpool.p;
  c->plan.ipool = c->d_ipool.p;
  c->d_theta.alloc(c->P);
  c->d_out.alloc(1 + c->P);
  c->d_status.alloc(1);
  c->d_data.alloc(std::max(1, c->nbins_total));
  c->d_mu.alloc(std::max(1, c->nbins_total));
  c->d_Sseg.alloc((size_t)std::max(1, c->plan.G));
  c->d_bin.alloc((size_t)6 * std::max(1, c->plan.KT));
  c->d_pre.alloc((size_t)c->plan.pre_total);
  {
    // fine bin of every segment (static), arrival counters and segment moments
    const int G = std::max(1, c->plan.G), KT = std::max(1, c->plan.KT);
    std::vector<int> seg_kt(G, 0);
    for (int kt = 0; kt < c->plan.KT; ++kt) {
      const int* info = &c->ipool[c->plan.kt_info + 5 * kt];
      for (int s2 = 0; s2 < info[2]; ++s2) seg_kt[info[0] + s2 * info[1]] = kt;
    }
    c->d_seg_kt.upload(seg_kt, c->stream);
    c->d_seg_cnt.alloc(G);
    c->d_kt_cnt.alloc(KT);
    c->d_kt_need.alloc(KT);
    c->d_segm.alloc((size_t)(MAX_MOM + 1) * G);
    hip_check(hipMemsetAsync(c->d_seg_cnt.p, 0, sizeof(int) * G, c->stream), "hipMemsetAsync");
    hip_check(hipMemsetAsync(c->d_kt_cnt.p, 0, sizeof(int) * KT, c->stream), "hipMemsetAsync");
  }
  hip_check(hipHostMalloc((void**)&c->h_stage, sizeof(double) * (2 + 2 * c->P + c->nbins_total)),
            "hipHostMalloc");
  hip_check(hipHostMalloc((void**)&c->h_status, sizeof(int32_t) * 4), "hipHostMalloc");
  hip_check(hipMemsetAsync(c->d_data.p, 0, sizeof(double) * std::max(1, c->nbins_total), c->stream),
            "hipMemsetAsync");
}

// Fine bin of every event: the largest k with y_k <= E, y_k = y0 + k*width
// (edges evaluated exactly as written, no fused multiply-add); -1 / K outside.
#pragma clang fp contract(off)
int fine_bin(double E, double y0, double wf, int K) {
  double t = std::floor((E - y0) / wf);
  int k;
  if (!(t > -2.0)) k = -1;
  else if (t > (double)K + 1.0) k = K;
  else k = (int)t;
  auto edge = [&](int j) {
    const double step = wf * (double)j;
    return y0 + step;
  };
  if (k > K) k = K;
  if (k < -1) k = -1;
  while (k >= 0 && E < edge(k)) --k;
  while (k + 1 <= K && E >= edge(k + 1)) ++k;
  return k;  // in [-1, K]
}
#pragma clang fp contract(on)

void drop_fit_graph(nf_ctx* c) {
  if (c->fit_graph) (void)hipGraphExecDestroy(c->fit_graph);
  c->fit_graph = nullptr;
  if (c->bf_graph) (void)hipGraphExecDestroy(c->bf_graph);
  c->bf_graph = nullptr;
  c->bf_graph_B = 0;
  if (c->ev_graph) (void)hipGraphExecDestroy(c->ev_graph);
  c->ev_graph = nullptr;
  c->ev_n = 0;
}

// The fold's inputs among the parameters: oscillation slots and every norm
// parameter of every source (the fold applies the source norms).
std::vector<double> fold_key(const nf_ctx* c, const double* theta) {
  std::vector<double> k;
  for (int j = 0; j < NSLOT; ++j)
    if (c->osc.slot_param[j] >= 0) k.push_back(theta[c->osc.slot_param[j]]);
  for (const auto& d : c->ds)
    for (const auto& nl : d.srcnorm)
      for (int q : nl) k.push_back(theta[q]);
  return k;
}

// Every path except the cached host evaluation expects the fold kernel's
// accumulation rows to be zero at launch: clear rows that were kept.
void release_rows(nf_ctx* c) {
  if (!c->rows_kept) return;
  hip_check(launch_zero(c->d_bin.p, 6 * (int64_t)std::max(1, c->plan.KT), c->stream), "zero launch");
  c->rows_kept = false;
}

void rebuild_events(nf_ctx* c) {
  drop_fit_graph(c);
  c->rows_kept = false;  // the rows are cleared below
  c->bt_cap = 0;  // batch partials depend on the work-item count
  std::vector<int> seg_item(c->plan.G + 1, 0);
  std::vector<double> Wseg(c->plan.G, 0.0);
  std::vector<WorkItem> items;
  int64_t total = 0;
  for (auto& d : c->ds) total += (int64_t)d.w.size();
  std::vector<double> u64;
  std::vector<float> u32, w;
  if (c->mode == NF_M64) u64.reserve(total + 4); else u32.reserve(total + 4);
  w.reserve(total + 4);
  const int64_t chunk = c->chunk;
  for (auto& d : c->ds) {
    int64_t local = 0;
    for (int s = 0; s < d.S; ++s) {
      for (int k = 0; k < d.K; ++k) {
        const int g = d.seg0 + s * d.K + k;
        seg_item[g] = (int)items.size();
        if (!d.has_events) continue;
        const int64_t cnt = d.seg_count[s * d.K + k];
        const int64_t base = (int64_t)w.size();
        for (int64_t off = 0; off < cnt; off += chunk) {
          WorkItem it;
          it.begin = base + off;
          it.count = (int32_t)std::min<int64_t>(chunk, cnt - off);
          it.seg = g;
          items.push_back(it);
        }
        Wseg[g] = d.Wseg[s * d.K + k];
        if (c->mode == NF_M64) u64.insert(u64.end(), d.u64.begin() + local, d.u64.begin() + local + cnt);
        else u32.insert(u32.end(), d.u32.begin() + local, d.u32.begin() + local + cnt);
        w.insert(w.end(), d.w.begin() + local, d.w.begin() + local + cnt);
        local += cnt;
      }
    }
  }
  seg_item[c->plan.G] = (int)items.size();
  if (items.size() > (size_t)0x7fffffff) fail(NF_EINVAL, "too many work items");
  // 4 zero-weight events after the last one: the fold's prefetching loads of
  // positions past an item's end are redirected here
  c->zpad = (int64_t)w.size();
  if (c->mode == NF_M64) u64.insert(u64.end(), 4, 0.0); else u32.insert(u32.end(), 4, 0.0f);
  w.insert(w.end(), 4, 0.0f);
  c->nitems = (int)items.size();
  if (c->mode == NF_M64) c->d_u64.upload(u64, c->stream); else c->d_u32.upload(u32, c->stream);
  c->d_w.upload(w, c->stream);
  c->d_items.upload(items, c->stream);
  c->d_seg_item.upload(seg_item, c->stream);
  {
    // per-item epilogue records (segment weight, fine-bin row, source, item range)
    std::vector<int> seg_kt(std::max(1, c->plan.G), 0);
    for (int kt = 0; kt < c->plan.KT; ++kt) {
      const int* info = &c->ipool[c->plan.kt_info + 5 * kt];
      for (int s2 = 0; s2 < info[2]; ++s2) seg_kt[info[0] + s2 * info[1]] = kt;
    }
    std::vector<ItemEpi> epi(std::max<size_t>(1, items.size()));
    for (size_t i = 0; i < items.size(); ++i) {
      const int g = items[i].seg, kt = seg_kt[g];
      const int* info = &c->ipool[c->plan.kt_info + 5 * kt];
      ItemEpi& e = epi[i];
      e.W = Wseg[g];
      e.row = 6 * info[4] + (kt - info[4]);
      e.K = info[1];
      e.first = seg_item[g];
      e.nseg = seg_item[g + 1] - seg_item[g];
      const int fs = info[3] + (g - info[0]) / info[1];
      for (int q = 0; q < NLMAX; ++q) e.nl[q] = c->ipool[c->plan.fs_nl + NLMAX * fs + q];
      e.pad_[0] = e.pad_[1] = 0;
    }
    c->d_epi.upload(epi, c->stream);
  }
  c->d_Wseg.upload(Wseg, c->stream);
  {
    std::vector<double> Lseg(std::max(1, c->plan.G), 0.0);
    for (auto& d : c->ds)
      for (int s = 0; s < d.S; ++s)
        for (int k = 0; k < d.K; ++k) Lseg[d.seg0 + s * d.K + k] = d.baselines[s];
    c->d_Lseg.upload(Lseg, c->stream);
  }
  c->d_part.alloc((size_t)MAX_MOM * std::max(1, c->nitems));
  {
    // segments with work items per fine bin; fine bins and segments without
    // events are never written by the fold, so they start (and stay) zero
    std::vector<int> need(std::max(1, c->plan.KT), 0);
    for (int kt = 0; kt < c->plan.KT; ++kt) {
      const int* info = &c->ipool[c->plan.kt_info + 5 * kt];
      for (int s2 = 0; s2 < info[2]; ++s2) {
        const int g = info[0] + s2 * info[1];
        if (seg_item[g + 1] > seg_item[g]) ++need[kt];
      }
    }
    c->d_kt_need.upload(need, c->stream);
    hip_check(hipMemsetAsync(c->d_Sseg.p, 0, sizeof(double) * std::max(1, c->plan.G), c->stream), "memset");
    hip_check(hipMemsetAsync(c->d_bin.p, 0, sizeof(double) * 6 * std::max(1, c->plan.KT), c->stream), "memset");
    hip_check(hipMemsetAsync(c->d_seg_cnt.p, 0, sizeof(int) * std::max(1, c->plan.G), c->stream), "memset");
    hip_check(hipMemsetAsync(c->d_kt_cnt.p, 0, sizeof(int) * std::max(1, c->plan.KT), c->stream), "memset");
  }
  c->plan.G = (int)Wseg.size();
  c->plan.nitems = c->nitems;
  c->plan.seg_item = c->d_seg_item.p;
  c->plan.Wseg = c->d_Wseg.p;
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

void set_events_impl(nf_ctx* c, int dsi, int64_t n, const double* e_true, const double* e_reco,
                     const uint8_t* source, const float* weight, int on_device) {
  if (dsi < 0 || dsi >= (int)c->ds.size()) fail(NF_EINVAL, "dataset index out of range");
  if (n < 0) fail(NF_EINVAL, "negative event count");
  if (n > 0 && (!e_true || !e_reco)) fail(NF_EINVAL, "null energy pointer");
  HostDataset& d = c->ds[dsi];
  std::vector<double> et(n), er(n);
  std::vector<uint8_t> src(n, 0);
  std::vector<float> wt(n, 1.0f);
  if (n > 0) {
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    hip_check(hipMemcpy(et.data(), e_true, n * sizeof(double), kind), "copy e_true");
    hip_check(hipMemcpy(er.data(), e_reco, n * sizeof(double), kind), "copy e_reco");
    if (source) hip_check(hipMemcpy(src.data(), source, n, kind), "copy source");
    if (weight) hip_check(hipMemcpy(wt.data(), weight, n * sizeof(float), kind), "copy weight");
  }
  const int K = d.K, S = d.S;
  std::vector<int> key(n);
  std::vector<int64_t> cnt((size_t)S * K, 0);
  int64_t dropped = 0;
  for (int64_t e = 0; e < n; ++e) {
    if (!(std::isfinite(et[e]) && et[e] > 0.0)) fail(NF_EINVAL, "e_true must be finite and > 0");
    if (!std::isfinite(er[e])) fail(NF_EINVAL, "e_reco must be finite");
    if (!std::isfinite(wt[e])) fail(NF_EINVAL, "weights must be finite");
    if (src[e] >= S) fail(NF_EINVAL, "source index out of range");
    const int k = fine_bin(er[e], d.y0, d.wf, K);
    if (k < 0 || k >= K) {
      key[e] = -1;
      ++dropped;
      continue;
    }
    key[e] = src[e] * K + k;
    ++cnt[key[e]];
  }
  // stable counting sort; segments padded to a multiple of 4 with zero weights
  std::vector<int64_t> padded(cnt.size()), start(cnt.size() + 1, 0);
  for (size_t g = 0; g < cnt.size(); ++g) {
    padded[g] = (cnt[g] + 3) & ~int64_t(3);
    start[g + 1] = start[g] + padded[g];
  }
  const int64_t npad = start.back();
  std::vector<double> u64;
  std::vector<float> u32;
  if (c->mode == NF_M64) u64.assign(npad, 0.0); else u32.assign(npad, 0.0f);
  std::vector<float> w(npad, 0.0f);
  std::vector<double> Wseg(cnt.size(), 0.0);
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  for (int64_t e = 0; e < n; ++e) {
    const int g = key[e];
    if (g < 0) continue;
    const double u = d.baselines[g / K] / et[e];
    const int64_t pos = fill[g]++;
    if (c->mode == NF_M64) u64[pos] = u; else u32[pos] = (float)u;
    w[pos] = wt[e];
    Wseg[g] += (double)wt[e];
  }
  d.u64.swap(u64);
  d.u32.swap(u32);
  d.w.swap(w);
  d.seg_count.swap(padded);
  d.Wseg.swap(Wseg);
  d.dropped = dropped;
  d.has_events = true;
  rebuild_events(c);
}

void require_ready(nf_ctx* c, bool need_data) {
  for (auto& d : c->ds) {
    if (!d.has_events) fail(NF_ESTATE, "events not set for dataset '" + d.name + "'");
    if (need_data && !d.has_data) fail(NF_ESTATE, "data not set for dataset '" + d.name + "'");
  }
}

FitArgs fit_args(nf_ctx* c) {
  FitArgs f{};
  f.hdr = c->f_hdr.p;
  f.x = c->f_x.p;
  f.g = c->f_g.p;
  f.p = c->f_p.p;
  f.d2 = c->f_d2.p;
  f.freem = c->f_fr.p;
  f.S = c->f_S.p;
  f.Y = c->f_Y.p;
  f.rho = c->f_rho.p;
  f.gam = c->f_gam.p;
  f.theta_next = c->d_theta.p;
  f.m = c->fit_m;
  return f;
}

// Scratch of one single evaluation: fold partials, per-segment moments and
// spectra, fine-bin rows and arrival counters (the context's own buffers, or
// the static array of the allocation-free entry point).
struct EvalScratch {
  double* part;
  double* segm;
  double* Sseg;
  double* bin;
  int* seg_cnt;
  int* kt_cnt;
  double* pre;
};

void enqueue_eval(nf_ctx* c, const double* theta_dev, double* out_dev, int32_t* status_dev, double* mu_dev,
                  int want_nll, int want_grad, bool fit = false, bool timed = true, bool reuse_fold = false,
                  bool keep_rows = false, const EvalScratch* scr = nullptr) {
  const EvalScratch own{c->d_part.p, c->d_segm.p, c->d_Sseg.p, c->d_bin.p, c->d_seg_cnt.p, c->d_kt_cnt.p,
                        c->d_pre.p};
  const EvalScratch& sc = scr ? *scr : own;
  FoldArgs fa{};
  fa.u = c->mode == NF_M64 ? (const void*)c->d_u64.p : (const void*)c->d_u32.p;
  fa.w = c->d_w.p;
  fa.items = c->d_items.p;
  fa.nitems = c->nitems;
  fa.zpad = c->zpad;
  fa.theta = theta_dev;
  fa.osc = c->osc;
  fa.Lseg = c->d_Lseg.p;
  fa.part = sc.part;
  fa.plan = c->plan;
  fa.pre = sc.pre;
  fa.npre = 3 * c->plan.D + 1;
  FoldFuse& fu = fa.fuse;
  fu.epi = c->d_epi.p;
  fu.seg_item = c->d_seg_item.p;
  fu.seg_kt = c->d_seg_kt.p;
  fu.kt_need = c->d_kt_need.p;
  fu.kt_info = c->d_ipool.p + c->plan.kt_info;
  fu.fs_nl = c->d_ipool.p + c->plan.fs_nl;
  fu.seg_cnt = sc.seg_cnt;
  fu.kt_cnt = sc.kt_cnt;
  fu.segm = sc.segm;
  fu.Sseg = sc.Sseg;
  fu.bin = sc.bin;
  fu.G = c->plan.G;
  fu.atomic_rows = c->deterministic ? 0 : 1;
  TailArgs ta{};
  ta.plan = c->plan;
  ta.theta = theta_dev;
  ta.data = c->d_data.p;
  ta.out = out_dev;
  ta.status = status_dev;
  ta.mu_out = mu_dev;
  ta.Sseg = sc.Sseg;
  ta.bin = sc.bin;
  ta.pre = sc.pre;
  ta.want_grad = want_grad;
  ta.want_nll = want_nll;
  ta.keep_rows = keep_rows ? 1 : 0;
  if (fit) {
    ta.has_fit = 1;
    ta.fit = fit_args(c);
    ta.skip = &c->f_hdr.p->status;
    fa.skip = &c->f_hdr.p->status;
  }
  hipEvent_t* ev = nullptr;
  if (c->timing && !fit && timed) {
    if (c->tcount == c->tev.size()) {
      std::array<hipEvent_t, 4> t{};
      // timing-only events: no system-scope fence (no cache write-back or
      // invalidation around the timed kernels)
      for (auto& e : t) hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
      c->tev.push_back(t);
    }
    ev = c->tev[c->tcount++].data();
  }
  if (reuse_fold) {
    // the rows of the last fold are still in place: the launch runs only its
    // parameter-pass workgroups
    FoldArgs pa = fa;
    pa.nitems = 0;
    hip_check(launch_fold(c->mode, pa, c->fold_block, c->stream, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr),
              "parameter pass launch");
  } else {
    hip_check(launch_fold(c->mode, fa, c->fold_block, c->stream, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr),
              "fold launch");
  }
  hip_check(launch_tail(ta, c->tail_threads, c->stream, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr),
            "tail launch");
}

int eval_host(nf_ctx* c, const double* theta, double* nll, double* grad, double* mu) {
  const bool want_nll = nll != nullptr;
  require_ready(c, want_nll);
  if (!theta) fail(NF_EINVAL, "theta is null");
  for (int i = 0; i < c->P; ++i)
    if (!std::isfinite(theta[i])) fail(NF_EINVAL, "theta[" + std::to_string(i) + "] is not finite");
  double* h_theta = c->h_stage;
  double* h_out = c->h_stage + c->P;
  double* h_mu = c->h_stage + 2 * c->P + 1;
  std::memcpy(h_theta, theta, sizeof(double) * c->P);
  hip_check(hipMemcpyAsync(c->d_theta.p, h_theta, sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream),
            "theta H2D");
  bool reuse = false;
  if (c->stage_cache) {
    std::vector<double> key = fold_key(c, theta);
    reuse = c->rows_kept && key == c->cache_key;
    if (!reuse) {
      release_rows(c);
      c->cache_key.swap(key);
    }
  } else {
    release_rows(c);
  }
  enqueue_eval(c, c->d_theta.p, c->d_out.p, c->d_status.p, mu ? c->d_mu.p : nullptr, want_nll ? 1 : 0,
               grad ? 1 : 0, false, true, reuse, c->stage_cache != 0);
  if (c->stage_cache) c->rows_kept = true;
  if (want_nll)
    hip_check(hipMemcpyAsync(h_out, c->d_out.p, sizeof(double) * (grad ? 1 + c->P : 1), hipMemcpyDeviceToHost,
                             c->stream), "out D2H");
  hip_check(hipMemcpyAsync(c->h_status, c->d_status.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream),
            "status D2H");
  if (mu)
    hip_check(hipMemcpyAsync(h_mu, c->d_mu.p, sizeof(double) * c->nbins_total, hipMemcpyDeviceToHost, c->stream),
              "mu D2H");
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (want_nll) {
    *nll = h_out[0];
    if (grad) std::memcpy(grad, h_out + 1, sizeof(double) * c->P);
  }
  if (mu) std::memcpy(mu, h_mu, sizeof(double) * c->nbins_total);
  if (*c->h_status & ST_DOMAIN) {
    c->err = "expectation <= 0, energy map not monotone, or oscillation parameter out of domain";
    return NF_WDOMAIN;
  }
  return NF_OK;
}

constexpr int FIT_CHUNK = 8;  // iterations per graph launch

// Public fit status: 0 converged, 2 iteration limit, 3 line search failed, 4 domain.
int public_status(int s) { return s == FIT_CONVERGED ? 0 : s; }

void ensure_fit_buffers(nf_ctx* c) {
  if (c->f_hdr.p) return;
  const size_t P = c->P, m = c->fit_m;
  c->f_hdr.alloc(1);
  c->f_x.alloc(P); c->f_g.alloc(P); c->f_p.alloc(P); c->f_d2.alloc(P); c->f_fr.alloc(P);
  c->f_S.alloc(m * P); c->f_Y.alloc(m * P); c->f_rho.alloc(m); c->f_gam.alloc(m);
  hip_check(hipHostMalloc((void**)&c->h_hdr, sizeof(FitHeader)), "hipHostMalloc");
}

void ensure_fit_graph(nf_ctx* c) {
  if (c->fit_graph) return;
  hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    for (int i = 0; i < FIT_CHUNK; ++i)
      enqueue_eval(c, c->d_theta.p, c->d_out.p, c->d_status.p, nullptr, 1, 1, true);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(c->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  hip_check(hipStreamEndCapture(c->stream, &g), "hipStreamEndCapture");
  const hipError_t e = hipGraphInstantiate(&c->fit_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, "hipGraphInstantiate");
}

// Diagonal preconditioner: prior variance, else covariance-block diagonal,
// else (5% of the start value, at least 1e-3)^2, a scale guess, stored
// negated so that the minimiser can tell it from a variance.
std::vector<double> preconditioner(nf_ctx* c, const double* start) {
  std::vector<double> d2(c->P, -1.0);
  const DevPlan& pl = c->plan;
  for (int j = 0; j < pl.ngauss; ++j) d2[c->ipool[pl.gidx + j]] = 1.0 / c->dpool[pl.ginv + j];
  for (int b = 0; b < pl.nblk; ++b) {
    const int b0 = c->ipool[pl.blk_ptr + b], b1 = c->ipool[pl.blk_ptr + b + 1], n = b1 - b0;
    const double* Vi = c->dpool.data() + c->ipool[pl.blk_inv + b];
    for (int r = 0; r < n; ++r) {
      const int i = c->ipool[pl.blk_idx + b0 + r];
      if (d2[i] < 0) d2[i] = 1.0 / Vi[(size_t)r * n + r];  // conditional variance scale
    }
  }
  for (int i = 0; i < c->P; ++i)
    if (d2[i] < 0) {
      const double s = 0.05 * std::max(std::fabs(start[i]), 0.02);
      d2[i] = -(s * s);
    }
  return d2;
}

// Warm starts (nf_fit_opts.warm_start): B start vectors (B x P, host) and the
// observed counts of each fit (B x all bins); writes the B start vectors with
// the surrogate's inputs replaced by the best of the start grid fitted on the
// surrogate to each fit's counts.
std::vector<double> surrogate_starts(nf_ctx* c, int B, const double* start, const std::vector<double>& obs) {
  auto& s = c->sur;
  if (!s.net) fail(NF_ESTATE, "warm start requested but no surrogate is attached (nf_set_surrogate)");
  const int S = s.n_starts, Ni = s.n_in, No = s.n_out;
  const int64_t N = (int64_t)B * S;
  std::vector<float> X((size_t)N * Ni), Nobs((size_t)N * No), F((size_t)N);
  for (int f = 0; f < B; ++f)
    for (int k = 0; k < S; ++k) {
      const int64_t r = (int64_t)f * S + k;
      std::memcpy(&X[(size_t)r * Ni], &s.starts[(size_t)k * Ni], sizeof(float) * Ni);
      for (int j = 0; j < No; ++j) Nobs[(size_t)r * No + j] = (float)obs[(size_t)f * No + j];
    }
  for (int64_t o = 0; o < N; o += s.max_batch) {
    const int n = (int)std::min<int64_t>(s.max_batch, N - o);
    const int code = nf_mlp_fit_inputs(s.net, n, &X[(size_t)o * Ni], &Nobs[(size_t)o * No], s.out_mean.data(),
                                       s.out_std.data(), s.x_prior.data(), s.x_weight.data(), s.iters, s.lr,
                                       &F[(size_t)o]);
    if (code < 0) fail(code, std::string("surrogate warm start: ") + nf_mlp_last_error(s.net));
  }
  const size_t P = c->P;
  std::vector<double> out(start, start + (size_t)B * P);
  for (int f = 0; f < B; ++f) {
    int best = -1;
    for (int k = 0; k < S; ++k) {
      const float v = F[(size_t)f * S + k];
      if (std::isfinite(v) && (best < 0 || v < F[(size_t)f * S + best])) best = k;
    }
    if (best < 0) continue;  // no finite surrogate fit: keep the given start
    const float* x = &X[((size_t)f * S + best) * Ni];
    for (int i = 0; i < Ni; ++i) {
      const double xi = std::min(1.0, std::max(-1.0, (double)x[i]));
      out[(size_t)f * P + s.idx[i]] = s.center[i] + s.half[i] * xi;
    }
  }
  return out;
}

bool want_warm(const nf_fit_opts* opts) { return opts && opts->warm_start == NF_SURROGATE; }

int fit_impl(nf_ctx* c, const double* start, const uint8_t* fixed, const nf_fit_opts* opts,
             nf_fit_result* res) {
  require_ready(c, true);
  if (!start || !res) fail(NF_EINVAL, "start and result are required");
  for (int i = 0; i < c->P; ++i)
    if (!std::isfinite(start[i])) fail(NF_EINVAL, "start[" + std::to_string(i) + "] is not finite");
  std::vector<double> warm;
  if (want_warm(opts)) {
    std::vector<double> obs(std::max(1, c->nbins_total));
    hip_check(hipMemcpy(obs.data(), c->d_data.p, sizeof(double) * c->nbins_total, hipMemcpyDeviceToHost), "D2H");
    warm = surrogate_starts(c, 1, start, obs);
    // the exact fold judges the proposal: it replaces the start only if its
    // NLL is lower
    double f0 = INFINITY, f1 = INFINITY;
    (void)eval_host(c, start, &f0, nullptr, nullptr);
    (void)eval_host(c, warm.data(), &f1, nullptr, nullptr);
    if (!(f1 < f0)) warm.assign(start, start + c->P);
    start = warm.data();
  }
  const double tol = (opts && opts->edm_tol > 0) ? opts->edm_tol : 1e-7;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 1000;
  ensure_fit_buffers(c);
  const std::vector<double> d2 = preconditioner(c, start);
  std::vector<double> fr(c->P, 1.0);
  for (int i = 0; i < c->P; ++i)
    if (fixed ? fixed[i] != 0 : c->fixed_default[i]) fr[i] = 0.0;
  FitHeader h{};
  h.status = FIT_RUNNING;
  h.phase = 0;
  h.max_iter = max_iter;
  h.edm_tol = tol;
  h.alpha = 1.0;
  *c->h_hdr = h;
  hip_check(hipMemcpyAsync(c->f_hdr.p, c->h_hdr, sizeof(FitHeader), hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->d_theta.p, start, sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->f_d2.p, d2.data(), sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->f_fr.p, fr.data(), sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  release_rows(c);
  ensure_fit_graph(c);
  const int64_t max_evals = (int64_t)max_iter * 50 + 200;
  for (int64_t launched = 0;; launched += FIT_CHUNK) {
    hip_check(hipGraphLaunch(c->fit_graph, c->stream), "hipGraphLaunch");
    hip_check(hipMemcpyAsync(c->h_hdr, c->f_hdr.p, sizeof(FitHeader), hipMemcpyDeviceToHost, c->stream), "D2H");
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (c->h_hdr->status != FIT_RUNNING) break;
    if (launched + FIT_CHUNK >= max_evals) {
      c->h_hdr->status = FIT_MAXITER;
      break;
    }
  }
  const FitHeader fh = *c->h_hdr;
  std::vector<double> x(c->P);
  hip_check(hipMemcpy(x.data(), c->f_x.p, sizeof(double) * c->P, hipMemcpyDeviceToHost), "D2H");
  res->nll = fh.f;
  res->edm = fh.edm;
  res->status = public_status(fh.status);
  res->iters = fh.iter;
  res->evals = fh.nevals;
  if (res->theta) std::memcpy(res->theta, x.data(), sizeof(double) * c->P);
  if (fh.status == FIT_DOMAIN) {
    c->err = "start point out of the model's domain";
    return NF_WDOMAIN;
  }
  int code = fh.status == FIT_CONVERGED ? NF_OK : NF_WNOCONV;
  if (code != NF_OK) c->err = fh.status == FIT_MAXITER ? "iteration limit reached" : "line search failed";
  if (opts && opts->want_cov && res->cov) {
    std::vector<int> fi;
    for (int i = 0; i < c->P; ++i)
      if (fr[i] != 0.0) fi.push_back(i);
    const int n = (int)fi.size();
    std::vector<double> Hm((size_t)n * n), th(x), gp(c->P), gm(c->P);
    double fdum;
    for (int a = 0; a < n; ++a) {
      const int j = fi[a];
      const double hstep = 1e-3 * std::sqrt(std::fabs(d2[j]));
      th[j] = x[j] + hstep;
      eval_host(c, th.data(), &fdum, gp.data(), nullptr);
      th[j] = x[j] - hstep;
      eval_host(c, th.data(), &fdum, gm.data(), nullptr);
      th[j] = x[j];
      for (int b = 0; b < n; ++b) Hm[(size_t)b * n + a] = (gp[fi[b]] - gm[fi[b]]) / (2.0 * hstep);
    }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < a; ++b) {
        const double v = 0.5 * (Hm[(size_t)a * n + b] + Hm[(size_t)b * n + a]);
        Hm[(size_t)a * n + b] = Hm[(size_t)b * n + a] = v;
      }
    std::vector<double> inv;
    std::fill(res->cov, res->cov + (size_t)c->P * c->P, 0.0);
    if (spd_inverse(Hm, n, inv)) {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) res->cov[(size_t)fi[a] * c->P + fi[b]] = inv[(size_t)a * n + b];
    } else {
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) res->cov[(size_t)fi[a] * c->P + fi[b]] = NAN;
      c->err = "Hessian at the minimum is not positive definite";
      if (code == NF_OK) code = NF_WNOCONV;
    }
  }
  return code;
}

// ---------------------------------------------------------------- batches
void ensure_batch(nf_ctx* c, int B) {
  if (B <= c->bt_cap) return;
  drop_fit_graph(c);
  const size_t P = c->P, m = c->fit_m, G = std::max(1, c->plan.G), KT = std::max(1, c->plan.KT);
  const size_t NM = MAX_MOM, NI = std::max(1, c->nitems);
  c->bt_theta.alloc(B * P);
  c->bt_part.alloc(B * NM * NI);
  c->bt_out.alloc(B * (1 + P));
  c->bt_Sseg.alloc(B * G);
  c->bt_bin.alloc(B * 6 * KT);
  c->bt_segtmp.alloc(B * 5 * G);
  c->bt_osc_last.alloc(B * 4);
  c->bt_status.alloc(B);
  c->bt_didx.alloc(B);
  c->bt_pidx.alloc(B);
  c->bt_fold_theta.alloc(B * P);
  c->bt_mu.alloc(B * (size_t)std::max(1, c->nbins_total));
  c->bf_hdr.alloc(B);
  c->bf_x.alloc(B * P); c->bf_g.alloc(B * P); c->bf_p.alloc(B * P); c->bf_d2.alloc(B * P); c->bf_fr.alloc(B * P);
  c->bf_S.alloc(B * m * P); c->bf_Y.alloc(B * m * P); c->bf_rho.alloc(B * m); c->bf_gam.alloc(B * m);
  c->bh_hdr.resize(B);
  c->bt_cap = B;
}

BatchFoldArgs batch_fold_args(nf_ctx* c, int B, bool fit) {
  BatchFoldArgs a{};
  a.u = c->mode == NF_M64 ? (const void*)c->d_u64.p : (const void*)c->d_u32.p;
  a.w = c->d_w.p;
  a.items = c->d_items.p;
  a.nitems = c->nitems;
  a.P = c->P;
  a.B = B;
  a.theta = c->bt_theta.p;
  a.osc = c->osc;
  a.Lseg = c->d_Lseg.p;
  a.part = c->bt_part.p;
  a.hdr = fit ? c->bf_hdr.p : nullptr;
  a.osc_last = fit ? c->bt_osc_last.p : nullptr;
  return a;
}

BatchTailArgs batch_tail_args(nf_ctx* c, int B, bool fit, bool want_grad, bool use_didx) {
  BatchTailArgs a{};
  a.plan = c->plan;
  a.B = B;
  a.theta = c->bt_theta.p;
  a.part = c->bt_part.p;
  a.data = c->bt_data.p;
  a.data_idx = use_didx ? c->bt_didx.p : nullptr;
  a.out = c->bt_out.p;
  a.status = c->bt_status.p;
  a.Sseg = c->bt_Sseg.p;
  a.bin = c->bt_bin.p;
  a.segtmp = c->bt_segtmp.p;
  a.osc_last = fit ? c->bt_osc_last.p : nullptr;
  a.want_grad = want_grad ? 1 : 0;
  a.want_nll = 1;
  a.has_fit = fit ? 1 : 0;
  if (fit) {
    FitArgs f{};
    f.hdr = c->bf_hdr.p;
    f.x = c->bf_x.p; f.g = c->bf_g.p; f.p = c->bf_p.p; f.d2 = c->bf_d2.p; f.freem = c->bf_fr.p;
    f.S = c->bf_S.p; f.Y = c->bf_Y.p; f.rho = c->bf_rho.p; f.gam = c->bf_gam.p;
    f.theta_next = c->bt_theta.p;
    f.m = c->fit_m;
    a.fit = f;
  }
  return a;
}

// whether a bin-stage workgroup of nt threads fits this model's LDS
bool tail_fits(const nf_ctx* c, int nt) { return tail_lds_bytes(c->plan, nt) <= (size_t)c->max_lds; }

int batch_threads(nf_ctx* c) {
  if (c->batch_threads_opt) return c->batch_threads_opt;
  return c->plan.G > 2048 ? 512 : 256;
}

void check_didx(nf_ctx* c, int B, const int* didx) {
  if (c->bt_nsets <= 0) fail(NF_ESTATE, "batch data not set (nf_set_data_batch)");
  for (int f = 0; f < B; ++f) {
    const int r = didx ? didx[f] : f;
    if (r < 0 || r >= c->bt_nsets) fail(NF_EINVAL, "data index out of range for fit " + std::to_string(f));
  }
}

// ---------------------------------------------------------------- autotuner
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    hip_check(hipEventCreateWithFlags(&a, hipEventDisableSystemFence), "hipEventCreate");
    hip_check(hipEventCreateWithFlags(&b, hipEventDisableSystemFence), "hipEventCreate");
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  double us_per(int n) {
    hip_check(hipEventSynchronize(b), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
    return 1e3 * ms / n;
  }
};

// mean device time of one evaluation (fold + bin stages + NLL + gradient) at d_theta
double time_single(nf_ctx* c, int n) {
  release_rows(c);
  EventPair ev;
  for (int i = 0; i < 2; ++i) enqueue_eval(c, c->d_theta.p, c->d_out.p, c->d_status.p, nullptr, 1, 1);
  hip_check(hipEventRecord(ev.a, c->stream), "hipEventRecord");
  for (int i = 0; i < n; ++i) enqueue_eval(c, c->d_theta.p, c->d_out.p, c->d_status.p, nullptr, 1, 1);
  hip_check(hipEventRecord(ev.b, c->stream), "hipEventRecord");
  return ev.us_per(n);
}

// mean device time of one batched evaluation of B fits (bt_theta, data row 0)
double time_batch(nf_ctx* c, int B, int n) {
  EventPair ev;
  auto once = [&] {
    hip_check(launch_fold_batch(c->mode, batch_fold_args(c, B, false), c->stream, c->batch_tile), "batch fold");
    hip_check(launch_batch_tail(batch_tail_args(c, B, false, true, true), batch_threads(c), c->stream),
              "batch tail");
  };
  once();
  hip_check(hipEventRecord(ev.a, c->stream), "hipEventRecord");
  for (int i = 0; i < n; ++i) once();
  hip_check(hipEventRecord(ev.b, c->stream), "hipEventRecord");
  return ev.us_per(n);
}

// Sweep the launch choices on this context's model and events and keep the
// fastest: bin-stage threads, then work-item size x fold workgroup size for
// the single evaluation; bin-stage threads per fit for batched launches of
// `batch` fits when batch data are set (batch > 0).
int autotune_impl(nf_ctx* c, const double* theta, int evals, int batch, int64_t* best, double* best_us) {
  require_ready(c, true);
  if (!theta || evals < 0 || batch < 0 || (evals == 0 && batch == 0))
    fail(NF_EINVAL, "theta, evals >= 0, batch >= 0 and evals + batch > 0 are required");
  for (int i = 0; i < c->P; ++i)
    if (!std::isfinite(theta[i])) fail(NF_EINVAL, "theta contains a non-finite value");
  const int timing = c->timing;
  c->timing = 0;
  hip_check(hipMemcpy(c->d_theta.p, theta, sizeof(double) * c->P, hipMemcpyHostToDevice), "H2D");
  // the current choice is timed first and a candidate replaces the best so far
  // only when it is faster by more than this margin, so that timing noise does
  // not move the launch configuration between equivalent choices
  constexpr double MARGIN = 0.01;
  auto better = [](double t, double t_best) { return t < t_best * (1.0 - MARGIN); };
  double t_best = 0.0;
  if (evals > 0) {  // single-evaluation choices
    int nt_best = c->tail_threads;
    t_best = time_single(c, evals);
    for (int nt : {256, 512, 1024}) {
      if (nt == nt_best || !tail_fits(c, nt)) continue;
      c->tail_threads = nt;
      const double t = time_single(c, evals);
      if (better(t, t_best)) { t_best = t; nt_best = nt; }
    }
    c->tail_threads = nt_best;
    const int64_t ch_cur = c->chunk;
    const int fb_cur = c->fold_block;
    int64_t ch_best = c->chunk;
    int fb_best = c->fold_block;
    t_best = time_single(c, evals);
    for (int64_t ch : {1024, 2048, 4096, 8192}) {
      if (ch != c->chunk) {
        c->chunk = ch;
        rebuild_events(c);
      }
      for (int fb : {64, 128, 256}) {
        if (ch == ch_cur && fb == fb_cur) continue;  // the current choice, timed above
        c->fold_block = fb;
        const double t = time_single(c, evals);
        if (better(t, t_best)) { t_best = t; ch_best = ch; fb_best = fb; }
      }
    }
    if (ch_best != c->chunk) {
      c->chunk = ch_best;
      rebuild_events(c);
    }
    c->fold_block = fb_best;
  }
  int bt_best = c->batch_threads_opt, ft_best = c->batch_tile;
  double tb_best = 0.0;
  if (batch > 0 && c->bt_nsets > 0) {
    ensure_batch(c, batch);
    // every fit of the timed batch folds at its own oscillation point (as at
    // the start of a batch of fits): the free oscillation slots of theta are
    // spread by up to +-1% across the rows
    std::vector<double> th((size_t)batch * c->P);
    for (int f = 0; f < batch; ++f) {
      std::memcpy(&th[(size_t)f * c->P], theta, sizeof(double) * c->P);
      for (int j = 0; j < NSLOT; ++j) {
        const int q = c->osc.slot_param[j];
        if (q >= 0) th[(size_t)f * c->P + q] *= 1.0 + 0.01 * ((double)((f * 7 + j * 13) % 21) / 10.0 - 1.0);
      }
    }
    std::vector<int> didx(batch, 0);
    hip_check(hipMemcpy(c->bt_theta.p, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice), "H2D");
    hip_check(hipMemcpy(c->bt_didx.p, didx.data(), sizeof(int) * batch, hipMemcpyHostToDevice), "H2D");
    tb_best = time_batch(c, batch, std::max(1, evals / 4));
    const int bt_cur = bt_best, ft_cur = ft_best;
    for (int ft : {1, 2, 4, 8})
      for (int nt : {256, 512, 1024}) {
        if ((ft == ft_cur && nt == bt_cur) || !tail_fits(c, nt)) continue;
        c->batch_tile = ft;
        c->batch_threads_opt = nt;
        const double t = time_batch(c, batch, std::max(1, evals / 4));
        if (better(t, tb_best)) { tb_best = t; bt_best = nt; ft_best = ft; }
      }
    c->batch_threads_opt = bt_best;
    c->batch_tile = ft_best;
  }
  drop_fit_graph(c);
  c->timing = timing;
  if (best) {
    best[0] = c->chunk;
    best[1] = c->fold_block;
    best[2] = c->tail_threads;
    best[3] = c->batch_threads_opt;
    best[4] = c->batch_tile;
  }
  if (best_us) {
    best_us[0] = t_best;
    best_us[1] = tb_best;
  }
  return NF_OK;
}

// Expectations for B parameter vectors. Rows whose oscillation slots are equal
// share one fold: the batched fold runs over the distinct oscillation points
// only, and each row's bin stages read the partials of its point.
int expected_batch_impl(nf_ctx* c, int B, const double* theta, double* mu) {
  require_ready(c, false);
  if (B <= 0 || !theta || !mu) fail(NF_EINVAL, "B > 0, theta and mu are required");
  const int P = c->P;
  for (int64_t i = 0; i < (int64_t)B * P; ++i)
    if (!std::isfinite(theta[i])) fail(NF_EINVAL, "theta contains a non-finite value");
  std::map<std::array<double, NSLOT>, int> points;
  std::vector<int> pidx(B);
  std::vector<double> ftheta;
  for (int f = 0; f < B; ++f) {
    std::array<double, NSLOT> key{};
    for (int q = 0; q < NSLOT; ++q) {
      const int i = c->osc.slot_param[q];
      key[q] = i >= 0 ? theta[(size_t)f * P + i] : c->osc.slot_value[q];
    }
    auto it = points.find(key);
    if (it == points.end()) {
      it = points.emplace(key, (int)points.size()).first;
      ftheta.insert(ftheta.end(), theta + (size_t)f * P, theta + (size_t)(f + 1) * P);
    }
    pidx[f] = it->second;
  }
  const int U = (int)points.size();
  ensure_batch(c, B);
  hip_check(hipMemcpyAsync(c->bt_fold_theta.p, ftheta.data(), sizeof(double) * U * P, hipMemcpyHostToDevice,
                           c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bt_theta.p, theta, sizeof(double) * B * P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bt_pidx.p, pidx.data(), sizeof(int) * B, hipMemcpyHostToDevice, c->stream), "H2D");
  BatchFoldArgs fa = batch_fold_args(c, U, false);
  fa.theta = c->bt_fold_theta.p;
  hip_check(launch_fold_batch(c->mode, fa, c->stream, c->batch_tile), "batch fold");
  BatchTailArgs ta = batch_tail_args(c, B, false, false, false);
  ta.part_idx = c->bt_pidx.p;
  ta.data = nullptr;
  ta.want_nll = 0;
  ta.out = nullptr;
  ta.mu_out = c->bt_mu.p;
  hip_check(launch_batch_tail(ta, batch_threads(c), c->stream), "batch tail");
  std::vector<int32_t> st(B);
  hip_check(hipMemcpyAsync(mu, c->bt_mu.p, sizeof(double) * (size_t)B * c->nbins_total, hipMemcpyDeviceToHost,
                           c->stream), "D2H");
  hip_check(hipMemcpyAsync(st.data(), c->bt_status.p, sizeof(int32_t) * B, hipMemcpyDeviceToHost, c->stream), "D2H");
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (int f = 0; f < B; ++f)
    if (st[f] & ST_DOMAIN) {
      c->err = "some parameter vectors are out of domain";
      return NF_WDOMAIN;
    }
  return NF_OK;
}

int eval_batch_impl(nf_ctx* c, int B, const double* theta, const int* didx, double* nll, double* grad) {
  require_ready(c, false);
  if (B <= 0 || !theta || !nll) fail(NF_EINVAL, "B > 0, theta and nll are required");
  check_didx(c, B, didx);
  for (int64_t i = 0; i < (int64_t)B * c->P; ++i)
    if (!std::isfinite(theta[i])) fail(NF_EINVAL, "theta contains a non-finite value");
  ensure_batch(c, B);
  hip_check(hipMemcpyAsync(c->bt_theta.p, theta, sizeof(double) * B * c->P, hipMemcpyHostToDevice, c->stream), "H2D");
  if (didx) hip_check(hipMemcpyAsync(c->bt_didx.p, didx, sizeof(int) * B, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(launch_fold_batch(c->mode, batch_fold_args(c, B, false), c->stream, c->batch_tile), "batch fold");
  hip_check(launch_batch_tail(batch_tail_args(c, B, false, grad != nullptr, didx != nullptr), batch_threads(c),
                              c->stream), "batch tail");
  std::vector<double> out((size_t)B * (1 + c->P));
  std::vector<int32_t> st(B);
  hip_check(hipMemcpyAsync(out.data(), c->bt_out.p, sizeof(double) * out.size(), hipMemcpyDeviceToHost, c->stream), "D2H");
  hip_check(hipMemcpyAsync(st.data(), c->bt_status.p, sizeof(int32_t) * B, hipMemcpyDeviceToHost, c->stream), "D2H");
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  bool dom = false;
  for (int f = 0; f < B; ++f) {
    nll[f] = out[(size_t)f * (1 + c->P)];
    if (grad) std::memcpy(grad + (size_t)f * c->P, &out[(size_t)f * (1 + c->P) + 1], sizeof(double) * c->P);
    dom = dom || (st[f] & ST_DOMAIN);
  }
  if (dom) {
    c->err = "some evaluations are out of domain (NLL = +inf)";
    return NF_WDOMAIN;
  }
  return NF_OK;
}

template <typename F>
int guarded(nf_ctx* c, F&& f) {
  if (!c) return NF_EINVAL;
  try {
    c->err.clear();
    return f();
  } catch (const ApiError& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return NF_ENOMEM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return NF_EINVAL;
  }
}

// FIT_CHUNK iterations of the batched fits of c on stream s: per iteration
// the batched fold, then the bin stages, adjoint and L-BFGS step of every fit.
hipError_t batch_fit_iterations(nf_ctx* c, int B, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < FIT_CHUNK && e == hipSuccess; ++i) {
    e = launch_fold_batch(c->mode, batch_fold_args(c, B, true), s, c->batch_tile);
    if (e == hipSuccess) e = launch_batch_tail(batch_tail_args(c, B, true, true, true), batch_threads(c), s);
  }
  return e;
}

void ensure_batch_fit_graph(nf_ctx* c, int B) {
  if (c->bf_graph && c->bf_graph_B == B) return;
  if (c->bf_graph) (void)hipGraphExecDestroy(c->bf_graph);
  c->bf_graph = nullptr;
  hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const hipError_t e = batch_fit_iterations(c, B, c->stream);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess && g) (void)hipGraphDestroy(g);
  hip_check(e, "batch capture launch");
  hip_check(e2, "hipStreamEndCapture");
  const hipError_t e3 = hipGraphInstantiate(&c->bf_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e3, "hipGraphInstantiate");
  c->bf_graph_B = B;
}

// Host side of a batched fit before its first iteration: argument checks,
// start points, preconditioners, free-parameter masks, data rows and fresh
// fit headers, uploaded on the context's stream (synchronised on return).
// Returns the iteration limit in graph iterations.
int64_t batch_fit_prepare(nf_ctx* c, int B, const double* start, const uint8_t* fixed, const int* didx,
                          const nf_fit_opts* opts) {
  require_ready(c, false);
  if (B <= 0 || !start) fail(NF_EINVAL, "B > 0 and start are required");
  check_didx(c, B, didx);
  for (int64_t i = 0; i < (int64_t)B * c->P; ++i)
    if (!std::isfinite(start[i])) fail(NF_EINVAL, "start contains a non-finite value");
  std::vector<double> warm;
  if (want_warm(opts)) {
    const size_t nb = (size_t)c->nbins_total;
    std::vector<double> all((size_t)c->bt_nsets * nb), obs((size_t)B * nb);
    hip_check(hipMemcpy(all.data(), c->bt_data.p, sizeof(double) * all.size(), hipMemcpyDeviceToHost), "D2H");
    for (int f = 0; f < B; ++f)
      std::memcpy(&obs[f * nb], &all[(size_t)(didx ? didx[f] : f) * nb], sizeof(double) * nb);
    warm = surrogate_starts(c, B, start, obs);
    // the exact fold judges every proposal: it replaces its fit's start only
    // if its NLL is lower
    std::vector<double> n0(B), n1(B);
    (void)eval_batch_impl(c, B, start, didx, n0.data(), nullptr);
    (void)eval_batch_impl(c, B, warm.data(), didx, n1.data(), nullptr);
    for (int f = 0; f < B; ++f)
      if (!(n1[f] < n0[f])) std::memcpy(&warm[(size_t)f * c->P], start + (size_t)f * c->P, sizeof(double) * c->P);
    start = warm.data();
  }
  const double tol = (opts && opts->edm_tol > 0) ? opts->edm_tol : 1e-7;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 1000;
  ensure_batch(c, B);
  const size_t P = c->P;
  std::vector<double> d2(B * P), fr(B * P);
  for (int f = 0; f < B; ++f) {
    const std::vector<double> d = preconditioner(c, start + (size_t)f * P);
    std::memcpy(&d2[(size_t)f * P], d.data(), sizeof(double) * P);
    for (size_t i = 0; i < P; ++i) fr[(size_t)f * P + i] = (fixed ? fixed[i] != 0 : c->fixed_default[i]) ? 0.0 : 1.0;
  }
  std::vector<int> rows(B);
  for (int f = 0; f < B; ++f) rows[f] = didx ? didx[f] : f;
  FitHeader h{};
  h.status = FIT_RUNNING;
  h.max_iter = max_iter;
  h.edm_tol = tol;
  h.alpha = 1.0;
  std::fill(c->bh_hdr.begin(), c->bh_hdr.begin() + B, h);
  std::vector<double> nanv((size_t)B * 4, NAN);
  hip_check(hipMemcpyAsync(c->bf_hdr.p, c->bh_hdr.data(), sizeof(FitHeader) * B, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bt_theta.p, start, sizeof(double) * B * P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bf_d2.p, d2.data(), sizeof(double) * B * P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bf_fr.p, fr.data(), sizeof(double) * B * P, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bt_osc_last.p, nanv.data(), sizeof(double) * B * 4, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipMemcpyAsync(c->bt_didx.p, rows.data(), sizeof(int) * B, hipMemcpyHostToDevice, c->stream), "H2D");
  hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return (int64_t)max_iter * 50 + 200;
}

// Enqueue the copy of the fit headers to the host on stream s (the caller
// synchronises s before reading them).
void batch_fit_headers_d2h(nf_ctx* c, int B, hipStream_t s) {
  hip_check(hipMemcpyAsync(c->bh_hdr.data(), c->bf_hdr.p, sizeof(FitHeader) * B, hipMemcpyDeviceToHost, s), "D2H");
}

int batch_fit_running(const nf_ctx* c, int B) {
  int running = 0;
  for (int f = 0; f < B; ++f) running += c->bh_hdr[f].status == FIT_RUNNING;
  return running;
}

void batch_fit_stop(nf_ctx* c, int B) {
  for (int f = 0; f < B; ++f)
    if (c->bh_hdr[f].status == FIT_RUNNING) c->bh_hdr[f].status = FIT_MAXITER;
}

// Outputs of a finished batched fit (each pointer nullable); NF_WNOCONV when
// some fit did not converge.
int batch_fit_collect(nf_ctx* c, int B, double* theta_out, double* nll_out, double* edm_out, int* status_out,
                      int* iters_out, int* evals_out) {
  if (theta_out)
    hip_check(hipMemcpy(theta_out, c->bf_x.p, sizeof(double) * B * c->P, hipMemcpyDeviceToHost), "D2H");
  bool all_ok = true;
  for (int f = 0; f < B; ++f) {
    const FitHeader& fh = c->bh_hdr[f];
    if (nll_out) nll_out[f] = fh.f;
    if (edm_out) edm_out[f] = fh.edm;
    if (status_out) status_out[f] = public_status(fh.status);
    if (iters_out) iters_out[f] = fh.iter;
    if (evals_out) evals_out[f] = fh.nevals;
    all_ok = all_ok && fh.status == FIT_CONVERGED;
  }
  if (!all_ok) {
    c->err = "some fits did not converge (see status)";
    return NF_WNOCONV;
  }
  return NF_OK;
}

int fit_batch_impl(nf_ctx* c, int B, const double* start, const uint8_t* fixed, const int* didx,
                   const nf_fit_opts* opts, double* theta_out, double* nll_out, double* edm_out, int* status_out,
                   int* iters_out, int* evals_out) {
  const int64_t max_evals = batch_fit_prepare(c, B, start, fixed, didx, opts);
  ensure_batch_fit_graph(c, B);
  for (int64_t launched = 0;; launched += FIT_CHUNK) {
    hip_check(hipGraphLaunch(c->bf_graph, c->stream), "hipGraphLaunch");
    batch_fit_headers_d2h(c, B, c->stream);
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (!batch_fit_running(c, B)) break;
    if (launched + FIT_CHUNK >= max_evals) {
      batch_fit_stop(c, B);
      break;
    }
  }
  return batch_fit_collect(c, B, theta_out, nll_out, edm_out, status_out, iters_out, evals_out);
}

// Batched fits of several contexts advanced together: one HIP graph holds
// FIT_CHUNK iterations of every member, each member's launches on a branch of
// its own (forked from and joined to the first member's stream), so the
// members' kernels run side by side; the graph is replayed, and every
// member's headers are polled after each replay, until all fits of all
// members have stopped.
int fit_batch_group_impl(int n, const nf_batch_member* mem, const nf_fit_opts* opts) {
  if (n < 1 || !mem) return NF_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (!mem[k].ctx) return NF_EINVAL;
    for (int j = 0; j < k; ++j)
      if (mem[j].ctx == mem[k].ctx) {
        mem[k].ctx->err = "a context appears twice in the group";
        return NF_EINVAL;
      }
  }
  std::vector<int64_t> limit(n);
  for (int k = 0; k < n; ++k) {
    nf_ctx* c = mem[k].ctx;
    const int code = guarded(c, [&] {
      limit[k] = batch_fit_prepare(c, mem[k].B, mem[k].start, mem[k].fixed, mem[k].data_idx, opts);
      return NF_OK;
    });
    if (code != NF_OK) return code;
  }
  nf_ctx* c0 = mem[0].ctx;
  return guarded(c0, [&] {
    hipStream_t s0 = c0->stream;
    std::vector<hipStream_t> side(n, nullptr);
    std::vector<hipEvent_t> ev(n, nullptr);
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&] {
      if (exec) (void)hipGraphExecDestroy(exec);
      for (auto& x : side)
        if (x) (void)hipStreamDestroy(x);
      for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    };
    try {
      for (int k = 0; k < n; ++k) {
        hip_check(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming), "hipEventCreate");
        if (k > 0) hip_check(hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking), "hipStreamCreate");
      }
      hip_check(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      hipError_t e = hipEventRecord(ev[0], s0);
      for (int k = 1; k < n && e == hipSuccess; ++k) e = hipStreamWaitEvent(side[k], ev[0], 0);
      for (int k = 0; k < n && e == hipSuccess; ++k)
        e = batch_fit_iterations(mem[k].ctx, mem[k].B, k == 0 ? s0 : side[k]);
      for (int k = 1; k < n && e == hipSuccess; ++k) {
        e = hipEventRecord(ev[k], side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s0, ev[k], 0);
      }
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(s0, &g);
      if (e != hipSuccess && g) (void)hipGraphDestroy(g);
      hip_check(e, "group capture");
      hip_check(e2, "hipStreamEndCapture");
      const hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      hip_check(e3, "hipGraphInstantiate");
      std::vector<bool> done(n, false);
      for (int64_t launched = 0;; launched += FIT_CHUNK) {
        hip_check(hipGraphLaunch(exec, s0), "hipGraphLaunch");
        for (int k = 0; k < n; ++k) batch_fit_headers_d2h(mem[k].ctx, mem[k].B, s0);
        hip_check(hipStreamSynchronize(s0), "hipStreamSynchronize");
        bool any = false;
        for (int k = 0; k < n; ++k) {
          if (done[k]) continue;
          if (!batch_fit_running(mem[k].ctx, mem[k].B)) {
            done[k] = true;
          } else if (launched + FIT_CHUNK >= limit[k]) {
            batch_fit_stop(mem[k].ctx, mem[k].B);
            done[k] = true;
          } else {
            any = true;
          }
        }
        if (!any) break;
      }
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
    int worst = NF_OK;
    for (int k = 0; k < n; ++k) {
      const nf_batch_member& m = mem[k];
      const int code = batch_fit_collect(m.ctx, m.B, m.theta_out, m.nll_out, m.edm_out, m.status_out, m.iters_out,
                                         m.evals_out);
      if (code != NF_OK) worst = code;
    }
    if (worst != NF_OK) c0->err = "some fits did not converge (see each member's status)";
    return worst;
  });
}


}  // namespace

extern "C" {

int nf_create(nf_ctx** out, const char* model_json, int mode, void* hip_stream) {
  if (!out) return NF_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  if (!model_json) { g_create_error = "model_json is null"; return NF_EINVAL; }
  if (mode != NF_M64 && mode != NF_M32) { g_create_error = "mode must be NF_M64 or NF_M32"; return NF_EINVAL; }
  nf_ctx* c = nullptr;
  try {
    c = new nf_ctx();
    c->mode = mode;
    parse_model(c, model_json);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(NF_EDEVICE, "no HIP device available");
    if (hip_stream) c->stream = static_cast<hipStream_t>(hip_stream);
    else {
      hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate");
      c->own_stream = true;
    }
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    c->scratch_dev = scratch_address();
    if (!c->scratch_dev) fail(NF_EDEVICE, "hipGetSymbolAddress of the static scratch array failed");
    int maxlds = 0;
    hip_check(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "attribute");
    c->max_lds = maxlds;
    // budget for 512 bin-stage threads (the default); 1024 threads need a
    // larger reduction scratch and are refused where they do not fit
    while (c->plan.fit_m > 4 && tail_lds_bytes(c->plan, 512) > (size_t)maxlds) c->plan.fit_m -= 2;
    c->fit_m = c->plan.fit_m;
    const size_t need = tail_lds_bytes(c->plan, 512);
    if (need > (size_t)maxlds)
      fail(NF_EINVAL, "model too large for one workgroup's LDS (" + std::to_string(need) + " > " +
                          std::to_string(maxlds) + " bytes)");
    if (maxlds > 65536) hip_check(tail_set_lds_limit((size_t)maxlds), "hipFuncSetAttribute");
    upload_plan(c);
    hip_check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    *out = c;
    return NF_OK;
  } catch (const ApiError& e) {
    g_create_error = e.what();
    delete c;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    delete c;
    return NF_ENOMEM;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    delete c;
    return NF_EINVAL;
  }
}

void nf_destroy(nf_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

const char* nf_last_error(const nf_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int nf_num_params(const nf_ctx* ctx) { return ctx ? ctx->P : NF_EINVAL; }
int nf_num_datasets(const nf_ctx* ctx) { return ctx ? (int)ctx->ds.size() : NF_EINVAL; }
int nf_num_bins(const nf_ctx* ctx, int d) {
  if (!ctx || d < 0 || d >= (int)ctx->ds.size()) return NF_EINVAL;
  return ctx->ds[d].Nb;
}
int nf_param_index(const nf_ctx* ctx, const char* name) {
  if (!ctx || !name) return NF_EINVAL;
  auto it = ctx->index.find(name);
  return it == ctx->index.end() ? NF_EINVAL : it->second;
}

int nf_set_events(nf_ctx* ctx, int dataset, int64_t n, const double* e_true, const double* e_reco,
                  const uint8_t* source, const float* weight, int on_device) {
  return guarded(ctx, [&] {
    set_events_impl(ctx, dataset, n, e_true, e_reco, source, weight, on_device);
    return NF_OK;
  });
}

int64_t nf_dropped_events(const nf_ctx* ctx, int dataset) {
  if (!ctx || dataset < 0 || dataset >= (int)ctx->ds.size()) return NF_EINVAL;
  return ctx->ds[dataset].dropped;
}

int nf_set_data(nf_ctx* ctx, int dataset, int nbins, const double* counts, int on_device) {
  return guarded(ctx, [&] {
    if (dataset < 0 || dataset >= (int)ctx->ds.size()) fail(NF_EINVAL, "dataset index out of range");
    HostDataset& d = ctx->ds[dataset];
    if (nbins != d.Nb) fail(NF_EINVAL, "nbins does not match the dataset's analysis bins");
    if (!counts) fail(NF_EINVAL, "counts is null");
    std::vector<double> v(nbins);
    hip_check(hipMemcpy(v.data(), counts, sizeof(double) * nbins,
                        on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost), "copy counts");
    for (double x : v)
      if (!(std::isfinite(x) && x >= 0.0)) fail(NF_EINVAL, "counts must be finite and >= 0");
    d.data = v;
    hip_check(hipMemcpyAsync(ctx->d_data.p + d.bins0, d.data.data(), sizeof(double) * nbins,
                             hipMemcpyHostToDevice, ctx->stream), "data H2D");
    hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    d.has_data = true;
    return NF_OK;
  });
}

int nf_eval_nll(nf_ctx* ctx, const double* theta, double* nll) {
  return guarded(ctx, [&] {
    if (!nll) fail(NF_EINVAL, "nll is null");
    return eval_host(ctx, theta, nll, nullptr, nullptr);
  });
}

int nf_eval_nll_grad(nf_ctx* ctx, const double* theta, double* nll, double* grad) {
  return guarded(ctx, [&] {
    if (!nll || !grad) fail(NF_EINVAL, "null output");
    return eval_host(ctx, theta, nll, grad, nullptr);
  });
}

int nf_expected(nf_ctx* ctx, const double* theta, double* mu) {
  return guarded(ctx, [&] {
    if (!mu) fail(NF_EINVAL, "mu is null");
    return eval_host(ctx, theta, nullptr, nullptr, mu);
  });
}

int nf_eval_device(nf_ctx* ctx, const double* theta_dev, double* out_dev, int32_t* status_dev, int want_grad) {
  return guarded(ctx, [&] {
    require_ready(ctx, true);
    if (!theta_dev || !out_dev) fail(NF_EINVAL, "null device pointer");
    release_rows(ctx);
    enqueue_eval(ctx, theta_dev, out_dev, status_dev, nullptr, 1, want_grad ? 1 : 0);
    return NF_OK;
  });
}

int nf_eval_device_noalloc(nf_ctx* ctx, const double* theta_dev, double* out_dev, int32_t* status_dev,
                           int want_grad) {
  return guarded(ctx, [&] {
    require_ready(ctx, true);
    if (!theta_dev || !out_dev) fail(NF_EINVAL, "null device pointer");
    nf_ctx* c = ctx;
    if (!c->scratch_dev) fail(NF_EDEVICE, "no static scratch array on this device");
    // layout: the part that must start at zero (fine-bin rows, per-segment
    // spectra of segments without events, arrival counters) first, cleared by
    // a fill kernel on every call; then fold partials and segment moments,
    // which every call writes before it reads them
    const size_t G = (size_t)std::max(1, c->plan.G), KT = (size_t)std::max(1, c->plan.KT);
    const size_t NI = (size_t)std::max(1, c->nitems);
    const size_t NM = (size_t)num_moments(c->osc.formula);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_bin = 0;
    const size_t o_Sseg = o_bin + up(sizeof(double) * 6 * KT);
    const size_t o_seg_cnt = o_Sseg + up(sizeof(double) * G);
    const size_t o_kt_cnt = o_seg_cnt + up(sizeof(int) * G);
    const size_t zero_end = o_kt_cnt + up(sizeof(int) * KT);
    const size_t o_part = zero_end;
    const size_t o_segm = o_part + up(sizeof(double) * NM * NI);
    const size_t o_pre = o_segm + up(sizeof(double) * (MAX_MOM + 1) * G);
    const size_t total = o_pre + up(sizeof(double) * (size_t)c->plan.pre_total);
    if (total > (size_t)NF_NOALLOC_SCRATCH_BYTES)
      fail(NF_EINVAL, "this context needs " + std::to_string(total) + " bytes of evaluation scratch, more than "
                      "the " + std::to_string((size_t)NF_NOALLOC_SCRATCH_BYTES) + " of the static array; use nf_eval_device");
    unsigned char* base = static_cast<unsigned char*>(c->scratch_dev);
    const EvalScratch sc{reinterpret_cast<double*>(base + o_part), reinterpret_cast<double*>(base + o_segm),
                         reinterpret_cast<double*>(base + o_Sseg), reinterpret_cast<double*>(base + o_bin),
                         reinterpret_cast<int*>(base + o_seg_cnt), reinterpret_cast<int*>(base + o_kt_cnt),
                         reinterpret_cast<double*>(base + o_pre)};
    hip_check(launch_zero(reinterpret_cast<double*>(base), (int64_t)(zero_end / sizeof(double)), c->stream),
              "zero launch");
    enqueue_eval(c, theta_dev, out_dev, status_dev, nullptr, 1, want_grad ? 1 : 0, false, false, false, false, &sc);
    return NF_OK;
  });
}

int nf_eval_device_many(nf_ctx* ctx, int n, const double* theta_dev, double* out_dev, int32_t* status_dev,
                        int want_grad) {
  return guarded(ctx, [&] {
    require_ready(ctx, true);
    if (n < 1 || n > NF_MAX_GRAPH_EVALS) fail(NF_EINVAL, "n must be in 1.." + std::to_string(NF_MAX_GRAPH_EVALS));
    if (!theta_dev || !out_dev) fail(NF_EINVAL, "null device pointer");
    nf_ctx* c = ctx;
    release_rows(c);
    const int g = want_grad ? 1 : 0;
    if (!(c->ev_graph && c->ev_n == n && c->ev_grad == g && c->ev_theta == theta_dev && c->ev_out == out_dev &&
          c->ev_status == status_dev)) {
      if (c->ev_graph) (void)hipGraphExecDestroy(c->ev_graph);
      c->ev_graph = nullptr;
      c->ev_n = 0;
      hip_check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        for (int i = 0; i < n; ++i)
          enqueue_eval(c, theta_dev + (size_t)i * c->P, out_dev + (size_t)i * (1 + c->P),
                       status_dev ? status_dev + i : nullptr, nullptr, 1, g, false, false);
      } catch (...) {
        hipGraph_t gr = nullptr;
        (void)hipStreamEndCapture(c->stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      hipGraph_t gr = nullptr;
      hip_check(hipStreamEndCapture(c->stream, &gr), "hipStreamEndCapture");
      const hipError_t e = hipGraphInstantiate(&c->ev_graph, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      hip_check(e, "hipGraphInstantiate");
      c->ev_n = n;
      c->ev_grad = g;
      c->ev_theta = theta_dev;
      c->ev_out = out_dev;
      c->ev_status = status_dev;
    }
    hip_check(hipGraphLaunch(c->ev_graph, c->stream), "hipGraphLaunch");
    return NF_OK;
  });
}

int nf_set_option(nf_ctx* ctx, const char* key, int64_t value) {
  return guarded(ctx, [&] {
    if (!key) fail(NF_EINVAL, "key is null");
    const std::string k = key;
    if (k == "chunk") {
      if (value < 256 || value % 256 != 0 || value > (1 << 24)) fail(NF_EINVAL, "chunk must be a multiple of 256");
      ctx->chunk = value;
      bool any = false;
      for (auto& d : ctx->ds) any = any || d.has_events;
      if (any) rebuild_events(ctx);
    } else if (k == "fold_block") {
      if (value != 64 && value != 128 && value != 256) fail(NF_EINVAL, "fold_block must be 64, 128 or 256");
      ctx->fold_block = (int)value;
      drop_fit_graph(ctx);
    } else if (k == "tail_threads") {
      if (value != 256 && value != 512 && value != 1024) fail(NF_EINVAL, "tail_threads must be 256, 512 or 1024");
      if (!tail_fits(ctx, (int)value)) fail(NF_EINVAL, "not enough LDS for " + std::to_string(value) + " threads");
      ctx->tail_threads = (int)value;
      drop_fit_graph(ctx);
    } else if (k == "batch_threads") {
      if (value != 0 && value != 256 && value != 512 && value != 1024)
        fail(NF_EINVAL, "batch_threads must be 0, 256, 512 or 1024");
      if (value && !tail_fits(ctx, (int)value)) fail(NF_EINVAL, "not enough LDS for " + std::to_string(value) + " threads");
      ctx->batch_threads_opt = (int)value;
      drop_fit_graph(ctx);
    } else if (k == "batch_fit_tile") {
      if (value != 1 && value != 2 && value != 4 && value != 8) fail(NF_EINVAL, "batch_fit_tile must be 1, 2, 4 or 8");
      ctx->batch_tile = (int)value;
      drop_fit_graph(ctx);
    } else if (k == "deterministic") {
      if (value != 0 && value != 1) fail(NF_EINVAL, "deterministic must be 0 or 1");
      ctx->deterministic = (int)value;
      drop_fit_graph(ctx);
    } else if (k == "timing") {
      ctx->timing = value ? 1 : 0;
      ctx->tcount = 0;
    } else if (k == "stage_cache") {
      if (value != 0 && value != 1) fail(NF_EINVAL, "stage_cache must be 0 or 1");
      ctx->stage_cache = (int)value;
      if (!value) release_rows(ctx);
    } else {
      fail(NF_EINVAL, "unknown option '" + k + "'");
    }
    return NF_OK;
  });
}

int nf_get_option(nf_ctx* ctx, const char* key, int64_t* value) {
  return guarded(ctx, [&] {
    if (!key || !value) fail(NF_EINVAL, "key and value are required");
    const std::string k = key;
    if (k == "chunk") *value = ctx->chunk;
    else if (k == "fold_block") *value = ctx->fold_block;
    else if (k == "tail_threads") *value = ctx->tail_threads;
    else if (k == "batch_threads") *value = ctx->batch_threads_opt;
    else if (k == "batch_fit_tile") *value = ctx->batch_tile;
    else if (k == "deterministic") *value = ctx->deterministic;
    else if (k == "timing") *value = ctx->timing;
    else if (k == "stage_cache") *value = ctx->stage_cache;
    else fail(NF_EINVAL, "unknown option '" + k + "'");
    return NF_OK;
  });
}

int nf_set_data_batch(nf_ctx* ctx, int nsets, const double* counts, int on_device) {
  return guarded(ctx, [&] {
    if (nsets <= 0 || !counts) fail(NF_EINVAL, "nsets > 0 and counts are required");
    const size_t n = (size_t)nsets * ctx->nbins_total;
    std::vector<double> v(n);
    hip_check(hipMemcpy(v.data(), counts, sizeof(double) * n, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost),
              "copy counts");
    for (double x : v)
      if (!(std::isfinite(x) && x >= 0.0)) fail(NF_EINVAL, "counts must be finite and >= 0");
    ctx->bt_data.upload(v, ctx->stream);
    hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    ctx->bt_nsets = nsets;
    drop_fit_graph(ctx);
    return NF_OK;
  });
}

int nf_timing_overhead(nf_ctx* ctx, int n, double* us) {
  return guarded(ctx, [&] {
    if (n < 1 || !us) fail(NF_EINVAL, "n >= 1 and us are required");
    hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
      EventPair ev;
      hip_check(hipEventRecord(ev.a, ctx->stream), "hipEventRecord");
      hip_check(hipEventRecord(ev.b, ctx->stream), "hipEventRecord");
      total += ev.us_per(1);
    }
    *us = total / n;
    return NF_OK;
  });
}

int nf_autotune(nf_ctx* ctx, const double* theta, int evals, int batch, int64_t* best, double* best_us) {
  return guarded(ctx, [&] { return autotune_impl(ctx, theta, evals, batch, best, best_us); });
}

int nf_expected_batch(nf_ctx* ctx, int B, const double* theta, double* mu) {
  return guarded(ctx, [&] { return expected_batch_impl(ctx, B, theta, mu); });
}

int nf_eval_batch(nf_ctx* ctx, int B, const double* theta, const int* data_idx, double* nll, double* grad) {
  return guarded(ctx, [&] { return eval_batch_impl(ctx, B, theta, data_idx, nll, grad); });
}

int nf_fit_batch(nf_ctx* ctx, int B, const double* start, const uint8_t* fixed, const int* data_idx,
                 const nf_fit_opts* opts, double* theta_out, double* nll_out, double* edm_out, int* status_out,
                 int* iters_out, int* evals_out) {
  return guarded(ctx, [&] {
    return fit_batch_impl(ctx, B, start, fixed, data_idx, opts, theta_out, nll_out, edm_out, status_out, iters_out,
                          evals_out);
  });
}

int nf_set_surrogate(nf_ctx* ctx, nf_mlp* net, int n_in, const int* param_index, const double* center,
                     const double* half, const float* out_mean, const float* out_std, const float* x_prior,
                     const float* x_weight, int n_starts, const float* starts, int iters, float lr) {
  return guarded(ctx, [&] {
    auto& s = ctx->sur;
    if (!net) {
      s = nf_ctx::Surrogate{};
      return NF_OK;
    }
    int ni = 0, no = 0, mb = 0;
    if (mlp_shape(net, &ni, &no, &mb) != NF_OK) fail(NF_EINVAL, "bad network handle");
    if (n_in != ni) fail(NF_EINVAL, "n_in differs from the network's input width");
    if (no != ctx->nbins_total) fail(NF_EINVAL, "the network's outputs must cover every analysis bin");
    if (n_starts < 1 || iters < 1 || !(lr > 0.f)) fail(NF_EINVAL, "n_starts, iters and lr must be positive");
    if (!param_index || !center || !half || !out_mean || !out_std || !x_prior || !x_weight || !starts)
      fail(NF_EINVAL, "null array");
    for (int i = 0; i < n_in; ++i) {
      if (param_index[i] < 0 || param_index[i] >= ctx->P) fail(NF_EINVAL, "parameter index out of range");
      if (!std::isfinite(center[i]) || !(half[i] > 0.0)) fail(NF_EINVAL, "center must be finite and half > 0");
    }
    nf_ctx::Surrogate t;
    t.net = net;
    t.n_in = n_in;
    t.n_out = no;
    t.max_batch = mb;
    t.n_starts = n_starts;
    t.iters = iters;
    t.lr = lr;
    t.idx.assign(param_index, param_index + n_in);
    t.center.assign(center, center + n_in);
    t.half.assign(half, half + n_in);
    t.out_mean.assign(out_mean, out_mean + no);
    t.out_std.assign(out_std, out_std + no);
    t.x_prior.assign(x_prior, x_prior + n_in);
    t.x_weight.assign(x_weight, x_weight + n_in);
    t.starts.assign(starts, starts + (size_t)n_starts * n_in);
    s = std::move(t);
    return NF_OK;
  });
}

int nf_fit_batch_group(int n, const nf_batch_member* members, const nf_fit_opts* opts) {
  return fit_batch_group_impl(n, members, opts);
}

int nf_fit(nf_ctx* ctx, const double* start, const uint8_t* fixed, const nf_fit_opts* opts,
           nf_fit_result* result) {
  return guarded(ctx, [&] { return fit_impl(ctx, start, fixed, opts, result); });
}

int nf_timing(nf_ctx* ctx, int reset, int64_t* count, double* fold_ms, double* tail_ms) {
  return guarded(ctx, [&] {
    hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    double f = 0.0, t = 0.0;
    for (size_t i = 0; i < ctx->tcount; ++i) {
      float a = 0.f, b = 0.f;
      hip_check(hipEventElapsedTime(&a, ctx->tev[i][0], ctx->tev[i][1]), "hipEventElapsedTime");
      hip_check(hipEventElapsedTime(&b, ctx->tev[i][2], ctx->tev[i][3]), "hipEventElapsedTime");
      f += a;
      t += b;
    }
    if (count) *count = (int64_t)ctx->tcount;
    if (fold_ms) *fold_ms = f;
    if (tail_ms) *tail_ms = t;
    if (reset) ctx->tcount = 0;
    return NF_OK;
  });
}

}  // extern "C"
