// Flat, device-readable description of a model (built once by the host
// runtime from the JSON description) and of the sorted event stream.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace nufold {

constexpr int FORM_EQ1 = 0;  // Eq. 1: slots sin2_2t13, dm2_ee, sin2_t12, dm2_21
constexpr int FORM_3NU = 1;  // exact vacuum 3-flavour: sin2_t12, sin2_t13, dm2_21, dm2_31
constexpr int FORM_4NU = 2;  // vacuum 3+1: sin2_t13, dm2_31, sin2_2t14, dm2_41 (sin2_t12, dm2_21 constants)
constexpr int FORM_MATTER = 3;  // exact 3-flavour in matter of constant density: the 3nu slots (rho Y_e constant)
constexpr int NSLOT = 4;
constexpr int MAX_MOM = 12;  // per-segment moments produced by the fold
constexpr int MAX_SOURCES = 64;
constexpr int FLUX_FW_MAX = 8;  // flux modes non-zero in one fine bin (fixed-width rows)
// Oscillation coefficient rows: row 0 gives S, rows 1..4 dS/d(slot j), each a
// linear combination of (W, M_1..M_NM) stored at CF_STRIDE doubles per row.
constexpr int CF_STRIDE = 16;
constexpr int CF_SIZE = 5 * CF_STRIDE;

// 2 k, k = 1/(4 hbar c) in MeV/(eV^2 m) with the exact SI-2019 value of hbar c;
// the fold phase x = 2 k dm2 L/E is twice the phase of Eq. 1.
constexpr double TWO_PHASE_K = 2.0 * 1.266932679039099;
constexpr double UNIT_1EM3 = 1e-3;
constexpr double UNIT_1EM5 = 1e-5;

// Matter potential of electron antineutrinos: A = 2 sqrt(2) G_F N_e E in
// eV^2 is MATTER_A_PER_MEV rho Y_e E[MeV] for a density rho in g/cm^3 with
// Y_e electrons per nucleon (N_e = rho Y_e N_A per cm^3, one gram per mole of
// nucleons), from G_F = 1.1663787e-5 GeV^-2, hbar c = 1.973269804593025e-14
// GeV cm (exact SI-2019 value) and N_A = 6.02214076e23 / mol:
//   sqrt(2) G_F (hbar c)^3 N_A = 7.6325e-14 eV per g/cm^3, times 2 E = 2e6 eV per MeV.
constexpr double MATTER_GF = 1.1663787e-5;
constexpr double MATTER_HBARC_CM = 1.973269804593025e-14;
constexpr double MATTER_NA = 6.02214076e23;
constexpr double MATTER_A_PER_MEV = 2.0e6 * 1.4142135623730950488 * MATTER_GF * MATTER_HBARC_CM * MATTER_HBARC_CM *
                                    MATTER_HBARC_CM * MATTER_NA * 1e9;

// moments the fold produces per segment (the matter form: S and its four slot
// derivatives directly)
__host__ __device__ inline int num_moments(int formula) {
  return formula == FORM_EQ1 ? 4 : formula == FORM_3NU ? 6 : formula == FORM_MATTER ? 5 : 12;
}

struct OscPlan {
  int formula;
  int slot_param[NSLOT];   // parameter index, or -1 for a constant
  int fp32_phase;          // 1: the fold forms phases from FP32 frequencies (M32); the
                           // coefficient rows then carry the first-order frequency correction
  int pad_;
  double slot_value[NSLOT];
  double cst[2];           // FORM_4NU: the fixed sin2_t12 and dm2_21 (1e-5 eV^2);
                           // FORM_MATTER: cst[0] = MATTER_A_PER_MEV rho Y_e
};

// A contiguous run of sorted events that all belong to one segment
// (dataset, source, fine bin). begin and count are multiples of 4.
struct WorkItem {
  int64_t begin;
  int32_t count;
  int32_t seg;
};

// What the single evaluation's fold epilogue needs about a work item, read at
// the start of the wavefront so nothing is loaded after the event stream.
constexpr int NLMAX = 8;  // norm parameters multiplying one source
struct ItemEpi {
  double W;           // summed weights of the item's segment
  int32_t row;        // the segment's fine bin in the row block: 6 kt0 + (kt - kt0)
  int32_t K;          // row stride (fine bins of the dataset)
  int32_t first;      // first work item of the segment
  int32_t nseg;       // work items of the segment
  int32_t nl[NLMAX];  // the source's norm parameters (-1: none)
  int32_t pad_[2];
};
static_assert(sizeof(ItemEpi) == 64, "ItemEpi is 64 bytes");

struct BkgPlan {
  double scale;
  int rate;    // parameter index or -1 (rate fixed at 1)
  int tmpl;    // dpool offset of Nb template values
  int shape;   // ipool offset of Nb parameter indices (-1 entries: none), or -1
  int pad_;
};

struct DsPlan {
  double y0, wf;
  int K, Nb, S, M, nbkg;
  int seg0;         // global segment index of (source 0, fine bin 0); segment = seg0 + s*K + k
  int kt0;          // global index of fine bin 0 of this dataset
  int fs0;          // flat (all-dataset) index of source 0
  int edges;        // dpool: Nb + 1 analysis edges
  int data;         // offset into the data vector (Nb counts)
  int bins0;        // offset into concatenated analysis bins (same as data)
  int srcnorm_ptr;  // ipool: S + 1 absolute ipool offsets of each source's norm list
  int nl0, nl;      // ipool offset and total length of this dataset's norm lists
  int fx_row;       // ipool: K + 1 absolute offsets into fx_mode / dpool fx_coef (CSR over k)
  int fx_mode;      // ipool base of CSR mode indices (0..M-1)
  int fx_coef;      // dpool base of CSR coefficients
  int md_col;       // ipool: M + 1 absolute offsets (CSC over modes)
  int md_k;         // ipool base of CSC fine-bin indices
  int md_coef;      // dpool base of CSC coefficients
  int md_param;     // ipool: M parameter indices
  int nnz;          // number of non-zero basis entries
  int cidx[3];      // energy-scale parameters c0, c1, c2 (-1: fixed at 0)
  int bkg0;         // index of the first BkgPlan
  int blob, blob_n; // dpool offset and length of the static blob (layout: blob_layout)
  int fw;           // flux basis entries per fine bin in the blob's fixed-width rows (>= 1)
  int pre0;         // this dataset's block of the parameter-pass buffer (layout: pre_layout; even)
  int pad_[2];
};

static_assert(sizeof(DsPlan) % sizeof(double) == 0, "DsPlan is copied as doubles");
constexpr int DSPLAN_DOUBLES = (int)(sizeof(DsPlan) / sizeof(double));

// Per-dataset static inputs of the bin stages, packed contiguously. Offsets
// count doubles; the integer arrays hold 32-bit integers, two per double
// slot. The first hpart doubles are what the stages read from LDS: the
// parameters of the background rates and shapes (read by the analysis-bin
// pass; the first `early` doubles), then the flux modes by column and the
// source norm lists (read only by the gradient's last pass). The rest (edges,
// background templates, the flux basis by fine bin in rows of fixed width fw,
// unused entries with parameter -1) is read by the parameter pass, each
// thread into registers, every load independent of the others.
struct BlobLayout {
  int brt, shp, early, mdc, mdcol, mdk, mdp, nlp, nli, hpart;
  int edges, tmpl, bsc, fcf, fpar, total;
};
__host__ __device__ inline BlobLayout blob_layout(int E, int B, int Nb, int nnz, int M, int S, int nl, int K,
                                                  int fw) {
  auto ints = [](int n) { return (n + 1) / 2; };  // double slots for n int32 values
  BlobLayout L;
  int o = 0;
  L.brt = o; o += ints(B);        // rate parameter of each background (-1: none)
  L.shp = o; o += ints(B * Nb);   // shape parameter of each (background, bin) (-1: none)
  o += o & 1;
  L.early = o;                    // (16-byte aligned)
  L.mdc = o; o += nnz;           // flux basis by mode (CSC): coefficients,
  L.mdcol = o; o += ints(M + 1);  // column pointers,
  L.mdk = o; o += ints(nnz);      // fine bin of each entry,
  L.mdp = o; o += ints(M);        // parameter of each mode
  L.nlp = o; o += ints(S + 1);    // norm list of each source: pointers,
  L.nli = o; o += ints(nl);       // parameter indices
  o += o & 1;                     // the global part starts 16-byte aligned
  L.hpart = o;
  L.edges = o; o += E;
  L.tmpl = o; o += B * Nb;
  L.bsc = o; o += B;
  L.fcf = o; o += K * fw;         // flux basis by fine bin, fw entries per bin: coefficients,
  L.fpar = o; o += ints(K * fw);  // parameter of each entry (-1: unused)
  L.total = o;
  return L;
}

// One dataset's block of the parameter-pass buffer (written by the fold
// launch for the single evaluation), in the order the bin stages hold it in
// LDS, so that one copy moves it: 1 + F per fine bin, the background
// expectation and its rate and shape factors per analysis bin, then per
// mapped edge t, y, 1 / f'(y) and the fine bin (int32, two per slot).
// Offsets in doubles; the total is even (16-byte aligned blocks).
struct PreLayout {
  int F1, B, bkr, bks, et, ey, eq, ek, total;
};
__host__ __device__ inline PreLayout pre_layout(int K, int Nb, int NB) {
  PreLayout L;
  const int E = Nb + 1, BN = NB * Nb;
  int o = 0;
  L.F1 = o; o += K;
  L.B = o; o += Nb;
  L.bkr = o; o += BN;
  L.bks = o; o += BN;
  L.et = o; o += E;
  L.ey = o; o += E;
  L.eq = o; o += E;
  L.ek = o; o += (E + 1) / 2;
  o += o & 1;
  L.total = o;
  return L;
}

struct DevPlan {
  int P, D, G, nitems, nbins_total;
  int KT, FS;            // total fine bins, total sources over all datasets
  int max_K, max_Nb, max_S, max_B, max_M, max_nnz, max_nl;
  OscPlan osc;
  const DsPlan* ds;
  DsPlan ds0;            // copy of ds[0] (read from the kernel arguments)
  const BkgPlan* bkg;
  const double* dpool;
  const int* ipool;
  int seg_fs;            // ipool: G flat source index of each segment
  int kt_ds;             // ipool: KT dataset index of each global fine bin
  int fs_ptr;            // ipool: 2 FS, [begin, end) absolute ipool offsets of each source's norm list
  int max_blob;          // largest LDS part (hpart) of a static blob
  int fit_m;             // minimiser history length (LDS is reserved for it)
  int kt_info;           // ipool: 5 KT: first segment, stride K, sources S, first flat source, kt0
  int fs_nl;             // ipool: NLMAX FS norm-list parameter indices per flat source (-1 padded)
  int kt_row;            // ipool: KT + 1 flux-basis row pointers per global fine bin (relative)
  int kt_par;            // ipool base: parameter index of each row entry
  int kt_coef;           // dpool base: coefficient of each row entry
  int NR;                // prior rows: ngauss Gaussian rows, then one row per block-prior entry
  int prow_blk;          // ipool: NR - ngauss block index of each block-prior row
  const int* seg_item;   // G + 1: work-item range of each segment
  const double* Wseg;    // G: sum of weights of each segment (static)
  // priors
  int ngauss;
  int gidx, gmean, ginv;        // ipool / dpool / dpool offsets (ginv = 1/sigma^2)
  int nblk;
  int blk_ptr;                  // ipool: nblk + 1 offsets into blk_idx (and blk_mean)
  int blk_idx;                  // ipool base
  int blk_mean;                 // dpool base (aligned with blk_idx)
  int blk_inv;                  // ipool: nblk offsets into dpool of row-major V^-1
  // parameter-pass buffer of the single evaluation (doubles; written by extra
  // workgroups of the fold launch, read by the bin stages): one block per
  // dataset (DsPlan::pre0, pre_layout), then one contiguous block of
  int pre_prv;   // NR: gradient contribution of each prior row,
  int pre_pri;   // (NR + 1) / 2: parameter of each prior row (int32),
  int pre_misc;  // 2 + D: prior NLL, parameter-domain flag, energy-map domain flag per dataset
  int pre_glob;  // doubles of that block (pre_prv .. pre_misc + 2 + D)
  int max_pre;   // largest dataset block
  int pre_total; // doubles of the buffer
};

}  // namespace nufold
